"""Write the oracle's FC-Gram table files under oracle/data/ (calls only oracle.fcgram).

usage: python -m oracle.make_tables [d ...]
"""
import sys

from oracle import fcgram


def main(argv):
    ds = [int(a) for a in argv] or [5]
    for d in ds:
        t = fcgram.compute_tables(d=d)
        path = fcgram.table_path(d=d)
        fcgram.write_tables(t, path)
        print("wrote", path, "cond %.3e" % t["cond"], "resid", t["residuals"])


if __name__ == "__main__":
    main(sys.argv[1:])
