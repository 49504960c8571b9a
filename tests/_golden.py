"""Readers for the text fixtures under tests/golden/ (each cites its source)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def kat_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([int(t, 16) for t in line.split()])
    return rows


def paper_values():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_values.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (t.strip() for t in line.split("=", 1))
                vals[k] = float(v)
    return vals
