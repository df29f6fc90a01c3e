"""Readers for the text fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def philox_kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((tuple(v[0:4]), tuple(v[4:6]), tuple(v[6:10])))
    return rows
