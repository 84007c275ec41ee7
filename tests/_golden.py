"""Reader for the hand-worked text fixtures under tests/golden/."""
import os
from fractions import Fraction

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read(name):
    """Return {key: [list of rows of Fractions/str]} for one fixture file."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            row = []
            for t in vals:
                try:
                    row.append(Fraction(t))
                except ValueError:
                    row.append(t)
            out.setdefault(key, []).append(row)
    return out
