"""Reader for the text fixtures under tests/golden/ (exact rationals)."""
import os
from fractions import Fraction

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_fixture(name):
    """Returns {key: [list of Fraction rows]} (keys may repeat, e.g. 'edge')."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out.setdefault(key, []).append([Fraction(v) for v in vals])
    return out


def as_floats(row):
    return [float(v) for v in row]
