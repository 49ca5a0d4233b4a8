"""Readers for the transcribed fixtures under tests/golden/."""
import json
import os
from fractions import Fraction

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_matrix(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([Fraction(tok) for tok in line.split()])
    return rows


def paper_values():
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        return json.load(fh)
