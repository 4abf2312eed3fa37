"""Readers for the text fixtures under tests/golden/ (numbers printed in
the paper; each file states where every block comes from)."""
import os
from fractions import Fraction

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def sections(name: str) -> dict:
    out, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                out[cur] = []
                continue
            out[cur].append(line.split())
    return out


def matrices() -> dict:
    """Printed matrices as lists of lists of Fractions."""
    return {k: [[Fraction(v) for v in row] for row in rows]
            for k, rows in sections("matrices.txt").items()}


def paper_tables() -> dict:
    return sections("paper_tables.txt")
