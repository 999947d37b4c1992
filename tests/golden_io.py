"""Readers for the text fixtures under tests/golden/ (no arithmetic of the method)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _entry(tok: str) -> complex:
    tok = tok.strip()
    if tok.endswith("i"):
        coef = tok[:-1]
        if coef in ("", "+"):
            return 1j
        if coef == "-":
            return -1j
        return complex(0.0, float(coef))
    return complex(float(tok), 0.0)


def read_projectors(name: str) -> dict:
    """{('+', mu) or ('-', mu): 4x4 complex ndarray} with mu = 1..4."""
    out, key, rows = {}, None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("P"):
                key, rows = (line[1], int(line[2])), []
                continue
            rows.append([_entry(t) for t in line.split()])
            if len(rows) == 4:
                out[key] = np.array(rows, dtype=np.complex128)
    return out
