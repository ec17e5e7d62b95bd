"""Loaders for the hand-derived fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def quarter_turns():
    """Returns (z [3, 4] complex128, expected: dict (i, j) -> (ReG, ImG, plv, iplv, ciplv))."""
    sigs = {}
    pairs = {}
    with open(os.path.join(HERE, "quarter_turns.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "sig":
                bar = tok.index("|")
                q = [int(v) for v in tok[2:bar]]
                a = [float(v) for v in tok[bar + 1:]]
                sigs[int(tok[1])] = [amp * (1j ** qq) for qq, amp in zip(q, a)]
            elif tok[0] == "pair":
                pairs[(int(tok[1]), int(tok[2]))] = tuple(float(v) for v in tok[3:8])
    z = np.array([sigs[k] for k in sorted(sigs)], dtype=np.complex128)
    # i**q in floating point leaves ~1e-16 residue on the zero component; snap it
    z = np.round(z.real, 12) + 1j * np.round(z.imag, 12)
    return z, pairs
