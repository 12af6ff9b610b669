"""Loader for the printed-matrix fixtures in tests/golden/printed_matrices.txt."""
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _ev(expr, names):
    if expr.strip() == "":
        return np.nan
    return float(eval(expr, {"__builtins__": {}}, dict(names)))


def printed_matrices(names, corrected=True, which=None):
    """Evaluate every printed matrix for the symbol values in ``names``."""
    mats, fixes, cur, rows = {}, [], None, []
    with open(os.path.join(HERE, "printed_matrices.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("matrix "):
                cur, rows = line.split()[1], []
            elif line == "end":
                mats[cur] = rows
                cur = None
            elif line.startswith("fix "):
                _, m, r, c, v = line.split(None, 4)
                fixes.append((m, int(r) - 1, int(c) - 1, v))
            else:
                rows.append(line.split(";"))
    out = {}
    for k, rows in mats.items():
        if which is not None and k not in which:
            continue
        out[k] = np.array([[_ev(e, names) for e in r] for r in rows])
    if corrected:
        for m, r, c, v in fixes:
            if m in out:
                out[m][r, c] = _ev(v, names)
    return out
