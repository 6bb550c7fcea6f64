"""gamma_2(P_n x C_m) from the paper's closed form (a pin, not the oracle).

gamma_2 = ceil(b_n * m / a_n) + alpha_n(m mod a_n)   (Section 4, with a_n, b_n
from Table 4 and alpha from Table 6), plus the cycle-5 exceptions stated after
the formula, and gamma_2(C_m) = ceil(m / 2) for the one-vertex path (the
textbook value for the 2-domination number of a cycle).  The table is read from
``tests/golden/table6_alpha.txt``.
"""
from __future__ import annotations

import os

_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load():
    rows, exc = {}, {}
    with open(os.path.join(_GOLDEN, "table6_alpha.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            t = line.split()
            if t[0] == "EXC":
                exc[(int(t[1]), int(t[2]))] = int(t[3])
                continue
            n, a, b = int(t[0]), int(t[1]), int(t[2])
            ks = set() if t[3] == "-" else {int(x) for x in t[3].split(",")}
            rows[n] = (a, b, ks, int(t[4]))
    return rows, exc


_ROWS, _EXC = _load()


def gamma2_closed_form(n: int, m: int) -> int:
    if m < 3:
        raise ValueError("m >= 3")
    if n == 1:
        return (m + 1) // 2
    if (n, m) in _EXC:
        return _EXC[(n, m)]
    a, b, ks, min_m = _ROWS[n]
    alpha = 1 if (m % a in ks and m >= min_m) else 0
    return -((-b * m) // a) + alpha
