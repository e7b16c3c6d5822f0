"""Writes gauss_exact.json: closed-form Gauss-Legendre rules for 1..5 nodes.

The nodes are the roots of the Legendre polynomial P_N (the paper's Sec. 2.1
recurrence) and the weights the standard Gauss weights (the rule of eq. gauss,
Sec. 2.3).  Closed forms (textbook, e.g. Abramowitz & Stegun Table 25.4):
  N=1: x = 0, w = 2
  N=2: x = +-1/sqrt3, w = 1
  N=3: x = 0, +-sqrt(3/5); w = 8/9, 5/9
  N=4: x = +-sqrt(3/7 -+ 2/7 sqrt(6/5)); w = (18 +- sqrt30)/36
  N=5: x = 0, +-1/3 sqrt(5 -+ 2 sqrt(10/7)); w = 128/225, (322 +- 13 sqrt70)/900
evaluated here in 50-digit decimal arithmetic, ordered x decreasing.
"""
import json
import os
from decimal import Decimal as D, getcontext

getcontext().prec = 50


def sq(v):
    return D(v).sqrt()


def rule(N):
    if N == 1:
        pts = [(D(0), D(2))]
    elif N == 2:
        pts = [(1 / sq(3), D(1))]
    elif N == 3:
        pts = [(D(0), D(8) / 9), (sq(D(3) / 5), D(5) / 9)]
    elif N == 4:
        pts = [(sq(D(3) / 7 - D(2) / 7 * sq(D(6) / 5)), (18 + sq(30)) / 36),
               (sq(D(3) / 7 + D(2) / 7 * sq(D(6) / 5)), (18 - sq(30)) / 36)]
    else:
        pts = [(D(0), D(128) / 225),
               (sq(5 - 2 * sq(D(10) / 7)) / 3, (322 + 13 * sq(70)) / 900),
               (sq(5 + 2 * sq(D(10) / 7)) / 3, (322 - 13 * sq(70)) / 900)]
    full = {}
    for x, w in pts:
        full[x] = w
        full[-x] = w
    xs = sorted(full, reverse=True)
    return {"x": [float(v) for v in xs], "w": [float(full[v]) for v in xs]}


if __name__ == "__main__":
    out = {"source": "closed-form Gauss-Legendre rules (textbook), see make_gauss_exact.py",
           "rules": {str(N): rule(N) for N in range(1, 6)}}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "gauss_exact.json"), "w") as f:
        json.dump(out, f, indent=1)
