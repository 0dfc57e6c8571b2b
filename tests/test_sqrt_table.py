"""Pin of the library's square-root table (csrc/sqrt_table.inc, Sec. 4.4).

The paper approximates sqrt on [0,1] by six (1,1)-rational pieces with an
error below 1e-3.  The table compiled into the library must: span [0,1] in six
pieces; stay below 1e-3 on each piece (dense sampling); be the minimax fit of
each piece, which for a (1,1) rational approximation of sqrt is characterised
by an error curve with four alternating extrema of equal magnitude; and so
agree with the oracle's table, which is fitted by a different method (Remez
exchange instead of differential correction).
"""
import os
import re

import numpy as np

import sqrt_fit

INC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2405_13409_amd", "csrc", "sqrt_table.inc")


def _table():
    txt = open(INC).read()
    ends = [float(v) for v in re.search(r"kSqrtPieceEnds\[7\] = \{([^}]*)\}", txt).group(1).split(",")]
    coef = [float(v) for v in re.search(r"kSqrtCoef\[24\] = \{([^}]*)\}", txt).group(1).split(",")]
    return np.array(ends), np.array(coef).reshape(6, 4)


def _extrema(x, e):
    """Alternating extrema of e: the ends and the interior local extrema, with
    runs of one sign merged to their largest member."""
    idx = [0] + list(np.nonzero((e[1:-1] - e[:-2]) * (e[2:] - e[1:-1]) <= 0)[0] + 1) + [len(e) - 1]
    out = []
    for i in idx:
        if out and np.sign(e[i]) == np.sign(e[out[-1]]):
            if abs(e[i]) > abs(e[out[-1]]):
                out[-1] = i
        else:
            out.append(i)
    return np.array(out)


def test_table_bound_and_alternation():
    ends, coef = _table()
    assert len(ends) == 7 and ends[0] == 0.0 and ends[-1] == 1.0 and np.all(np.diff(ends) > 0)
    for i in range(6):
        a, b = ends[i], ends[i + 1]
        x = np.linspace(a, b, 400001)
        c0, c1, d0, d1 = coef[i]
        assert np.all(d0 + d1 * x > 0)
        e = (c0 + c1 * x) / (d0 + d1 * x) - np.sqrt(x)
        emax = np.abs(e).max()
        assert emax < 1e-3, (i, emax)
        ext = _extrema(x, e)
        big = ext[np.abs(e[ext]) > 0.99 * emax]
        # four alternating extrema of (nearly) the same magnitude
        assert len(big) >= 4, (i, e[ext])
        assert np.all(np.sign(e[big][1:]) == -np.sign(e[big][:-1]))


def test_table_matches_oracle_fit():
    ends, coef = _table()
    ocoef, _ = sqrt_fit.fit_table()
    assert np.allclose(ends, sqrt_fit.BREAKPOINTS)
    for i in range(6):
        a, b = ends[i], ends[i + 1]
        x = np.linspace(a, b, 20001)
        lib = (coef[i][0] + coef[i][1] * x) / (coef[i][2] + coef[i][3] * x)
        orc = (ocoef[i][0] + ocoef[i][1] * x) / (ocoef[i][2] + ocoef[i][3] * x)
        assert np.abs(lib - orc).max() < 1e-6 * max(1e-3, np.sqrt(b))
