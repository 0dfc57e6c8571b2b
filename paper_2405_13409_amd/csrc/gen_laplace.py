"""Generate straight-line HIP code for the one-bounce elimination phase.

For a bivariate system a(u,v) (total degree TA, u-degree TA) and b(u,v) (total
degree TB, u-degree >= N), the emitted device function builds the N x N Bezout
matrix of Eq. (eq_bezout) whose entries are polynomials in v,
    B_ij(v) = sum_{k=0}^{min(i, N-1-j)} a_{i-k}(v) b_{j+1+k}(v) - b_{i-k}(v) a_{j+1+k}(v),
and expands its determinant by Laplace expansion (Sec. 5.2) into the explicit
coefficients of r(v).  The expansion is memoised bottom-up over column subsets:
the minor of rows r..N-1 on the column set S is the cofactor sum along row r
of the entries times the minors of rows r+1..N-1.  Every degree is known at
generation time, so structurally-zero entries and minors are skipped and each
polynomial lives in a fixed-size register array.

Run:  python gen_laplace.py > laplace_gen.inc
"""
from __future__ import annotations

import itertools
import sys

VARIANTS = [
    # name, N, TA, TB
    ("r_interp", 3, 2, 4),
    ("r_flat", 1, 1, 2),
    ("t_interp", 6, 2, 6),
    ("t_flat", 4, 1, 4),
]


def tri_idx(D, i, j):
    """index of u^i v^j in the triangular layout of a degree-D bivariate polynomial"""
    return i * (D + 1) - i * (i - 1) // 2 + j


def emit(name, N, TA, TB, out):
    w = out.append
    DR = N * (TA + TB - 1) - N * (N - 1)
    w(f"// ---- {name}: Bezout {N}x{N}, deg a = {TA}, deg b = {TB}, deg r = {DR}")
    w("template <typename R>")
    w(f"__device__ __forceinline__ void elim_{name}(const R* __restrict__ A, const R* __restrict__ B, R* __restrict__ r)")
    w("{")

    def adeg(i):
        return TA - i if i <= TA else -1

    def bdeg(i):
        return TB - i if i <= TB and i <= N else -1

    def aco(i, k):
        return f"A[{tri_idx(TA, i, k)}]"

    def bco(i, k):
        return f"B[{tri_idx(TB, i, k)}]"

    # Bezout entries
    deg = {}
    for i in range(N):
        for j in range(N):
            terms = []
            for k in range(0, min(i, N - 1 - j) + 1):
                p, q = i - k, j + 1 + k
                if p == q:
                    continue  # a_p b_p - b_p a_p vanishes identically
                if adeg(p) >= 0 and bdeg(q) >= 0:
                    terms.append(("ab", p, q))
                if bdeg(p) >= 0 and adeg(q) >= 0:
                    terms.append(("ba", p, q))
            d = TA + TB - 1 - i - j
            if not terms or d < 0:
                deg[(i, j)] = -1
                continue
            deg[(i, j)] = d
            w(f"  R e{i}_{j}[{d + 1}];")
            acc = {m: [] for m in range(d + 1)}
            for kind, p, q in terms:
                if kind == "ab":
                    for s in range(adeg(p) + 1):
                        for t in range(bdeg(q) + 1):
                            acc[s + t].append(f"{aco(p, s)} * {bco(q, t)}")
                else:
                    for s in range(bdeg(p) + 1):
                        for t in range(adeg(q) + 1):
                            acc[s + t].append(f"-{bco(p, s)} * {aco(q, t)}")
            for m in range(d + 1):
                if acc[m]:
                    expr = acc[m][0]
                    for tterm in acc[m][1:]:
                        if tterm.startswith("-"):
                            expr = f"fma(-{tterm[1:].split(' * ')[0]}, {tterm.split(' * ')[1]}, {expr})"
                        else:
                            a_, b_ = tterm.split(" * ")
                            expr = f"fma({a_}, {b_}, {expr})"
                    if expr.startswith("-"):
                        expr = f"-({expr[1:]})"
                    w(f"  e{i}_{j}[{m}] = {expr};")
                else:
                    w(f"  e{i}_{j}[{m}] = R(0);")

    # bottom-up minors
    minors = {}  # (row, frozenset cols) -> degree
    for k in range(1, N + 1):
        r0 = N - k
        for S in itertools.combinations(range(N), k):
            parts = []
            for pos, j in enumerate(S):
                if deg[(r0, j)] < 0:
                    continue
                rest = tuple(c for c in S if c != j)
                if k > 1:
                    if rest not in minors:
                        continue
                    md = minors[rest]
                else:
                    md = 0
                parts.append((pos, j, rest, deg[(r0, j)] + md))
            if not parts:
                continue
            d = max(p[3] for p in parts)
            minors[S] = d
            mname = "m_" + "_".join(map(str, S))
            w(f"  R {mname}[{d + 1}];")
            for m in range(d + 1):
                w(f"  {mname}[{m}] = R(0);")
            for pos, j, rest, dd in parts:
                sg = "-" if pos % 2 else ""
                ed = deg[(r0, j)]
                if k == 1:
                    for m in range(ed + 1):
                        w(f"  {mname}[{m}] = {sg}e{r0}_{j}[{m}];" if not sg else f"  {mname}[{m}] = -e{r0}_{j}[{m}];")
                else:
                    rn = "m_" + "_".join(map(str, rest))
                    rd = minors[rest]
                    for s in range(ed + 1):
                        for t in range(rd + 1):
                            if sg:
                                w(f"  {mname}[{s + t}] = fma(-e{r0}_{j}[{s}], {rn}[{t}], {mname}[{s + t}]);")
                            else:
                                w(f"  {mname}[{s + t}] = fma(e{r0}_{j}[{s}], {rn}[{t}], {mname}[{s + t}]);")
    full = tuple(range(N))
    fname = "m_" + "_".join(map(str, full))
    fd = minors[full]
    for m in range(DR + 1):
        w(f"  r[{m}] = {fname}[{m}];" if m <= fd else f"  r[{m}] = R(0);")
    w("}")
    w("")
    return DR


def main():
    out = ["// Generated by gen_laplace.py -- do not edit.", ""]
    for name, N, TA, TB in VARIANTS:
        emit(name, N, TA, TB, out)
    sys.stdout.write("\n".join(out) + "\n")


if __name__ == "__main__":
    main()
