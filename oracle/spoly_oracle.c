/*
 * spoly_oracle.c -- plain, slow FP64 CPU oracle of the specular-polynomial
 * solver (Fan et al., "Specular Polynomials", ACM TOG 43(4), 2024).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP path; the two are compared on the same
 * seeded inputs.
 *
 * What it computes, in the paper's order (Sec. 4 then Sec. 5):
 *   coefficient phase  -- bivariate a(u,v), b(u,v) from the vertex constraints
 *                         (coplanarity Eq. eq_coplane; product form Eq.
 *                         eq_pf_result for R; square form Eq. eq_cpf_result
 *                         for T) and, for two bounces, the rational coordinate
 *                         mapping Eq. eq_rct with the refracted direction
 *                         Eq. eq_refr_rational and the piecewise rational
 *                         square-root approximation (Sec. 4.4);
 *   elimination phase  -- Bezout matrix Eq. eq_bezout (Sec. 5.1); for one bounce
 *                         its determinant is expanded by Laplace expansion into
 *                         explicit coefficients of r(v) (Sec. 5.2);
 *   univariate solve   -- one bounce: recursive derivative isolation plus
 *                         bisection on each monotone piece (Sec. 5.2); two
 *                         bounces: sign of det R(v) by Gaussian elimination at
 *                         `pieces`+1 uniform points of [0,1] and `bisect_iters`
 *                         bisection steps on every sign change (Sec. 5.2);
 *   path phase         -- u from a(u)|_v (Sec. 5.3), FP64 Newton polish
 *                         (Sec. 7, one Newton iteration fixes the refraction
 *                         approximation), path-space check of h x n = 0
 *                         (Eq. eq_ch) with side rules, inside-triangle test.
 *
 * Everything is double precision; nothing is blocked, fused or reordered
 * beyond what those steps say.  Readings of points the paper leaves open are
 * listed in the design notes and repeated at the place they apply.
 */
#define _GNU_SOURCE
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXSOL 16

/* ------------------------------------------------------------------ op counter
 * Floating-point operations of the method, by stage, counted in the
 * polynomial and root-finding primitives (one per add, multiply or divide,
 * two per multiply-add) and as fixed per-call figures in the short geometric
 * routines.  Stages: 0 coefficient phase, 1 elimination (one vertex: Bezout
 * matrix and Laplace expansion; two vertices: the det-sign samples of the
 * scan), 2 root finding in v (one vertex: isolation; two vertices: the
 * bisection samples), 3 path phase (u roots, polish, validation).  The
 * Laplace expansion counts each minor once (memoised cost) and a bisection
 * counts its steps down to the paper's 1e-9 only; diagnostics count nothing.
 * Per thread; read by or_opcount_*.                                         */
static __thread uint64_t g_ops[4];
static __thread int g_stage;
static __thread int g_count = 1;
#define OPS(n) (g_ops[g_stage] += g_count ? (uint64_t)(n) : 0u)

/* ------------------------------------------------------------------ params */
typedef struct {
    double tau;          /* path-space tolerance on |h^ x n^| (reading: 1e-6)          */
    double u_margin;     /* u search interval [-m, 1-v+m] before polish                 */
    double dedup;        /* solutions closer than this in (u,v) are one solution        */
    int32_t polish_iters;/* max Newton iterations of the polish                         */
    int32_t pieces;      /* uniform pieces of [0,1] for the >=2-bounce scan (100)       */
    int32_t bisect_iters;/* bisection steps per sign change (10)                        */
    int32_t det_method;  /* sign of det R(v): 0 Gaussian elimination on the Bezout matrix, */
                         /* 1 product formula over the real roots of a(.,v),             */
                         /* 2 the same product with near-double root pairs left out,     */
                         /* 3 as 2 with b evaluated from its defining products and the   */
                         /*   roots where x2 is at infinity left out (the default)       */
} or_params;

typedef struct {
    int32_t query;       /* instance index                                              */
    int32_t flags;
    double u1, v1, u2, v2;
    double residual;     /* max over the chain of |h^ x n^|                             */
    double edge;         /* min over the chain of min(u, v, 1-u-v)                      */
} or_sol;

typedef struct {
    int32_t n_vroots;    /* roots of the univariate problem found in [0,1]              */
    int32_t n_cand;      /* (u,v) candidates sent to polish                             */
    int32_t n_valid;     /* reported solutions                                          */
    int32_t flags;       /* OR_F_* below                                                */
    double tangency;     /* min |r(c)|/max|r_k| over critical points c of r in [0,1]   */
    double min_gap;      /* smallest gap between consecutive v roots (1 if < 2 roots)   */
} or_diag;

enum { OR_F_DEGENERATE = 1, OR_F_EDGE2 = 2, OR_F_AXIS_Z = 4, OR_F_AXIS_Y = 8,
       OR_F_FLAT1 = 16, OR_F_FLAT2 = 32, OR_F_OVERFLOW = 64 };

/* ------------------------------------------------------------------ arena */
typedef struct { char *base; size_t cap, top; } arena;

static void *ar_alloc(arena *A, size_t n)
{
    n = (n + 15) & ~(size_t)15;
    if (A->top + n > A->cap) { fprintf(stderr, "oracle arena exhausted\n"); abort(); }
    void *p = A->base + A->top;
    A->top += n;
    memset(p, 0, n);
    return p;
}

/* ------------------------------------------------------------------ 3-vectors */
typedef struct { double x, y, z; } v3;
static v3 V(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 vadd(v3 a, v3 b) { return V(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vsub(v3 a, v3 b) { return V(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vmul(v3 a, double s) { return V(a.x * s, a.y * s, a.z * s); }
static double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 vcross(v3 a, v3 b)
{
    return V(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double vlen(v3 a) { return sqrt(vdot(a, a)); }
static v3 vnorm(v3 a) { double l = vlen(a); return l > 0 ? vmul(a, 1.0 / l) : a; }
static v3 vload(const double *p, int64_t i) { return V(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }

/* ------------------------------------------------------------------ bivariate polynomials
 * p(u,v) = sum_{i+j<=d} c[i*(d+1)+j] u^i v^j.  Degrees are tracked by
 * construction (structure), never inferred from coefficient values.          */
typedef struct { int d; double *c; } bp;

static bp bp_new(arena *A, int d)
{
    bp p;
    p.d = d < 0 ? 0 : d;
    p.c = (double *)ar_alloc(A, sizeof(double) * (size_t)(p.d + 1) * (size_t)(p.d + 1));
    return p;
}
static double bp_at(bp p, int i, int j)
{
    if (i < 0 || j < 0 || i + j > p.d) return 0.0;
    return p.c[i * (p.d + 1) + j];
}
static bp bp_const(arena *A, double k) { bp p = bp_new(A, 0); p.c[0] = k; return p; }
static bp bp_lin(arena *A, double k0, double ku, double kv)
{
    bp p = bp_new(A, 1);
    p.c[0] = k0;          /* u^0 v^0 */
    p.c[1] = kv;          /* u^0 v^1 */
    p.c[2] = ku;          /* u^1 v^0 */
    return p;
}
static bp bp_mul(arena *A, bp a, bp b)
{
    bp r = bp_new(A, a.d + b.d);
    for (int i = 0; i <= a.d; ++i)
        for (int j = 0; i + j <= a.d; ++j) {
            double x = a.c[i * (a.d + 1) + j];
            if (x == 0.0) continue;
            for (int k = 0; k <= b.d; ++k)
                for (int l = 0; k + l <= b.d; ++l)
                    r.c[(i + k) * (r.d + 1) + (j + l)] += x * b.c[k * (b.d + 1) + l];
            OPS(2 * (b.d + 1) * (b.d + 2) / 2);
        }
    return r;
}
/* sa*a + sb*b */
static bp bp_lc(arena *A, double sa, bp a, double sb, bp b)
{
    bp r = bp_new(A, a.d > b.d ? a.d : b.d);
    for (int i = 0; i <= r.d; ++i)
        for (int j = 0; i + j <= r.d; ++j)
            r.c[i * (r.d + 1) + j] = sa * bp_at(a, i, j) + sb * bp_at(b, i, j);
    OPS(3 * (r.d + 1) * (r.d + 2) / 2);
    return r;
}
static bp bp_add(arena *A, bp a, bp b) { return bp_lc(A, 1.0, a, 1.0, b); }
static bp bp_sub(arena *A, bp a, bp b) { return bp_lc(A, 1.0, a, -1.0, b); }
static bp bp_scale(arena *A, bp a, double s) { return bp_lc(A, s, a, 0.0, a); }

/* value and partial derivatives at (u,v), by direct summation */
static void bp_eval3(bp p, double u, double v, double *f, double *fu, double *fv)
{
    double s = 0, su = 0, sv = 0;
    OPS(8 * (p.d + 1) * (p.d + 2) / 2);
    for (int i = 0; i <= p.d; ++i)
        for (int j = 0; i + j <= p.d; ++j) {
            double c = p.c[i * (p.d + 1) + j];
            s += c * pow(u, i) * pow(v, j);
            if (i > 0) su += c * i * pow(u, i - 1) * pow(v, j);
            if (j > 0) sv += c * j * pow(u, i) * pow(v, j - 1);
        }
    *f = s; if (fu) *fu = su; if (fv) *fv = sv;
}

/* vectors of bivariate polynomials */
typedef struct { bp x, y, z; } bv;
static bv bv_affine(arena *A, v3 p0, v3 eu, v3 ev)     /* p0 + u eu + v ev */
{
    bv r;
    r.x = bp_lin(A, p0.x, eu.x, ev.x);
    r.y = bp_lin(A, p0.y, eu.y, ev.y);
    r.z = bp_lin(A, p0.z, eu.z, ev.z);
    return r;
}
static bv bv_const(arena *A, v3 c)
{
    bv r; r.x = bp_const(A, c.x); r.y = bp_const(A, c.y); r.z = bp_const(A, c.z); return r;
}
static bv bv_add(arena *A, bv a, bv b) { bv r = {bp_add(A, a.x, b.x), bp_add(A, a.y, b.y), bp_add(A, a.z, b.z)}; return r; }
static bv bv_sub(arena *A, bv a, bv b) { bv r = {bp_sub(A, a.x, b.x), bp_sub(A, a.y, b.y), bp_sub(A, a.z, b.z)}; return r; }
static bv bv_smul(arena *A, bp s, bv a) { bv r = {bp_mul(A, s, a.x), bp_mul(A, s, a.y), bp_mul(A, s, a.z)}; return r; }
static bv bv_kmul(arena *A, double k, bv a) { bv r = {bp_scale(A, a.x, k), bp_scale(A, a.y, k), bp_scale(A, a.z, k)}; return r; }
static bv bv_vmul(arena *A, bp s, v3 c)   /* s * constant vector */
{
    bv r = {bp_scale(A, s, c.x), bp_scale(A, s, c.y), bp_scale(A, s, c.z)}; return r;
}
static bp bv_dot(arena *A, bv a, bv b)
{
    return bp_add(A, bp_add(A, bp_mul(A, a.x, b.x), bp_mul(A, a.y, b.y)), bp_mul(A, a.z, b.z));
}
static bp bv_dotc(arena *A, bv a, v3 c)
{
    return bp_add(A, bp_add(A, bp_scale(A, a.x, c.x), bp_scale(A, a.y, c.y)), bp_scale(A, a.z, c.z));
}
static bv bv_cross(arena *A, bv a, bv b)
{
    bv r;
    r.x = bp_sub(A, bp_mul(A, a.y, b.z), bp_mul(A, a.z, b.y));
    r.y = bp_sub(A, bp_mul(A, a.z, b.x), bp_mul(A, a.x, b.z));
    r.z = bp_sub(A, bp_mul(A, a.x, b.y), bp_mul(A, a.y, b.x));
    return r;
}

/* ------------------------------------------------------------------ univariate polynomials in v */
typedef struct { int d; double *c; } up;   /* sum_{k<=d} c[k] v^k ; d < 0 means the zero polynomial */

static up up_new(arena *A, int d)
{
    up p; p.d = d;
    p.c = (double *)ar_alloc(A, sizeof(double) * (size_t)(d < 0 ? 1 : d + 1));
    return p;
}
static up up_mul(arena *A, up a, up b)
{
    if (a.d < 0 || b.d < 0) return up_new(A, -1);
    up r = up_new(A, a.d + b.d);
    for (int i = 0; i <= a.d; ++i)
        for (int j = 0; j <= b.d; ++j) r.c[i + j] += a.c[i] * b.c[j];
    OPS(2 * (a.d + 1) * (b.d + 1));
    return r;
}
static up up_lc(arena *A, double sa, up a, double sb, up b)
{
    int d = a.d > b.d ? a.d : b.d;
    up r = up_new(A, d);
    for (int k = 0; k <= d; ++k)
        r.c[k] = (k <= a.d ? sa * a.c[k] : 0.0) + (k <= b.d ? sb * b.c[k] : 0.0);
    OPS(3 * (d + 1));
    return r;
}
static double up_eval(const double *c, int d, double v)
{
    OPS(2 * (d + 1));
    double s = 0.0;
    for (int k = d; k >= 0; --k) s = s * v + c[k];
    return s;
}
/* coefficient of u^i in p(u,v), as a polynomial in v of degree p.d - i */
static up bp_ucoef(arena *A, bp p, int i)
{
    if (i > p.d) return up_new(A, -1);
    up r = up_new(A, p.d - i);
    for (int j = 0; j <= p.d - i; ++j) r.c[j] = p.c[i * (p.d + 1) + j];
    return r;
}

/* ------------------------------------------------------------------ Bezout resultant, Eq. (eq_bezout)
 * (i,j) entry, 0 <= i,j < n:
 *     sum_{k=0}^{min(i, n-1-j)} a_{i-k} b_{j+1+k} - b_{i-k} a_{j+1+k}
 * with a_m = b_m = 0 beyond the polynomial's u-degree.  n is the structural
 * u-degree of the system (never inferred from values).                      */
static void bezout_poly(arena *A, const up *ac, const up *bc, int n, up *M /* n*n */)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            up s = up_new(A, -1);
            int kmax = i < n - 1 - j ? i : n - 1 - j;
            for (int k = 0; k <= kmax; ++k) {
                up t1 = up_mul(A, ac[i - k], bc[j + 1 + k]);
                up t2 = up_mul(A, bc[i - k], ac[j + 1 + k]);
                s = up_lc(A, 1.0, s, 1.0, up_lc(A, 1.0, t1, -1.0, t2));
            }
            M[i * n + j] = s;
        }
}

/* Laplace (cofactor) expansion along the first remaining row, Sec. 5.2.
 * Rows r..n-1, columns given by `mask`.                                      */
static __thread unsigned char g_minor_seen[1 << 12];
static up laplace(arena *A, const up *M, int n, int r, unsigned mask)
{
    if (r == n) { up one = up_new(A, 0); one.c[0] = 1.0; return one; }
    /* op counter: a minor (rows r.., columns `mask`) is counted once */
    int saved = g_count;
    if (r == 0) memset(g_minor_seen, 0, sizeof(g_minor_seen));
    if (g_minor_seen[mask]) g_count = 0;
    g_minor_seen[mask] = 1;
    up acc = up_new(A, -1);
    int pos = 0;
    for (int j = 0; j < n; ++j) {
        if (!(mask & (1u << j))) continue;
        up e = M[r * n + j];
        if (e.d >= 0) {
            up minor = laplace(A, M, n, r + 1, mask & ~(1u << j));
            up t = up_mul(A, e, minor);
            acc = up_lc(A, 1.0, acc, (pos & 1) ? -1.0 : 1.0, t);
        }
        ++pos;
    }
    g_count = saved;
    return acc;
}

/* ------------------------------------------------------------------ univariate root isolation (Sec. 5.2)
 * The zeros of p' split [lo,hi] into monotone pieces; a piece whose end values
 * have strictly different signs holds exactly one root, found by bisection.
 * Reading: sgn(0) := +1.  The oracle bisects until the interval stops
 * shrinking (full double precision), which is finer than the paper's 1e-9.   */
static int sgn(double x) { return x < 0.0 ? -1 : 1; }

static double bisect_full(const double *c, int d, double l, double r, int sl)
{
    int saved = g_count;
    for (int it = 0; it < 2000; ++it) {
        double m = 0.5 * (l + r);
        if (!(m > l && m < r)) break;
        if (!(r - l > 1e-9)) g_count = 0;   /* op counter: the paper's 1e-9 */
        if (sgn(up_eval(c, d, m)) == sl) l = m; else r = m;
    }
    g_count = saved;
    return 0.5 * (l + r);
}

/* roots of sum c[k] x^k (degree d) in [lo,hi]; returns count, ascending */
static int isolate(arena *A, const double *c, int d, double lo, double hi, double *roots, int cap)
{
    double *crit = NULL;
    int nc = 0;
    if (d >= 2) {
        double *dc = (double *)ar_alloc(A, sizeof(double) * (size_t)d);
        for (int k = 1; k <= d; ++k) dc[k - 1] = k * c[k];
        OPS(d);
        crit = (double *)ar_alloc(A, sizeof(double) * (size_t)d);
        nc = isolate(A, dc, d - 1, lo, hi, crit, d);
    }
    int nr = 0;
    double l = lo, fl = up_eval(c, d, lo);
    for (int k = 0; k <= nc; ++k) {
        double r = (k < nc) ? crit[k] : hi;
        double fr = up_eval(c, d, r);
        if (r > l && sgn(fl) != sgn(fr)) {
            double x = bisect_full(c, d, l, r, sgn(fl));
            if (nr == 0 || x - roots[nr - 1] > 1e-12) {
                if (nr < cap) roots[nr++] = x;
            }
        }
        l = r; fl = fr;
    }
    return nr;
}

/* ------------------------------------------------------------------ path-space check (Eq. eq_ch)
 * Reading of the check the paper delegates to prior work: with
 * wi = normalize(x_prev - x), wo = normalize(x_next - x),
 * h = eta_in wi + eta_out wo (the generalised half vector of Eq. eq_ch up to sign),
 * a vertex is admissible iff |h^ x n^| <= tau and (wi.n)(wo.n) > 0 for
 * reflection, < 0 for refraction.                                             */
static int vertex_law(v3 xp, v3 x, v3 xn, v3 nrm, double eta_in, double eta_out, int refract, double *res)
{
    OPS(70);
    double ln = vlen(nrm);
    if (!(ln > 1e-12)) { *res = 1e300; return 0; }
    v3 nh = vmul(nrm, 1.0 / ln);
    v3 wi = vnorm(vsub(xp, x)), wo = vnorm(vsub(xn, x));
    v3 h = vadd(vmul(wi, eta_in), vmul(wo, eta_out));
    double lh = vlen(h);
    if (!(lh > 0)) { *res = 1e300; return 0; }
    double r = vlen(vcross(vmul(h, 1.0 / lh), nh));
    *res = r;
    double side = vdot(wi, nh) * vdot(wo, nh);
    int ok_side = refract ? (side < 0.0) : (side > 0.0);
    return ok_side;
}

static double edge_dist(double u, double v)
{
    double w = 1.0 - u - v, m = u < v ? u : v;
    return m < w ? m : w;
}

static int bary_inside(double u, double v) { return u >= 0.0 && v >= 0.0 && u + v <= 1.0; }

/* ------------------------------------------------------------------ axis / tangent rules
 * Square form (Eq. eq_cpf_result): b = x^ by default, another axis when the
 * projection degenerates.  On the coplanarity curve both sides of Eq.
 * eq_angrel2 are parallel to the incidence-plane normal m, so the projection
 * degenerates where m.b -> 0.  Reading: with m_c = normalize((c - xa) x (xb - xa))
 * at the triangle centroid c, take x^ if |m_c.x^| >= 1/2, else z^ if
 * |m_c.z^| >= 1/2, else y^.
 * Product form (Eq. eq_pf_result): t = n x e1 by default; along the
 * coplanarity curve d.t = (e1.m)(d.(n x m)), so it degenerates when e1 lies in
 * the incidence plane.  Reading: switch to t = n x e2 iff |e1^.m_c| < 1/4 and
 * |e2^.m_c| > |e1^.m_c|.                                                       */
static int pick_axis(v3 c, v3 xa, v3 xb, v3 *axis)
{
    v3 m = vcross(vsub(c, xa), vsub(xb, xa));
    double l = vlen(m);
    if (!(l > 0)) { *axis = V(1, 0, 0); return 0; }
    m = vmul(m, 1.0 / l);
    if (fabs(m.x) >= 0.5) { *axis = V(1, 0, 0); return 0; }
    if (fabs(m.z) >= 0.5) { *axis = V(0, 0, 1); return OR_F_AXIS_Z; }
    *axis = V(0, 1, 0);
    return OR_F_AXIS_Y;
}

static int pick_edge2(v3 c, v3 xa, v3 xb, v3 e1, v3 e2)
{
    v3 m = vcross(vsub(c, xa), vsub(xb, xa));
    double l = vlen(m);
    if (!(l > 0)) return 0;
    m = vmul(m, 1.0 / l);
    double g1 = fabs(vdot(vnorm(e1), m)), g2 = fabs(vdot(vnorm(e2), m));
    return (g1 < 0.25 && g2 > g1) ? 1 : 0;
}

/* ------------------------------------------------------------------ one bounce: coefficient phase
 * R  (Sec. 4.5):  a = ((P u - x0) x (x2 - x0)) . N u                       (Eq. eq_coplane)
 *                 b = ((Pu-x0).Nu)((x2-Pu).t) + ((x2-Pu).Nu)((Pu-x0).t),
 *                     t = N u x e                                          (Eq. eq_pf_result)
 * T  (Sec. 4.5):  b = eta0^2 |x2-Pu|^2 (((Pu-x0) x Nu).b)^2
 *                   - eta1^2 |Pu-x0|^2 (((x2-Pu) x Nu).b)^2                 (Eq. eq_cpf_result)
 * Returns the structural u-degree of b (the Bezout size n).                 */
typedef struct { v3 p0, e1, e2, n0, dn1, dn2; int flat; } tri_t;

static tri_t load_tri(const double *P, const double *N, const int32_t *tri, int64_t t)
{
    tri_t T;
    int32_t i0 = tri[3 * t], i1 = tri[3 * t + 1], i2 = tri[3 * t + 2];
    v3 p0 = vload(P, i0), p1 = vload(P, i1), p2 = vload(P, i2);
    v3 n0 = vload(N, i0), n1 = vload(N, i1), n2 = vload(N, i2);
    T.p0 = p0; T.e1 = vsub(p1, p0); T.e2 = vsub(p2, p0);
    T.n0 = n0; T.dn1 = vsub(n1, n0); T.dn2 = vsub(n2, n0);
    T.flat = (n0.x == n1.x && n0.y == n1.y && n0.z == n1.z && n0.x == n2.x && n0.y == n2.y && n0.z == n2.z);
    return T;
}
static v3 tri_x(const tri_t *T, double u, double v) { return vadd(T->p0, vadd(vmul(T->e1, u), vmul(T->e2, v))); }
static v3 tri_n(const tri_t *T, double u, double v) { return vadd(T->n0, vadd(vmul(T->dn1, u), vmul(T->dn2, v))); }

static bv tri_xpoly(arena *A, const tri_t *T) { return bv_affine(A, T->p0, T->e1, T->e2); }
static bv tri_npoly(arena *A, const tri_t *T)
{
    if (T->flat) return bv_const(A, T->n0);
    return bv_affine(A, T->n0, T->dn1, T->dn2);
}

static int coeffs_1b(arena *A, const tri_t *T, v3 x0, v3 x2, int refract, double eta0, double eta1,
                     bp *pa, bp *pb, int *flags)
{
    int f = T->flat ? 0 : 1;
    bv x1 = tri_xpoly(A, T);
    bv n = tri_npoly(A, T);
    bv d0 = bv_sub(A, x1, bv_const(A, x0));         /* x1 - x0 */
    bv d1 = bv_sub(A, bv_const(A, x2), x1);         /* x2 - x1 */
    v3 w = vsub(x2, x0);
    /* a: endpoint-difference coplanarity */
    *pa = bv_dot(A, bv_cross(A, d0, bv_const(A, w)), n);
    v3 c = tri_x(T, 1.0 / 3.0, 1.0 / 3.0);
    if (!refract) {
        int use2 = pick_edge2(c, x0, x2, T->e1, T->e2);
        if (use2) *flags |= OR_F_EDGE2;
        bv t = bv_cross(A, n, bv_const(A, use2 ? T->e2 : T->e1));
        *pb = bp_add(A, bp_mul(A, bv_dot(A, d0, n), bv_dot(A, d1, t)),
                        bp_mul(A, bv_dot(A, d0, t), bv_dot(A, d1, n)));
        /* with t = n x e1 the u^(2+2f) term cancels: e1.(dn1 x e1) = 0 */
        return use2 ? 2 + 2 * f : 1 + 2 * f;
    } else {
        v3 ax;
        *flags |= pick_axis(c, x0, x2, &ax);
        bp l = bv_dotc(A, bv_cross(A, d0, n), ax);
        bp r = bv_dotc(A, bv_cross(A, d1, n), ax);
        bp t1 = bp_mul(A, bv_dot(A, d1, d1), bp_mul(A, l, l));
        bp t2 = bp_mul(A, bv_dot(A, d0, d0), bp_mul(A, r, r));
        *pb = bp_lc(A, eta0 * eta0, t1, -eta1 * eta1, t2);
        return 4 + 2 * f;
    }
}


/* Numerical u-degree of p, at most `cap` (the structural degree).  A top row of
 * u-powers is dropped when it is exactly zero or below 1e-10 times the row under
 * it: exact algebraic cancellations of the input family (parallel flat
 * triangles; sphere normals equal to position/radius) leave such rows as
 * rounding residues, while the natural decay of the coefficients of a small
 * triangle is orders of magnitude slower.  Dropped rows are set to zero.     */
static double row_max(bp p, int i)
{
    double m = 0.0;
    for (int j = 0; i + j <= p.d; ++j) m = fmax(m, fabs(p.c[i * (p.d + 1) + j]));
    return m;
}
static int numeric_udeg(bp p, int cap)
{
    int d = cap < p.d ? cap : p.d;
    while (d > 0) {
        double top = row_max(p, d), below = row_max(p, d - 1);
        if (top == 0.0 || top < 1e-10 * below) --d;
        else break;
    }
    for (int i = d + 1; i <= p.d; ++i)
        for (int j = 0; i + j <= p.d; ++j) p.c[i * (p.d + 1) + j] = 0.0;
    return d;
}

/* FP64 Newton on the bivariate system (a,b) = 0 (Sec. 7 polish reading).
 * Returns 1 if the last step was below 1e-10.                               */
static int polish_ab(bp a, bp b, int iters, double *pu, double *pv)
{
    double u = *pu, v = *pv, step = 1e300;
    for (int it = 0; it < iters; ++it) {
        double fa, au, av, fb, bu, bvv;
        bp_eval3(a, u, v, &fa, &au, &av);
        bp_eval3(b, u, v, &fb, &bu, &bvv);
        double det = au * bvv - av * bu;
        OPS(12);
        if (!(det != 0.0) || !isfinite(det)) break;
        double du = (fa * bvv - av * fb) / det;
        double dv = (au * fb - fa * bu) / det;
        u -= du; v -= dv;
        step = fabs(du) + fabs(dv);
        if (!(step > 1e-16)) break;
    }
    *pu = u; *pv = v;
    return step <= 1e-10;
}

static int add_solution(or_sol *S, int n, double dedup, or_sol s)
{
    for (int k = 0; k < n; ++k)
        if (fabs(S[k].u1 - s.u1) < dedup && fabs(S[k].v1 - s.v1) < dedup) return n;
    if (n < OR_MAXSOL) S[n++] = s;
    return n;
}

/* one (x0, x2, triangle) instance */
static void solve_1b(arena *A, const tri_t *T, v3 x0, v3 x2, int refract, double eta0, double eta1,
                     const or_params *prm, int32_t qid, or_sol *out, int32_t *nout, or_diag *dg)
{
    memset(dg, 0, sizeof(*dg));
    dg->min_gap = 1.0;
    dg->tangency = 1e300;
    if (T->flat) dg->flags |= OR_F_FLAT1;
    bp a, b;
    g_stage = 0;
    int nb = coeffs_1b(A, T, x0, x2, refract, eta0, eta1, &a, &b, &dg->flags);
    int ma = numeric_udeg(a, a.d);
    nb = numeric_udeg(b, nb);
    int n = ma > nb ? ma : nb;
    if (n < 1) { dg->flags |= OR_F_DEGENERATE; *nout = 0; return; }
    /* elimination: coefficient polynomials a_i(v), b_i(v), i = 0..n */
    up *ac = (up *)ar_alloc(A, sizeof(up) * (size_t)(n + 1));
    up *bc = (up *)ar_alloc(A, sizeof(up) * (size_t)(n + 1));
    for (int i = 0; i <= n; ++i) { ac[i] = bp_ucoef(A, a, i); bc[i] = bp_ucoef(A, b, i); }
    up *M = (up *)ar_alloc(A, sizeof(up) * (size_t)(n * n));
    g_stage = 1;
    bezout_poly(A, ac, bc, n, M);
    up r = laplace(A, M, n, 0, (1u << n) - 1u);
    double scale = 0.0;
    for (int k = 0; k <= r.d; ++k) scale = fmax(scale, fabs(r.c[k]));
    int nsol = 0;
    if (r.d < 0 || !(scale > 0.0) || !isfinite(scale)) {
        dg->flags |= OR_F_DEGENERATE;
        *nout = 0;
        return;
    }
    /* tangency diagnostic at the critical points of r (not part of the method) */
    int saved = g_count;
    g_count = 0;
    if (r.d >= 2) {
        double *dc = (double *)ar_alloc(A, sizeof(double) * (size_t)r.d);
        for (int k = 1; k <= r.d; ++k) dc[k - 1] = k * r.c[k];
        double crit[64];
        int ncr = isolate(A, dc, r.d - 1, 0.0, 1.0, crit, 64);
        for (int k = 0; k < ncr; ++k)
            dg->tangency = fmin(dg->tangency, fabs(up_eval(r.c, r.d, crit[k])) / scale);
    }
    g_count = saved;
    g_stage = 2;
    double vr[64];
    int nv = isolate(A, r.c, r.d, 0.0, 1.0, vr, 64);
    g_stage = 3;
    dg->n_vroots = nv;
    for (int k = 1; k < nv; ++k) dg->min_gap = fmin(dg->min_gap, vr[k] - vr[k - 1]);
    for (int k = 0; k < nv; ++k) {
        double v = vr[k];
        /* path phase: u from a(u)|_v */
        int da = ma;
        double *auc = (double *)ar_alloc(A, sizeof(double) * (size_t)(da + 1));
        for (int i = 0; i <= da; ++i) auc[i] = up_eval(ac[i].c, ac[i].d, v);
        double ur[64];
        int nu = isolate(A, auc, da, -prm->u_margin, 1.0 - v + prm->u_margin, ur, 64);
        for (int m = 0; m < nu; ++m) {
            double u = ur[m], vv = v;
            dg->n_cand++;
            if (!polish_ab(a, b, prm->polish_iters, &u, &vv)) continue;
            if (!bary_inside(u, vv)) continue;
            v3 x1 = tri_x(T, u, vv), nn = tri_n(T, u, vv);
            double res;
            if (!vertex_law(x0, x1, x2, nn, eta0, eta1, refract, &res)) continue;
            if (!(res <= prm->tau)) continue;
            or_sol s;
            memset(&s, 0, sizeof(s));
            s.query = qid; s.u1 = u; s.v1 = vv; s.u2 = 0; s.v2 = 0;
            s.residual = res; s.edge = edge_dist(u, vv); s.flags = dg->flags;
            nsol = add_solution(out, nsol, prm->dedup, s);
        }
    }
    dg->n_valid = nsol;
    *nout = nsol;
}

/* ------------------------------------------------------------------ exported: one bounce
 * P,N: [nv*3] vertex positions / normals; tri: [nt*3]; x0s: [n0*3]; x2s: [n2*3];
 * queries q_x0[q], q_x2[q], q_tri[q].  Output: out[q*OR_MAXSOL + k], k < count[q].  */
int or_solve_1bounce(const double *P, const double *N, const int32_t *tri, int64_t nt,
                     const double *x0s, const double *x2s,
                     const int32_t *q_x0, const int32_t *q_x2, const int32_t *q_tri, int64_t nq,
                     int32_t refract, double eta0, double eta1, const or_params *prm,
                     or_sol *out, int32_t *count, or_diag *diag)
{
    (void)nt;
    int bad = 0;
#pragma omp parallel
    {
        arena A;
        A.cap = (size_t)8 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < nq; ++q) {
            A.top = 0;
            tri_t T = load_tri(P, N, tri, q_tri[q]);
            solve_1b(&A, &T, vload(x0s, q_x0[q]), vload(x2s, q_x2[q]), refract, eta0, eta1, prm,
                     (int32_t)q, out + q * OR_MAXSOL, count + q, diag + q);
        }
        free(A.base);
    }
    return bad;
}

/* ------------------------------------------------------------------ exported helpers for the pin tests */

/* bivariate coefficients of the one-bounce system, dense (d+1)^2 arrays  */
int or_coeffs_1bounce(const double *P, const double *N, const int32_t *tri, int64_t t,
                      const double *x0, const double *x2, int32_t refract, double eta0, double eta1,
                      double *a_out, int32_t *da, double *b_out, int32_t *db, int32_t *n_bez, int32_t *flags)
{
    arena A; A.cap = (size_t)8 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    tri_t T = load_tri(P, N, tri, t);
    bp a, b; int fl = 0;
    int nb = coeffs_1b(&A, &T, vload(x0, 0), vload(x2, 0), refract, eta0, eta1, &a, &b, &fl);
    int ma = numeric_udeg(a, a.d);
    nb = numeric_udeg(b, nb);
    int n = ma > nb ? ma : nb;
    *da = a.d; *db = b.d; *n_bez = n; *flags = fl;
    memcpy(a_out, a.c, sizeof(double) * (size_t)(a.d + 1) * (size_t)(a.d + 1));
    memcpy(b_out, b.c, sizeof(double) * (size_t)(b.d + 1) * (size_t)(b.d + 1));
    free(A.base);
    return 0;
}

/* Bezout + Laplace of given bivariate a, b (dense, degrees da, db) with Bezout size n.
 * r_out receives the coefficients of r(v); returns its degree.  */
int or_resultant_laplace(const double *a_in, int32_t da, const double *b_in, int32_t db, int32_t n, double *r_out)
{
    arena A; A.cap = (size_t)32 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    bp a = bp_new(&A, da), b = bp_new(&A, db);
    memcpy(a.c, a_in, sizeof(double) * (size_t)(da + 1) * (size_t)(da + 1));
    memcpy(b.c, b_in, sizeof(double) * (size_t)(db + 1) * (size_t)(db + 1));
    up *ac = (up *)ar_alloc(&A, sizeof(up) * (size_t)(n + 1));
    up *bc = (up *)ar_alloc(&A, sizeof(up) * (size_t)(n + 1));
    for (int i = 0; i <= n; ++i) { ac[i] = bp_ucoef(&A, a, i); bc[i] = bp_ucoef(&A, b, i); }
    up *M = (up *)ar_alloc(&A, sizeof(up) * (size_t)(n * n));
    bezout_poly(&A, ac, bc, n, M);
    up r = laplace(&A, M, n, 0, (1u << n) - 1u);
    for (int k = 0; k <= r.d; ++k) r_out[k] = r.c[k];
    int d = r.d;
    free(A.base);
    return d;
}

/* real roots of sum c[k] x^k in [lo,hi] by the recursive isolation */
int or_isolate(const double *c, int32_t d, double lo, double hi, double *roots, int32_t cap)
{
    arena A; A.cap = (size_t)8 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    int n = isolate(&A, c, d, lo, hi, roots, cap);
    free(A.base);
    return n;
}

/* ================================================================== two bounces (RR, RT, TR, TT)
 * Chain x0 -> x1 on T1 -> x2 on T2 -> x3, reflection (R) or refraction (T) at
 * each vertex, IORs eta[0] (segment x0x1), eta[1] (x1x2), eta[2] (x2x3); a
 * reflection has equal IORs on both of its segments.
 *
 * Coefficient phase (Sec. 4.4-4.5):
 *   d0 = x1 - x0, n1 = N1 u.
 *   Direction x1 -> x2 (Eq. eq_431_di):
 *   R at x1: Dt = |n1|^2 d0 - 2 (d0.n1) n1, the reflected direction scaled by
 *     |n1|^2 (exact, polynomial);
 *   T at x1: beta = n1^2 d0^2 - eta'^2 (n1^2 d0^2 - (d0.n1)^2),
 *   eta' = eta0/eta1                                             (Eq. eq_refr_rational)
 *   sqrt(beta) ~ sqrt(S) R_p(beta/S), R_p(s) = (c0 + c1 s)/(d0 + d1 s)   (Sec. 4.4)
 *     reading: S = n1^2 d0^2 at the centroid of T1 (a per-tuple constant) and the
 *     piece p is the one that holds beta/S at the centroid.
 *   Dt = den * eta' (d0 n1^2 - (d0.n1) n1) + sgn(d0.n1) sqrt(S) num n1
 *     (Eq. eq_refr_rational times den = d0 + d1 beta/S; the sign orients n1
 *     against the incoming ray)
 *   mapping onto T2 (Eq. eq_rct): q = x1 - p20,
 *     ut = (Dt x e22).q,  vt = (q x e21).Dt,  kappa = (Dt x e22).e21
 *   X2 = kappa p20 + ut e21 + vt e22 (= kappa x2),  M2 = kappa n20 + ut dn21 + vt dn22 (= kappa n2),
 *   D2 = kappa x3 - X2 (= kappa d2).
 *   Since d1 = x2 - x1 is parallel to Dt, Dt replaces d1 in both constraints at x2:
 *   a = (Dt x (x3 - x1)) . M2                                         (Eq. eq_coplane)
 *   T at x2: b = eta1^2 |D2|^2 ((Dt x M2).b)^2 - eta2^2 |Dt|^2 ((D2 x M2).b)^2
 *                                                                      (Eq. eq_cpf_result)
 *   R at x2: b = (Dt.M2)(D2.t) + (Dt.t)(D2.M2), t = M2 x e              (Eq. eq_pf_result)
 *            with e = e21 of T2, or e22 by the product-form rule at x2.
 *   Structural degrees with f = 1 for interpolated normals, D = deg Dt
 *   (R: 1 + 2 f1; T: 3 + 4 f1): deg a = 2D + 1 + f2; deg b = 6D + 2 + 2 f2 (T at
 *   x2) or 4D + 1 + 2 f2 (R at x2); u-degree = total degree.
 */
typedef struct { double bp[7]; double c[6][4]; } or_sqrtfit;  /* breakpoints, (c0,c1,d0,d1) per piece */

static int coeffs_2v(arena *A, const tri_t *T1, const tri_t *T2, v3 x0, v3 x3, const double *eta,
                     int ev1, int ev2, const or_sqrtfit *fit, bp *pa, bp *pb, int *flags)
{
    int f1 = T1->flat ? 0 : 1, f2 = T2->flat ? 0 : 1;
    bv x1 = tri_xpoly(A, T1);
    bv n1 = tri_npoly(A, T1);
    bv d0 = bv_sub(A, x1, bv_const(A, x0));
    bp nn = bv_dot(A, n1, n1), dn = bv_dot(A, d0, n1);
    v3 c1 = tri_x(T1, 1.0 / 3.0, 1.0 / 3.0);
    bv Dt;
    int D;
    if (ev1 == 0) {
        /* reflection: |n1|^2 d0 - 2 (d0.n1) n1 */
        Dt = bv_sub(A, bv_smul(A, nn, d0), bv_kmul(A, 2.0, bv_smul(A, dn, n1)));
        D = 1 + 2 * f1;
    } else {
        double etap = eta[0] / eta[1];
        bp dd = bv_dot(A, d0, d0);
        bp nndd = bp_mul(A, nn, dd);
        bp beta = bp_lc(A, 1.0 - etap * etap, nndd, etap * etap, bp_mul(A, dn, dn));
        /* per-tuple constants at the centroid of T1 */
        v3 nc1 = tri_n(T1, 1.0 / 3.0, 1.0 / 3.0);
        v3 d0c = vsub(c1, x0);
        double S = vdot(nc1, nc1) * vdot(d0c, d0c);
        double dnc = vdot(d0c, nc1);
        double sc = 1.0 - etap * etap * (1.0 - dnc * dnc / S);   /* beta/S at the centroid */
        int p = 0;
        for (int k = 1; k < 6; ++k) if (sc >= fit->bp[k]) p = k;
        double q0 = fit->c[p][0], q1 = fit->c[p][1], r0 = fit->c[p][2], r1 = fit->c[p][3];
        bp num = bp_lc(A, q1 / S, beta, q0, bp_const(A, 1.0));
        bp den = bp_lc(A, r1 / S, beta, r0, bp_const(A, 1.0));
        double sg = dnc < 0.0 ? -1.0 : 1.0;
        bv tang = bv_sub(A, bv_smul(A, nn, d0), bv_smul(A, dn, n1));          /* d0 n^2 - (d0.n) n */
        Dt = bv_add(A, bv_kmul(A, etap, bv_smul(A, den, tang)), bv_kmul(A, sg * sqrt(S), bv_smul(A, num, n1)));
        D = 3 + 4 * f1;
    }
    /* rational coordinate mapping onto T2 */
    bv q = bv_sub(A, x1, bv_const(A, T2->p0));
    bv Dxe22 = bv_cross(A, Dt, bv_const(A, T2->e2));
    bp ut = bv_dot(A, Dxe22, q);
    bp vt = bv_dot(A, bv_cross(A, q, bv_const(A, T2->e1)), Dt);
    bp ka = bv_dotc(A, Dxe22, T2->e1);
    bv X2 = bv_add(A, bv_vmul(A, ka, T2->p0), bv_add(A, bv_vmul(A, ut, T2->e1), bv_vmul(A, vt, T2->e2)));
    bv M2 = f2 ? bv_add(A, bv_vmul(A, ka, T2->n0), bv_add(A, bv_vmul(A, ut, T2->dn1), bv_vmul(A, vt, T2->dn2)))
               : bv_vmul(A, ka, T2->n0);
    bv D2 = bv_sub(A, bv_vmul(A, ka, x3), X2);
    *pa = bv_dot(A, bv_cross(A, Dt, bv_sub(A, bv_const(A, x3), x1)), M2);
    v3 c2 = tri_x(T2, 1.0 / 3.0, 1.0 / 3.0);
    if (ev2 == 0) {
        int use2 = pick_edge2(c2, c1, x3, T2->e1, T2->e2);
        if (use2) *flags |= OR_F_EDGE2;
        bv t = bv_cross(A, M2, bv_const(A, use2 ? T2->e2 : T2->e1));
        *pb = bp_add(A, bp_mul(A, bv_dot(A, Dt, M2), bv_dot(A, D2, t)),
                        bp_mul(A, bv_dot(A, Dt, t), bv_dot(A, D2, M2)));
        return 4 * D + 1 + 2 * f2;  /* structural u-degree of b */
    }
    v3 ax;
    *flags |= pick_axis(c2, c1, x3, &ax);
    bp l = bv_dotc(A, bv_cross(A, Dt, M2), ax);
    bp r = bv_dotc(A, bv_cross(A, D2, M2), ax);
    bp t1 = bp_mul(A, bv_dot(A, D2, D2), bp_mul(A, l, l));
    bp t2 = bp_mul(A, bv_dot(A, Dt, Dt), bp_mul(A, r, r));
    *pb = bp_lc(A, eta[1] * eta[1], t1, -eta[2] * eta[2], t2);
    return 6 * D + 2 + 2 * f2;  /* structural u-degree of b */
}

/* sign of det of the numeric Bezout matrix at v, by Gaussian elimination with
 * partial pivoting (Sec. 5.2).  Only the sign is formed (the product of the
 * pivots under- or overflows for large n).  Reading: sgn(0) := +1.          */
static int det_sign_at(arena *A, bp a, bp b, int n, double v)
{
    size_t mark = A->top;
    double *ai = (double *)ar_alloc(A, sizeof(double) * (size_t)(n + 2));
    double *bi = (double *)ar_alloc(A, sizeof(double) * (size_t)(n + 2));
    for (int i = 0; i <= n; ++i) {
        ai[i] = 0.0; bi[i] = 0.0;
        if (i <= a.d) for (int j = a.d - i; j >= 0; --j) ai[i] = ai[i] * v + a.c[i * (a.d + 1) + j];
        if (i <= b.d) for (int j = b.d - i; j >= 0; --j) bi[i] = bi[i] * v + b.c[i * (b.d + 1) + j];
    }
    double *M = (double *)ar_alloc(A, sizeof(double) * (size_t)n * (size_t)n);
    OPS(2 * (a.d + 1) * (a.d + 2) / 2 + 2 * (b.d + 1) * (b.d + 2) / 2);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            int kmax = i < n - 1 - j ? i : n - 1 - j;
            for (int k = 0; k <= kmax; ++k) s += ai[i - k] * bi[j + 1 + k] - bi[i - k] * ai[j + 1 + k];
            OPS(4 * (kmax + 1));
            M[i * n + j] = s;
        }
    int sign = 1;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(M[k * n + k]);
        for (int i = k + 1; i < n; ++i) if (fabs(M[i * n + k]) > best) { best = fabs(M[i * n + k]); p = i; }
        if (!(best > 0.0)) { A->top = mark; return 1; }   /* det == 0 */
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = M[k * n + j]; M[k * n + j] = M[p * n + j]; M[p * n + j] = t; }
            sign = -sign;
        }
        double piv = M[k * n + k];
        if (piv < 0) sign = -sign;
        for (int i = k + 1; i < n; ++i) {
            double l = M[i * n + k] / piv;
            OPS(1);
            if (l == 0.0) continue;
            for (int j = k + 1; j < n; ++j) M[i * n + j] -= l * M[k * n + j];
            OPS(2 * (n - k - 1));
        }
    }
    A->top = mark;
    return sign;
}

/* exact reflection (ev1 = 0) or refraction (ev1 = 1) at x1 and intersection
 * with T2's plane.  Returns 0 on total internal reflection or when the plane
 * is behind / parallel.                                                     */
static int trace_x2(const tri_t *T1, const tri_t *T2, v3 x0, double u1, double v1, int ev1, double etap,
                    double *u2, double *v2, v3 *x1o, v3 *x2o)
{
    OPS(90);
    v3 x1 = tri_x(T1, u1, v1);
    v3 n = vnorm(tri_n(T1, u1, v1));
    v3 di = vnorm(vsub(x1, x0));
    double c = vdot(di, n);
    v3 dt;
    if (ev1 == 0) {
        dt = vsub(di, vmul(n, 2.0 * c));
    } else {
        if (c > 0) { n = vmul(n, -1.0); c = -c; }          /* orient n against the incoming ray */
        double ci = -c;
        double k = 1.0 - etap * etap * (1.0 - ci * ci);
        if (k < 0.0) return 0;
        dt = vadd(vmul(di, etap), vmul(n, etap * ci - sqrt(k)));
    }
    /* Moller-Trumbore without bounds */
    v3 pv = vcross(dt, T2->e2);
    double det = vdot(T2->e1, pv);
    if (!(fabs(det) > 0.0)) return 0;
    v3 tv = vsub(x1, T2->p0);
    double uu = vdot(tv, pv) / det;
    v3 qv = vcross(tv, T2->e1);
    double vv = vdot(dt, qv) / det;
    double t = vdot(T2->e2, qv) / det;
    if (!(t > 0.0)) return 0;
    *u2 = uu; *v2 = vv; *x1o = x1; *x2o = tri_x(T2, uu, vv);
    return 1;
}

/* F(u1,v1): (h2^ x n2^) on a fixed tangent basis of T2, x2 from the exact ray */
static int tt_residual(const tri_t *T1, const tri_t *T2, v3 x0, v3 x3, const double *eta, int ev1,
                       v3 ta, v3 tb, double u1, double v1, double F[2])
{
    double u2, v2; v3 x1, x2;
    if (!trace_x2(T1, T2, x0, u1, v1, ev1, eta[0] / eta[1], &u2, &v2, &x1, &x2)) return 0;
    OPS(75);
    v3 n2 = vnorm(tri_n(T2, u2, v2));
    v3 wi = vnorm(vsub(x1, x2)), wo = vnorm(vsub(x3, x2));
    v3 h = vnorm(vadd(vmul(wi, eta[1]), vmul(wo, eta[2])));
    v3 g = vcross(h, n2);
    F[0] = vdot(g, ta); F[1] = vdot(g, tb);
    return 1;
}

/* Newton polish with a central-difference Jacobian (reading of the one
 * Newton iteration of Sec. 7, applied to the exact constraints).            */
static int polish_tt(const tri_t *T1, const tri_t *T2, v3 x0, v3 x3, const double *eta, int ev1, int iters,
                     double *pu, double *pv)
{
    v3 nc = vnorm(tri_n(T2, 1.0 / 3.0, 1.0 / 3.0));
    v3 ref = fabs(nc.x) < 0.9 ? V(1, 0, 0) : V(0, 1, 0);
    v3 ta = vnorm(vcross(nc, ref)), tb = vcross(nc, ta);
    double u = *pu, v = *pv, step = 1e300;
    const double h = 1e-6;
    for (int it = 0; it < iters; ++it) {
        double F[2], Fu1[2], Fu0[2], Fv1[2], Fv0[2];
        if (!tt_residual(T1, T2, x0, x3, eta, ev1, ta, tb, u, v, F)) return 0;
        if (!tt_residual(T1, T2, x0, x3, eta, ev1, ta, tb, u + h, v, Fu1)) return 0;
        if (!tt_residual(T1, T2, x0, x3, eta, ev1, ta, tb, u - h, v, Fu0)) return 0;
        if (!tt_residual(T1, T2, x0, x3, eta, ev1, ta, tb, u, v + h, Fv1)) return 0;
        if (!tt_residual(T1, T2, x0, x3, eta, ev1, ta, tb, u, v - h, Fv0)) return 0;
        OPS(24);
        double J00 = (Fu1[0] - Fu0[0]) / (2 * h), J10 = (Fu1[1] - Fu0[1]) / (2 * h);
        double J01 = (Fv1[0] - Fv0[0]) / (2 * h), J11 = (Fv1[1] - Fv0[1]) / (2 * h);
        double det = J00 * J11 - J01 * J10;
        if (!(det != 0.0) || !isfinite(det)) return 0;
        double du = (F[0] * J11 - J01 * F[1]) / det;
        double dv = (J00 * F[1] - J10 * F[0]) / det;
        u -= du; v -= dv;
        step = fabs(du) + fabs(dv);
        if (!(step > 1e-15)) break;
    }
    *pu = u; *pv = v;
    return step <= 1e-10;
}


/* Sign of det R(v) through the resultant's product formula.  With
 * det R(v) = C lc_u(b)^(n - deg a) Res_u(a, b) (C a nonzero constant) and
 * Res_u(a, b) = lc_u(a)^(deg b) prod_{a(alpha)=0} b(alpha), where complex
 * conjugate roots contribute |b(alpha)|^2 > 0, the sign of det R(v) is, up to
 * the constant sign of C lc(b)^(n - deg a) (lc(b) is a constant for the TT
 * system), sgn(lc(a))^(deg b) times the product of sgn b(alpha) over the REAL
 * roots alpha of a(., v).  The real roots are isolated (Sec. 5.2 isolation) on
 * [-B, B] with B = 2 max_k |a_{m-k}/a_m|^(1/k) (Fujiwara's bound on every root),
 * in the scaled variable w = u/B.                                            */
static int res_sign_product(arena *A, bp a, int ma, bp b, int n, double v)
{
    size_t mark = A->top;
    double *ai = (double *)ar_alloc(A, sizeof(double) * (size_t)(ma + 1));
    double *bi = (double *)ar_alloc(A, sizeof(double) * (size_t)(b.d + 1));
    for (int i = 0; i <= ma; ++i) {
        double s = 0.0;
        for (int j = a.d - i; j >= 0; --j) s = s * v + a.c[i * (a.d + 1) + j];
        ai[i] = s;
    }
    for (int i = 0; i <= b.d; ++i) {
        double s = 0.0;
        for (int j = b.d - i; j >= 0; --j) s = s * v + b.c[i * (b.d + 1) + j];
        bi[i] = s;
    }
    /* The factor sgn(lc(a))^(deg b) is left out: it is +1 when deg_u b is even
     * (a refraction at x2: 6D + 2 + 2 f2) and a constant sign when lc_u(a) is a
     * constant (no top row of a dropped).  Otherwise (deg b odd: a reflection
     * at x2) each zero of lc_u(a)(v) in [0,1] adds a sign change that is not a
     * root of the resultant; its v yields no admissible path and the path phase
     * rejects it. */
    int sign = 1;
    (void)n;
    if (ai[ma] == 0.0) { A->top = mark; return 1; }
    double B = 0.0;
    for (int k = 1; k <= ma; ++k) B = fmax(B, pow(fabs(ai[ma - k] / ai[ma]), 1.0 / k));
    B = 2.0 * B;
    if (!(B > 0.0)) B = 1.0;
    double *w = (double *)ar_alloc(A, sizeof(double) * (size_t)(ma + 1));
    double pw = 1.0;
    for (int k = 0; k <= ma; ++k) { w[k] = ai[k] * pw; pw *= B; }
    double roots[64];
    int nr = isolate(A, w, ma, -1.0, 1.0, roots, 64);
    for (int k = 0; k < nr; ++k) {
        double al = roots[k] * B, s = 0.0;
        for (int i = b.d; i >= 0; --i) s = s * al + bi[i];
        if (s < 0.0) sign = -sign;
    }
    A->top = mark;
    return sign;
}

/* Paired product sign (det_method 2, the two-vertex default): the product
 * formula of res_sign_product, where two consecutive real roots of a(., v)
 * closer than 1e-4 max(1, |alpha|) contribute nothing.  Reading: such a pair
 * contributes b(alpha1) b(alpha2) ~ b(alpha)^2 > 0 unless b vanishes between
 * two nearly equal roots, and the pair does occur away from any solution:
 * where the direction x1 -> x2 turns parallel to T2's plane (x2 at infinity)
 * a(., v) has a near-double real pair far outside T1 at which b nearly vanishes
 * too, and there the FP64 values of b are rounding noise whose signs flip from
 * one v to the next (their 60-digit values do not).                        */
static int res_sign_paired(arena *A, bp a, int ma, bp b, double v)
{
    size_t mark = A->top;
    double *ai = (double *)ar_alloc(A, sizeof(double) * (size_t)(ma + 1));
    double *bi = (double *)ar_alloc(A, sizeof(double) * (size_t)(b.d + 1));
    /* a_i(v), b_i(v) by Horner, the root bound and the scaling to [-1, 1] */
    OPS((a.d + 1) * (a.d + 2) + (b.d + 1) * (b.d + 2) + 5 * ma + 2);
    for (int i = 0; i <= ma; ++i) {
        double s = 0.0;
        for (int j = a.d - i; j >= 0; --j) s = s * v + a.c[i * (a.d + 1) + j];
        ai[i] = s;
    }
    for (int i = 0; i <= b.d; ++i) {
        double s = 0.0;
        for (int j = b.d - i; j >= 0; --j) s = s * v + b.c[i * (b.d + 1) + j];
        bi[i] = s;
    }
    int sign = 1;
    if (ai[ma] == 0.0) { A->top = mark; return 1; }
    double B = 0.0;
    for (int k = 1; k <= ma; ++k) B = fmax(B, pow(fabs(ai[ma - k] / ai[ma]), 1.0 / k));
    B = 2.0 * B;
    if (!(B > 0.0)) B = 1.0;
    double *w = (double *)ar_alloc(A, sizeof(double) * (size_t)(ma + 1));
    double pw = 1.0;
    for (int k = 0; k <= ma; ++k) { w[k] = ai[k] * pw; pw *= B; }
    double roots[64];
    int nr = isolate(A, w, ma, -1.0, 1.0, roots, 64);
    for (int k = 0; k < nr; ++k) {
        double al = roots[k] * B;
        OPS(1);
        if (k + 1 < nr && roots[k + 1] * B - al <= 1e-4 * fmax(1.0, fabs(al))) { ++k; continue; }
        double s = 0.0;
        for (int i = b.d; i >= 0; --i) s = s * al + bi[i];
        OPS(2 * (b.d + 1));
        if (s < 0.0) sign = -sign;
    }
    A->top = mark;
    return sign;
}

/* Per-tuple constants of a two-vertex chain, to evaluate b(u, v) at a point
 * from the same defining products coeffs_2v expands (the mapped direction
 * Dt at x1, the homogeneous coordinates (kappa, ut, vt) of x2 on T2's plane,
 * M2, D2 and the product or square form at x2).                            */
typedef struct {
    tri_t T1, T2;
    v3 x0, x3, ax, edge;
    double eta1, eta2, etap, S, q0, q1, r0, r1, sg, n2len;
    int ev1, ev2, f2;
} chain2v;

static void chain2v_setup(chain2v *C, const tri_t *T1, const tri_t *T2, v3 x0, v3 x3, const double *eta,
                          int ev1, int ev2, const or_sqrtfit *fit)
{
    memset(C, 0, sizeof(*C));
    C->T1 = *T1; C->T2 = *T2; C->x0 = x0; C->x3 = x3;
    C->eta1 = eta[1]; C->eta2 = eta[2]; C->ev1 = ev1; C->ev2 = ev2;
    C->f2 = T2->flat ? 0 : 1;
    C->etap = eta[0] / eta[1];
    v3 c1 = tri_x(T1, 1.0 / 3.0, 1.0 / 3.0);
    if (ev1 != 0) {
        v3 nc1 = tri_n(T1, 1.0 / 3.0, 1.0 / 3.0);
        v3 d0c = vsub(c1, x0);
        C->S = vdot(nc1, nc1) * vdot(d0c, d0c);
        double dnc = vdot(d0c, nc1);
        double sc = 1.0 - C->etap * C->etap * (1.0 - dnc * dnc / C->S);
        int p = 0;
        for (int k = 1; k < 6; ++k) if (sc >= fit->bp[k]) p = k;
        C->q0 = fit->c[p][0]; C->q1 = fit->c[p][1]; C->r0 = fit->c[p][2]; C->r1 = fit->c[p][3];
        C->sg = dnc < 0.0 ? -1.0 : 1.0;
    }
    v3 c2 = tri_x(T2, 1.0 / 3.0, 1.0 / 3.0);
    if (ev2 == 0) C->edge = pick_edge2(c2, c1, x3, T2->e1, T2->e2) ? T2->e2 : T2->e1;
    else pick_axis(c2, c1, x3, &C->ax);
    C->n2len = vlen(vcross(T2->e1, T2->e2));
}

/* b(u, v) from its defining products, and |kappa| / (|Dt| |e1 x e2|) of T2:
 * the sine of the angle between the mapped ray from x1 and T2's plane (0
 * when x2 is at infinity).                                                 */
static double b2v_value(const chain2v *C, double u, double v, double *kratio)
{
    OPS(160);
    const tri_t *T1 = &C->T1, *T2 = &C->T2;
    v3 x1 = tri_x(T1, u, v), n1 = tri_n(T1, u, v);
    v3 d0 = vsub(x1, C->x0);
    double nn = vdot(n1, n1), dn = vdot(d0, n1);
    v3 Dt;
    if (C->ev1 == 0) {
        Dt = vsub(vmul(d0, nn), vmul(n1, 2.0 * dn));
    } else {
        double e2p = C->etap * C->etap;
        double beta = (1.0 - e2p) * nn * vdot(d0, d0) + e2p * dn * dn;
        double num = C->q1 / C->S * beta + C->q0, den = C->r1 / C->S * beta + C->r0;
        v3 tang = vsub(vmul(d0, nn), vmul(n1, dn));
        Dt = vadd(vmul(tang, C->etap * den), vmul(n1, C->sg * sqrt(C->S) * num));
    }
    v3 q = vsub(x1, T2->p0);
    v3 Dxe22 = vcross(Dt, T2->e2);
    double ut = vdot(Dxe22, q), vt = vdot(vcross(q, T2->e1), Dt), ka = vdot(Dxe22, T2->e1);
    v3 X2 = vadd(vmul(T2->p0, ka), vadd(vmul(T2->e1, ut), vmul(T2->e2, vt)));
    v3 M2 = vmul(T2->n0, ka);
    if (C->f2) M2 = vadd(M2, vadd(vmul(T2->dn1, ut), vmul(T2->dn2, vt)));
    v3 D2 = vsub(vmul(C->x3, ka), X2);
    double ld = vlen(Dt) * C->n2len;
    *kratio = ld > 0.0 ? fabs(ka) / ld : 0.0;
    if (C->ev2 == 0) {
        v3 t = vcross(M2, C->edge);
        return vdot(Dt, M2) * vdot(D2, t) + vdot(Dt, t) * vdot(D2, M2);
    }
    double l = vdot(vcross(Dt, M2), C->ax), r = vdot(vcross(D2, M2), C->ax);
    return C->eta1 * C->eta1 * vdot(D2, D2) * l * l - C->eta2 * C->eta2 * vdot(Dt, Dt) * r * r;
}

/* Sign of the resultant at v by the product formula over the real roots of
 * a(., v) (paired as in res_sign_paired), with two readings for the chain:
 * b at each root is evaluated from its defining products (the expanded
 * coefficients lose every digit at roots far from the triangle), and roots
 * where the mapped ray runs within 1e-4 rad of parallel to T2's plane are
 * left out.  There x2 is at infinity, no path can lie, and kappa divides both
 * a and b when T2 is flat or its vertex normals are proportional to its
 * positions (a sphere), which makes the resultant vanish identically and
 * the sign of such a factor a matter of rounding.                         */
#define OR_KAPPA_SKIP 1e-4
static int res_sign_chain(arena *A, bp a, int ma, const chain2v *C, double v)
{
    size_t mark = A->top;
    double *ai = (double *)ar_alloc(A, sizeof(double) * (size_t)(ma + 1));
    OPS((a.d + 1) * (a.d + 2) + 5 * ma + 2);
    for (int i = 0; i <= ma; ++i) {
        double s = 0.0;
        for (int j = a.d - i; j >= 0; --j) s = s * v + a.c[i * (a.d + 1) + j];
        ai[i] = s;
    }
    int sign = 1;
    if (ai[ma] == 0.0) { A->top = mark; return 1; }
    double B = 0.0;
    for (int k = 1; k <= ma; ++k) B = fmax(B, pow(fabs(ai[ma - k] / ai[ma]), 1.0 / k));
    B = 2.0 * B;
    if (!(B > 0.0)) B = 1.0;
    double *w = (double *)ar_alloc(A, sizeof(double) * (size_t)(ma + 1));
    double pw = 1.0;
    for (int k = 0; k <= ma; ++k) { w[k] = ai[k] * pw; pw *= B; }
    double roots[64];
    int nr = isolate(A, w, ma, -1.0, 1.0, roots, 64);
    for (int k = 0; k < nr; ++k) {
        double al = roots[k] * B;
        OPS(1);
        if (k + 1 < nr && roots[k + 1] * B - al <= 1e-4 * fmax(1.0, fabs(al))) { ++k; continue; }
        double kr;
        double s = b2v_value(C, al, v, &kr);
        if (kr < OR_KAPPA_SKIP) continue;
        if (s < 0.0) sign = -sign;
    }
    A->top = mark;
    return sign;
}

static void solve_2v(arena *A, const tri_t *T1, const tri_t *T2, v3 x0, v3 x3, const double *eta,
                     int ev1, int ev2, const or_sqrtfit *fit, const or_params *prm, int32_t qid,
                     or_sol *out, int32_t *nout, or_diag *dg)
{
    memset(dg, 0, sizeof(*dg));
    dg->min_gap = 1.0; dg->tangency = 1e300;
    if (T1->flat) dg->flags |= OR_F_FLAT1;
    if (T2->flat) dg->flags |= OR_F_FLAT2;
    bp a, b;
    g_stage = 0;
    int nb = coeffs_2v(A, T1, T2, x0, x3, eta, ev1, ev2, fit, &a, &b, &dg->flags);
    int ma = numeric_udeg(a, a.d);
    nb = numeric_udeg(b, nb);
    int n = ma > nb ? ma : nb;
    if (n < 1) { dg->flags |= OR_F_DEGENERATE; *nout = 0; return; }
    /* piecewise sign scan of det R(v) on [0,1] */
    int P = prm->pieces;
    int *sg = (int *)ar_alloc(A, sizeof(int) * (size_t)(P + 1));
    chain2v C;
    if (prm->det_method == 3) chain2v_setup(&C, T1, T2, x0, x3, eta, ev1, ev2, fit);
#define DETSIGN(vv) (prm->det_method == 3 ? res_sign_chain(A, a, ma, &C, (vv)) : \
                     prm->det_method == 2 ? res_sign_paired(A, a, ma, b, (vv)) : \
                     prm->det_method == 1 ? res_sign_product(A, a, ma, b, n, (vv)) : det_sign_at(A, a, b, n, (vv)))
    g_stage = 1;
    for (int j = 0; j <= P; ++j) sg[j] = DETSIGN((double)j / P);
    g_stage = 2;
    double vr[OR_MAXSOL * 8];
    int nv = 0;
    for (int j = 0; j < P; ++j) {
        if (sg[j] == sg[j + 1]) continue;
        double l = (double)j / P, r = (double)(j + 1) / P;
        int sl = sg[j];
        for (int it = 0; it < prm->bisect_iters; ++it) {
            double m = 0.5 * (l + r);
            if (DETSIGN(m) == sl) l = m; else r = m;
        }
        if (nv < OR_MAXSOL * 8) vr[nv++] = 0.5 * (l + r);
    }
    dg->n_vroots = nv;
    for (int k = 1; k < nv; ++k) dg->min_gap = fmin(dg->min_gap, vr[k] - vr[k - 1]);
    g_stage = 3;
    int nsol = 0;
    double etap = eta[0] / eta[1];
    for (int k = 0; k < nv; ++k) {
        double v = vr[k];
        double *auc = (double *)ar_alloc(A, sizeof(double) * (size_t)(ma + 1));
        for (int i = 0; i <= ma; ++i) {
            double s = 0.0;
            for (int j = a.d - i; j >= 0; --j) s = s * v + a.c[i * (a.d + 1) + j];
            auc[i] = s;
        }
        OPS((a.d + 1) * (a.d + 2));
        double ur[64];
        int nu = isolate(A, auc, ma, -prm->u_margin, 1.0 - v + prm->u_margin, ur, 64);
        for (int m = 0; m < nu; ++m) {
            double u = ur[m], vv = v;
            dg->n_cand++;
            if (!polish_tt(T1, T2, x0, x3, eta, ev1, prm->polish_iters, &u, &vv)) continue;
            if (!bary_inside(u, vv)) continue;
            double u2, v2; v3 x1, x2;
            if (!trace_x2(T1, T2, x0, u, vv, ev1, etap, &u2, &v2, &x1, &x2)) continue;
            if (!bary_inside(u2, v2)) continue;
            double r1, r2;
            if (!vertex_law(x0, x1, x2, tri_n(T1, u, vv), eta[0], eta[1], ev1, &r1)) continue;
            if (!vertex_law(x1, x2, x3, tri_n(T2, u2, v2), eta[1], eta[2], ev2, &r2)) continue;
            double res = fmax(r1, r2);
            if (!(res <= prm->tau)) continue;
            or_sol s;
            memset(&s, 0, sizeof(s));
            s.query = qid; s.u1 = u; s.v1 = vv; s.u2 = u2; s.v2 = v2;
            s.residual = res; s.edge = fmin(edge_dist(u, vv), edge_dist(u2, v2)); s.flags = dg->flags;
            nsol = add_solution(out, nsol, prm->dedup, s);
        }
    }
    dg->n_valid = nsol;
    *nout = nsol;
}

/* chain[0], chain[1]: event at x1 and at x2 (0 = reflection, 1 = refraction) */
int or_solve_2v(const double *P, const double *N, const int32_t *tri, int64_t nt,
                const double *x0s, const double *x3s,
                const int32_t *q_x0, const int32_t *q_x3, const int32_t *q_t1, const int32_t *q_t2, int64_t nq,
                const double *eta, const int32_t *chain, const or_sqrtfit *fit, const or_params *prm,
                or_sol *out, int32_t *count, or_diag *diag)
{
    (void)nt;
#pragma omp parallel
    {
        arena A;
        A.cap = (size_t)64 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < nq; ++q) {
            A.top = 0;
            tri_t T1 = load_tri(P, N, tri, q_t1[q]);
            tri_t T2 = load_tri(P, N, tri, q_t2[q]);
            solve_2v(&A, &T1, &T2, vload(x0s, q_x0[q]), vload(x3s, q_x3[q]), eta, chain[0], chain[1], fit, prm,
                     (int32_t)q, out + q * OR_MAXSOL, count + q, diag + q);
        }
        free(A.base);
    }
    return 0;
}

int or_solve_tt(const double *P, const double *N, const int32_t *tri, int64_t nt,
                const double *x0s, const double *x3s,
                const int32_t *q_x0, const int32_t *q_x3, const int32_t *q_t1, const int32_t *q_t2, int64_t nq,
                const double *eta, const or_sqrtfit *fit, const or_params *prm,
                or_sol *out, int32_t *count, or_diag *diag)
{
    const int32_t tt[2] = {1, 1};
    return or_solve_2v(P, N, tri, nt, x0s, x3s, q_x0, q_x3, q_t1, q_t2, nq, eta, tt, fit, prm, out, count, diag);
}

/* two-vertex coefficients for the pin tests (dense (d+1)^2 arrays, capacity 49*49) */
int or_coeffs_2v(const double *P, const double *N, const int32_t *tri, int64_t t1, int64_t t2,
                 const double *x0, const double *x3, const double *eta, const int32_t *chain, const or_sqrtfit *fit,
                 double *a_out, int32_t *da, double *b_out, int32_t *db, int32_t *n_bez, int32_t *flags)
{
    arena A; A.cap = (size_t)64 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    tri_t T1 = load_tri(P, N, tri, t1), T2 = load_tri(P, N, tri, t2);
    bp a, b; int fl = 0;
    int nb = coeffs_2v(&A, &T1, &T2, vload(x0, 0), vload(x3, 0), eta, chain[0], chain[1], fit, &a, &b, &fl);
    int ma = numeric_udeg(a, a.d);
    nb = numeric_udeg(b, nb);
    int n = ma > nb ? ma : nb;
    *da = a.d; *db = b.d; *n_bez = n; *flags = fl;
    memcpy(a_out, a.c, sizeof(double) * (size_t)(a.d + 1) * (size_t)(a.d + 1));
    memcpy(b_out, b.c, sizeof(double) * (size_t)(b.d + 1) * (size_t)(b.d + 1));
    free(A.base);
    return 0;
}

int or_coeffs_tt(const double *P, const double *N, const int32_t *tri, int64_t t1, int64_t t2,
                 const double *x0, const double *x3, const double *eta, const or_sqrtfit *fit,
                 double *a_out, int32_t *da, double *b_out, int32_t *db, int32_t *n_bez, int32_t *flags)
{
    const int32_t tt[2] = {1, 1};
    return or_coeffs_2v(P, N, tri, t1, t2, x0, x3, eta, tt, fit, a_out, da, b_out, db, n_bez, flags);
}

/* sign of det R(v) for given bivariate a, b and Bezout size n */
int or_det_sign(const double *a_in, int32_t da, const double *b_in, int32_t db, int32_t n, double v)
{
    arena A; A.cap = (size_t)16 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    bp a = bp_new(&A, da), b = bp_new(&A, db);
    memcpy(a.c, a_in, sizeof(double) * (size_t)(da + 1) * (size_t)(da + 1));
    memcpy(b.c, b_in, sizeof(double) * (size_t)(db + 1) * (size_t)(db + 1));
    int s = det_sign_at(&A, a, b, n, v);
    free(A.base);
    return s;
}

/* sign of det R(v) through the product formula over the real roots of
 * a(., v) (u-degree ma), for given bivariate a, b                          */
int or_res_sign(const double *a_in, int32_t da, const double *b_in, int32_t db, int32_t ma, double v)
{
    arena A; A.cap = (size_t)16 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    bp a = bp_new(&A, da), b = bp_new(&A, db);
    memcpy(a.c, a_in, sizeof(double) * (size_t)(da + 1) * (size_t)(da + 1));
    memcpy(b.c, b_in, sizeof(double) * (size_t)(db + 1) * (size_t)(db + 1));
    int s = res_sign_product(&A, a, ma, b, 0, v);
    free(A.base);
    return s;
}

/* paired product sign (det_method 2) for given bivariate a, b */
int or_res_sign_paired(const double *a_in, int32_t da, const double *b_in, int32_t db, int32_t ma, double v)
{
    arena A; A.cap = (size_t)16 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    bp a = bp_new(&A, da), b = bp_new(&A, db);
    memcpy(a.c, a_in, sizeof(double) * (size_t)(da + 1) * (size_t)(da + 1));
    memcpy(b.c, b_in, sizeof(double) * (size_t)(db + 1) * (size_t)(db + 1));
    int s = res_sign_paired(&A, a, ma, b, v);
    free(A.base);
    return s;
}

/* Op counts by stage (ops[4 q + s]) of each query, solved one at a time on
 * the calling thread with the same arithmetic as or_solve_1bounce.         */
int or_opcount_1bounce(const double *P, const double *N, const int32_t *tri,
                       const double *x0s, const double *x2s,
                       const int32_t *q_x0, const int32_t *q_x2, const int32_t *q_tri, int64_t nq,
                       int32_t refract, double eta0, double eta1, const or_params *prm, uint64_t *ops)
{
    arena A;
    A.cap = (size_t)8 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    or_sol out[OR_MAXSOL];
    for (int64_t q = 0; q < nq; ++q) {
        A.top = 0;
        memset(g_ops, 0, sizeof(g_ops));
        g_count = 1;
        int32_t cnt; or_diag dg;
        tri_t T = load_tri(P, N, tri, q_tri[q]);
        solve_1b(&A, &T, vload(x0s, q_x0[q]), vload(x2s, q_x2[q]), refract, eta0, eta1, prm, (int32_t)q,
                 out, &cnt, &dg);
        for (int k = 0; k < 4; ++k) ops[4 * q + k] = g_ops[k];
    }
    free(A.base);
    return 0;
}

int or_opcount_2v(const double *P, const double *N, const int32_t *tri,
                  const double *x0s, const double *x3s,
                  const int32_t *q_x0, const int32_t *q_x3, const int32_t *q_t1, const int32_t *q_t2, int64_t nq,
                  const double *eta, const int32_t *chain, const or_sqrtfit *fit, const or_params *prm,
                  uint64_t *ops)
{
    arena A;
    A.cap = (size_t)64 << 20; A.top = 0; A.base = (char *)malloc(A.cap);
    or_sol out[OR_MAXSOL];
    for (int64_t q = 0; q < nq; ++q) {
        A.top = 0;
        memset(g_ops, 0, sizeof(g_ops));
        g_count = 1;
        int32_t cnt; or_diag dg;
        tri_t T1 = load_tri(P, N, tri, q_t1[q]), T2 = load_tri(P, N, tri, q_t2[q]);
        solve_2v(&A, &T1, &T2, vload(x0s, q_x0[q]), vload(x3s, q_x3[q]), eta, chain[0], chain[1], fit, prm,
                 (int32_t)q, out, &cnt, &dg);
        for (int k = 0; k < 4; ++k) ops[4 * q + k] = g_ops[k];
    }
    free(A.base);
    return 0;
}

/* host threads of the parallel solves (OpenMP); returns the previous count */
int or_set_threads(int n)
{
    int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
}

int or_maxsol(void) { return OR_MAXSOL; }

/* ================================================================== Normal-cone cull twin (FP64)
 * keep[(j0*n2 + j2)*nt + t] = 1 unless the cone of generalised half vectors
 * h = eta0 w0 + eta1 w2 (w0, w2: unit directions from a point of the
 * triangle's bounding sphere to x0 and x2) cannot meet the cone of the vertex
 * normals: with chord bounds |w - a| <= 2 sin(theta/2), h lies within
 * asin(delta/L) of H = eta0 a0 + eta1 a2 (L = |H|, delta = eta0 ch0 + eta1 ch2);
 * h x n = 0 needs the angle between the lines of H and of the normal-cone axis
 * to be at most theta_n + asin(delta/L).  `margin` (radians) widens the test.  */
int or_cull_1bounce(const double *P, const double *N, const int32_t *tri, int64_t nt,
                    const double *x0s, int64_t n0, const double *x2s, int64_t n2,
                    double eta0, double eta1, double margin, uint8_t *keep)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; ++t) {
        v3 p[3], n[3];
        for (int k = 0; k < 3; ++k) { p[k] = vload(P, tri[3 * t + k]); n[k] = vnorm(vload(N, tri[3 * t + k])); }
        v3 c = vmul(vadd(vadd(p[0], p[1]), p[2]), 1.0 / 3.0);
        double rad = fmax(fmax(vlen(vsub(p[0], c)), vlen(vsub(p[1], c))), vlen(vsub(p[2], c)));
        v3 an = vadd(vadd(n[0], n[1]), n[2]);
        double lan = vlen(an);
        an = vnorm(an);
        double thn = 0.0;
        for (int k = 0; k < 3; ++k) thn = fmax(thn, acos(fmin(1.0, fmax(-1.0, vdot(an, n[k])))));
        for (int64_t j0 = 0; j0 < n0; ++j0)
            for (int64_t j2 = 0; j2 < n2; ++j2) {
                int k = 1;
                v3 va = vsub(vload(x0s, j0), c), vb = vsub(vload(x2s, j2), c);
                double da = vlen(va), db = vlen(vb);
                if (lan > 0.5 && thn < M_PI / 2 && da > rad && db > rad) {
                    v3 aa = vmul(va, 1.0 / da), ab = vmul(vb, 1.0 / db);
                    double sa = rad / da, sb = rad / db;
                    double cha = sqrt(fmax(0.0, 2.0 - 2.0 * sqrt(fmax(0.0, 1.0 - sa * sa))));
                    double chb = sqrt(fmax(0.0, 2.0 - 2.0 * sqrt(fmax(0.0, 1.0 - sb * sb))));
                    v3 H = vadd(vmul(aa, eta0), vmul(ab, eta1));
                    double L = vlen(H), delta = eta0 * cha + eta1 * chb;
                    if (delta < L) {
                        double lim = thn + asin(delta / L) + margin;
                        if (lim < M_PI / 2) {
                            double cphi = fabs(vdot(an, H)) / L;
                            k = cphi >= cos(lim);
                        }
                    }
                }
                keep[(j0 * n2 + j2) * nt + t] = (uint8_t)k;
            }
    }
    return 0;
}

/* ================================================================== Normal-cone cull twin for two vertices (FP64)
 * Tuple (x0, T1, T2, x3) is kept unless one of the two vertices fails the
 * half-vector / normal-cone test of or_cull_1bounce: at x1 the directions go to
 * x0 (eta[0]) and into the cone from T1 to T2 (eta[1]); at x2 they go into
 * the cone from T2 to T1 (eta[1]) and to x3 (eta[2]).  The cone between the
 * bounding spheres of two triangles has axis c_b - c_a and half angle
 * asin((r_a + r_b)/|c_b - c_a|).  keep: [n0, n3, nt, nt] bytes.            */
typedef struct { v3 c, an; double rad, thn; int ok; } or_cone;

static or_cone tri_cone(const double *P, const double *N, const int32_t *tri, int64_t t)
{
    or_cone k;
    v3 p[3], n[3];
    for (int j = 0; j < 3; ++j) { p[j] = vload(P, tri[3 * t + j]); n[j] = vnorm(vload(N, tri[3 * t + j])); }
    k.c = vmul(vadd(vadd(p[0], p[1]), p[2]), 1.0 / 3.0);
    k.rad = fmax(fmax(vlen(vsub(p[0], k.c)), vlen(vsub(p[1], k.c))), vlen(vsub(p[2], k.c)));
    v3 an = vadd(vadd(n[0], n[1]), n[2]);
    k.ok = vlen(an) > 0.5;
    k.an = vnorm(an);
    k.thn = 0.0;
    for (int j = 0; j < 3; ++j) k.thn = fmax(k.thn, acos(fmin(1.0, fmax(-1.0, vdot(k.an, n[j])))));
    return k;
}

/* direction cone (axis a, chord bound ch = 2 sin(theta/2)); returns 0 if unbounded */
static int dir_cone(v3 from, double r, v3 to, double *ch, v3 *a)
{
    v3 d = vsub(to, from);
    double l = vlen(d);
    if (!(l > r)) return 0;
    *a = vmul(d, 1.0 / l);
    double s = r / l;
    *ch = sqrt(fmax(0.0, 2.0 - 2.0 * sqrt(fmax(0.0, 1.0 - s * s))));
    return 1;
}

static int vertex_cone_keep(const or_cone *k, v3 aa, double cha, double ea, v3 ab, double chb, double eb, double margin)
{
    if (!k->ok || !(k->thn < M_PI / 2)) return 1;
    v3 H = vadd(vmul(aa, ea), vmul(ab, eb));
    double L = vlen(H), delta = ea * cha + eb * chb;
    if (!(delta < L)) return 1;
    double lim = k->thn + asin(delta / L) + margin;
    if (lim >= M_PI / 2) return 1;
    return fabs(vdot(k->an, H)) / L >= cos(lim);
}

int or_cull_tt(const double *P, const double *N, const int32_t *tri, int64_t nt,
               const double *x0s, int64_t n0, const double *x3s, int64_t n3,
               const double *eta, double margin, uint8_t *keep)
{
    or_cone *K = (or_cone *)malloc(sizeof(or_cone) * (size_t)nt);
    for (int64_t t = 0; t < nt; ++t) K[t] = tri_cone(P, N, tri, t);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t1 = 0; t1 < nt; ++t1)
        for (int64_t t2 = 0; t2 < nt; ++t2)
            for (int64_t j0 = 0; j0 < n0; ++j0)
                for (int64_t j3 = 0; j3 < n3; ++j3) {
                    uint8_t k = 0;
                    if (t1 != t2) {
                        const or_cone *A1 = &K[t1], *A2 = &K[t2];
                        v3 x0 = vload(x0s, j0), x3 = vload(x3s, j3);
                        double ch0, ch12, ch21, ch3;
                        v3 a0, a12, a21, a3;
                        int b0 = dir_cone(A1->c, A1->rad, x0, &ch0, &a0);
                        int b12 = dir_cone(A1->c, A1->rad + A2->rad, A2->c, &ch12, &a12);
                        int b21 = dir_cone(A2->c, A1->rad + A2->rad, A1->c, &ch21, &a21);
                        int b3 = dir_cone(A2->c, A2->rad, x3, &ch3, &a3);
                        int k1 = (b0 && b12) ? vertex_cone_keep(A1, a0, ch0, eta[0], a12, ch12, eta[1], margin) : 1;
                        int k2 = (b21 && b3) ? vertex_cone_keep(A2, a21, ch21, eta[1], a3, ch3, eta[2], margin) : 1;
                        k = (uint8_t)(k1 && k2);
                    }
                    keep[((j0 * n3 + j3) * nt + t1) * nt + t2] = k;
                }
    free(K);
    return 0;
}
