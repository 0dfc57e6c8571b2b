// One specular vertex (systems R and T of Sec. 4.5): coefficient phase,
// Bezout elimination with Laplace expansion, recursive root isolation in v,
// u from a(u)|_v, FP64 Newton polish, path-space validation and wave-ballot
// compaction -- one instance per lane, everything in registers.
#include "spoly_dev.hpp"
#include "laplace_gen.inc"
#include "onebounce.hpp"

namespace spoly {

constexpr int kMaxLaneSol = 4;
constexpr double kNearDoubleU = 1e-3;   // u-root pairs closer than this are tried from their midpoint
constexpr double kRefineWindow = 0.005; // FP32 reflection: refine v when the nearest u misses the triangle by less
// FP32 reflection: refine v when a(u)|v has a complex u pair this close to the
// real axis with its real part in (or this close to) the triangle.  Near a fold
// of the coplanarity curve (a double u root) the pair's imaginary part grows
// like the square root of the error in v: a v error of 1e-5, typical of the
// FP32 resultant, can open a pair 0.05 wide at a solution 1e-6 from the fold.
// At the roots of the FP64 resultant such pairs do not occur (none among
// 8245 roots of 30000 glints candidates), so the hand-offs stay rare.
constexpr double kComplexWindow = 0.1;
// FP32 reflection: a candidate whose r(v) comes within this fraction of sum |r_k|
// of zero at v = 0, v = 1 or a critical point in [0,1] without the isolation
// seeing a sign change there (or with one that rounding may have moved) is
// solved in FP64 instead: a near-double root (the relabelled e2 system has
// such pairs, one root valid and one superfluous) or a root next to an end of
// [0,1] can vanish from, or move out of, the FP32 r(v).
constexpr double kTangentFrac = 1e-3;

struct Geo {            // FP64 geometry of one instance (after the edge relabelling)
    V3<double> p0, e1, e2, n0, dn1, dn2, x0, x2;
    int axis;           // square-form projection axis (T)
    bool flat;          // all three vertex normals equal
    bool swapped;       // vertices 1 and 2 exchanged: (u, v) of the kernel = (v, u) of the mesh
};

// ---------------------------------------------------------------- rules (FP64, as the oracle)
// Product form tangent t = n x e1 unless e1 nearly lies in the incidence plane
// (|e1^.m_c| < 1/4 and e2 does better), then t = n x e2.  Instead of using the
// u-degree-4 system of t = n x e2, the kernel exchanges the triangle's
// vertices 1 and 2: the system is then of the t = n x e1 shape in (u', v') =
// (v, u), whose Bezout size is 3 in u'.
__device__ __forceinline__ bool pick_edge2(V3<double> c, V3<double> xa, V3<double> xb, V3<double> e1, V3<double> e2)
{
    V3<double> m = cross(c - xa, xb - xa);
    double l = len(m);
    if (!(l > 0.0)) return false;
    m = m * (1.0 / l);
    double g1 = fabs(dot(normalized(e1), m)), g2 = fabs(dot(normalized(e2), m));
    return g1 < 0.25 && g2 > g1;
}
// Square form axis: x^ if |m_c.x^| >= 1/2, else z^ if |m_c.z^| >= 1/2, else y^.
__device__ __forceinline__ int pick_axis(V3<double> c, V3<double> xa, V3<double> xb)
{
    V3<double> m = cross(c - xa, xb - xa);
    double l = len(m);
    if (!(l > 0.0)) return 0;
    m = m * (1.0 / l);
    if (fabs(m.x) >= 0.5) return 0;
    if (fabs(m.z) >= 0.5) return 2;
    return 1;
}

// ---------------------------------------------------------------- coefficient phase
// a = ((x1 - x0) x (x2 - x0)) . n                          (Eq. eq_coplane)
// R: b = (d0.n)(d1.t) + (d0.t)(d1.n), t = n x e1           (Eq. eq_pf_result)
// T: b = eta0^2 |d1|^2 ((d0 x n).ax)^2 - eta1^2 |d0|^2 ((d1 x n).ax)^2   (Eq. eq_cpf_result)
template <typename R, int EV, int F>
struct Sys {
    static constexpr int TA = 1 + F;
    static constexpr int TB = EV == SPOLY_R ? 2 + 2 * F : 4 + 2 * F;
    static constexpr int N = EV == SPOLY_R ? 1 + 2 * F : 4 + 2 * F;
    static constexpr int DR = N * (TA + TB - 1) - N * (N - 1);
};

template <typename R, int F>
struct NormalPoly;
template <typename R>
struct NormalPoly<R, 0> {
    static __device__ __forceinline__ VP<R, 0> make(const Geo& g) { return vp_const(cvt<R>(g.n0)); }
};
template <typename R>
struct NormalPoly<R, 1> {
    static __device__ __forceinline__ VP<R, 1> make(const Geo& g)
    {
        return vp_affine(cvt<R>(g.n0), cvt<R>(g.dn1), cvt<R>(g.dn2));
    }
};

template <typename R, int EV, int F>
__device__ __forceinline__ void build_ab(const Geo& g, double eta0, double eta1, P2<R, 1 + F>& a,
                                         P2<R, Sys<R, EV, F>::TB>& b)
{
    VP<R, 1> x1 = vp_affine(cvt<R>(g.p0), cvt<R>(g.e1), cvt<R>(g.e2));
    auto n = NormalPoly<R, F>::make(g);
    VP<R, 1> d0 = x1 - vp_const(cvt<R>(g.x0));
    VP<R, 1> d1 = vp_const(cvt<R>(g.x2)) - x1;
    VP<R, 0> w = vp_const(cvt<R>(g.x2 - g.x0));
    a = vdot(vcross(d0, w), n);
    if constexpr (EV == SPOLY_R) {
        auto t = vcross(n, vp_const(cvt<R>(g.e1)));
        auto full = vdot(d0, n) * vdot(d1, t) + vdot(d0, t) * vdot(d1, n);
        b = full;
    } else {
        auto l = vcomp(vcross(d0, n), g.axis);
        auto r = vcomp(vcross(d1, n), g.axis);
        auto t1 = vdot(d1, d1) * (l * l);
        auto t2 = vdot(d0, d0) * (r * r);
        b = lc(R(eta0 * eta0), t1, R(-eta1 * eta1), t2);
    }
}

template <typename R, int D>
__device__ __forceinline__ R normalise(P2<R, D>& p)
{
    R m = R(0);
#pragma unroll
    for (int k = 0; k < tri_size(D); ++k) m = fmax(m, fabs(p.c[k]));
    if (m > R(0)) {
        R s = R(1) / m;
#pragma unroll
        for (int k = 0; k < tri_size(D); ++k) p.c[k] *= s;
    }
    return m;
}

template <typename R, int EV, int F>
__device__ __forceinline__ void eliminate(const R* A, const R* B, R* r)
{
    if constexpr (EV == SPOLY_R && F == 1) elim_r_interp<R>(A, B, r);
    else if constexpr (EV == SPOLY_R && F == 0) elim_r_flat<R>(A, B, r);
    else if constexpr (EV == SPOLY_T && F == 1) elim_t_interp<R>(A, B, r);
    else elim_t_flat<R>(A, B, r);
}

// ---------------------------------------------------------------- univariate solve (Sec. 5.2)
// Recursive isolation on [0,1]: the roots of p' split [0,1] into monotone
// pieces; a piece with a strict sign change (sgn(0) := +1) holds one root,
// bisected until the interval is shorter than eps.  Roots are kept in the slot
// of the piece they come from (no compaction, so every register index is a
// compile-time constant); ok[k] marks a root in slot k.
template <typename R, int D>
__device__ __forceinline__ R bisect(const R (&c)[D + 1], R lo, R hi, bool neg_lo, R eps)
{
    for (int it = 0; it < 80; ++it) {
        if (!(hi - lo > eps)) break;
        R m = (lo + hi) * R(0.5);
        if (!(m > lo && m < hi)) break;
        bool neg = horner<R, D>(c, m) < R(0);
        if (neg == neg_lo) lo = m;
        else hi = m;
    }
    return (lo + hi) * R(0.5);
}

template <typename R, int D>
__device__ __forceinline__ void scan_pieces(const R (&c)[D + 1], const R (&bp)[D], const bool (&bok)[D],
                                            R (&rt)[D + 1], bool (&ok)[D + 1], R eps, R* minabs = nullptr)
{
    R lo = R(0), flo = horner<R, D>(c, R(0));
    R last = R(-1e30);
    if (minabs) *minabs = fabs(flo);
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        ok[k] = false;
        rt[k] = R(0);
        bool has = (k < D) ? bok[k] : true;
        R hi = (k < D) ? bp[k] : R(1);
        if (has) {
            R fhi = horner<R, D>(c, hi);
            if (minabs) *minabs = fmin(*minabs, fabs(fhi));
            if (hi > lo && ((flo < R(0)) != (fhi < R(0)))) {
                R x = bisect<R, D>(c, lo, hi, flo < R(0), eps);
                if (x - last > R(1e-12)) {
                    rt[k] = x;
                    ok[k] = true;
                    last = x;
                }
            }
            lo = hi;
            flo = fhi;
        }
    }
}

// With minabs, the smallest |c| over the piece ends (0, 1 and the critical
// points in between) is returned there.
template <typename R, int D>
__device__ __forceinline__ void isolate01(const R (&c)[D + 1], R (&rt)[D + 1], bool (&ok)[D + 1], R eps,
                                          R* minabs = nullptr)
{
    R bp[D];
    bool bok[D];
    if constexpr (D == 1) {
        bok[0] = false;
        bp[0] = R(0);
    } else {
        R dc[D];
#pragma unroll
        for (int k = 0; k < D; ++k) dc[k] = c[k + 1] * R(k + 1);
        R brt[D];
        bool bbok[D];
        isolate01<R, D - 1>(dc, brt, bbok, eps);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            bp[k] = brt[k];
            bok[k] = bbok[k];
        }
    }
    scan_pieces<R, D>(c, bp, bok, rt, ok, eps, minabs);
}

// ---------------------------------------------------------------- path phase (FP64)
// a, b and their partial derivatives evaluated directly from the geometry.
template <int EV>
__device__ __forceinline__ void eval_ab(const Geo& g, double eta0, double eta1, double u, double v, double& fa,
                                        double& au, double& av, double& fb, double& bu, double& bv)
{
    V3<double> x1 = g.p0 + g.e1 * u + g.e2 * v;
    V3<double> n = g.n0 + g.dn1 * u + g.dn2 * v;
    V3<double> d0 = x1 - g.x0, d1 = g.x2 - x1, w = g.x2 - g.x0;
    V3<double> cw = cross(d0, w);
    fa = dot(cw, n);
    au = dot(cross(g.e1, w), n) + dot(cw, g.dn1);
    av = dot(cross(g.e2, w), n) + dot(cw, g.dn2);
    if constexpr (EV == SPOLY_R) {
        V3<double> t = cross(n, g.e1), tu = cross(g.dn1, g.e1), tv = cross(g.dn2, g.e1);
        double p = dot(d0, n), q = dot(d1, t), r = dot(d0, t), s = dot(d1, n);
        double pu = dot(g.e1, n) + dot(d0, g.dn1), pv = dot(g.e2, n) + dot(d0, g.dn2);
        double qu = -dot(g.e1, t) + dot(d1, tu), qv = -dot(g.e2, t) + dot(d1, tv);
        double ru = dot(g.e1, t) + dot(d0, tu), rv = dot(g.e2, t) + dot(d0, tv);
        double su = -dot(g.e1, n) + dot(d1, g.dn1), sv = -dot(g.e2, n) + dot(d1, g.dn2);
        fb = p * q + r * s;
        bu = pu * q + p * qu + ru * s + r * su;
        bv = pv * q + p * qv + rv * s + r * sv;
    } else {
        auto comp = [&](V3<double> x) { return g.axis == 0 ? x.x : (g.axis == 1 ? x.y : x.z); };
        double l = comp(cross(d0, n)), r = comp(cross(d1, n));
        double lu = comp(cross(g.e1, n) + cross(d0, g.dn1)), lv = comp(cross(g.e2, n) + cross(d0, g.dn2));
        double ru = comp(cross(g.e1 * -1.0, n) + cross(d1, g.dn1)), rv = comp(cross(g.e2 * -1.0, n) + cross(d1, g.dn2));
        double s1 = dot(d1, d1), s0 = dot(d0, d0);
        double s1u = -2.0 * dot(d1, g.e1), s1v = -2.0 * dot(d1, g.e2);
        double s0u = 2.0 * dot(d0, g.e1), s0v = 2.0 * dot(d0, g.e2);
        double k0 = eta0 * eta0, k1 = eta1 * eta1;
        fb = k0 * s1 * l * l - k1 * s0 * r * r;
        bu = k0 * (s1u * l * l + 2.0 * s1 * l * lu) - k1 * (s0u * r * r + 2.0 * s0 * r * ru);
        bv = k0 * (s1v * l * l + 2.0 * s1 * l * lv) - k1 * (s0v * r * r + 2.0 * s0 * r * rv);
    }
}

template <int EV>
__device__ __forceinline__ bool polish(const Geo& g, double eta0, double eta1, int iters, double& u, double& v)
{
    double step = 1e300;
    for (int it = 0; it < iters; ++it) {
        double fa, au, av, fb, bu, bv;
        eval_ab<EV>(g, eta0, eta1, u, v, fa, au, av, fb, bu, bv);
        double det = au * bv - av * bu;
        if (!(det != 0.0) || !isfinite(det)) break;
        double du = (fa * bv - av * fb) / det;
        double dv = (au * fb - fa * bu) / det;
        u -= du;
        v -= dv;
        step = fabs(du) + fabs(dv);
        // Newton converges quadratically at a simple solution: after a step
        // below 1e-13 the error left is far below FP64 rounding, and further
        // steps only move within the rounding of the residual.
        if (!(step > 1e-13)) break;
    }
    return step <= 1e-10;
}

// Path-space check of Eq. eq_ch: wi, wo unit directions to the neighbours,
// h = eta_in wi + eta_out wo; admissible iff |h^ x n^| <= tau and the sides
// agree with the event ((wi.n)(wo.n) > 0 for R, < 0 for T).
__device__ __forceinline__ bool vertex_law(V3<double> xp, V3<double> x, V3<double> xn, V3<double> nrm, double ein,
                                           double eout, bool refract, double& res)
{
    double ln = len(nrm);
    if (!(ln > 1e-12)) {
        res = 1e300;
        return false;
    }
    V3<double> nh = nrm * (1.0 / ln);
    V3<double> wi = normalized(xp - x), wo = normalized(xn - x);
    V3<double> h = wi * ein + wo * eout;
    double lh = len(h);
    if (!(lh > 0.0)) {
        res = 1e300;
        return false;
    }
    res = len(cross(h * (1.0 / lh), nh));
    double side = dot(wi, nh) * dot(wo, nh);
    return refract ? side < 0.0 : side > 0.0;
}

struct LaneSols {
    double u[kMaxLaneSol], v[kMaxLaneSol], res[kMaxLaneSol], edge[kMaxLaneSol];
    int n;
    int over;  // solutions past the kMaxLaneSol kept (counted, not written)
};

__device__ __forceinline__ void push_sol(LaneSols& S, double u, double v, double res, double edge, double dedup)
{
    bool dup = false;
#pragma unroll
    for (int k = 0; k < kMaxLaneSol; ++k)
        if (k < S.n && fabs(S.u[k] - u) < dedup && fabs(S.v[k] - v) < dedup) dup = true;
    if (dup) return;
#pragma unroll
    for (int k = 0; k < kMaxLaneSol; ++k)
        if (k == S.n) {
            S.u[k] = u;
            S.v[k] = v;
            S.res[k] = res;
            S.edge[k] = edge;
        }
    if (S.n < kMaxLaneSol) S.n++;
    else S.over++;
}

// Coefficients and elimination: r(v), normalised.  Returns false for a
// degenerate instance (r not finite or identically zero).
template <typename R, int EV, int F>
__device__ __forceinline__ bool front_poly(const Geo& g, const OneBounceArgs& A, R (&r)[Sys<R, EV, F>::DR + 1])
{
    using Y = Sys<R, EV, F>;
    P2<R, Y::TA> a;
    P2<R, Y::TB> b;
    build_ab<R, EV, F>(g, A.eta0, A.eta1, a, b);
    normalise(a);
    normalise(b);
    eliminate<R, EV, F>(a.c, b.c, r);
    R rmax = R(0);
    bool finite = true;
#pragma unroll
    for (int k = 0; k <= Y::DR; ++k) {
        rmax = fmax(rmax, fabs(r[k]));
        finite = finite && isfinite(r[k]);
    }
    return finite && rmax > R(0);
}

// r(v) not finite or identically zero (the test front_poly applies)
template <typename R, int D>
__device__ __forceinline__ bool front_poly_degenerate(const R (&r)[D + 1])
{
    R rmax = R(0);
    bool finite = true;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        rmax = fmax(rmax, fabs(r[k]));
        finite = finite && isfinite(r[k]);
    }
    return !(finite && rmax > R(0));
}

// Coefficients, elimination and isolation: the roots of r(v) in [0,1] in
// ascending order.  Returns their number (degen set for a degenerate instance).
// In FP32, `uncertain` is set when r comes within kTangentFrac of zero at a
// piece end (see kTangentFrac); FP64 never sets it.
template <typename R, int EV, int F>
__device__ __forceinline__ int front_roots(const Geo& g, const OneBounceArgs& A, R (&rt)[Sys<R, EV, F>::DR + 1],
                                           bool (&ok)[Sys<R, EV, F>::DR + 1], int& degen, bool& uncertain)
{
    using Y = Sys<R, EV, F>;
    R r[Y::DR + 1];
    uncertain = false;
    if (!front_poly<R, EV, F>(g, A, r)) {
        degen = 1;
#pragma unroll
        for (int k = 0; k <= Y::DR; ++k) ok[k] = false;
        return 0;
    }

    if constexpr (sizeof(R) == 4) {
        R minabs;
        isolate01<R, Y::DR>(r, rt, ok, R(A.iso_eps), &minabs);
        R l1 = R(0);
#pragma unroll
        for (int k = 0; k <= Y::DR; ++k) l1 += fabs(r[k]);
        uncertain = !(minabs > R(kTangentFrac) * l1);
    } else {
        isolate01<R, Y::DR>(r, rt, ok, R(A.iso_eps));
    }
    int n = 0;
#pragma unroll
    for (int k = 0; k <= Y::DR; ++k) n += ok[k] ? 1 : 0;
    return n;
}

// FP64 coefficients of a(u, v) as a polynomial in u (u-degree TA, constant leading term)
template <int F>
__device__ __forceinline__ P2<double, 1 + F> a_fp64(const Geo& g)
{
    VP<double, 1> x1 = vp_affine(g.p0, g.e1, g.e2);
    auto n = NormalPoly<double, F>::make(g);
    VP<double, 1> d0 = x1 - vp_const(g.x0);
    return vdot(vcross(d0, vp_const(g.x2 - g.x0)), n);
}

// Determinant of the Bezout matrix of a(., v0) and b(., v0) for reflection,
// evaluated in FP64 from the geometry at a fixed v0: the same construction as
// the generated elimination (B_ij = sum_k a_{i-k} b_{j+1+k} - b_{i-k} a_{j+1+k},
// b truncated at the Bezout size), i.e. r(v0) up to a positive factor.
template <int F>
__device__ __forceinline__ double bezout_det_r(const Geo& g, double v0)
{
    constexpr int N = 1 + 2 * F;
    const V3<double> P = g.p0 + g.e2 * v0;
    const V3<double> E = g.e1, w = g.x2 - g.x0;
    const V3<double> N0 = F ? g.n0 + g.dn2 * v0 : g.n0;
    const V3<double> N1 = F ? g.dn1 : V3<double>{0.0, 0.0, 0.0};
    const V3<double> D0 = P - g.x0, D1 = g.x2 - P;
    const V3<double> A0 = cross(D0, w), A1 = cross(E, w);
    double a[4] = {dot(A0, N0), dot(A0, N1) + dot(A1, N0), dot(A1, N1), 0.0};
    const V3<double> T0 = cross(N0, E), T1 = cross(N1, E);
    const double dn[3] = {dot(D0, N0), dot(D0, N1) + dot(E, N0), dot(E, N1)};
    const double d1t[3] = {dot(D1, T0), dot(D1, T1) - dot(E, T0), -dot(E, T1)};
    const double d0t[3] = {dot(D0, T0), dot(D0, T1) + dot(E, T0), dot(E, T1)};
    const double d1n[3] = {dot(D1, N0), dot(D1, N1) - dot(E, N0), -dot(E, N1)};
    double b[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) b[i + j] += dn[i] * d1t[j] + d0t[i] * d1n[j];
    auto av = [&](int p) { return p <= 2 ? a[p] : 0.0; };
    auto bv = [&](int p) { return p <= N ? b[p] : 0.0; };
    double B[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double e = 0.0;
#pragma unroll
            for (int k = 0; k <= (i < N - 1 - j ? i : N - 1 - j); ++k) {
                const int pp = i - k, qq = j + 1 + k;
                if (pp != qq) e += av(pp) * bv(qq) - bv(pp) * av(qq);
            }
            B[i][j] = e;
        }
    double det;
    if constexpr (N == 1) {
        det = B[0][0];
    } else {
        det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
              B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    }
    return det;
}

// FP64 refinement of a root v of r found in FP32: secant iterations on the
// FP64 Bezout determinant started at v and v + 1e-6 (up to six; two suffice
// from an FP32-accurate root).  FP32 coefficients can move a simple root by
// ~1e-3 when the elimination cancels, and u from a(u)|v is only as good as v.
// The FP32 value is kept if the iteration leaves [v - 0.05, v + 0.05].
template <int F>
__device__ __forceinline__ double refine_v64(const Geo& g, double v)
{
    double xa = v, xb = v + 1e-6;
    double fa = bezout_det_r<F>(g, xa), fb = bezout_det_r<F>(g, xb);
    for (int it = 0; it < 6; ++it) {
        const double den = fb - fa;
        if (!(den != 0.0) || !isfinite(den)) break;
        const double xn = xb - fb * (xb - xa) / den;
        if (!(fabs(xn - v) <= 0.05)) return v;
        xa = xb;
        fa = fb;
        xb = xn;
        fb = bezout_det_r<F>(g, xb);
        if (fb == 0.0 || fabs(xb - xa) <= 4e-16 * fmax(1.0, fabs(xb))) break;
    }
    return isfinite(xb) && fabs(xb - v) <= 0.05 ? xb : v;
}

// One root v of r: u from a(u)|v, FP64 polish, closed-triangle and path-space checks.
// Real u roots of a(u)|v (ascending) from the FP64 coefficients; `near`
// reports a complex pair within kComplexWindow of the real axis over the
// triangle (the case a slightly wrong v produces near a fold).
template <int F>
__device__ __forceinline__ int u_roots(const P2<double, 1 + F>& a64, double v, double (&us)[2], bool& near)
{
    constexpr int TA = 1 + F;
    double c[TA + 1];
#pragma unroll
    for (int i = 0; i <= TA; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = TA - i; j >= 0; --j) s = fma(s, v, a64.c[tri_idx(TA, i, j)]);
        c[i] = s;
    }
    us[0] = us[1] = 0.0;
    near = false;
    if constexpr (TA == 2) {
        const double qa = c[2], qb = c[1], qc = c[0];
        if (qa != 0.0) {
            const double disc = qb * qb - 4.0 * qa * qc;
            if (disc > 0.0) {
                const double qq = -0.5 * (qb + copysign(sqrt(disc), qb));
                const double r1 = qq / qa, r2 = qc / qq;
                us[0] = fmin(r1, r2);
                us[1] = fmax(r1, r2);
                return 2;
            }
            const double re = -qb / (2.0 * qa);
            near = -disc <= 4.0 * kComplexWindow * kComplexWindow * qa * qa && re >= -kComplexWindow &&
                   re <= 1.0 - v + kComplexWindow;
            if (-disc <= kNearDoubleU * kNearDoubleU * qa * qa) {
                // The two u roots are within kNearDoubleU of each other or a
                // complex pair that close to the real axis: v is known only to
                // the isolation tolerance, so a solution with a near-double u
                // root can show a slightly negative discriminant.  Its vertex
                // is the start point; the FP64 polish (whose Jacobian does not
                // vanish there at a simple solution) and validation decide.
                us[0] = -qb / (2.0 * qa);
                return 1;
            }
            return 0;
        }
        if (qb != 0.0) {
            us[0] = -qc / qb;
            return 1;
        }
        return 0;
    } else {
        if (c[1] != 0.0) {
            us[0] = -c[0] / c[1];
            return 1;
        }
        return 0;
    }
}

// With kDefer the FP64 refinement of v is not done here: the root is reported
// (return false, nothing emitted) so that the caller can hand its candidate to
// the FP64 solve instead.
template <int EV, int F, bool kDefer = false>
__device__ __forceinline__ bool back_root(const Geo& g, const OneBounceArgs& A, const P2<double, 1 + F>& a64, double v,
                                          LaneSols& S, int& ncand)
{
    double us[2];
    bool near = false;
    int nu = u_roots<F>(a64, v, us, near);
    if constexpr (EV == SPOLY_R) {
        // FP32 roots: when no u lands in the triangle but one is close (or
        // the pair is nearly real), v may be the culprit: refine it in FP64
        // and solve for u again.
        if (A.refine_v) {
            bool in = false, close = near;
            for (int m = 0; m < nu; ++m) {
                in = in || (us[m] >= -A.u_margin && us[m] <= 1.0 - v + A.u_margin);
                close = close || (us[m] >= -kRefineWindow && us[m] <= 1.0 + kRefineWindow - v);
            }
            if (!in && close) {
                if constexpr (kDefer) return false;
                v = refine_v64<F>(g, v);
                nu = u_roots<F>(a64, v, us, near);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        if (m >= nu) continue;
        double u = us[m], vv = v;
        if (!(u >= -A.u_margin && u <= 1.0 - v + A.u_margin)) continue;
        ncand++;
        if (!polish<EV>(g, A.eta0, A.eta1, A.polish_iters, u, vv)) continue;
        if (!(u >= 0.0 && vv >= 0.0 && u + vv <= 1.0)) continue;
        V3<double> x1 = g.p0 + g.e1 * u + g.e2 * vv;
        V3<double> nn = g.n0 + g.dn1 * u + g.dn2 * vv;
        double res;
        if (!vertex_law(g.x0, x1, g.x2, nn, A.eta0, A.eta1, EV == SPOLY_T, res)) continue;
        if (!(res <= A.tau)) continue;
        double w = 1.0 - u - vv;
        double edge = fmin(fmin(u, vv), w);
        push_sol(S, u, vv, res, edge, A.dedup);
    }
    return true;
}

template <typename R, int EV, int F>
__device__ __forceinline__ void solve_instance(const Geo& g, const OneBounceArgs& A, LaneSols& S, int& nvr,
                                               int& ncand, int& degen)
{
    using Y = Sys<R, EV, F>;
    R rt[Y::DR + 1];
    bool ok[Y::DR + 1];
    bool uncertain = false;
    const int n = front_roots<R, EV, F>(g, A, rt, ok, degen, uncertain);
    if constexpr (sizeof(R) == 4) {
        if (uncertain) {
            // rare (a near-tangent or near-end r): the whole candidate in FP64
            solve_instance<double, EV, F>(g, A, S, nvr, ncand, degen);
            return;
        }
    }
    nvr += n;
    const P2<double, 1 + F> a64 = a_fp64<F>(g);
#pragma unroll
    for (int k = 0; k <= Y::DR; ++k)
        if (ok[k]) back_root<EV, F>(g, A, a64, double(rt[k]), S, ncand);
}

__device__ __forceinline__ V3<double> ld3(const double* x, const double* y, const double* z, int i)
{
    return {x[i], y[i], z[i]};
}

// Geometry of query q (FP64), with the vertex relabelling of the product form.
// Returns the triangle id.
template <int EV>
__device__ __forceinline__ int setup_geo(const OneBounceArgs& A, int64_t q, Geo& g)
{
    const int tid = A.q_tri[q];
    const int i0 = A.tri[3 * tid], i1 = A.tri[3 * tid + 1], i2 = A.tri[3 * tid + 2];
    V3<double> P0 = ld3(A.px, A.py, A.pz, i0), P1 = ld3(A.px, A.py, A.pz, i1), P2v = ld3(A.px, A.py, A.pz, i2);
    V3<double> N0 = ld3(A.nx, A.ny, A.nz, i0), N1 = ld3(A.nx, A.ny, A.nz, i1), N2 = ld3(A.nx, A.ny, A.nz, i2);
    const int j0 = A.q_x0[q], j2 = A.q_x2[q];
    g.x0 = ld3(A.x0x, A.x0y, A.x0z, j0);
    g.x2 = ld3(A.x2x, A.x2y, A.x2z, j2);
    g.flat = N0.x == N1.x && N0.y == N1.y && N0.z == N1.z && N0.x == N2.x && N0.y == N2.y && N0.z == N2.z;
    const V3<double> c = P0 + (P1 - P0) * (1.0 / 3.0) + (P2v - P0) * (1.0 / 3.0);
    bool swapped = false;
    if constexpr (EV == SPOLY_R) swapped = pick_edge2(c, g.x0, g.x2, P1 - P0, P2v - P0);
    if (swapped) {
        V3<double> t = P1; P1 = P2v; P2v = t;
        t = N1; N1 = N2; N2 = t;
    }
    g.p0 = P0; g.e1 = P1 - P0; g.e2 = P2v - P0;
    g.n0 = N0; g.dn1 = N1 - N0; g.dn2 = N2 - N0;
    g.swapped = swapped;
    g.axis = (EV == SPOLY_T) ? pick_axis(c, g.x0, g.x2) : 0;
    return tid;
}

// Solution records of one lane: compaction (block- or wave-wide), counters and
// per-query diagnostics.  Every lane must call it.
__device__ __forceinline__ void emit_lane(const OneBounceArgs& A, int64_t q, bool active, int64_t qid_offset, int tid,
                                          bool swapped, const LaneSols& S, int nvr, int ncand, int degen,
                                          unsigned long long* slots, bool write_nvr)
{
    const int cnt = active ? S.n : 0;
    const int incl = wave_incl_scan(cnt);
    const int total = __shfl(incl, kWave - 1, kWave);
    unsigned long long base = 0;
    if (slots) {
        base = block_reserve((unsigned long long)total, A.out_count, slots);
    } else if (total > 0) {
        if (lane_id() == kWave - 1) base = atomicAdd(A.out_count, (unsigned long long)total);
        base = __shfl(base, kWave - 1, kWave);
    }
    const unsigned long long first = base + (unsigned long long)(incl - cnt);
#pragma unroll
    for (int k = 0; k < kMaxLaneSol; ++k) {
        if (k < cnt) {
            unsigned long long idx = first + k;
            if (idx < (unsigned long long)A.cap) {
                spoly_solution s;
                s.query = int32_t(q + qid_offset);
                s.tri[0] = tid;
                s.tri[1] = -1;
                s.flags = 0;
                s.u[0] = swapped ? S.v[k] : S.u[k];
                s.v[0] = swapped ? S.u[k] : S.v[k];
                s.u[1] = 0.0;
                s.v[1] = 0.0;
                s.residual = float(S.res[k]);
                s.edge = float(S.edge[k]);
                A.out[idx] = s;
            }
        }
    }
    if (A.counters) {
        unsigned long long s0 = wave_sum_u64(active ? nvr : 0);
        unsigned long long s1 = wave_sum_u64(active ? ncand : 0);
        unsigned long long s2 = wave_sum_u64(active ? degen : 0);
        unsigned long long s3 = wave_sum_u64(active ? S.over : 0);
        if (lane_id() == 0) {
            if (s0) atomicAdd(A.counters + 0, s0);
            if (s1) atomicAdd(A.counters + 1, s1);
            if (s2) atomicAdd(A.counters + 2, s2);
            if (s3) atomicAdd(A.counters + 3, s3);
        }
    }
    if (A.diag_q && active) {
        if (write_nvr) A.diag_q[2 * q] = nvr;
        A.diag_q[2 * q + 1] = S.n;
    }
}

// One instance per lane; every lane of the wave must call it (the compaction
// is wave-wide).  Output records carry query id q + qid_offset.  With `slots`
// (LDS, kMaxBlockWaves + 1 values) every thread of the block must call it and
// the output range is reserved once per block; without, once per wave.
template <typename R, int EV>
__device__ __forceinline__ void onebounce_lane(const OneBounceArgs& A, int64_t q, bool active, int64_t qid_offset,
                                               unsigned long long* slots = nullptr)
{
    LaneSols S;
    S.n = 0;
    S.over = 0;
    int nvr = 0, ncand = 0, degen = 0;
    int tid = -1;
    bool swapped = false;
    if (active) {
        Geo g;
        tid = setup_geo<EV>(A, q, g);
        swapped = g.swapped;
        bool finite = isfinite(dot(g.p0, g.e1) + dot(g.e2, g.n0) + dot(g.dn1, g.dn2) + dot(g.x0, g.x2));
        if (!finite) degen = 1;
        else if (g.flat) solve_instance<R, EV, 0>(g, A, S, nvr, ncand, degen);
        else solve_instance<R, EV, 1>(g, A, S, nvr, ncand, degen);
    }
    emit_lane(A, q, active, qid_offset, tid, swapped, S, nvr, ncand, degen, slots, true);
}

template <typename R, int EV>
__global__ void __launch_bounds__(256) k_onebounce(OneBounceArgs A)
{
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    onebounce_lane<R, EV>(A, q, q < A.nq, 0, s_slots);
}

// ---------------------------------------------------------------- two-phase solve
// Front: one candidate per lane; candidates with 1..kObEmit roots are appended
// (block-wide reservation) to the item list; a candidate with more roots, or
// one that finds the list full, is solved in place.
template <typename R, int D>
__device__ __forceinline__ void gather_roots(const R (&rt)[D + 1], const bool (&ok)[D + 1], double (&vr)[kObEmit])
{
    int j = 0;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        if (ok[k]) {
#pragma unroll
            for (int i = 0; i < kObEmit; ++i)
                if (i == j) vr[i] = double(rt[k]);
            ++j;
        }
    }
}

template <typename R, int EV, int F>
__device__ __forceinline__ int front_collect(const Geo& g, const OneBounceArgs& A, double (&vr)[kObEmit], int& degen,
                                             bool& uncertain)
{
    using Y = Sys<R, EV, F>;
    R rt[Y::DR + 1];
    bool ok[Y::DR + 1];
    const int n = front_roots<R, EV, F>(g, A, rt, ok, degen, uncertain);
    gather_roots<R, Y::DR>(rt, ok, vr);
    return n;
}

// Item emission of the front phase (every thread of the block must call it):
// one item per candidate with 1..kObEmit roots, one full-list entry per
// candidate with more, counters and per-query diagnostics.
__device__ __forceinline__ void emit_items(const OneBounceArgs& A, int64_t q, bool active, int nvr, int degen,
                                           const double (&vr)[kObEmit], unsigned long long* s_slots,
                                           bool force_full = false)
{
    const bool full = active && (nvr > kObEmit || force_full);
    const bool want = active && !full && nvr > 0;
    const int wi = want ? 1 : 0, wf = full ? 1 : 0;
    const int ii = wave_incl_scan(wi), fi = wave_incl_scan(wf);
    const unsigned long long bi = block_reserve((unsigned long long)__shfl(ii, kWave - 1, kWave), A.items_count,
                                                s_slots);
    const unsigned long long bf = block_reserve((unsigned long long)__shfl(fi, kWave - 1, kWave),
                                                A.items_count + 1, s_slots);
    if (want) {
        const unsigned long long idx = bi + (unsigned long long)(ii - wi);
        A.items_q[idx] = int32_t(q);
        A.items_n[idx] = nvr;
#pragma unroll
        for (int i = 0; i < kObEmit; ++i)
            if (i < nvr) A.items_v[kObEmit * idx + i] = vr[i];
    }
    if (full) A.full_q[bf + (unsigned long long)(fi - wf)] = int32_t(q);
    if (A.counters) {
        const unsigned long long s0 = wave_sum_u64(active ? nvr : 0);
        const unsigned long long s2 = wave_sum_u64(active ? degen : 0);
        if (lane_id() == 0) {
            if (s0) atomicAdd(A.counters + 0, s0);
            if (s2) atomicAdd(A.counters + 2, s2);
        }
    }
    if (A.diag_q && active) {
        A.diag_q[2 * q] = nvr;
        A.diag_q[2 * q + 1] = 0;
    }
}

// Fused front (reflection): coefficients, elimination and isolation in one
// kernel, one candidate per lane.
template <typename R, int EV>
__device__ __forceinline__ void ob_front_body(const OneBounceArgs& A)
{
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool active = q < A.nq;
    int nvr = 0, degen = 0;
    bool uncertain = false;
    double vr[kObEmit];
#pragma unroll
    for (int i = 0; i < kObEmit; ++i) vr[i] = 0.0;
    if (active) {
        Geo g;
        setup_geo<EV>(A, q, g);
        const bool finite = isfinite(dot(g.p0, g.e1) + dot(g.e2, g.n0) + dot(g.dn1, g.dn2) + dot(g.x0, g.x2));
        if (!finite) degen = 1;
        else if (g.flat) nvr = front_collect<R, EV, 0>(g, A, vr, degen, uncertain);
        else nvr = front_collect<R, EV, 1>(g, A, vr, degen, uncertain);
    }
    emit_items(A, q, active, nvr, degen, vr, s_slots, uncertain);
}

template <typename R, int EV>
__global__ void __launch_bounds__(256) k_ob_front(OneBounceArgs A)
{
    ob_front_body<R, EV>(A);
}

// FP32: six waves per SIMD (80 VGPRs and a few bytes of spill) run faster than
// the five the compiler picks by itself (86 VGPRs); the FP64 instance would
// spill heavily at that target and keeps its own allocation.
template <>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) k_ob_front<float, SPOLY_R>(OneBounceArgs A)
{
    ob_front_body<float, SPOLY_R>(A);
}

// Front phase in two kernels (refraction).  k_ob_coef builds r(v) for every candidate and
// lists, in list order, the candidates whose r may have a root in [0,1]
// (their r and a status: 0 interpolated normals, 1 flat).  k_ob_iso isolates
// the listed ones with full waves and emits items.  The split keeps the
// isolation off the lanes of the ~70% of candidates without a root, and it
// separates the FP64 elimination (which needs every vector register) from the
// isolation (three waves per SIMD).  For reflection in FP32 the fused front
// is faster: its elimination is light and the list traffic would cost more
// than the isolation it saves.
//
// Exclusion test: with Bernstein coefficients b_k of r on [0,1],
// r(v) = sum_k b_k B_k(v) with B_k >= 0 and sum_k B_k = 1, so r(v) >= min_k b_k
// (and <= max_k b_k) on [0,1].  If every b_k exceeds `margin` in the same
// sign, where margin bounds the rounding of the b_k and of the Horner
// evaluations of the isolation (about (3 D + 4) units in the last place of
// sum |r_j|), the isolation cannot see a sign change and the candidate has no
// root of r in [0,1].
template <typename R, int D>
__device__ __forceinline__ bool no_root01(const R (&r)[D + 1])
{
    R l1 = R(0);
#pragma unroll
    for (int j = 0; j <= D; ++j) l1 += fabs(r[j]);
    const R margin = (sizeof(R) == 4 ? R(1e-5) : R(1e-13)) * l1;
    bool pos = true, neg = true;
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        R bk = R(0);
#pragma unroll
        for (int j = 0; j <= k; ++j) bk = fma(R(binom(k, j) / binom(D, j)), r[j], bk);
        pos = pos && bk > margin;
        neg = neg && bk < -margin;
    }
    return pos || neg;
}

// r(v) of listed candidate i, coefficient k: rlist[k * cap + i]
template <typename R, int EV, int F>
__device__ __forceinline__ bool coef_list(const Geo& g, const OneBounceArgs& A, R (&r)[Sys<R, EV, F>::DR + 1])
{
    return front_poly<R, EV, F>(g, A, r) && !no_root01<R, Sys<R, EV, F>::DR>(r);
}

template <typename R, int EV>
__global__ void __launch_bounds__(256) k_ob_coef(OneBounceArgs A)
{
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    constexpr int D1 = Sys<R, EV, 1>::DR, D0 = Sys<R, EV, 0>::DR;
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool active = q < A.nq;
    int degen = 0, flat = 0;
    bool listed = false;
    R r[D1 + 1];
#pragma unroll
    for (int k = 0; k <= D1; ++k) r[k] = R(0);
    if (active) {
        Geo g;
        setup_geo<EV>(A, q, g);
        const bool finite = isfinite(dot(g.p0, g.e1) + dot(g.e2, g.n0) + dot(g.dn1, g.dn2) + dot(g.x0, g.x2));
        if (!finite) {
            degen = 1;
        } else if (g.flat) {
            flat = 1;
            R r0[D0 + 1];
            listed = coef_list<R, EV, 0>(g, A, r0);
            degen = front_poly_degenerate<R, D0>(r0) ? 1 : 0;
#pragma unroll
            for (int k = 0; k <= D0; ++k) r[k] = r0[k];
        } else {
            listed = coef_list<R, EV, 1>(g, A, r);
            degen = front_poly_degenerate<R, D1>(r) ? 1 : 0;
        }
    }
    const int wl = listed ? 1 : 0;
    const int il = wave_incl_scan(wl);
    const unsigned long long bl = block_reserve((unsigned long long)__shfl(il, kWave - 1, kWave),
                                                A.items_count + 2, s_slots);
    if (listed) {
        const unsigned long long i = bl + (unsigned long long)(il - wl);
        R* rl = reinterpret_cast<R*>(A.rlist);
        A.iso_q[i] = int32_t(q);
        A.iso_st[i] = flat;
#pragma unroll
        for (int k = 0; k <= D1; ++k)
            if (!flat || k <= D0) rl[k * A.items_cap + i] = r[k];
    }
    if (A.counters) {
        const unsigned long long s2 = wave_sum_u64(active ? degen : 0);
        if (lane_id() == 0 && s2) atomicAdd(A.counters + 2, s2);
    }
    if (A.diag_q && active && !listed) {
        A.diag_q[2 * q] = 0;
        A.diag_q[2 * q + 1] = 0;
    }
}

// Register target of the FP64 isolation: left to itself the compiler uses all
// 512 registers of one wave; at three waves per SIMD it compiles without
// scratch (about 160 VGPRs), and four waves (128 VGPRs, 104 bytes of spill)
// measured 0.17 ms faster over the glints refraction list.
template <typename R, int EV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_ob_iso(OneBounceArgs A)
{
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    constexpr int D1 = Sys<R, EV, 1>::DR, D0 = Sys<R, EV, 0>::DR;
    const R* rl = reinterpret_cast<const R*>(A.rlist);
    const int64_t n_list = int64_t(A.items_count[2]);
    for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < n_list; b0 += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = b0 + threadIdx.x;
        const bool active = i < n_list;
        int nvr = 0;
        int64_t q = 0;
        double vr[kObEmit];
#pragma unroll
        for (int k = 0; k < kObEmit; ++k) vr[k] = 0.0;
        if (active) {
            q = A.iso_q[i];
            if (A.iso_st[i] == 1) {
                R r[D0 + 1], rt[D0 + 1];
                bool ok[D0 + 1];
#pragma unroll
                for (int k = 0; k <= D0; ++k) r[k] = rl[k * A.items_cap + i];
                isolate01<R, D0>(r, rt, ok, R(A.iso_eps));
#pragma unroll
                for (int k = 0; k <= D0; ++k) nvr += ok[k] ? 1 : 0;
                gather_roots<R, D0>(rt, ok, vr);
            } else {
                R r[D1 + 1], rt[D1 + 1];
                bool ok[D1 + 1];
#pragma unroll
                for (int k = 0; k <= D1; ++k) r[k] = rl[k * A.items_cap + i];
                isolate01<R, D1>(r, rt, ok, R(A.iso_eps));
#pragma unroll
                for (int k = 0; k <= D1; ++k) nvr += ok[k] ? 1 : 0;
                gather_roots<R, D1>(rt, ok, vr);
            }
        }
        emit_items(A, q, active, nvr, 0, vr, s_slots);
    }
}

// Back: persistent blocks stride over the item list, one candidate per lane.
// The next item's record (query, root count, roots) is loaded one iteration
// ahead, so that its latency overlaps this item's work and only the geometry
// gathers that depend on it remain on the critical path.
template <int EV>
__global__ void __launch_bounds__(256) k_ob_back(OneBounceArgs A)
{
    static_assert(kObEmit == 2, "the record carried ahead holds two roots");
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    const int64_t n_items = int64_t(*A.items_count);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t qn = 0;
    int nrn = 0;
    double vn0 = 0.0, vn1 = 0.0;
    auto load_item = [&](int64_t i) {
        if (i < n_items) {
            qn = A.items_q[i];
            nrn = A.items_n[i];
            vn0 = A.items_v[kObEmit * i];
            vn1 = A.items_v[kObEmit * i + 1];
        }
    };
    load_item(int64_t(blockIdx.x) * blockDim.x + threadIdx.x);
    for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < n_items; b0 += stride) {
        const int64_t i = b0 + threadIdx.x;
        const bool active = i < n_items;
        const int64_t qc = qn;
        const int nr = nrn;
        const double v0 = vn0, v1 = vn1;
        load_item(i + stride);
        LaneSols S;
        S.n = 0;
        S.over = 0;
        int ncand = 0, tid = -1;
        bool swapped = false, defer = false;
        int64_t q = 0;
        if (active) {
            q = qc;
            Geo g;
            tid = setup_geo<EV>(A, q, g);
            swapped = g.swapped;
            bool ok = true;
            if (g.flat) {
                const P2<double, 1> a64 = a_fp64<0>(g);
                for (int j = 0; j < nr && ok; ++j)
                    ok = back_root<EV, 0, true>(g, A, a64, j == 0 ? v0 : v1, S, ncand);
            } else {
                const P2<double, 2> a64 = a_fp64<1>(g);
                for (int j = 0; j < nr && ok; ++j)
                    ok = back_root<EV, 1, true>(g, A, a64, j == 0 ? v0 : v1, S, ncand);
            }
            if (!ok) {
                // An FP32 root whose u misses the triangle narrowly: the whole
                // candidate goes to the FP64 solve of the full list, so that
                // the waves here do not wait for the refinement of few lanes.
                defer = true;
                S.n = 0;
                S.over = 0;
                ncand = 0;
            }
        }
        if (A.refine_v) {
            const int wf = defer ? 1 : 0, fi = wave_incl_scan(wf);
            const unsigned long long bf = block_reserve((unsigned long long)__shfl(fi, kWave - 1, kWave),
                                                        A.items_count + 1, s_slots);
            if (defer) A.full_q[bf + (unsigned long long)(fi - wf)] = int32_t(q);
        }
        emit_lane(A, q, active, 0, tid, swapped, S, 0, ncand, 0, s_slots, false);
    }
}

// The full list: candidates with more than kObEmit roots, and FP32 candidates
// whose root count the FP64 check doubts, solved from scratch in FP64.
template <int EV>
__global__ void __launch_bounds__(256) k_ob_full(OneBounceArgs A)
{
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    const int64_t n_full = int64_t(A.items_count[1]);
    for (int64_t b0 = int64_t(blockIdx.x) * blockDim.x; b0 < n_full; b0 += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = b0 + threadIdx.x;
        const bool active = i < n_full;
        LaneSols S;
        S.n = 0;
        S.over = 0;
        int ncand = 0, tid = -1, nv = 0, dg = 0;
        bool swapped = false;
        int64_t q = 0;
        if (active) {
            q = A.full_q[i];
            Geo g;
            tid = setup_geo<EV>(A, q, g);
            swapped = g.swapped;
            if (g.flat) solve_instance<double, EV, 0>(g, A, S, nv, ncand, dg);
            else solve_instance<double, EV, 1>(g, A, S, nv, ncand, dg);
        }
        emit_lane(A, q, active, 0, tid, swapped, S, 0, ncand, 0, s_slots, false);
    }
}

__global__ void k_zero_items(unsigned long long* p)
{
    p[0] = 0ull;   // items
    p[1] = 0ull;   // full list
    p[2] = 0ull;   // refraction: candidates listed for isolation
}

hipError_t launch_onebounce_2phase(const OneBounceArgs& A, int ev, int prec, int back_blocks, hipStream_t stream,
                                   hipEvent_t* stage_events)
{
    if (A.nq <= 0) return hipSuccess;
    if (A.items_cap < A.nq || (ev == SPOLY_T && !A.rlist)) return hipErrorInvalidValue;
    int stage = 0;
    auto mark = [&]() {
        if (stage_events) (void)hipEventRecord(stage_events[stage], stream);
        ++stage;
    };
    mark();
    hipLaunchKernelGGL(k_zero_items, dim3(1), dim3(1), 0, stream, A.items_count);
    const dim3 block(256), grid(unsigned((A.nq + 255) / 256));
    const dim3 bgrid(unsigned(back_blocks > 0 ? back_blocks : 1));
    const dim3 fgrid(bgrid);   // the full list can be long (deferred FP32 roots): fill the chip
    // Refraction always runs in FP64 (see launch_onebounce).
    if (ev == SPOLY_R && prec == SPOLY_FP64) {
        hipLaunchKernelGGL((k_ob_front<double, SPOLY_R>), grid, block, 0, stream, A);
        mark();
        hipLaunchKernelGGL((k_ob_back<SPOLY_R>), bgrid, block, 0, stream, A);
        mark();
        hipLaunchKernelGGL((k_ob_full<SPOLY_R>), fgrid, block, 0, stream, A);
        mark();
    } else if (ev == SPOLY_R) {
        hipLaunchKernelGGL((k_ob_front<float, SPOLY_R>), grid, block, 0, stream, A);
        mark();
        hipLaunchKernelGGL((k_ob_back<SPOLY_R>), bgrid, block, 0, stream, A);
        mark();
        hipLaunchKernelGGL((k_ob_full<SPOLY_R>), fgrid, block, 0, stream, A);
        mark();
    } else {
        hipLaunchKernelGGL((k_ob_coef<double, SPOLY_T>), grid, block, 0, stream, A);
        mark();
        hipLaunchKernelGGL((k_ob_iso<double, SPOLY_T>), bgrid, block, 0, stream, A);
        mark();
        hipLaunchKernelGGL((k_ob_back<SPOLY_T>), bgrid, block, 0, stream, A);
        mark();
        hipLaunchKernelGGL((k_ob_full<SPOLY_T>), fgrid, block, 0, stream, A);
        mark();
    }
    return hipGetLastError();
}

hipError_t launch_onebounce(const OneBounceArgs& A, int ev, int prec, hipStream_t stream)
{
    if (A.nq <= 0) return hipSuccess;
    dim3 block(256), grid(unsigned((A.nq + 255) / 256));
    // Refraction always runs in FP64: its degree-12 resultant, expanded and
    // isolated in FP32, loses roots of the square form (a difference of two
    // nearly equal squares over a small triangle), while FP32 and FP64 have the
    // same non-packed VALU rate on this chip.
    if (ev == SPOLY_R && prec == SPOLY_FP64) hipLaunchKernelGGL((k_onebounce<double, SPOLY_R>), grid, block, 0, stream, A);
    else if (ev == SPOLY_R) hipLaunchKernelGGL((k_onebounce<float, SPOLY_R>), grid, block, 0, stream, A);
    else hipLaunchKernelGGL((k_onebounce<double, SPOLY_T>), grid, block, 0, stream, A);
    return hipGetLastError();
}

}  // namespace spoly
