// Two specular vertices (Sec. 4.5: chains RR, RT, TR and TT): one wave per
// (x0, T1, T2, x3) tuple.
//   coefficient phase  (wave-cooperative, LDS): the coplanarity polynomial
//       a(u,v) = (Dt x (x3 - x1)) . M2 of the mapped system (Eq. eq_rct), with
//       Dt the reflected direction (Eq. eq_431_di, scaled by |n1|^2) or the
//       refracted one (Eq. eq_refr_rational with the piecewise rational square
//       root);
//   elimination + scan (lane per sample of v): the sign of det R(v) of the
//       Bezout matrix (Eq. eq_bezout) at v_j = j/pieces, j = 0..pieces, and at
//       the bisection midpoints (Sec. 5.2).  det R(v) = C lc(b)^k Res_u(a, b)(v),
//       and Res_u(a,b) = lc(a)^deg b prod_{a(alpha)=0} b(alpha); complex roots
//       pair up into |b|^2 > 0, so, up to a sign that is constant where lc_u(a)
//       keeps its sign, it is the product of sgn b(alpha, v) over the real roots
//       alpha of a(., v), near-double root pairs left out.  Real roots come from the
//       recursive isolation of Sec. 5.2 on Fujiwara's root bound; b is the
//       square-form (Eq. eq_cpf_result, refraction at x2) or product-form (Eq.
//       eq_pf_result, reflection at x2) polynomial, evaluated through its
//       defining products of the mapped quantities.
//   path phase (lane per v root): u from a(u)|_v, exact reflection or
//       refraction at x1 and intersection with T2's plane, FP64 Newton polish
//       on h2 x n2 = 0, validation at both vertices, wave-ballot compaction.
#include "spoly_dev.hpp"
#include "twobounce.hpp"

namespace spoly {

constexpr int kDA = 16;        // structural degree bound of a(u,v) (interpolated normals at both vertices)
constexpr int kTTMaxSol = 4;   // solutions kept per lane

// ------------------------------------------------------------------ geometry (per tuple, FP64)
struct TTGeo {
    V3<double> p1, e11, e12, n10, dn11, dn12;   // T1
    V3<double> p2, e21, e22, n20, dn21, dn22;   // T2
    V3<double> x0, x3;
    double eta0, eta1, eta2, etap;
    double S, sq0, sq1, sr0, sr1, sg, sqrtS;    // square-root approximation of this tuple
    int axis;
    int f1, f2;                                 // 1 = interpolated normals, 0 = flat
    int ev1, ev2;                               // SPOLY_R or SPOLY_T at x1, x2
    V3<double> edge2;                           // product-form edge of T2 (reflection at x2)
    double n2len;                               // |e21 x e22|
};

__device__ __forceinline__ V3<double> ld3t(const double* x, const double* y, const double* z, int i)
{
    return {x[i], y[i], z[i]};
}

// Square-form axis: x^ if |m_c.x^| >= 1/2, else z^ if |m_c.z^| >= 1/2, else y^,
// with m_c the normal of the plane through the previous vertex, the centroid
// and the next vertex (the incidence plane where the projection must not vanish).
__device__ __forceinline__ int tt_axis(V3<double> c, V3<double> xa, V3<double> xb)
{
    V3<double> m = cross(c - xa, xb - xa);
    double l = len(m);
    if (!(l > 0.0)) return 0;
    m = m * (1.0 / l);
    if (fabs(m.x) >= 0.5) return 0;
    if (fabs(m.z) >= 0.5) return 2;
    return 1;
}

// Product-form edge at x2: e21 unless it nearly lies in the incidence plane
// (|e21^.m_c| < 1/4 and e22 does better), then e22.
__device__ __forceinline__ V3<double> tt_edge(V3<double> c, V3<double> xa, V3<double> xb, V3<double> e1,
                                              V3<double> e2)
{
    V3<double> m = cross(c - xa, xb - xa);
    double l = len(m);
    if (!(l > 0.0)) return e1;
    m = m * (1.0 / l);
    double g1 = fabs(dot(normalized(e1), m)), g2 = fabs(dot(normalized(e2), m));
    return (g1 < 0.25 && g2 > g1) ? e2 : e1;
}

__device__ void tt_setup(const TTArgs& A, int64_t q, TTGeo& g)
{
    const int t1 = A.q_tris[2 * q], t2 = A.q_tris[2 * q + 1];
    V3<double> P[6], Nn[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int i = A.tri[3 * t1 + k], j = A.tri[3 * t2 + k];
        P[k] = ld3t(A.px, A.py, A.pz, i);
        Nn[k] = ld3t(A.nx, A.ny, A.nz, i);
        P[3 + k] = ld3t(A.px, A.py, A.pz, j);
        Nn[3 + k] = ld3t(A.nx, A.ny, A.nz, j);
    }
    g.p1 = P[0]; g.e11 = P[1] - P[0]; g.e12 = P[2] - P[0];
    g.n10 = Nn[0]; g.dn11 = Nn[1] - Nn[0]; g.dn12 = Nn[2] - Nn[0];
    g.p2 = P[3]; g.e21 = P[4] - P[3]; g.e22 = P[5] - P[3];
    g.n20 = Nn[3]; g.dn21 = Nn[4] - Nn[3]; g.dn22 = Nn[5] - Nn[3];
    auto same = [](V3<double> a, V3<double> b) { return a.x == b.x && a.y == b.y && a.z == b.z; };
    g.f1 = (same(Nn[0], Nn[1]) && same(Nn[0], Nn[2])) ? 0 : 1;
    g.f2 = (same(Nn[3], Nn[4]) && same(Nn[3], Nn[5])) ? 0 : 1;
    g.x0 = ld3t(A.x0x, A.x0y, A.x0z, A.q_x0[q]);
    g.x3 = ld3t(A.x3x, A.x3y, A.x3z, A.q_x3[q]);
    g.eta0 = A.eta0; g.eta1 = A.eta1; g.eta2 = A.eta2;
    g.etap = A.eta0 / A.eta1;
    // per-tuple constants of the square-root approximation at the centroid of T1:
    // S = |n|^2 |d0|^2, piece from beta/S = 1 - eta'^2 (1 - cos^2), sign orienting n
    V3<double> c1 = g.p1 + g.e11 * (1.0 / 3.0) + g.e12 * (1.0 / 3.0);
    V3<double> nc1 = g.n10 + g.dn11 * (1.0 / 3.0) + g.dn12 * (1.0 / 3.0);
    V3<double> d0c = c1 - g.x0;
    g.S = dot(nc1, nc1) * dot(d0c, d0c);
    double dnc = dot(d0c, nc1);
    double sc = 1.0 - g.etap * g.etap * (1.0 - dnc * dnc / g.S);
    int p = 0;
#pragma unroll
    for (int k = 1; k < 6; ++k)
        if (sc >= A.sqrt_bp[k]) p = k;
    g.sq0 = A.sqrt_c[4 * p + 0]; g.sq1 = A.sqrt_c[4 * p + 1];
    g.sr0 = A.sqrt_c[4 * p + 2]; g.sr1 = A.sqrt_c[4 * p + 3];
    g.sg = dnc < 0.0 ? -1.0 : 1.0;
    g.sqrtS = sqrt(g.S);
    V3<double> c2 = g.p2 + g.e21 * (1.0 / 3.0) + g.e22 * (1.0 / 3.0);
    g.axis = tt_axis(c2, c1, g.x3);
    g.ev1 = A.ev1;
    g.ev2 = A.ev2;
    g.edge2 = tt_edge(c2, c1, g.x3, g.e21, g.e22);
    g.n2len = len(cross(g.e21, g.e22));
}

// ------------------------------------------------------------------ LDS bivariate polynomials (wave-cooperative)
// Dense (d+1) x (d+1) storage, c[i*(d+1)+j] = coefficient of u^i v^j, zero for i+j > d.
struct LP {
    double* c;
    int d;
};

__device__ __forceinline__ void sync_wave() { __syncthreads(); }

__device__ __forceinline__ void lp_zero(LP p)
{
    const int n = (p.d + 1) * (p.d + 1);
    for (int o = lane_id(); o < n; o += kWave) p.c[o] = 0.0;
}
// p = k0 + ku u + kv v (p.d >= 1)
__device__ __forceinline__ void lp_set_lin(LP p, double k0, double ku, double kv)
{
    lp_zero(p);
    sync_wave();
    if (lane_id() == 0) {
        p.c[0] = k0;
        p.c[1] = kv;
        if (p.d >= 1) p.c[p.d + 1] = ku;
    }
}
// C += s * A * B   (C.d >= A.d + B.d)
__device__ void lp_mul_acc(LP C, LP A, LP B, double s)
{
    const int dc = A.d + B.d;
    const int n = (C.d + 1) * (C.d + 1);
    for (int o = lane_id(); o < n; o += kWave) {
        const int i = o / (C.d + 1), j = o % (C.d + 1);
        if (i + j > dc) continue;
        double acc = 0.0;
        const int k0 = i - B.d > 0 ? i - B.d : 0;
        const int k1 = i < A.d ? i : A.d;
        for (int k = k0; k <= k1; ++k) {
            const int rb = B.d - (i - k);          // v-degree room left in B's row i-k
            const int l0 = j - rb > 0 ? j - rb : 0;
            const int l1 = j < A.d - k ? j : A.d - k;
            for (int l = l0; l <= l1; ++l)
                acc = fma(A.c[k * (A.d + 1) + l], B.c[(i - k) * (B.d + 1) + (j - l)], acc);
        }
        C.c[o] = fma(s, acc, C.c[o]);
    }
}
// C += s * A  (C.d >= A.d)
__device__ void lp_axpy(LP C, LP A, double s)
{
    const int n = (A.d + 1) * (A.d + 1);
    for (int o = lane_id(); o < n; o += kWave) {
        const int i = o / (A.d + 1), j = o % (A.d + 1);
        if (i + j > A.d) continue;
        C.c[i * (C.d + 1) + j] = fma(s, A.c[o], C.c[i * (C.d + 1) + j]);
    }
}
__device__ __forceinline__ void lp_addc(LP C, double k)
{
    if (lane_id() == 0) C.c[0] += k;
}

// LDS budget per wave (doubles)
constexpr int sq(int d) { return (d + 1) * (d + 1); }
constexpr int kLdsDoubles = 3 * sq(1) /*X1*/ + 3 * sq(1) /*N1*/ + 3 * sq(1) /*D0*/ + 3 * sq(2) /*NN,DD,DN*/ +
                            sq(4) /*BETA*/ + 2 * sq(4) /*NUM,DEN*/ + 3 * sq(3) /*TANG*/ + 3 * sq(7) /*DT*/ +
                            3 * sq(7) /*DXE*/ + 3 * sq(8) /*UT,VT,KA*/ + 3 * sq(8) /*M2*/ + 3 * sq(1) /*W*/ +
                            3 * sq(8) /*CR*/ + sq(kDA) /*A*/ + 3 * sq(1) /*Q*/;

// Build a(u,v) into A (degree 2D + 1 + f2 <= 16); returns its structural degree.
__device__ int tt_build_a(const TTGeo& g, double* lds, LP& Aout)
{
    const int D = g.ev1 == SPOLY_R ? 1 + 2 * g.f1 : 3 + 4 * g.f1;
    double* p = lds;
    auto take = [&](int d) { LP r{p, d}; p += sq(d); return r; };
    LP X1[3], N1[3], D0[3], Q[3], W[3];
    for (int k = 0; k < 3; ++k) X1[k] = take(1);
    for (int k = 0; k < 3; ++k) N1[k] = take(1);
    for (int k = 0; k < 3; ++k) D0[k] = take(1);
    for (int k = 0; k < 3; ++k) Q[k] = take(1);
    for (int k = 0; k < 3; ++k) W[k] = take(1);
    LP NN = take(2), DD = take(2), DN = take(2);
    LP BETA = take(4), NUM = take(4), DEN = take(4);
    LP TANG[3], DT[3], DXE[3], M2[3], CR[3];
    for (int k = 0; k < 3; ++k) TANG[k] = take(3);
    for (int k = 0; k < 3; ++k) DT[k] = take(7);
    for (int k = 0; k < 3; ++k) DXE[k] = take(7);
    LP UT = take(8), VT = take(8), KA = take(8);
    for (int k = 0; k < 3; ++k) M2[k] = take(8);
    for (int k = 0; k < 3; ++k) CR[k] = take(8);
    LP A = take(kDA);
    auto comp = [](V3<double> v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); };
    for (int k = 0; k < 3; ++k) {
        lp_set_lin(X1[k], comp(g.p1, k), comp(g.e11, k), comp(g.e12, k));
        lp_set_lin(N1[k], comp(g.n10, k), g.f1 ? comp(g.dn11, k) : 0.0, g.f1 ? comp(g.dn12, k) : 0.0);
        lp_set_lin(D0[k], comp(g.p1 - g.x0, k), comp(g.e11, k), comp(g.e12, k));
        lp_set_lin(Q[k], comp(g.p1 - g.p2, k), comp(g.e11, k), comp(g.e12, k));
        lp_set_lin(W[k], comp(g.x3 - g.p1, k), -comp(g.e11, k), -comp(g.e12, k));
    }
    // flat T1: N1 has degree 0 (its linear part is zero); degrees below follow the structure
    for (int k = 0; k < 3; ++k) N1[k].d = g.f1;   // storage stride stays (1+1) only when d = 1
    sync_wave();
    // Re-store N1 with its structural degree so that stride matches d.
    if (!g.f1) {
        for (int k = 0; k < 3; ++k)
            if (lane_id() == 0) N1[k].c[0] = comp(g.n10, k);
        sync_wave();
    }
    const double ep = g.etap;
    lp_zero(NN); lp_zero(DD); lp_zero(DN);
    sync_wave();
    for (int k = 0; k < 3; ++k) {
        LP nn{NN.c, 2 * g.f1}, dn{DN.c, 1 + g.f1};
        lp_mul_acc(nn, N1[k], N1[k], 1.0);
        lp_mul_acc(DD, D0[k], D0[k], 1.0);
        lp_mul_acc(dn, D0[k], N1[k], 1.0);
        sync_wave();
    }
    LP nnS{NN.c, 2 * g.f1}, dnS{DN.c, 1 + g.f1};
    LP dt[3];
    if (g.ev1 == SPOLY_R) {
        // reflected direction |n1|^2 d0 - 2 (d0.n1) n1
        for (int k = 0; k < 3; ++k) {
            dt[k] = LP{DT[k].c, D};
            lp_zero(dt[k]);
        }
        sync_wave();
        for (int k = 0; k < 3; ++k) {
            lp_mul_acc(dt[k], nnS, D0[k], 1.0);
            lp_mul_acc(dt[k], dnS, N1[k], -2.0);
        }
        sync_wave();
    } else {
    const int db = 2 + 2 * g.f1;
    LP beta{BETA.c, db}, num{NUM.c, db}, den{DEN.c, db};
    lp_zero(beta);
    sync_wave();
    lp_mul_acc(beta, nnS, DD, 1.0 - ep * ep);
    sync_wave();
    lp_mul_acc(beta, dnS, dnS, ep * ep);
    sync_wave();
    lp_zero(num); lp_zero(den);
    sync_wave();
    lp_axpy(num, beta, g.sq1 / g.S);
    lp_axpy(den, beta, g.sr1 / g.S);
    sync_wave();
    lp_addc(num, g.sq0);
    lp_addc(den, g.sr0);
    sync_wave();
    const int dt_ = 1 + 2 * g.f1;
    LP tang[3];
    for (int k = 0; k < 3; ++k) {
        tang[k] = LP{TANG[k].c, dt_};
        dt[k] = LP{DT[k].c, D};
        lp_zero(tang[k]);
        lp_zero(dt[k]);
    }
    sync_wave();
    for (int k = 0; k < 3; ++k) {
        lp_mul_acc(tang[k], nnS, D0[k], 1.0);
        lp_mul_acc(tang[k], dnS, N1[k], -1.0);
    }
    sync_wave();
    for (int k = 0; k < 3; ++k) {
        lp_mul_acc(dt[k], den, tang[k], ep);
        lp_mul_acc(dt[k], num, N1[k], g.sg * g.sqrtS);
    }
    sync_wave();
    }
    // DXE = Dt x e22 (constant vector): linear combinations
    LP dxe[3];
    for (int k = 0; k < 3; ++k) {
        dxe[k] = LP{DXE[k].c, D};
        lp_zero(dxe[k]);
    }
    sync_wave();
    const V3<double> e = g.e22;
    lp_axpy(dxe[0], dt[1], e.z); lp_axpy(dxe[0], dt[2], -e.y);
    lp_axpy(dxe[1], dt[2], e.x); lp_axpy(dxe[1], dt[0], -e.z);
    lp_axpy(dxe[2], dt[0], e.y); lp_axpy(dxe[2], dt[1], -e.x);
    sync_wave();
    LP ut{UT.c, D + 1}, vt{VT.c, D + 1}, ka{KA.c, D};
    lp_zero(ut); lp_zero(vt); lp_zero(ka);
    sync_wave();
    // ut = DXE . Q ;  ka = DXE . e21 ;  vt = (Q x e21) . Dt = sum_k Dt_k (Q x e21)_k
    for (int k = 0; k < 3; ++k) {
        lp_mul_acc(ut, dxe[k], Q[k], 1.0);
        lp_axpy(ka, dxe[k], comp(g.e21, k));
    }
    sync_wave();
    {
        const V3<double> f = g.e21;
        // (Q x f)_0 = Q1 f2 - Q2 f1, (Q x f)_1 = Q2 f0 - Q0 f2, (Q x f)_2 = Q0 f1 - Q1 f0
        lp_mul_acc(vt, dt[0], Q[1], f.z); lp_mul_acc(vt, dt[0], Q[2], -f.y);
        lp_mul_acc(vt, dt[1], Q[2], f.x); lp_mul_acc(vt, dt[1], Q[0], -f.z);
        lp_mul_acc(vt, dt[2], Q[0], f.y); lp_mul_acc(vt, dt[2], Q[1], -f.x);
    }
    sync_wave();
    const int dm = D + g.f2;
    LP m2[3];
    for (int k = 0; k < 3; ++k) {
        m2[k] = LP{M2[k].c, dm};
        lp_zero(m2[k]);
    }
    sync_wave();
    for (int k = 0; k < 3; ++k) {
        lp_axpy(m2[k], ka, comp(g.n20, k));
        if (g.f2) {
            lp_axpy(m2[k], ut, comp(g.dn21, k));
            lp_axpy(m2[k], vt, comp(g.dn22, k));
        }
    }
    sync_wave();
    // CR = Dt x W, W = x3 - x1
    LP cr[3];
    for (int k = 0; k < 3; ++k) {
        cr[k] = LP{CR[k].c, D + 1};
        lp_zero(cr[k]);
    }
    sync_wave();
    lp_mul_acc(cr[0], dt[1], W[2], 1.0); lp_mul_acc(cr[0], dt[2], W[1], -1.0);
    lp_mul_acc(cr[1], dt[2], W[0], 1.0); lp_mul_acc(cr[1], dt[0], W[2], -1.0);
    lp_mul_acc(cr[2], dt[0], W[1], 1.0); lp_mul_acc(cr[2], dt[1], W[0], -1.0);
    sync_wave();
    const int da = 2 * D + 1 + g.f2;
    LP a{A.c, da};
    lp_zero(a);
    sync_wave();
    for (int k = 0; k < 3; ++k) lp_mul_acc(a, cr[k], m2[k], 1.0);
    sync_wave();
    Aout = a;
    return da;
}

// Numerical u-degree (the same rule as the reference solver): drop a top row of
// u-powers while it is zero or below 1e-10 times the row under it.
__device__ int tt_udeg(LP a)
{
    auto rowmax = [&](int i) {
        double m = 0.0;
        for (int j = 0; i + j <= a.d; ++j) m = fmax(m, fabs(a.c[i * (a.d + 1) + j]));
        return m;
    };
    int d = a.d;
    while (d > 0) {
        double top = rowmax(d), below = rowmax(d - 1);
        if (top == 0.0 || top < 1e-10 * below) --d;
        else break;
    }
    return d;
}

// ------------------------------------------------------------------ recursive isolation, runtime-sized input
// Real roots of sum_{k<=DMAX} c[k] x^k on [lo, hi]: level d works on the
// (DMAX-d)-th derivative divided by (DMAX-d)! (coefficients c[k+m] C(k+m, m)),
// whose piece ends are the roots of the level below; each piece with a strict
// sign change (sgn(0) := +1) is solved by safeguarded Newton (bisection
// fallback keeps the bracket) to full precision.

// f and f' of the level polynomial q_k = c[k+m] C(k+m, m), k = 0..d (the m-th
// derivative of sum c_k x^k divided by m!), read straight from c.
template <int DMAX, int d>
__device__ __forceinline__ void horner_lv(const double (&c)[DMAX + 1], double x, double& f, double& fp)
{
    constexpr int m = DMAX - d;
    f = c[d + m] * binom(d + m, m);
    fp = 0.0;
#pragma unroll
    for (int k = d - 1; k >= 0; --k) {
        fp = fma(fp, x, f);
        f = fma(f, x, c[k + m] * binom(k + m, m));
    }
}

// Roots of the derivative levels (d < DMAX) only split the next level into
// monotone pieces: they stop at 1e-9 relative, three orders below the
// near-double pair gap of the det-sign product (closer roots are left out of
// it), so a coarser piece end cannot change which roots a sign change brackets;
// the roots of the polynomial itself are refined to full precision.
template <int DMAX, int d>
__device__ __forceinline__ double refine(const double (&c)[DMAX + 1], double l, double r, bool neg_l)
{
    constexpr double tol = d == DMAX ? 4e-16 : 1e-9;
    double x = 0.5 * (l + r);
    for (int it = 0; it < 100; ++it) {
        double f, fp;
        horner_lv<DMAX, d>(c, x, f, fp);
        if (f == 0.0) return x;
        if ((f < 0.0) == neg_l) l = x;
        else r = x;
        double xn = x - f / fp;
        if (!(xn > l && xn < r)) xn = 0.5 * (l + r);
        if (!(r - l > 0.0) || xn == x) return xn;
        if (fabs(xn - x) <= tol * fmax(1.0, fabs(x))) return xn;
        x = xn;
    }
    return x;
}

// Level d of the recursion: rt[k] for the slots k set in the returned mask.
// The piece ends are the roots of level d-1 (bit mask `bmask`, values bp).
template <int DMAX, int d>
__device__ __forceinline__ unsigned iso_level(const double (&c)[DMAX + 1], double lo, double hi,
                                              double (&rt)[DMAX + 1])
{
    double bp[DMAX + 1];
    unsigned bmask = 0u;
    if constexpr (d > 1) bmask = iso_level<DMAX, d - 1>(c, lo, hi, bp);
    // pass 1: bit k set if piece k (ending at bp[k], or at hi for k = d) has a strict sign change
    unsigned mask = 0u;
    {
        double l = lo, f_lo, dummy;
        horner_lv<DMAX, d>(c, lo, f_lo, dummy);
#pragma unroll
        for (int k = 0; k <= d; ++k) {
            const bool has = (k < d) ? ((bmask >> k) & 1u) != 0u : true;
            const double r = (k < d) ? bp[k] : hi;
            if (has) {
                double f_r, dd;
                horner_lv<DMAX, d>(c, r, f_r, dd);
                if (r > l && ((f_lo < 0.0) != (f_r < 0.0))) mask |= 1u << k;
                l = r;
                f_lo = f_r;
            }
        }
    }
    // pass 2: one refinement per sign-change piece of this lane
    unsigned todo = mask;
    while (todo) {
        const int k = __builtin_ctz(todo);
        todo &= todo - 1u;
        double l = lo, r = hi;
#pragma unroll
        for (int j = 0; j < d; ++j) {
            if (((bmask >> j) & 1u) && j < k) l = bp[j];
            if (j == k) r = bp[j];
        }
        double f_l, dd;
        horner_lv<DMAX, d>(c, l, f_l, dd);
        const double x = refine<DMAX, d>(c, l, r, f_l < 0.0);
#pragma unroll
        for (int j = 0; j <= d; ++j)
            if (j == k) rt[j] = x;
    }
    // pass 3: slot order, near-duplicates dropped
    unsigned okm = 0u;
    double last = -1e300;
#pragma unroll
    for (int k = 0; k <= d; ++k) {
        if ((mask >> k) & 1u) {
            if (rt[k] - last > 1e-12 * fmax(1.0, fabs(rt[k]))) {
                okm |= 1u << k;
                last = rt[k];
            }
        }
    }
    return okm;
}

// ------------------------------------------------------------------ b(u,v) through its defining products
// b(u, v) from its defining products; with kr, also |kappa| / (|Dt| |e21 x e22|),
// the sine of the angle between the mapped ray from x1 and T2's plane
__device__ __forceinline__ double tt_b_eval(const TTGeo& g, double u, double v, double* kr = nullptr)
{
    V3<double> x1 = g.p1 + g.e11 * u + g.e12 * v;
    V3<double> n1 = g.n10 + (g.dn11 * u + g.dn12 * v) * double(g.f1);
    V3<double> d0 = x1 - g.x0;
    double nn = dot(n1, n1), dn = dot(d0, n1);
    V3<double> Dt;
    if (g.ev1 == SPOLY_R) {
        Dt = d0 * nn - n1 * (2.0 * dn);
    } else {
        double dd = dot(d0, d0);
        double beta = (1.0 - g.etap * g.etap) * nn * dd + g.etap * g.etap * dn * dn;
        double num = g.sq0 + g.sq1 * beta / g.S, den = g.sr0 + g.sr1 * beta / g.S;
        Dt = (d0 * nn - n1 * dn) * (g.etap * den) + n1 * (g.sg * g.sqrtS * num);
    }
    V3<double> q = x1 - g.p2;
    V3<double> dxe = cross(Dt, g.e22);
    double ut = dot(dxe, q), vt = dot(cross(q, g.e21), Dt), ka = dot(dxe, g.e21);
    V3<double> X2 = g.p2 * ka + g.e21 * ut + g.e22 * vt;
    V3<double> M2 = g.n20 * ka + (g.dn21 * ut + g.dn22 * vt) * double(g.f2);
    V3<double> D2 = g.x3 * ka - X2;
    if (kr) {
        const double ld = len(Dt) * g.n2len;
        *kr = ld > 0.0 ? fabs(ka) / ld : 0.0;
    }
    if (g.ev2 == SPOLY_R) {
        const V3<double> t = cross(M2, g.edge2);
        return dot(Dt, M2) * dot(D2, t) + dot(Dt, t) * dot(D2, M2);
    }
    auto comp = [&](V3<double> w) { return g.axis == 0 ? w.x : (g.axis == 1 ? w.y : w.z); };
    double l = comp(cross(Dt, M2)), r = comp(cross(D2, M2));
    return g.eta1 * g.eta1 * dot(D2, D2) * l * l - g.eta2 * g.eta2 * dot(Dt, Dt) * r * r;
}

// a_i(v) for i <= kDA (zero above the numerical degree)
__device__ __forceinline__ void tt_acoef(const double* __restrict__ Ac, int da, int ma, double v, double (&c)[kDA + 1])
{
#pragma unroll
    for (int i = 0; i <= kDA; ++i) {
        double s = 0.0;
        if (i <= ma)
            for (int j = da - i; j >= 0; --j) s = fma(s, v, Ac[i * (da + 1) + j]);
        c[i] = s;
    }
}

// An upper bound of x^(1/k) for x >= 0, within 0.2% of it: the exponent is
// split off exactly (frexp) and only the logarithm of the mantissa and the
// fractional power of two go through single-precision transcendentals.  The
// bound only sizes the isolation interval, so a slightly larger value leaves
// the roots found unchanged.
__device__ __forceinline__ double root_k_upper(double x, int k)
{
    if (!(x > 0.0)) return 0.0;
    if (!isfinite(x)) return x;
    int e;
    const double mnt = frexp(x, &e);                        // x = mnt 2^e, mnt in [1/2, 1)
    const float t = (float(e) + log2f(float(mnt))) / float(k);
    const float fl = floorf(t);
    return ldexp(double(exp2f(t - fl)), int(fl)) * 1.002;
}

// Two consecutive real roots of a(., v) closer than kPairGap max(1, |alpha|)
// are left out of the product: together they contribute b(alpha)^2 > 0 unless
// b vanishes between them, and such pairs sit where x2 goes to infinity (far
// outside T1), where a and b nearly share a root and the values of b are
// rounding noise.
constexpr double kPairGap = 1e-4;

// Roots of a(., v) where the mapped ray from x1 runs within this angle (rad)
// of T2's plane put x2 at infinity: no path lies there, and where T2 is flat
// or its normals are proportional to its positions (a sphere) kappa divides
// both a and b, so the resultant vanishes identically and the sign of b at
// such a root is rounding.  They are left out of the product.
constexpr double kKappaSkip = 1e-4;

// sgn b at a root of a(., v) taken into the product: -1, or +1 (also for a
// root left out at x2 = infinity)
__device__ __forceinline__ bool factor_negative(const TTGeo& g, double u, double v)
{
    double kr;
    const double b = tt_b_eval(g, u, v, &kr);
    return kr >= kKappaSkip && b < 0.0;
}

// Product of sgn b(x B, v) over the real roots x in [-1, 1] of the scaled
// a(., v) (coefficients c, degree at most D), near-double pairs and roots at
// x2 = infinity left out.
template <int D>
__device__ __forceinline__ int sign_over_roots(const TTGeo& g, const double (&c)[kDA + 1], double B, double v)
{
    double cc[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) cc[k] = c[k];
    double rt[D + 1];
    unsigned okm = iso_level<D, D>(cc, -1.0, 1.0, rt);
    // roots in ascending order; a root waits in `p` until the next one shows
    // whether the two form a near-double pair (left out of the product)
    int s = 1;
    bool has_p = false;
    double p = 0.0;
    while (okm) {
        const int k = __builtin_ctz(okm);
        okm &= okm - 1u;
        double x = 0.0;
#pragma unroll
        for (int j = 0; j <= D; ++j)
            if (j == k) x = rt[j];
        x *= B;
        if (has_p && x - p <= kPairGap * fmax(1.0, fabs(p))) {
            has_p = false;
            continue;
        }
        if (has_p && factor_negative(g, p, v)) s = -s;
        p = x;
        has_p = true;
    }
    if (has_p && factor_negative(g, p, v)) s = -s;
    return s;
}

// sign of det R(v) (up to a constant sign): product of sgn b over the real roots of a(., v)
__device__ int tt_det_sign(const TTGeo& g, const double* __restrict__ Ac, int da, int ma, double v)
{
    double c[kDA + 1];
    tt_acoef(Ac, da, ma, v, c);
    double lead = 0.0;
#pragma unroll
    for (int i = 0; i <= kDA; ++i)
        if (i == ma) lead = c[i];
    if (lead == 0.0) return 1;
    double B = 0.0;
#pragma unroll
    for (int k = 1; k <= kDA; ++k) {
        double ck = 0.0;
#pragma unroll
        for (int i = 0; i <= kDA; ++i)
            if (i == ma - k) ck = c[i];
        if (k <= ma) B = fmax(B, root_k_upper(fabs(ck / lead), k));
    }
    B = 2.0 * B;
    if (!(B > 0.0)) B = 1.0;
    double pw = 1.0;
#pragma unroll
    for (int k = 0; k <= kDA; ++k) {
        c[k] *= pw;
        pw *= B;
    }
    if (ma <= 8) return sign_over_roots<8>(g, c, B, v);
    return ma <= 13 ? sign_over_roots<13>(g, c, B, v) : sign_over_roots<kDA>(g, c, B, v);
}

// ------------------------------------------------------------------ path phase (exact constraints, FP64)
__device__ bool tt_trace(const TTGeo& g, double u1, double v1, double& u2, double& v2, V3<double>& x1,
                         V3<double>& x2)
{
    x1 = g.p1 + g.e11 * u1 + g.e12 * v1;
    V3<double> n = normalized(g.n10 + g.dn11 * u1 + g.dn12 * v1);
    V3<double> di = normalized(x1 - g.x0);
    double c = dot(di, n);
    V3<double> dt;
    if (g.ev1 == SPOLY_R) {
        dt = di - n * (2.0 * c);
    } else {
        if (c > 0.0) {
            n = n * -1.0;
            c = -c;
        }
        double ci = -c;
        double k = 1.0 - g.etap * g.etap * (1.0 - ci * ci);
        if (k < 0.0) return false;
        dt = di * g.etap + n * (g.etap * ci - sqrt(k));
    }
    V3<double> pv = cross(dt, g.e22);
    double det = dot(g.e21, pv);
    if (!(fabs(det) > 0.0)) return false;
    V3<double> tv = x1 - g.p2;
    u2 = dot(tv, pv) / det;
    V3<double> qv = cross(tv, g.e21);
    v2 = dot(dt, qv) / det;
    double t = dot(g.e22, qv) / det;
    if (!(t > 0.0)) return false;
    x2 = g.p2 + g.e21 * u2 + g.e22 * v2;
    return true;
}

__device__ bool tt_F(const TTGeo& g, V3<double> ta, V3<double> tb, double u, double v, double F[2])
{
    double u2, v2;
    V3<double> x1, x2;
    if (!tt_trace(g, u, v, u2, v2, x1, x2)) return false;
    V3<double> n2 = normalized(g.n20 + g.dn21 * u2 + g.dn22 * v2);
    V3<double> wi = normalized(x1 - x2), wo = normalized(g.x3 - x2);
    V3<double> h = normalized(wi * g.eta1 + wo * g.eta2);
    V3<double> gg = cross(h, n2);
    F[0] = dot(gg, ta);
    F[1] = dot(gg, tb);
    return true;
}

// Newton on (h2^ x n2^) . (ta, tb) = 0 with a central-difference Jacobian.
__device__ bool tt_polish(const TTGeo& g, int iters, double& pu, double& pv)
{
    V3<double> nc = normalized(g.n20 + g.dn21 * (1.0 / 3.0) + g.dn22 * (1.0 / 3.0));
    V3<double> ref = fabs(nc.x) < 0.9 ? V3<double>{1.0, 0.0, 0.0} : V3<double>{0.0, 1.0, 0.0};
    V3<double> ta = normalized(cross(nc, ref)), tb = cross(nc, ta);
    double u = pu, v = pv, step = 1e300;
    const double h = 1e-6;
    for (int it = 0; it < iters; ++it) {
        double F[2], Fu1[2], Fu0[2], Fv1[2], Fv0[2];
        if (!tt_F(g, ta, tb, u, v, F) || !tt_F(g, ta, tb, u + h, v, Fu1) || !tt_F(g, ta, tb, u - h, v, Fu0) ||
            !tt_F(g, ta, tb, u, v + h, Fv1) || !tt_F(g, ta, tb, u, v - h, Fv0))
            return false;
        double J00 = (Fu1[0] - Fu0[0]) / (2 * h), J10 = (Fu1[1] - Fu0[1]) / (2 * h);
        double J01 = (Fv1[0] - Fv0[0]) / (2 * h), J11 = (Fv1[1] - Fv0[1]) / (2 * h);
        double det = J00 * J11 - J01 * J10;
        if (!(det != 0.0) || !isfinite(det)) return false;
        double du = (F[0] * J11 - J01 * F[1]) / det;
        double dv = (J00 * F[1] - J10 * F[0]) / det;
        u -= du;
        v -= dv;
        step = fabs(du) + fabs(dv);
        if (!(step > 1e-15)) break;
    }
    pu = u;
    pv = v;
    return step <= 1e-10;
}

__device__ __forceinline__ bool law(V3<double> xp, V3<double> x, V3<double> xn, V3<double> nrm, double ein,
                                    double eout, int ev, double& res)
{
    double ln = len(nrm);
    if (!(ln > 1e-12)) return false;
    V3<double> nh = nrm * (1.0 / ln);
    V3<double> wi = normalized(xp - x), wo = normalized(xn - x);
    V3<double> h = wi * ein + wo * eout;
    double lh = len(h);
    if (!(lh > 0.0)) return false;
    res = len(cross(h * (1.0 / lh), nh));
    const double side = dot(wi, nh) * dot(wo, nh);
    return ev == SPOLY_R ? side > 0.0 : side < 0.0;   // reflection: one side; refraction: opposite sides
}

// ------------------------------------------------------------------ the fused kernel
// One tuple per wave (the whole wave must call it); `lds` holds kLdsDoubles
// doubles and `sgeo` one TTGeo, both in LDS and private to the wave.  The
// tuple's geometry is the same for every lane, so it is kept in LDS rather
// than replicated in vector registers.  smask and cmask (LDS, kSignWords
// each) hold the scan's sign and sign-change bits.  Output records carry
// query id q + qid_offset.
__device__ __forceinline__ void tt_tuple(const TTArgs& A, int64_t q, double* lds, TTGeo* sgeo,
                                         unsigned long long* smask, unsigned long long* cmask, int64_t qid_offset)
{
    const int lane = lane_id();
    {
        TTGeo gl;
        tt_setup(A, q, gl);
        if (lane == 0) *sgeo = gl;
    }
    sync_wave();
    const TTGeo& g = *sgeo;
    LP a;
    const int da = tt_build_a(g, lds, a);
    const int ma = tt_udeg(a);
    sync_wave();
    int degen = 0;
    // ---- sign scan at v_j = j / pieces, 64 samples per round; bit j of
    // smask is set where the sign at v_j is negative, bit j of cmask where the
    // signs at v_j and v_{j+1} differ (piece j holds a sign change)
    const int P = A.pieces;
    const int nw = (P + 1 + kWave - 1) / kWave;   // sign words
    if (ma < 1) degen = 1;
    for (int w = 0; w < nw; ++w) {
        const int j = w * kWave + lane;
        const bool neg = !degen && j <= P && tt_det_sign(g, a.c, da, ma, double(j) / P) < 0;
        const unsigned long long bal = __ballot(neg);
        if (lane == 0) smask[w] = bal;
    }
    sync_wave();
    int nv = 0;
    for (int w = 0; w < nw; ++w) {
        const unsigned long long cur = smask[w], nxt = (w + 1 < nw) ? smask[w + 1] : 0ull;
        unsigned long long c = cur ^ ((cur >> 1) | (nxt << 63));
        const int valid = P - w * kWave;            // pieces j = w*64 + i with i < valid
        if (valid < kWave) c &= valid > 0 ? ((1ull << valid) - 1ull) : 0ull;
        if (degen) c = 0ull;
        nv += __popcll(c);
        if (lane == 0) cmask[w] = c;
    }
    sync_wave();
    // ---- bisection (Sec. 5.2), then the path phase (u from a(u)|v, polish,
    // validation) for the final midpoint of every sign-change piece.
    LaneTT S;
    S.n = 0;
    S.over = 0;
    int ncand = 0;
    auto path_phase = [&](const double v) {
        double c[kDA + 1];
        tt_acoef(a.c, da, ma, v, c);
        double ur[kDA + 1];
        unsigned um = iso_level<kDA, kDA>(c, -A.u_margin, 1.0 - v + A.u_margin, ur);
        while (um) {
            const int t = __builtin_ctz(um);
            um &= um - 1u;
            double u = 0.0, vv = v;
#pragma unroll
            for (int j = 0; j <= kDA; ++j)
                if (j == t) u = ur[j];
            ncand++;
            if (!tt_polish(g, A.polish_iters, u, vv)) continue;
            if (!(u >= 0.0 && vv >= 0.0 && u + vv <= 1.0)) continue;
            double u2, v2;
            V3<double> x1, x2;
            if (!tt_trace(g, u, vv, u2, v2, x1, x2)) continue;
            if (!(u2 >= 0.0 && v2 >= 0.0 && u2 + v2 <= 1.0)) continue;
            double r1, r2;
            if (!law(g.x0, x1, x2, g.n10 + g.dn11 * u + g.dn12 * vv, g.eta0, g.eta1, g.ev1, r1)) continue;
            if (!law(x1, x2, g.x3, g.n20 + g.dn21 * u2 + g.dn22 * v2, g.eta1, g.eta2, g.ev2, r2)) continue;
            const double res = fmax(r1, r2);
            if (!(res <= A.tau)) continue;
            const double e1 = fmin(fmin(u, vv), 1.0 - u - vv), e2 = fmin(fmin(u2, v2), 1.0 - u2 - v2);
            bool dup = false;
#pragma unroll
            for (int q2 = 0; q2 < kTTMaxSol; ++q2)
                if (q2 < S.n && fabs(S.u1[q2] - u) < A.dedup && fabs(S.v1[q2] - vv) < A.dedup) dup = true;
            if (dup) continue;
            if (S.n >= kTTMaxSol) {
                S.over++;
                continue;
            }
#pragma unroll
            for (int q2 = 0; q2 < kTTMaxSol; ++q2)
                if (q2 == S.n) {
                    S.u1[q2] = u; S.v1[q2] = vv; S.u2[q2] = u2; S.v2[q2] = v2;
                    S.res[q2] = res; S.edge[q2] = fmin(e1, e2);
                }
            S.n++;
        }
    };
    // sign of the scan at grid point j
    auto scan_sign = [&](int j) -> int { return ((smask[j >> 6] >> (j & 63)) & 1ull) ? -1 : 1; };
    // index of the k-th sign-change piece (k < nv)
    auto kth_piece = [&](int k) -> int {
        for (int w = 0; w < nw; ++w) {
            unsigned long long m = cmask[w];
            const int c = __popcll(m);
            if (k < c) {
                for (int i = 0; i < k; ++i) m &= m - 1ull;
                return w * kWave + __ffsll((long long)m) - 1;
            }
            k -= c;
        }
        return 0;
    };
    // Bits per round of the grouped bisection: groups of 2^b lanes evaluate the
    // 2^b - 1 midpoints that the next b bisection steps can visit, so b steps
    // cost one evaluation round; 64 / 2^b pieces share a round.  Chosen per
    // tuple for the fewest rounds; b = 1 is the plain one-lane-per-piece loop.
    const int iters = A.bisect_iters;
    int bits = 1;
    if (nv > 0 && nv <= 32 && iters > 0) {
        int best = iters * ((nv + kWave - 1) / kWave);
        for (int bb = 2; bb <= 5; ++bb) {
            const int rounds = (iters + bb - 1) / bb, per = kWave >> bb;
            const int cost = rounds * ((nv + per - 1) / per);
            if (cost < best) { best = cost; bits = bb; }
        }
    }
    if (bits == 1) {
        for (int base = 0; base < nv; base += kWave) {
            const int k = base + lane;
            const int piece = k < nv ? kth_piece(k) : 0;
            const int sl = scan_sign(piece);
            if (k >= nv) continue;
            double l = double(piece) / P, r = double(piece + 1) / P;
            for (int it = 0; it < iters; ++it) {
                const double mm = 0.5 * (l + r);
                if (tt_det_sign(g, a.c, da, ma, mm) == sl) l = mm;
                else r = mm;
            }
            path_phase(0.5 * (l + r));
        }
    } else {
        // Every round reproduces b sequential steps exactly: the candidate
        // midpoints are formed by the same halvings, and the step decisions
        // read the signs evaluated at them.
        const int gsz = 1 << bits, per = kWave >> bits;
        const int grp = lane >> bits, j = lane & (gsz - 1);
        double my_v = 0.0;
        for (int batch = 0; batch < nv; batch += per) {
            const int k = batch + grp;
            const bool act = k < nv;
            const int piece = act ? kth_piece(k) : 0;
            const int sl = scan_sign(piece);
            double l = double(piece) / P, r = double(piece + 1) / P;
            for (int left = iters; left > 0;) {
                const int bb = left < bits ? left : bits;
                const int top = 1 << (bb - 1);
                bool same = false;
                if (act && j >= 1 && j < (1 << bb)) {
                    double lo = l, hi = r, pt = 0.0;
                    int c = top, half = top >> 1;
                    for (int d = 0; d < bb; ++d) {   // node j of the in-order tree sits at depth < bb
                        const double mm = 0.5 * (lo + hi);
                        if (j == c) { pt = mm; break; }
                        if (j > c) { lo = mm; c += half; }
                        else { hi = mm; c -= half; }
                        half >>= 1;
                    }
                    same = tt_det_sign(g, a.c, da, ma, pt) == sl;
                }
                const unsigned long long bal = __ballot(same);
                const unsigned int gb = (unsigned int)((bal >> (grp << bits)) & ((1ull << gsz) - 1ull));
                int c = top, half = top >> 1;
                for (int st = 0; st < bb; ++st) {
                    const double mm = 0.5 * (l + r);
                    if ((gb >> c) & 1u) { l = mm; c += half; }
                    else { r = mm; c -= half; }
                    half >>= 1;
                }
                left -= bb;
            }
            const double v = 0.5 * (l + r);
            // hand the piece's v to lane k (lanes batch .. batch + per - 1)
            const int t = lane - batch;
            const double got = __shfl(v, (t >= 0 && t < per ? t : 0) << bits, kWave);
            if (t >= 0 && t < per && lane < nv) my_v = got;
        }
        if (lane < nv) path_phase(my_v);
    }
    // ---- de-duplicate across lanes (two v roots polishing onto one path), then compact
    // lanes compare against all earlier lanes' solutions through shuffles
    int keepmask = (1 << S.n) - 1;
    for (int src = 0; src < kWave; ++src) {
        const int ns = __shfl(S.n, src, kWave);
        if (ns == 0) continue;
#pragma unroll
        for (int s = 0; s < kTTMaxSol; ++s) {
            if (s >= ns) break;
            const double ou = __shfl(S.u1[s], src, kWave), ov = __shfl(S.v1[s], src, kWave);
            if (lane > src) {
#pragma unroll
                for (int t = 0; t < kTTMaxSol; ++t)
                    if (t < S.n && fabs(S.u1[t] - ou) < A.dedup && fabs(S.v1[t] - ov) < A.dedup)
                        keepmask &= ~(1 << t);
            }
        }
    }
    const int cnt = __popc(keepmask);
    const int incl = wave_incl_scan(cnt);
    const int total = __shfl(incl, kWave - 1, kWave);
    if (total > 0) {
        unsigned long long base = 0;
        if (lane == kWave - 1) base = atomicAdd(A.out_count, (unsigned long long)total);
        base = __shfl(base, kWave - 1, kWave);
        unsigned long long idx = base + (unsigned long long)(incl - cnt);
#pragma unroll
        for (int s = 0; s < kTTMaxSol; ++s) {
            if (!((keepmask >> s) & 1)) continue;
            if (idx < (unsigned long long)A.cap) {
                spoly_solution o;
                o.query = int32_t(q + qid_offset);
                o.tri[0] = A.q_tris[2 * q];
                o.tri[1] = A.q_tris[2 * q + 1];
                o.flags = 0;
                o.u[0] = S.u1[s]; o.v[0] = S.v1[s];
                o.u[1] = S.u2[s]; o.v[1] = S.v2[s];
                o.residual = float(S.res[s]);
                o.edge = float(S.edge[s]);
                A.out[idx] = o;
            }
            idx++;
        }
    }
    if (A.counters) {
        unsigned long long c1 = wave_sum_u64(ncand);
        unsigned long long c3 = wave_sum_u64(S.over);
        if (lane == 0) {
            if (c3) atomicAdd(A.counters + 3, c3);
            if (nv) atomicAdd(A.counters + 0, (unsigned long long)nv);
            if (c1) atomicAdd(A.counters + 1, c1);
            if (degen) atomicAdd(A.counters + 2, 1ull);
        }
    }
    if (A.diag_q && lane == 0) {
        A.diag_q[2 * q] = nv;
        A.diag_q[2 * q + 1] = total;
    }
}

// ------------------------------------------------------------------ normal-cone cull for two vertices
// Direction cone from a sphere (centre `from`, radius r) to a point or sphere at
// `to`: unit axis a, chord bound ch = 2 sin(theta/2), theta = asin(r/|to-from|).
__device__ __forceinline__ bool dir_cone_f(float3 from, float r, float3 to, float3& a, float& ch)
{
    float dx = to.x - from.x, dy = to.y - from.y, dz = to.z - from.z;
    float l = sqrtf(dx * dx + dy * dy + dz * dz);
    if (!(l > r * 1.0001f)) return false;
    float il = 1.0f / l;
    a = make_float3(dx * il, dy * il, dz * il);
    float s = r * il;
    ch = sqrtf(fmaxf(0.0f, 2.0f - 2.0f * sqrtf(fmaxf(0.0f, 1.0f - s * s))));
    return true;
}
// Can h = ea wa + eb wb (wa, wb in their cones) be parallel to a normal of the cone nc (axis, half angle)?
__device__ __forceinline__ bool vtx_keep(float4 nc, float3 aa, float cha, float ea, float3 ab, float chb, float eb,
                                         float margin)
{
    if (!(nc.w < 1.5707f)) return true;
    float hx = ea * aa.x + eb * ab.x, hy = ea * aa.y + eb * ab.y, hz = ea * aa.z + eb * ab.z;
    float L = sqrtf(hx * hx + hy * hy + hz * hz);
    float delta = (ea * cha + eb * chb) * 1.0001f + 1e-6f;
    if (!(delta < L)) return true;
    float lim = nc.w + asinf(fminf(1.0f, delta / L)) + margin;
    if (lim >= 1.5707f) return true;
    return fabsf(nc.x * hx + nc.y * hy + nc.z * hz) / L >= cosf(lim) * (1.0f - 1e-6f);
}

// (T1, T2) pairs passing the test at x2 for light j3 (independent of x0).
__global__ void __launch_bounds__(256) k_tt_pairs(CullTTArgs A, int j3)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t npair = int64_t(A.n_tris) * A.n_tris;
    bool keep = false;
    int t1 = 0, t2 = 0;
    if (idx < npair) {
        t1 = int(idx / A.n_tris);
        t2 = int(idx % A.n_tris);
        if (t1 != t2) {
            float4 a0 = A.tri_cone[2 * t1], b0 = A.tri_cone[2 * t2], b1 = A.tri_cone[2 * t2 + 1];
            float3 c1 = make_float3(a0.x, a0.y, a0.z), c2 = make_float3(b0.x, b0.y, b0.z);
            float3 x3 = make_float3(float(A.x3x[j3]), float(A.x3y[j3]), float(A.x3z[j3]));
            float3 a21, a3;
            float ch21, ch3;
            if (!dir_cone_f(c2, a0.w + b0.w, c1, a21, ch21) || !dir_cone_f(c2, b0.w, x3, a3, ch3)) keep = true;
            else keep = vtx_keep(b1, a21, ch21, A.eta1, a3, ch3, A.eta2, A.margin);
        }
    }
    const unsigned long long bal = __ballot(keep);
    const int total = __popcll(bal);
    if (total == 0) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(A.pair_count, (unsigned long long)total);
    base = __shfl(base, 0, kWave);
    if (keep) {
        unsigned long long o = base + __popcll(bal & ((1ull << lane_id()) - 1ull));
        if (o < (unsigned long long)A.pair_cap) A.pairs[o] = make_int2(t1, t2);
    }
}

constexpr int kTTCullPts = 64;

// (x0, pair) tuples passing the test at x1; one atomic per wave per 64 receivers.
__global__ void __launch_bounds__(256) k_tt_cull(CullTTArgs A, int j3, int64_t n_pairs)
{
    __shared__ unsigned long long s_bal[4][kTTCullPts];
    __shared__ unsigned long long s_slots[kMaxBlockWaves + 1];
    const int64_t npb = (n_pairs + 255) / 256;
    const int64_t pk = int64_t(blockIdx.x % npb) * 256 + threadIdx.x;
    const int r0 = int(blockIdx.x / npb) * kTTCullPts;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const bool ok = pk < n_pairs;
    int2 pr = make_int2(0, 0);
    float4 a0 = make_float4(0, 0, 0, 0), a1 = make_float4(0, 0, 0, 4.0f), b0 = make_float4(0, 0, 0, 0);
    float3 a12 = make_float3(0, 0, 0);
    float ch12 = 0.0f;
    bool unb = true;
    if (ok) {
        pr = A.pairs[pk];
        a0 = A.tri_cone[2 * pr.x];
        a1 = A.tri_cone[2 * pr.x + 1];
        b0 = A.tri_cone[2 * pr.y];
        unb = !dir_cone_f(make_float3(a0.x, a0.y, a0.z), a0.w + b0.w, make_float3(b0.x, b0.y, b0.z), a12, ch12);
    }
    const int nr = min(kTTCullPts, A.n0 - r0);
    int mine = 0;
    for (int k = 0; k < nr; ++k) {
        const int j0 = r0 + k;
        bool keep = false;
        if (ok) {
            float3 a0d;
            float ch0;
            float3 x0 = make_float3(float(A.x0x[j0]), float(A.x0y[j0]), float(A.x0z[j0]));
            if (unb || !dir_cone_f(make_float3(a0.x, a0.y, a0.z), a0.w, x0, a0d, ch0)) keep = true;
            else keep = vtx_keep(a1, a0d, ch0, A.eta0, a12, ch12, A.eta1, A.margin);
        }
        const unsigned long long bal = __ballot(keep);
        if (lane == 0) s_bal[w][k] = bal;
        mine += keep ? 1 : 0;
    }
    const int incl = wave_incl_scan(mine);
    const int total = __shfl(incl, kWave - 1, kWave);
    const unsigned long long base = block_reserve((unsigned long long)total, A.out_count, s_slots);
    if (total == 0) return;
    unsigned long long off = base;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int k = 0; k < nr; ++k) {
        const unsigned long long bal = s_bal[w][k];
        if ((bal >> lane) & 1ull) {
            const unsigned long long o = off + (unsigned long long)__popcll(bal & lt);
            if (o < (unsigned long long)A.cap) {
                A.out_x0[o] = r0 + k;
                A.out_x3[o] = j3;
                A.out_t1[o] = pr.x;
                A.out_t2[o] = pr.y;
            }
        }
        off += (unsigned long long)__popcll(bal);
    }
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_tt_pairs(const CullTTArgs& A, int j3, hipStream_t stream)
{
    const int64_t npair = int64_t(A.n_tris) * A.n_tris;
    if (npair <= 0) return hipSuccess;
    const int64_t nb = (npair + 255) / 256;
    if (nb > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tt_pairs, dim3(unsigned(nb)), dim3(256), 0, stream, A, j3);
    return hipGetLastError();
}

hipError_t launch_tt_cull(const CullTTArgs& A, int j3, int64_t n_pairs, hipStream_t stream)
{
    if (n_pairs <= 0 || A.n0 <= 0) return hipSuccess;
    const int64_t nb = ((n_pairs + 255) / 256) * ((A.n0 + kTTCullPts - 1) / kTTCullPts);
    if (nb > 2147483647LL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tt_cull, dim3(unsigned(nb)), dim3(256), 0, stream, A, j3, n_pairs);
    return hipGetLastError();
}

__global__ void __launch_bounds__(64) k_tt_solve(TTArgs A)
{
    __shared__ double lds[kLdsDoubles];
    __shared__ TTGeo sgeo;
    __shared__ unsigned long long smask[kSignWords], cmask[kSignWords];
    // grid-stride over tuples: a launch may hold at most 2^32 work-items
    for (int64_t q = blockIdx.x; q < A.nq; q += gridDim.x) {
        tt_tuple(A, q, lds, &sgeo, smask, cmask, 0);
        __syncthreads();
    }
}

hipError_t launch_tt_solve(const TTArgs& A, hipStream_t stream)
{
    if (A.nq <= 0) return hipSuccess;
    if (A.nq > 2147483647LL) return hipErrorInvalidValue;
    const int64_t blocks = A.nq < (int64_t(1) << 22) ? A.nq : (int64_t(1) << 22);
    hipLaunchKernelGGL(k_tt_solve, dim3(unsigned(blocks)), dim3(kWave), 0, stream, A);
    return hipGetLastError();
}

}  // namespace spoly
