/*
 * tail_oracle.c -- plain FP64 CPU oracle of the path-phase tail: the
 * visibility test and the contribution of every validated specular path
 * (Sec. 5.3, "The whole pipeline": a path is dropped when the segment from
 * any vertex to the next is blocked; each surviving connection contributes,
 * and several connections between the same two endpoints add up).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header or helper with the HIP path.
 *
 * Readings (the paper delegates both steps to prior work):
 *  - visibility: the segment x_i -> x_{i+1} (x_{k+1} the light) is blocked iff
 *    some triangle other than the ones carrying x_i and x_{i+1} meets it at a
 *    segment parameter t in [t_eps, 1 - t_eps] and closed barycentrics
 *    (Moller-Trumbore, every triangle tried: the brute-force definition);
 *  - contribution: the irradiance at x0, on the plane normal to the arriving
 *    ray, carried by the chain from an isotropic point light of intensity I:
 *    E = I * prod(F_i) * dw/dA, where dw/dA is the solid angle of light
 *    directions per unit of that area; F_i is the unpolarised Fresnel
 *    transmittance at a refraction (shading normal, the two media of the
 *    vertex) and a constant reflectance rho at a reflection.  The oracle takes
 *    dA/dw from central differences of a forward trace from the light
 *    through the planes of the chain's triangles (shading normals
 *    interpolated at each hit) onto the receiver plane, at two step sizes
 *    combined by Richardson extrapolation.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <string.h>

typedef struct { double x, y, z; } t3;
static t3 T3(double x, double y, double z) { t3 r = {x, y, z}; return r; }
static t3 tadd(t3 a, t3 b) { return T3(a.x + b.x, a.y + b.y, a.z + b.z); }
static t3 tsub(t3 a, t3 b) { return T3(a.x - b.x, a.y - b.y, a.z - b.z); }
static t3 tmul(t3 a, double s) { return T3(a.x * s, a.y * s, a.z * s); }
static double tdot(t3 a, t3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static t3 tcross(t3 a, t3 b) { return T3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double tlen(t3 a) { return sqrt(tdot(a, a)); }
static t3 tnorm(t3 a) { return tmul(a, 1.0 / tlen(a)); }
static t3 tload(const double *p, int64_t i) { return T3(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }

/* ------------------------------------------------------------------ visibility */

/* Moller-Trumbore of the segment p + t (q - p) against triangle (a, b, c).
 * Returns 1 on a hit (t in [teps, 1-teps], closed barycentrics) and writes
 * the distance of (t, u, v) from flipping that decision to *margin.         */
static int seg_tri(t3 p, t3 q, t3 a, t3 b, t3 c, double teps, double *margin)
{
    t3 d = tsub(q, p), e1 = tsub(b, a), e2 = tsub(c, a);
    t3 pv = tcross(d, e2);
    double det = tdot(e1, pv);
    if (det == 0.0) { *margin = INFINITY; return 0; }
    t3 tv = tsub(p, a);
    double u = tdot(tv, pv) / det;
    t3 qv = tcross(tv, e1);
    double v = tdot(d, qv) / det;
    double t = tdot(e2, qv) / det;
    double w = 1.0 - u - v;
    double in[5] = {u, v, w, t - teps, 1.0 - teps - t};
    int hit = 1;
    double m = INFINITY, out = -INFINITY;
    for (int j = 0; j < 5; ++j) {
        if (in[j] < 0.0) hit = 0;
        if (in[j] < m) m = in[j];
        if (-in[j] > out) out = -in[j];
    }
    *margin = hit ? m : out;
    return hit;
}

/* Blocked-segment mask of one path: bit i for x_i -> x_{i+1}; *margin is the
 * smallest decision margin over every (segment, triangle) pair tried.       */
static int32_t path_visibility(const double *P, const int32_t *tri, int64_t nt, const t3 *x, const int32_t *ptri,
                               int k, double teps, double *margin)
{
    int32_t mask = 0;
    double mm = INFINITY;
    for (int s = 0; s <= k; ++s) {
        int32_t skip_a = s >= 1 ? ptri[s - 1] : -1;   /* triangle of x_s */
        int32_t skip_b = s < k ? ptri[s] : -1;        /* triangle of x_{s+1} */
        for (int64_t t = 0; t < nt; ++t) {
            if (t == skip_a || t == skip_b) continue;
            double m;
            int h = seg_tri(x[s], x[s + 1], tload(P, tri[3 * t]), tload(P, tri[3 * t + 1]), tload(P, tri[3 * t + 2]),
                            teps, &m);
            if (h) mask |= 1 << s;
            if (m < mm) mm = m;
        }
    }
    *margin = mm;
    return mask;
}

/* ------------------------------------------------------------------ Fresnel */

/* Unpolarised Fresnel transmittance for light crossing from index n1 to n2
 * at incidence cosine ci (Fresnel's amplitude ratios for s and p).  Returns
 * 0 past the critical angle.                                               */
double ot_fresnel_t(double n1, double n2, double ci)
{
    ci = fabs(ci);
    double s2 = (n1 / n2) * (n1 / n2) * (1.0 - ci * ci);
    if (s2 >= 1.0) return 0.0;
    double ct = sqrt(1.0 - s2);
    double rs = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct);
    double rp = (n2 * ci - n1 * ct) / (n2 * ci + n1 * ct);
    return 1.0 - 0.5 * (rs * rs + rp * rp);
}

/* ------------------------------------------------------------------ forward trace */

typedef struct { t3 p0, e1, e2, n0, dn1, dn2; } ot_tri;

static ot_tri ot_load(const double *P, const double *N, const int32_t *tri, int64_t t)
{
    ot_tri T;
    t3 p0 = tload(P, tri[3 * t]), p1 = tload(P, tri[3 * t + 1]), p2 = tload(P, tri[3 * t + 2]);
    t3 n0 = tload(N, tri[3 * t]), n1 = tload(N, tri[3 * t + 1]), n2 = tload(N, tri[3 * t + 2]);
    T.p0 = p0; T.e1 = tsub(p1, p0); T.e2 = tsub(p2, p0);
    T.n0 = n0; T.dn1 = tsub(n1, n0); T.dn2 = tsub(n2, n0);
    return T;
}

/* Ray o + s d against the plane of T (no bounds); the hit point and the unit
 * interpolated normal there.  0 if parallel or behind.                     */
static int plane_hit(const ot_tri *T, t3 o, t3 d, t3 *x, t3 *n)
{
    t3 pv = tcross(d, T->e2);
    double det = tdot(T->e1, pv);
    if (det == 0.0) return 0;
    t3 tv = tsub(o, T->p0);
    double u = tdot(tv, pv) / det;
    t3 qv = tcross(tv, T->e1);
    double v = tdot(d, qv) / det;
    double s = tdot(T->e2, qv) / det;
    if (!(s > 0.0)) return 0;
    *x = tadd(T->p0, tadd(tmul(T->e1, u), tmul(T->e2, v)));
    *n = tnorm(tadd(T->n0, tadd(tmul(T->dn1, u), tmul(T->dn2, v))));
    return 1;
}

/* Mirror reflection of unit d about unit n, or Snell refraction from index n1
 * into n2.  0 on total internal reflection.                                 */
static int bend(t3 d, t3 n, int refract, double n1, double n2, t3 *out)
{
    double c = tdot(d, n);
    if (!refract) { *out = tsub(d, tmul(n, 2.0 * c)); return 1; }
    if (c > 0) { n = tmul(n, -1.0); c = -c; }
    double r = n1 / n2, ci = -c;
    double k = 1.0 - r * r * (1.0 - ci * ci);
    if (k < 0.0) return 0;
    *out = tnorm(tadd(tmul(d, r), tmul(n, r * ci - sqrt(k))));
    return 1;
}

/* Unit vectors a, b with (a, b, w) orthonormal (a fixed construction).     */
static void basis(t3 w, t3 *a, t3 *b)
{
    t3 h = fabs(w.x) < 0.6 ? T3(1, 0, 0) : (fabs(w.y) < 0.6 ? T3(0, 1, 0) : T3(0, 0, 1));
    *a = tnorm(tcross(w, h));
    *b = tcross(w, *a);
}

typedef struct {
    int k;
    const ot_tri *T;     /* T[0] carries x1, ... */
    const int32_t *ev;   /* 0 reflection, 1 refraction, per vertex */
    const double *eta;   /* eta[i]: index of the medium between x_i and x_{i+1} */
    t3 xl, wl, ea, eb;   /* light, direction to x_k and its tangent basis */
    t3 x0, w0, fa, fb;   /* receiver, arrival direction (x0 -> x1) and plane basis */
} trace_t;

/* Landing point of the light ray with direction wl + al ea + be eb on the
 * receiver plane, in (fa, fb) coordinates about x0.                         */
static int land(const trace_t *R, double al, double be, double y[2])
{
    t3 o = R->xl, d = tnorm(tadd(R->wl, tadd(tmul(R->ea, al), tmul(R->eb, be))));
    for (int i = R->k; i >= 1; --i) {
        t3 x, n;
        if (!plane_hit(&R->T[i - 1], o, d, &x, &n)) return 0;
        if (!bend(d, n, R->ev[i - 1], R->eta[i], R->eta[i - 1], &d)) return 0;
        o = x;
    }
    double den = tdot(d, R->w0);        /* plane through x0 normal to w0 */
    if (den == 0.0) return 0;
    double s = tdot(tsub(R->x0, o), R->w0) / den;
    t3 yp = tsub(tadd(o, tmul(d, s)), R->x0);
    y[0] = tdot(yp, R->fa);
    y[1] = tdot(yp, R->fb);
    return 1;
}

static int area_per_solid_angle(const trace_t *R, double h, double *out)
{
    double ya[2], yb[2], yc[2], yd[2];
    if (!land(R, h, 0, ya) || !land(R, -h, 0, yb) || !land(R, 0, h, yc) || !land(R, 0, -h, yd)) return 0;
    double j00 = (ya[0] - yb[0]) / (2 * h), j10 = (ya[1] - yb[1]) / (2 * h);
    double j01 = (yc[0] - yd[0]) / (2 * h), j11 = (yc[1] - yd[1]) / (2 * h);
    *out = fabs(j00 * j11 - j01 * j10);
    return 1;
}

/* ------------------------------------------------------------------ entry point
 * n paths of k (1 or 2) specular vertices.  Per path p: x0 = x0s[q_x0[p]],
 * light = xls[q_xl[p]], vertex i on triangle ptri[p k + i] at barycentrics
 * (pu, pv)[p k + i].  ev[k], eta[k+1] as in trace_t.  Outputs per path: the
 * blocked-segment mask, its decision margin, the Fresnel / reflectance
 * product, E (before visibility) and the relative change of E when the
 * difference step is quartered (a conditioning diagnostic).               */
int ot_tail(const double *P, const double *N, const int32_t *tri, int64_t nt, const double *x0s, const double *xls,
            const int32_t *q_x0, const int32_t *q_xl, const int32_t *ptri, const double *pu, const double *pv,
            int64_t n, int32_t k, const int32_t *ev, const double *eta, double intensity, double rho, double teps,
            double h, int32_t *mask, double *margin, double *fresnel, double *E, double *E_change)
{
    if (k < 1 || k > 2) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < n; ++p) {
        ot_tri T[2];
        t3 x[4];
        x[0] = tload(x0s, q_x0[p]);
        for (int i = 0; i < k; ++i) {
            T[i] = ot_load(P, N, tri, ptri[p * k + i]);
            x[i + 1] = tadd(T[i].p0, tadd(tmul(T[i].e1, pu[p * k + i]), tmul(T[i].e2, pv[p * k + i])));
        }
        x[k + 1] = tload(xls, q_xl[p]);
        mask[p] = path_visibility(P, tri, nt, x, ptri + p * k, k, teps, &margin[p]);

        double F = 1.0;
        for (int i = 1; i <= k; ++i) {
            if (!ev[i - 1]) { F *= rho; continue; }
            const ot_tri *Ti = &T[i - 1];
            double u = pu[p * k + i - 1], v = pv[p * k + i - 1];
            t3 nn = tnorm(tadd(Ti->n0, tadd(tmul(Ti->dn1, u), tmul(Ti->dn2, v))));
            t3 win = tnorm(tsub(x[i + 1], x[i]));       /* toward the light side */
            F *= ot_fresnel_t(eta[i], eta[i - 1], tdot(win, nn));
        }
        fresnel[p] = F;

        trace_t R;
        R.k = k; R.T = T; R.ev = ev; R.eta = eta;
        R.xl = x[k + 1]; R.wl = tnorm(tsub(x[k], x[k + 1]));
        basis(R.wl, &R.ea, &R.eb);
        R.x0 = x[0]; R.w0 = tnorm(tsub(x[1], x[0]));
        basis(R.w0, &R.fa, &R.fb);
        /* central differences at steps h and h/4, combined by Richardson
         * extrapolation (their error is c h^2 + O(h^4)); the change from the
         * h/4 value to the extrapolated one is the error estimate reported */
        double a1, a2;
        if (area_per_solid_angle(&R, h, &a1) && area_per_solid_angle(&R, 0.25 * h, &a2) && a1 > 0 && a2 > 0) {
            double ar = (16.0 * a2 - a1) / 15.0;
            if (!(ar > 0)) ar = a2;
            E[p] = intensity * F / ar;
            E_change[p] = fabs(a2 - ar) / ar;
        } else {
            E[p] = 0.0;
            E_change[p] = INFINITY;
        }
    }
    return 0;
}

/* Segment-triangle test alone (one pair per index), for the pins.          */
int ot_seg_tri(const double *p, const double *q, const double *a, const double *b, const double *c, int64_t n,
               double teps, int32_t *hit, double *margin)
{
    for (int64_t i = 0; i < n; ++i)
        hit[i] = seg_tri(tload(p, i), tload(q, i), tload(a, i), tload(b, i), tload(c, i), teps, &margin[i]);
    return 0;
}
