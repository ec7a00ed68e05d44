/*
 * FP64 oracle for the photon-plane workload (Section 6.7, reciprocal estimation inside the CMIS
 * framework): single scattering in a homogeneous medium lit by a rectangular area light, rendered
 * with photon planes whose balance-heuristic CMIS weight over the continuous technique space of
 * chord angles needs the reciprocal of an integral over that space.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: only the test suite, the smoke check and the CPU
 * baseline of the benchmarks load it; the HIP library never links or includes it.
 *
 * Scene block (27 doubles): light centre c[3], light axes U[3] and V[3] (orthonormal; the light
 * emits on the side of N = U x V, Lambertian, radiance Le), half extents eu, ev along U and V,
 * Le[3], camera[10] (position, target, up, vertical field of view in degrees), sigma_s, sigma_t,
 * t_max. The medium fills space, the phase function is isotropic, nothing occludes.
 *
 * What is computed:
 *   the single-scattered radiance along the eye ray o + t d, 0 < t <= t_max,
 *     L = int dt int_A dA(y) e^{-st t} ss (1/4pi) Le cos(theta_y) / R^2 e^{-st R},  R = |x - y|;
 *   a photon plane: y0 uniform on the light, chord angle alpha uniform in [0, pi), direction w
 *   cosine-distributed about N; the plane {y0 + s u_alpha + lambda w, lambda > 0} with the chord
 *   of the rectangle through y0 along u_alpha = cos(alpha) U + sin(alpha) V. An eye ray that
 *   meets it at x yields the path (camera, x, y = y0 + s u_alpha);
 *   the density of that path under chord angle alpha, measure dt dA(y):
 *     p(alpha, xbar) = (1/pi) (len(alpha; y) / A) (cos theta / pi) |u_alpha . (w x d)| / R^2,
 *   len(alpha; y) the length of the chord through y at angle alpha;
 *   the balance-heuristic CMIS estimate of one plane's hit (Section 6.7 with alpha the technique):
 *     f / int_0^pi p(alpha', xbar) dalpha' = ss Le e^{-st (t + R)} pi A / (4 J),
 *     J(y, m) = int_0^pi len(alpha; y) |u_alpha . m| dalpha,  m = w x d.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PL_PI 3.14159265358979323846

typedef struct { double x, y, z; } pv3;
static pv3 pv(double x, double y, double z) { pv3 r = {x, y, z}; return r; }
static pv3 padd(pv3 a, pv3 b) { return pv(a.x + b.x, a.y + b.y, a.z + b.z); }
static pv3 psub(pv3 a, pv3 b) { return pv(a.x - b.x, a.y - b.y, a.z - b.z); }
static pv3 pscl(pv3 a, double s) { return pv(a.x * s, a.y * s, a.z * s); }
static double pdot(pv3 a, pv3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static pv3 pcross(pv3 a, pv3 b) { return pv(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static pv3 pnorm(pv3 a) { return pscl(a, 1.0 / sqrt(pdot(a, a))); }

typedef struct {
    pv3 c, U, V, N;
    double eu, ev, area, le[3];
    pv3 cam_p, cam_f, cam_r, cam_u;
    double tan_half;
    double ss, st, tmax;
} plane_scene;

static void unpack(const double *b, plane_scene *s)
{
    s->c = pv(b[0], b[1], b[2]);
    s->U = pv(b[3], b[4], b[5]);
    s->V = pv(b[6], b[7], b[8]);
    s->N = pcross(s->U, s->V);
    s->eu = b[9]; s->ev = b[10];
    s->area = 4.0 * s->eu * s->ev;
    for (int k = 0; k < 3; ++k) s->le[k] = b[11 + k];
    const double *cam = b + 14;
    s->cam_p = pv(cam[0], cam[1], cam[2]);
    s->cam_f = pnorm(psub(pv(cam[3], cam[4], cam[5]), s->cam_p));
    s->cam_r = pnorm(pcross(s->cam_f, pv(cam[6], cam[7], cam[8])));
    s->cam_u = pcross(s->cam_r, s->cam_f);
    s->tan_half = tan(0.5 * cam[9] * PL_PI / 180.0);
    s->ss = b[24]; s->st = b[25]; s->tmax = b[26];
}

/* the eye ray through the centre of pixel (px, py) of a W x H image */
static pv3 pixel_dir(const plane_scene *s, int W, int H, int px, int py)
{
    const double aspect = (double)W / (double)H;
    const double x = (2.0 * (px + 0.5) / W - 1.0) * s->tan_half * aspect;
    const double y = (1.0 - 2.0 * (py + 0.5) / H) * s->tan_half;
    return pnorm(padd(s->cam_f, padd(pscl(s->cam_r, x), pscl(s->cam_u, y))));
}

/* Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n) */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(PL_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = -z; x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* length of the chord of [-eu, eu] x [-ev, ev] through (a, b) along (cos al, sin al) */
double or_planes_chord(double eu, double ev, double a, double b, double al)
{
    const double ca = cos(al), sa = sin(al);
    double lo = -1e300, hi = 1e300;
    if (fabs(ca) > 1e-300) {
        double t0 = (-eu - a) / ca, t1 = (eu - a) / ca;
        if (t0 > t1) { const double t = t0; t0 = t1; t1 = t; }
        lo = t0 > lo ? t0 : lo; hi = t1 < hi ? t1 : hi;
    } else if (a < -eu || a > eu) return 0.0;
    if (fabs(sa) > 1e-300) {
        double t0 = (-ev - b) / sa, t1 = (ev - b) / sa;
        if (t0 > t1) { const double t = t0; t0 = t1; t1 = t; }
        lo = t0 > lo ? t0 : lo; hi = t1 < hi ? t1 : hi;
    } else if (b < -ev || b > ev) return 0.0;
    return hi > lo ? hi - lo : 0.0;
}

static int cmp_d(const void *p, const void *q)
{
    const double a = *(const double *)p, b = *(const double *)q;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* J = int_0^pi len(alpha; a, b) |mu cos(alpha) + mv sin(alpha)| dalpha, by Gauss-Legendre on the
 * pieces between the angles where the integrand is not smooth: the directions from (a, b) to the
 * four corners (the chord's limiting sides change there) and the zero of the cosine factor */
double or_planes_J(double eu, double ev, double a, double b, double mu, double mv)
{
    double br[8];
    int nb = 0;
    br[nb++] = 0.0;
    br[nb++] = PL_PI;
    const double cx[4] = {-eu, eu, eu, -eu}, cy[4] = {-ev, -ev, ev, ev};
    for (int k = 0; k < 4; ++k) {
        double t = atan2(cy[k] - b, cx[k] - a);
        t = fmod(t + 2.0 * PL_PI, PL_PI);
        br[nb++] = t;
    }
    if (mu != 0.0 || mv != 0.0) br[nb++] = fmod(atan2(-mu, mv) + 2.0 * PL_PI, PL_PI);
    qsort(br, (size_t)nb, sizeof(double), cmp_d);
    enum { NG = 24 };
    double gx[NG], gw[NG];
    gauss_legendre(NG, gx, gw);
    double J = 0.0;
    for (int i = 0; i + 1 < nb; ++i) {
        const double lo = br[i], hi = br[i + 1];
        if (hi - lo < 1e-15) continue;
        const double h = 0.5 * (hi - lo), m = 0.5 * (hi + lo);
        for (int k = 0; k < NG; ++k) {
            const double al = m + h * gx[k];
            J += h * gw[k] * or_planes_chord(eu, ev, a, b, al) * fabs(mu * cos(al) + mv * sin(al));
        }
    }
    return J;
}

/* the single-scattered radiance (per unit Le) along the ray o + t d by quadrature: t on
 * [0, t_max] in `pieces` Gauss-Legendre pieces of nt nodes, y on the light in 4 x 4 sub-rectangles
 * of ny x ny nodes each */
static double ss_quadrature(const plane_scene *s, pv3 o, pv3 d, int nt, int ny)
{
    enum { PIECES = 8, SUB = 4 };
    double *tx = (double *)malloc(sizeof(double) * (size_t)(2 * (nt > ny ? nt : ny)));
    double *tw = tx + (nt > ny ? nt : ny);
    double *yx = (double *)malloc(sizeof(double) * (size_t)(2 * ny));
    double *yw = yx + ny;
    gauss_legendre(nt, tx, tw);
    gauss_legendre(ny, yx, yw);
    double L = 0.0;
    for (int p = 0; p < PIECES; ++p) {
        const double t0 = s->tmax * p / PIECES, t1 = s->tmax * (p + 1) / PIECES;
        for (int i = 0; i < nt; ++i) {
            const double t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * tx[i];
            const double wt = 0.5 * (t1 - t0) * tw[i];
            const pv3 x = padd(o, pscl(d, t));
            double inner = 0.0;
            for (int su = 0; su < SUB; ++su)
                for (int sv = 0; sv < SUB; ++sv) {
                    const double a0 = -s->eu + 2.0 * s->eu * su / SUB, a1 = a0 + 2.0 * s->eu / SUB;
                    const double b0 = -s->ev + 2.0 * s->ev * sv / SUB, b1 = b0 + 2.0 * s->ev / SUB;
                    for (int j = 0; j < ny; ++j)
                        for (int k = 0; k < ny; ++k) {
                            const double a = 0.5 * (a0 + a1) + 0.5 * (a1 - a0) * yx[j];
                            const double b = 0.5 * (b0 + b1) + 0.5 * (b1 - b0) * yx[k];
                            const double wy = 0.25 * (a1 - a0) * (b1 - b0) * yw[j] * yw[k];
                            const pv3 y = padd(s->c, padd(pscl(s->U, a), pscl(s->V, b)));
                            const pv3 r = psub(x, y);
                            const double R2 = pdot(r, r), R = sqrt(R2);
                            const double ct = pdot(r, s->N) / R;
                            if (ct <= 0.0) continue;
                            inner += wy * ct / R2 * exp(-s->st * R);
                        }
                }
            L += wt * exp(-s->st * t) * s->ss / (4.0 * PL_PI) * inner;
        }
    }
    free(tx);
    free(yx);
    return L;
}

/* per-pixel reference image [H][W][3]: the single-scattered radiance along each pixel's centre ray */
void or_planes_reference(const double *scene, int W, int H, int nt, int ny, double *img)
{
    plane_scene s;
    unpack(scene, &s);
    for (int py = 0; py < H; ++py)
        for (int px = 0; px < W; ++px) {
            const double L = ss_quadrature(&s, s.cam_p, pixel_dir(&s, W, H, px, py), nt, ny);
            for (int k = 0; k < 3; ++k) img[3 * ((size_t)py * W + px) + k] = L * s.le[k];
        }
}

/* the oracle's own random numbers: splitmix64 (Steele, Lea and Flood 2014) */
static uint64_t sm64(uint64_t *st)
{
    uint64_t z = (*st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double u01(uint64_t *st) { return (double)(sm64(st) >> 11) * (1.0 / 9007199254740992.0); }

typedef struct { pv3 y0, u, w; double smin, smax; } plane_t;

static void sample_plane(const plane_scene *s, uint64_t *rs, plane_t *P)
{
    const double a = (2.0 * u01(rs) - 1.0) * s->eu, b = (2.0 * u01(rs) - 1.0) * s->ev;
    const double al = PL_PI * u01(rs);
    const double r1 = u01(rs), r2 = u01(rs);
    /* cosine hemisphere about N */
    const double phi = 2.0 * PL_PI * r1, sr = sqrt(r2);
    const double wz = sqrt(1.0 - r2);
    P->y0 = padd(s->c, padd(pscl(s->U, a), pscl(s->V, b)));
    P->w = padd(pscl(s->N, wz), padd(pscl(s->U, sr * cos(phi)), pscl(s->V, sr * sin(phi))));
    P->u = padd(pscl(s->U, cos(al)), pscl(s->V, sin(al)));
    /* the chord's parameter range through (a, b) */
    const double ca = cos(al), sa = sin(al);
    double lo = -1e300, hi = 1e300;
    if (fabs(ca) > 1e-300) {
        double t0 = (-s->eu - a) / ca, t1 = (s->eu - a) / ca;
        if (t0 > t1) { const double t = t0; t0 = t1; t1 = t; }
        lo = t0 > lo ? t0 : lo; hi = t1 < hi ? t1 : hi;
    }
    if (fabs(sa) > 1e-300) {
        double t0 = (-s->ev - b) / sa, t1 = (s->ev - b) / sa;
        if (t0 > t1) { const double t = t0; t0 = t1; t1 = t; }
        lo = t0 > lo ? t0 : lo; hi = t1 < hi ? t1 : hi;
    }
    P->smin = lo; P->smax = hi;
}

/* one plane's CMIS estimate for the eye ray (o, d): 0 when the ray misses the plane */
static double plane_hit(const plane_scene *s, const plane_t *P, pv3 o, pv3 d)
{
    const pv3 n = pcross(P->u, P->w);
    const double den = pdot(d, n);
    if (den == 0.0) return 0.0;
    const double t = pdot(psub(P->y0, o), n) / den;
    if (!(t > 0.0 && t <= s->tmax)) return 0.0;
    const pv3 q = psub(padd(o, pscl(d, t)), P->y0);
    const double uw = pdot(P->u, P->w), det = 1.0 - uw * uw;
    const double qu = pdot(q, P->u), qw = pdot(q, P->w);
    const double sp = (qu - uw * qw) / det, lam = (qw - uw * qu) / det;
    if (!(lam > 0.0) || sp < P->smin || sp > P->smax) return 0.0;
    const pv3 y = padd(P->y0, pscl(P->u, sp));
    const pv3 m = pcross(P->w, d);
    const pv3 yc = psub(y, s->c);
    const double J = or_planes_J(s->eu, s->ev, pdot(yc, s->U), pdot(yc, s->V), pdot(m, s->U), pdot(m, s->V));
    if (!(J > 0.0)) return 0.0;
    return s->ss * exp(-s->st * (t + lam)) * PL_PI * s->area / (4.0 * J);
}

/* n_iter iterations of the photon-plane estimator with the exact J: per iteration M planes, every
 * pixel's centre ray gathers every plane it meets, value = (1/M) sum of the CMIS estimates x Le.
 * sum / sumsq [H][W][3] receive the per-iteration values and their squares. */
void or_planes_render(const double *scene, int W, int H, int M, int n_iter, uint64_t seed, double *sum,
                      double *sumsq)
{
    plane_scene s;
    unpack(scene, &s);
    plane_t *P = (plane_t *)malloc(sizeof(plane_t) * (size_t)M);
    memset(sum, 0, sizeof(double) * 3 * (size_t)W * H);
    memset(sumsq, 0, sizeof(double) * 3 * (size_t)W * H);
    for (int it = 0; it < n_iter; ++it) {
        /* the iteration's stream starts at a hashed state: consecutive start states would give
         * streams that are shifts of one another */
        uint64_t h = (uint64_t)it + 1u;
        uint64_t rs = sm64(&h) ^ seed;
        rs = sm64(&rs);
        for (int k = 0; k < M; ++k) sample_plane(&s, &rs, &P[k]);
        for (int py = 0; py < H; ++py)
            for (int px = 0; px < W; ++px) {
                const pv3 d = pixel_dir(&s, W, H, px, py);
                double v = 0.0;
                for (int k = 0; k < M; ++k) v += plane_hit(&s, &P[k], s.cam_p, d);
                v /= M;
                for (int c = 0; c < 3; ++c) {
                    const double x = v * s.le[c];
                    sum[3 * ((size_t)py * W + px) + c] += x;
                    sumsq[3 * ((size_t)py * W + px) + c] += x * x;
                }
            }
    }
    free(P);
}
