/*
 * pbh_oracle.c -- plain CPU FP64 oracle for the P3T distant-force path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path
 * (libpbh) never calls into it and shares no code with it.
 *
 * Built with -O2 -ffp-contract=off so that every double expression below is
 * evaluated as written (IEEE round-to-nearest, no fused multiply-add).
 *
 * What it computes (Arnold, Baumgardt & Wang 2021, Section 2.1):
 *   The P3T split divides gravity between the neighbour (irregular) force
 *   F_I = sum_j m_j K(r_ij) r_ij / r_ij^3 and the regular force
 *   F_R = (total) - F_I, with the changeover function K of eq. (duncan):
 *   K = 1 - g(x), g(x) = 35x^4 - 84x^5 + 70x^6 - 20x^7 for 0 <= x < 1,
 *   x = (r - r_in)/(r_cut - r_in), and K = 1 (0) below r_in (above r_cut).
 *   Hence the regular acceleration is sum_j m_j W(s) d_ij / s^3 with
 *   W = 1 - K and d_ij = x_j - x_i (attractive gravity, G = 1).
 *   Softening enters as s^2 = r^2 + eps^2 (eps = 0 recovers the paper).
 *   The regular potential Phi_R is the one whose radial derivative is
 *   W(s)/s^2 and which equals -1/s beyond r_cut; below r_in it is constant.
 *   The neighbour set of i is { j != i : r_ij^2 < r_cut^2 } (unsoftened).
 *   In this file r_cut is called r_out.
 *
 * Functions:
 *   orc_W, orc_phiR           the changeover weight and regular potential
 *   orc_direct                O(N^2) direct sum (all or a subset of targets)
 *   orc_full_direct           plain softened gravity (no split)
 *   orc_irregular             O(N^2) irregular force F_I, its time
 *                             derivative and the irregular potential
 *   orc_core                  core quantities from the 6 nearest neighbours
 *                             of a particle sample, by brute force
 *   orc_irr_derivs            its second and third time derivatives
 *   orc_hermite, orc_p3t      Hermite integration of F_I with block time
 *                             steps over one regular step, and the P3T loop
 *   orc_nbr_brute/orc_nbr_cells neighbour sets, brute force and cell list
 *   orc_keys                  Morton keys of the octree
 *   orc_tree                  Barnes-Hut octree walk with the same tree,
 *                             group and opening rules as the GPU path
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Changeover weight W = 1 - K (Section 2.1, eq. duncan)                     */
/* ------------------------------------------------------------------------ */

static double g_poly(double x)
{
    /* g(x) = 35 x^4 - 84 x^5 + 70 x^6 - 20 x^7 */
    double x2 = x * x;
    double x4 = x2 * x2;
    double x5 = x4 * x;
    double x6 = x5 * x;
    double x7 = x6 * x;
    return 35.0 * x4 - 84.0 * x5 + 70.0 * x6 - 20.0 * x7;
}

double orc_W(double s, double r_in, double r_out)
{
    if (s >= r_out) return 1.0;  /* wholly regular beyond the outer radius */
    if (s < r_in) return 0.0;    /* wholly irregular inside the inner radius */
    return g_poly((s - r_in) / (r_out - r_in));
}

/* ------------------------------------------------------------------------ */
/* Regular potential Phi_R(s), dPhi_R/ds = W(s)/s^2, Phi_R = -1/s past r_out */
/*                                                                          */
/* With D = r_out - r_in, a = r_in/D and t = s/D, g(t - a) = sum_k d_k t^k.  */
/* Integrating g(t-a)/t^2 term by term gives                                */
/*   G(t) = -d0/t + d1 ln t + sum_{k=2..7} d_k t^(k-1)/(k-1)                */
/* and Phi_R(s) = -1/r_out - (G(a+1) - G(s/D)) / D on [r_in, r_out).        */
/* ------------------------------------------------------------------------ */

typedef struct {
    double r_in, r_out, D, a;
    double d[8];
    double G1;      /* G(a + 1) */
    double inner;   /* Phi_R(r_in) */
    int mode;       /* 0: plain gravity (r_out = 0), 1: step (D = 0), 2: smooth */
} phir_t;

static double binom(int n, int k)
{
    double b = 1.0;
    for (int i = 1; i <= k; ++i) b = b * (double)(n - k + i) / (double)i;
    return b;
}

static double G_of_t(const phir_t* p, double t)
{
    double G = 0.0;
    if (p->d[0] != 0.0) G += -p->d[0] / t;
    if (p->d[1] != 0.0) G += p->d[1] * log(t);
    for (int k = 2; k <= 7; ++k) G += p->d[k] * pow(t, (double)(k - 1)) / (double)(k - 1);
    return G;
}

static double phir_eval(const phir_t* p, double s)
{
    if (p->mode == 0) return -1.0 / s;
    if (s >= p->r_out) return -1.0 / s;
    if (p->mode == 1) return -1.0 / p->r_out;  /* W = 0 everywhere below r_out */
    if (s < p->r_in) return p->inner;
    return -1.0 / p->r_out - (p->G1 - G_of_t(p, s / p->D)) / p->D;
}

static void phir_init(phir_t* p, double r_in, double r_out)
{
    static const double c[8] = {0, 0, 0, 0, 35.0, -84.0, 70.0, -20.0};
    memset(p, 0, sizeof(*p));
    p->r_in = r_in;
    p->r_out = r_out;
    p->D = r_out - r_in;
    if (r_out == 0.0) { p->mode = 0; return; }
    if (p->D == 0.0) { p->mode = 1; p->inner = -1.0 / r_out; return; }
    p->mode = 2;
    p->a = r_in / p->D;
    /* expand g(t - a) = sum_p c_p (t - a)^p = sum_k d_k t^k */
    for (int k = 0; k <= 7; ++k) {
        double dk = 0.0;
        for (int q = 4; q <= 7; ++q) {
            if (k > q) continue;
            double term = c[q] * binom(q, k);
            for (int e = 0; e < q - k; ++e) term = term * (-p->a);
            dk += term;
        }
        p->d[k] = dk;
    }
    p->G1 = G_of_t(p, p->a + 1.0);
    /* s = r_in takes the smooth branch; for r_in = 0 (a = 0) d0 = d1 = 0 and
       G is a polynomial, so Phi_R(0) is finite */
    p->inner = phir_eval(p, r_in);
}

double orc_phiR(double s, double r_in, double r_out)
{
    phir_t p;
    phir_init(&p, r_in, r_out);
    return phir_eval(&p, s);
}

/* Coefficients d_0..d_7 of g(t - a) and G(a+1), for tests. */
void orc_phiR_coeffs(double r_in, double r_out, double* d8, double* G1)
{
    phir_t p;
    phir_init(&p, r_in, r_out);
    for (int k = 0; k < 8; ++k) d8[k] = p.d[k];
    *G1 = p.G1;
}

/* ------------------------------------------------------------------------ */
/* O(N^2) direct sum of the regular force and potential                      */
/* ------------------------------------------------------------------------ */

/* One source j acting on target i (j != i): regular acceleration and potential. */
static void pair_regular(const phir_t* p, double eps2,
                         double xi, double yi, double zi,
                         double xj, double yj, double zj, double mj,
                         double* ax, double* ay, double* az, double* pot)
{
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    double r2 = dx * dx + dy * dy + dz * dz;
    double s2 = r2 + eps2;
    double s = sqrt(s2);
    double w = orc_W(s, p->r_in, p->r_out);
    if (p->mode == 0) w = 1.0;
    if (w != 0.0) {
        double f = mj * w / (s2 * s);
        *ax += f * dx;
        *ay += f * dy;
        *az += f * dz;
    }
    *pot += mj * phir_eval(p, s);
}

/*
 * Regular acceleration and potential by direct summation over all sources.
 * pos: [n][3], mass: [n]. If tgt != NULL only the n_tgt listed targets are
 * computed and acc/pot are [n_tgt][3] / [n_tgt]; otherwise all n.
 */
void orc_direct(int64_t n, const double* pos, const double* mass,
                double r_in, double r_out, double eps,
                int64_t n_tgt, const int64_t* tgt, double* acc, double* pot)
{
    phir_t p;
    phir_init(&p, r_in, r_out);
    double eps2 = eps * eps;
    int64_t nt = tgt ? n_tgt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tgt ? tgt[t] : t;
        double ax = 0, ay = 0, az = 0, ph = 0;
        double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            pair_regular(&p, eps2, xi, yi, zi, pos[3 * j], pos[3 * j + 1], pos[3 * j + 2],
                         mass[j], &ax, &ay, &az, &ph);
        }
        acc[3 * t] = ax;
        acc[3 * t + 1] = ay;
        acc[3 * t + 2] = az;
        pot[t] = ph;
    }
}

/* Plain softened gravity (the whole force, no changeover), for split checks. */
void orc_full_direct(int64_t n, const double* pos, const double* mass, double eps,
                     double* acc, double* pot)
{
    double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double ax = 0, ay = 0, az = 0, ph = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = pos[3 * j] - pos[3 * i];
            double dy = pos[3 * j + 1] - pos[3 * i + 1];
            double dz = pos[3 * j + 2] - pos[3 * i + 2];
            double s2 = dx * dx + dy * dy + dz * dz + eps2;
            double s = sqrt(s2);
            double f = mass[j] / (s2 * s);
            ax += f * dx;
            ay += f * dy;
            az += f * dz;
            ph += -mass[j] / s;
        }
        acc[3 * i] = ax;
        acc[3 * i + 1] = ay;
        acc[3 * i + 2] = az;
        pot[i] = ph;
    }
}

/* ------------------------------------------------------------------------ */
/* Irregular force, its time derivative and potential                        */
/* (Section 2.1: eq. fi, eq. fidot, eq. duncan, eq. duncan2)                 */
/*                                                                          */
/* With d = x_j - x_i, u = v_j - v_i and s^2 = |d|^2 + eps^2:                */
/*   F_I      = sum_{j != i} m_j K(s) d / s^3                                */
/*   dF_I/dt  = sum_{j != i} m_j { K(s) [u / s^3 - 3 (d.u) d / s^5]          */
/*                                 + (dK/dt) d / s^3 }                       */
/*   dK/dt    = -g'(x) (d.u) / (s (r_out - r_in)) for r_in <= s < r_out,     */
/*              0 elsewhere; g'(x) = 140 x^3 (1 - x)^3                       */
/*   Phi_I(s) = -1/s - Phi_R(s) (so Phi_I + Phi_R is plain softened gravity) */
/* The jerk is the time derivative of eq. fi taken term by term along the    */
/* particles' velocities (ds/dt = d.u / s). As printed, eq. fidot drops m_j  */
/* and K from its second term, and eq. duncan2 gives dK/dt the sign of       */
/* +g'(x) although K = 1 - g(x) decreases with x; this follows the           */
/* derivative. A step changeover (r_in = r_out) has K = 1 below r_out and    */
/* dK/dt = 0 (the jump carries no smooth derivative); r_out = 0 gives K = 0. */
/* ------------------------------------------------------------------------ */

/* K(s) and g'(x)/(r_out - r_in) for one pair (the latter 0 off the band). */
static void k_and_slope(const phir_t* p, double s, double* K, double* slope)
{
    *slope = 0.0;
    if (p->mode == 0 || s >= p->r_out) { *K = 0.0; return; }
    if (p->mode == 1 || s < p->r_in) { *K = 1.0; return; }
    double x = (s - p->r_in) / p->D;
    double omx = 1.0 - x;
    *K = 1.0 - g_poly(x);
    *slope = 140.0 * x * x * x * omx * omx * omx / p->D;
}

/*
 * pos, vel: [n][3]; mass: [n]. If tgt != NULL only the n_tgt listed targets
 * are computed and the outputs are [n_tgt][3] / [n_tgt]; otherwise all n.
 * jerk, pot and scale may be NULL. scale [n_tgt][3], if given, receives
 * per-target magnitude sums over the pairs with s < r_out, for error bounds:
 *   sum m_j / s^2,  sum m_j |u| (4/s^3 + max g' / (s^2 (r_out - r_in))),
 *   sum m_j (1/s + |Phi_R(s)|)
 * (max g' = 140/64; the second sum drops that term for a step changeover).
 */
void orc_irregular(int64_t n, const double* pos, const double* vel, const double* mass,
                   double r_in, double r_out, double eps,
                   int64_t n_tgt, const int64_t* tgt,
                   double* acc, double* jerk, double* pot, double* scale)
{
    phir_t p;
    phir_init(&p, r_in, r_out);
    double eps2 = eps * eps;
    int64_t nt = tgt ? n_tgt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tgt ? tgt[t] : t;
        double a[3] = {0, 0, 0}, jk[3] = {0, 0, 0}, ph = 0;
        double sa = 0, sj = 0, sp = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3], u[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = pos[3 * j + k] - pos[3 * i + k];
                u[k] = vel[3 * j + k] - vel[3 * i + k];
            }
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double s2 = r2 + eps2;
            double s = sqrt(s2);
            double K, slope;
            k_and_slope(&p, s, &K, &slope);
            if (p.mode == 0 || s >= p.r_out) continue;   /* K = 0 and Phi_I = 0 */
            double du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
            double s3 = s2 * s;
            double Kdot = -slope * du / s;
            for (int k = 0; k < 3; ++k) {
                a[k] += mass[j] * K * d[k] / s3;
                jk[k] += mass[j] * (K * (u[k] / s3 - 3.0 * du * d[k] / (s3 * s2)) + Kdot * d[k] / s3);
            }
            double phiR = phir_eval(&p, s);
            ph += mass[j] * (-1.0 / s - phiR);
            double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            sa += mass[j] / s2;
            sj += mass[j] * un * (4.0 / s3 + (p.mode == 2 ? (140.0 / 64.0) / (s2 * p.D) : 0.0));
            sp += mass[j] * (1.0 / s + fabs(phiR));
        }
        for (int k = 0; k < 3; ++k) {
            acc[3 * t + k] = a[k];
            if (jerk) jerk[3 * t + k] = jk[k];
        }
        if (pot) pot[t] = ph;
        if (scale) {
            scale[3 * t] = sa;
            scale[3 * t + 1] = sj;
            scale[3 * t + 2] = sp;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Second and third time derivatives of the irregular force                  */
/* (Section 2.1: the text after eq. dt -- the higher derivatives are         */
/* computed, so that the fourth-order criterion eq. dt sets the first step)  */
/*                                                                            */
/* Along a motion on which every particle has position x, velocity v,        */
/* acceleration acc and its time derivative jrk, each pair term of eq. fi is */
/* m_j h(s) d with h(s) = K(s) / s^3, d = x_j - x_i, d' = u = v_j - v_i,      */
/* d'' = w = acc_j - acc_i, d''' = z = jrk_j - jrk_i. With                    */
/*   s' = d.u / s,  s'' = (u.u + d.w - s'^2) / s,                            */
/*   s''' = (3 u.w + d.z - 3 s' s'') / s,                                    */
/* and h_s, h_ss, h_sss the derivatives of K s^-3 with respect to s,          */
/*   h'   = h_s s',   h'' = h_ss s'^2 + h_s s'',                             */
/*   h''' = h_sss s'^3 + 3 h_ss s' s'' + h_s s''',                            */
/*   F^(2) = sum m_j (h'' d + 2 h' u + h w),                                  */
/*   F^(3) = sum m_j (h''' d + 3 h'' u + 3 h' w + h z).                       */
/* In the band, with x = (s - r_in)/D: dK/ds = -g'(x)/D,                      */
/* d2K/ds2 = -g''(x)/D^2, d3K/ds3 = -g'''(x)/D^3, g' = 140 x^3 (1-x)^3,       */
/* g'' = 420 x^2 (1-x)^2 (1-2x), g''' = 840 x (1-x) (1 - 5x + 5x^2); all      */
/* three vanish at x = 0 and x = 1, so K is three times continuously          */
/* differentiable across both radii. Off the band K is constant.              */
/* ------------------------------------------------------------------------ */

/* K(s) and its first three derivatives with respect to s, Kd[0..3]. */
static void k_derivs(const phir_t* p, double s, double Kd[4])
{
    Kd[1] = Kd[2] = Kd[3] = 0.0;
    if (p->mode == 0 || s >= p->r_out) { Kd[0] = 0.0; return; }
    if (p->mode == 1 || s < p->r_in) { Kd[0] = 1.0; return; }
    double x = (s - p->r_in) / p->D;
    double omx = 1.0 - x;
    Kd[0] = 1.0 - g_poly(x);
    Kd[1] = -140.0 * x * x * x * omx * omx * omx / p->D;
    Kd[2] = -420.0 * x * x * omx * omx * (1.0 - 2.0 * x) / (p->D * p->D);
    Kd[3] = -840.0 * x * omx * (1.0 - 5.0 * x + 5.0 * x * x) / (p->D * p->D * p->D);
}

/* F^(2), F^(3) at particle i from every j != i with s < r_out */
static void irr_d23_at(const phir_t* p, double eps2, int64_t n, const double* xs, const double* vs,
                       const double* as, const double* js, const double* mass, int64_t i,
                       double* f2, double* f3)
{
    for (int k = 0; k < 3; ++k) f2[k] = f3[k] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double d[3], u[3], w[3], z[3];
        for (int k = 0; k < 3; ++k) {
            d[k] = xs[3 * j + k] - xs[3 * i + k];
            u[k] = vs[3 * j + k] - vs[3 * i + k];
            w[k] = as[3 * j + k] - as[3 * i + k];
            z[k] = js[3 * j + k] - js[3 * i + k];
        }
        double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
        double s = sqrt(s2);
        if (p->mode == 0 || s >= p->r_out) continue;
        double Kd[4];
        k_derivs(p, s, Kd);
        double du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
        double uw = u[0] * w[0] + u[1] * w[1] + u[2] * w[2];
        double dz = d[0] * z[0] + d[1] * z[1] + d[2] * z[2];
        double sd1 = du / s;
        double sd2 = (uu + dw - sd1 * sd1) / s;
        double sd3 = (3.0 * uw + dz - 3.0 * sd1 * sd2) / s;
        double s3 = s2 * s, s4 = s2 * s2, s5 = s4 * s, s6 = s4 * s2;
        double h = Kd[0] / s3;
        double hs = Kd[1] / s3 - 3.0 * Kd[0] / s4;
        double hss = Kd[2] / s3 - 6.0 * Kd[1] / s4 + 12.0 * Kd[0] / s5;
        double hsss = Kd[3] / s3 - 9.0 * Kd[2] / s4 + 36.0 * Kd[1] / s5 - 60.0 * Kd[0] / s6;
        double h1 = hs * sd1;
        double h2 = hss * sd1 * sd1 + hs * sd2;
        double h3 = hsss * sd1 * sd1 * sd1 + 3.0 * hss * sd1 * sd2 + hs * sd3;
        for (int k = 0; k < 3; ++k) {
            f2[k] += mass[j] * (h2 * d[k] + 2.0 * h1 * u[k] + h * w[k]);
            f3[k] += mass[j] * (h3 * d[k] + 3.0 * h2 * u[k] + 3.0 * h1 * w[k] + h * z[k]);
        }
    }
}

/*
 * F^(2), F^(3) of F_I [n_t][3] for all particles or the n_tgt listed targets,
 * along the motion given by pos, vel, acc, jrk [n][3].
 */
void orc_irr_derivs(int64_t n, const double* pos, const double* vel, const double* acc,
                    const double* jrk, const double* mass, double r_in, double r_out, double eps,
                    int64_t n_tgt, const int64_t* tgt, double* f2, double* f3)
{
    phir_t p;
    phir_init(&p, r_in, r_out);
    int64_t nt = tgt ? n_tgt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tgt ? tgt[t] : t;
        irr_d23_at(&p, eps * eps, n, pos, vel, acc, jrk, mass, i, f2 + 3 * t, f3 + 3 * t);
    }
}

/* ------------------------------------------------------------------------ */
/* Core quantities: the sampled core algorithm of Section 3.2 with the       */
/* density estimator of Casertano & Hut (1985), and the regularisation       */
/* parameters R_min, dT_min of Section 2.5                                   */
/*                                                                            */
/* For each sampled particle i: its 6 nearest neighbours among all n (j != i, */
/* unsoftened ((dx*dx + dy*dy) + dz*dz), ties to the lower index), and        */
/*   rho_i = (sum of the masses of the 5 nearest) / ((4 pi / 3) r_6^3)        */
/* the order-6 estimator with masses. Over the sample:                        */
/*   x_d = sum rho x / sum rho          density centre                        */
/*   r_c = sqrt(sum rho^2 |x - x_d|^2 / sum rho^2)   core radius              */
/*   rho_core = sum rho^2 / sum rho                  core density             */
/* Over all particles: N_core = #{ |x - x_d|^2 < r_c^2 }, and the half-mass   */
/* radius r_h = the smallest |x_k - x_d| whose sphere (inclusive) holds at    */
/* least half the total mass. R_min = 4 r_h / (n rho_core^(1/3)) and          */
/* dT_min = 0.01 sqrt(eta / 0.02) sqrt(R_min^3).                              */
/* ------------------------------------------------------------------------ */

/* 6 nearest neighbours of particle i by brute force; d2[6] ascending, idx[6]. */
static void knn6(int64_t n, const double* pos, int64_t i, double* d2, int64_t* idx)
{
    int cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = pos[3 * j] - pos[3 * i];
        double dy = pos[3 * j + 1] - pos[3 * i + 1];
        double dz = pos[3 * j + 2] - pos[3 * i + 2];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (cnt == 6 && !(r2 < d2[5])) continue;   /* equal distance: the lower index stays */
        int k = cnt < 6 ? cnt++ : 5;
        while (k > 0 && r2 < d2[k - 1]) {
            d2[k] = d2[k - 1];
            idx[k] = idx[k - 1];
            --k;
        }
        d2[k] = r2;
        idx[k] = j;
    }
}

static int cmp_dist(const void* a, const void* b)
{
    const double* x = (const double*)a;
    const double* y = (const double*)b;
    if (x[0] < y[0]) return -1;
    if (x[0] > y[0]) return 1;
    return (x[1] < y[1]) ? -1 : (x[1] > y[1]);
}

/*
 * pos [n][3], mass [n], n >= 7; sample [n_s] distinct particle indices.
 * rho [n_s] receives the per-sample densities (may be NULL); out[9] =
 * x_d (3), rho_core, r_c, N_core, r_h, R_min, dT_min.
 */
void orc_core(int64_t n, const double* pos, const double* mass, int64_t n_s, const int64_t* sample,
              double eta, double* rho, double* out)
{
    double* r = (double*)malloc(sizeof(double) * (size_t)n_s);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < n_s; ++s) {
        double d2[6];
        int64_t idx[6];
        knn6(n, pos, sample[s], d2, idx);
        double m5 = 0.0;
        for (int k = 0; k < 5; ++k) m5 += mass[idx[k]];
        double r6 = sqrt(d2[5]);
        r[s] = m5 / (4.0 / 3.0 * M_PI * (d2[5] * r6));
    }
    double sr = 0.0, srx[3] = {0, 0, 0};
    for (int64_t s = 0; s < n_s; ++s) {
        sr += r[s];
        for (int d = 0; d < 3; ++d) srx[d] += r[s] * pos[3 * sample[s] + d];
    }
    double xd[3];
    for (int d = 0; d < 3; ++d) xd[d] = srx[d] / sr;
    double sr2 = 0.0, sr2d2 = 0.0;
    for (int64_t s = 0; s < n_s; ++s) {
        double dd = 0.0;
        for (int d = 0; d < 3; ++d) {
            double v = pos[3 * sample[s] + d] - xd[d];
            dd += v * v;
        }
        sr2 += r[s] * r[s];
        sr2d2 += r[s] * r[s] * dd;
    }
    double rc = sqrt(sr2d2 / sr2);
    double rho_core = sr2 / sr;
    /* core membership and half-mass radius over all particles */
    double* dm = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    int64_t ncore = 0;
    double mtot = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double dd = 0.0;
        for (int d = 0; d < 3; ++d) {
            double v = pos[3 * i + d] - xd[d];
            dd += v * v;
        }
        if (dd < rc * rc) ++ncore;
        dm[2 * i] = dd;
        dm[2 * i + 1] = (double)i;
        mtot += mass[i];
    }
    qsort(dm, (size_t)n, 2 * sizeof(double), cmp_dist);
    double cum = 0.0, rh = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        cum += mass[(int64_t)dm[2 * k + 1]];
        if (cum >= 0.5 * mtot) {
            rh = sqrt(dm[2 * k]);
            break;
        }
    }
    double rmin = 4.0 * rh / ((double)n * cbrt(rho_core));
    double dtmin = 0.01 * sqrt(eta / 0.02) * sqrt(rmin * rmin * rmin);
    for (int d = 0; d < 3; ++d) out[d] = xd[d];
    out[3] = rho_core;
    out[4] = rc;
    out[5] = (double)ncore;
    out[6] = rh;
    out[7] = rmin;
    out[8] = dtmin;
    if (rho)
        for (int64_t s = 0; s < n_s; ++s) rho[s] = r[s];
    free(dm);
    free(r);
}

/* 6 nearest neighbours of the listed particles (for tests): d2 [n_s][6], idx [n_s][6]. */
void orc_knn6(int64_t n, const double* pos, int64_t n_s, const int64_t* sample, double* d2,
              int64_t* idx)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < n_s; ++s) knn6(n, pos, sample[s], d2 + 6 * s, idx + 6 * s);
}

/* ------------------------------------------------------------------------ */
/* Hermite integration of the irregular force with block time steps, and the */
/* P3T loop (Section 2.2: the integration algorithm and eq. p3t-jpred-x,      */
/* p3t-jpred-dx; eq. dt with eta; eq. dtmax: dt_max = dt_reg / 4)             */
/*                                                                            */
/* Over one regular step of length T every particle carries x, v, a = F_I,    */
/* j = dF_I/dt, its time tau_i and block step dt_i = dt_max / 2^k.            */
/*   start: tau = 0; a and j from the state (after the kick); the second and  */
/*          third derivatives a^(2), a^(3) of F_I along the motion under F_I  */
/*          (relative accelerations a_j - a_i and jerks j_j - j_i, computed   */
/*          by the derivative formulas above); dt from eq. dt with a^(0) =    */
/*          a + F_R, a^(1) = j, a^(2), a^(3), and dt_max where the           */
/*          denominator vanishes (an empty list: no irregular force).         */
/*   block: tau' = min(tau_i + dt_i); the active particles have              */
/*          tau_i + dt_i = tau'. All particles are predicted to tau' (d =     */
/*          tau' - tau_i):  x_p = x + d v + d^2/2 a + d^3/6 j,               */
/*          v_p = v + d a + d^2/2 j  (no regular force: the kicks carry it).  */
/*          Active particles get a1, j1 at the predicted state and the        */
/*          4th-order Hermite correction (d = dt_i, da = a - a1):            */
/*            a2 = (-6 da - d (4 j + 2 j1)) / d^2                             */
/*            a3 = (12 da + 6 d (j + j1)) / d^3                               */
/*            x = x_p + d^4/24 a2 + d^5/120 a3,  v = v_p + d^3/6 a2 + d^4/24 a3 */
/*          new step: eq. dt with a^(0) = a1 + F_R, a^(1) = j1,               */
/*          a^(2) = a2 + d a3, a^(3) = a3, at most twice the old step and     */
/*          dt_max, rounded down to dt_max / 2^k and to a divisor of tau'.    */
/*   until every particle is at tau = T (steps divide T, so they all meet).   */
/* Readings: eq. dt, its first-step use with computed derivatives and the    */
/* P3T predictor are the paper's; steps are set afresh after every regular   */
/* kick (the new routine that applies the kick also determines new steps);  */
/* the corrector is the standard 4th-order Hermite one (Makino & Aarseth     */
/* 1992), which the paper keeps from NBODY6.                                 */
/* ------------------------------------------------------------------------ */

/* Times are counted in integer ticks of dt_max / 2^HERM_KMAX (a regular step
   is 4 * 2^HERM_KMAX ticks), so block times add exactly; a time length in
   FP64 is ticks * (T / 2^(HERM_KMAX + 2)). */
#define HERM_KMAX 40

static double hnorm(const double* v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* block step in ticks: dt_max / 2^k not above `want`, dividing tau */
static int64_t block_step(double want, double dtmax, int64_t tau)
{
    double d = dtmax;
    int k = 0;
    while (d > want && k < HERM_KMAX) { d *= 0.5; ++k; }
    int64_t t = (int64_t)1 << (HERM_KMAX - k);
    while (tau % t != 0) t >>= 1;
    return t;
}

/* F_I and its derivative at particle i from all others (the definition) */
static void irr_at(const phir_t* p, double eps2, int64_t n, const double* xs, const double* vs,
                   const double* mass, int64_t i, double* a, double* jk)
{
    for (int k = 0; k < 3; ++k) a[k] = jk[k] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double d[3], u[3];
        for (int k = 0; k < 3; ++k) {
            d[k] = xs[3 * j + k] - xs[3 * i + k];
            u[k] = vs[3 * j + k] - vs[3 * i + k];
        }
        double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
        double s = sqrt(s2);
        double K, slope;
        k_and_slope(p, s, &K, &slope);
        if (p->mode == 0 || s >= p->r_out) continue;
        double du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
        double s3 = s2 * s;
        double Kdot = -slope * du / s;
        for (int k = 0; k < 3; ++k) {
            a[k] += mass[j] * K * d[k] / s3;
            jk[k] += mass[j] * (K * (u[k] / s3 - 3.0 * du * d[k] / (s3 * s2)) + Kdot * d[k] / s3);
        }
    }
}

/*
 * Integrate F_I over one regular step T in place (x, v [n][3]). fr [n][3] is
 * the regular force for the step criterion (may be NULL). stats (optional,
 * int64[3]): block steps, particle steps, smallest k. want_out (optional,
 * [4n]): per particle the step eq. dt asked for at the start, the one it
 * asked for at the particle's last corrector step (before the doubling cap
 * and the rounding to a block step), the length of that last step and of the
 * step before it (0 when the last step was the first of the regular step).
 */
void orc_hermite(int64_t n, double* x, double* v, const double* mass, const double* fr,
                 double r_in, double r_out, double eps, double T, double eta, int64_t* stats,
                 double* want_out)
{
    phir_t p;
    phir_init(&p, r_in, r_out);
    const double eps2 = eps * eps, dtmax = T / 4.0;
    const double unit = T / (double)((int64_t)1 << (HERM_KMAX + 2));
    const int64_t tend = (int64_t)1 << (HERM_KMAX + 2);
    double* a = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* jk = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    int64_t* tau = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* dt = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    double* xp = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* vp = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* a1 = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* j1 = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    char* act = (char*)malloc((size_t)n);
    int64_t nblock = 0, nsteps = 0, kmin = 0;
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) irr_at(&p, eps2, n, x, v, mass, i, a + 3 * i, jk + 3 * i);
    /* first steps: eq. dt with a^(2), a^(3) from the derivative formulas
       (xp, vp hold them here; they are overwritten by the first prediction) */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) irr_d23_at(&p, eps2, n, x, v, a, jk, mass, i, xp + 3 * i, vp + 3 * i);
    for (int64_t i = 0; i < n; ++i) {
        double at[3];
        for (int k = 0; k < 3; ++k) at[k] = a[3 * i + k] + (fr ? fr[3 * i + k] : 0.0);
        double n0 = hnorm(at), n1 = hnorm(jk + 3 * i), n2 = hnorm(xp + 3 * i), n3 = hnorm(vp + 3 * i);
        double num = n0 * n2 + n1 * n1, den = n1 * n3 + n2 * n2;
        double want = den > 0.0 ? sqrt(eta * num / den) : dtmax;
        if (want_out) want_out[i] = want;
        tau[i] = 0;
        dt[i] = block_step(want, dtmax, 0);
    }
    for (;;) {
        int64_t tn = tau[0] + dt[0];
        for (int64_t i = 1; i < n; ++i)
            if (tau[i] + dt[i] < tn) tn = tau[i] + dt[i];
        for (int64_t i = 0; i < n; ++i) {
            double d = (double)(tn - tau[i]) * unit;
            double d2 = d * d, d3 = d2 * d;
            for (int k = 0; k < 3; ++k) {
                xp[3 * i + k] = x[3 * i + k] + d * v[3 * i + k] + 0.5 * d2 * a[3 * i + k] + d3 / 6.0 * jk[3 * i + k];
                vp[3 * i + k] = v[3 * i + k] + d * a[3 * i + k] + 0.5 * d2 * jk[3 * i + k];
            }
            act[i] = (tau[i] + dt[i] == tn);
        }
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i)
            if (act[i]) irr_at(&p, eps2, n, xp, vp, mass, i, a1 + 3 * i, j1 + 3 * i);
        for (int64_t i = 0; i < n; ++i) {
            if (!act[i]) continue;
            double d = (double)dt[i] * unit, d2 = d * d, d3 = d2 * d, d4 = d3 * d, d5 = d4 * d;
            double a2[3], a3[3], a2e[3], at[3];
            for (int k = 0; k < 3; ++k) {
                double da = a[3 * i + k] - a1[3 * i + k];
                a2[k] = (-6.0 * da - d * (4.0 * jk[3 * i + k] + 2.0 * j1[3 * i + k])) / d2;
                a3[k] = (12.0 * da + 6.0 * d * (jk[3 * i + k] + j1[3 * i + k])) / d3;
                x[3 * i + k] = xp[3 * i + k] + d4 / 24.0 * a2[k] + d5 / 120.0 * a3[k];
                v[3 * i + k] = vp[3 * i + k] + d3 / 6.0 * a2[k] + d4 / 24.0 * a3[k];
                a[3 * i + k] = a1[3 * i + k];
                jk[3 * i + k] = j1[3 * i + k];
                a2e[k] = a2[k] + d * a3[k];
                at[k] = a1[3 * i + k] + (fr ? fr[3 * i + k] : 0.0);
            }
            double n0 = hnorm(at), n1 = hnorm(jk + 3 * i), n2 = hnorm(a2e), n3 = hnorm(a3);
            double num = n0 * n2 + n1 * n1, den = n1 * n3 + n2 * n2;
            double want = den > 0.0 ? sqrt(eta * num / den) : dtmax;
            if (want_out) {
                want_out[3 * n + i] = tau[i] > 0 ? want_out[2 * n + i] : 0.0;
                want_out[n + i] = want;
                want_out[2 * n + i] = d;
            }
            if (want > 2.0 * d) want = 2.0 * d;
            tau[i] = tn;
            dt[i] = block_step(want, dtmax, tn);
            ++nsteps;
            int64_t k = 0;
            for (int64_t q = (int64_t)1 << HERM_KMAX; q > dt[i]; q >>= 1) ++k;
            if (k > kmin) kmin = k;
        }
        ++nblock;
        if (tn == tend) break;
    }
    if (stats) { stats[0] = nblock; stats[1] = nsteps; stats[2] = kmin; }
    free(a); free(jk); free(tau); free(dt); free(xp); free(vp); free(a1); free(j1); free(act);
}

/*
 * P3T loop (Section 2.2): per step, kick v += T/2 F_R, integrate F_I over T
 * (orc_hermite), recompute F_R, kick again. F_R is the direct regular sum.
 * energy [steps+1] (optional): KE + 1/2 sum m (Phi_R + Phi_I), i.e. plain
 * softened gravity, before the first step and after each.
 */
void orc_p3t(int64_t n, double* x, double* v, const double* mass, double r_in, double r_out,
             double eps, double T, double eta, int steps, double* energy)
{
    double* fr = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* pr = (double*)malloc(sizeof(double) * (size_t)n);
    double* fa = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* pa = (double*)malloc(sizeof(double) * (size_t)n);
    orc_direct(n, x, mass, r_in, r_out, eps, n, NULL, fr, pr);
    for (int st = 0; st <= steps; ++st) {
        if (energy) {
            orc_full_direct(n, x, mass, eps, fa, pa);
            double e = 0.0;
            for (int64_t i = 0; i < n; ++i)
                e += 0.5 * mass[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2])
                     + 0.5 * mass[i] * pa[i];
            energy[st] = e;
        }
        if (st == steps) break;
        for (int64_t k = 0; k < 3 * n; ++k) v[k] += 0.5 * T * fr[k];
        orc_hermite(n, x, v, mass, fr, r_in, r_out, eps, T, eta, NULL, NULL);
        orc_direct(n, x, mass, r_in, r_out, eps, n, NULL, fr, pr);
        for (int64_t k = 0; k < 3 * n; ++k) v[k] += 0.5 * T * fr[k];
    }
    free(fr); free(pr); free(fa); free(pa);
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets: j != i with ((dx*dx + dy*dy) + dz*dz) < r_out*r_out       */
/* ------------------------------------------------------------------------ */

static int is_nbr(const double* pos, int64_t i, int64_t j, double rout2)
{
    double dx = pos[3 * j] - pos[3 * i];
    double dy = pos[3 * j + 1] - pos[3 * i + 1];
    double dz = pos[3 * j + 2] - pos[3 * i + 2];
    double r2 = dx * dx + dy * dy + dz * dz;
    return r2 < rout2;
}

/*
 * Brute force. Writes counts to off[0..n] as a CSR offset array (off[0] = 0)
 * and, if idx != NULL and the total fits in cap, the ascending neighbour
 * indices of each particle. Returns the total number of entries.
 */
int64_t orc_nbr_brute(int64_t n, const double* pos, double r_out,
                      int64_t* off, int32_t* idx, int64_t cap)
{
    double rout2 = r_out * r_out;
    off[0] = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && is_nbr(pos, i, j, rout2)) ++c;
        off[i + 1] = c;
    }
    for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
    int64_t total = off[n];
    if (idx && total <= cap) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int64_t w = off[i];
            for (int64_t j = 0; j < n; ++j)
                if (j != i && is_nbr(pos, i, j, rout2)) idx[w++] = (int32_t)j;
        }
    }
    return total;
}

/* Cell list with cells of side r_out: candidates come from the 27 cells around i. */
typedef struct { int64_t c[3]; int64_t i; } cellrec;

static int cell_cmp(const void* pa, const void* pb)
{
    const cellrec* a = (const cellrec*)pa;
    const cellrec* b = (const cellrec*)pb;
    for (int d = 0; d < 3; ++d) {
        if (a->c[d] < b->c[d]) return -1;
        if (a->c[d] > b->c[d]) return 1;
    }
    return (a->i < b->i) ? -1 : (a->i > b->i);
}

static int cell_key_cmp(const int64_t* c, const cellrec* r)
{
    for (int d = 0; d < 3; ++d) {
        if (c[d] < r->c[d]) return -1;
        if (c[d] > r->c[d]) return 1;
    }
    return 0;
}

/* first record whose cell is >= c */
static int64_t cell_lower(const cellrec* recs, int64_t n, const int64_t* c)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cell_key_cmp(c, &recs[mid]) > 0) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

int64_t orc_nbr_cells(int64_t n, const double* pos, double r_out,
                      int64_t* off, int32_t* idx, int64_t cap)
{
    off[0] = 0;
    if (!(r_out > 0.0) || n < 2) {
        for (int64_t i = 0; i < n; ++i) off[i + 1] = 0;
        return 0;
    }
    double lo[3] = {pos[0], pos[1], pos[2]};
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d)
            if (pos[3 * i + d] < lo[d]) lo[d] = pos[3 * i + d];
    cellrec* recs = (cellrec*)malloc(sizeof(cellrec) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) recs[i].c[d] = (int64_t)floor((pos[3 * i + d] - lo[d]) / r_out);
        recs[i].i = i;
    }
    qsort(recs, (size_t)n, sizeof(cellrec), cell_cmp);
    double rout2 = r_out * r_out;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
            if (!idx || off[n] > cap) break;
        }
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int64_t ci[3];
            for (int d = 0; d < 3; ++d) ci[d] = (int64_t)floor((pos[3 * i + d] - lo[d]) / r_out);
            int64_t cnt = 0;
            int64_t w = pass ? off[i] : 0;
            for (int ox = -1; ox <= 1; ++ox)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int oz = -1; oz <= 1; ++oz) {
                        int64_t c[3] = {ci[0] + ox, ci[1] + oy, ci[2] + oz};
                        for (int64_t k = cell_lower(recs, n, c); k < n && cell_key_cmp(c, &recs[k]) == 0; ++k) {
                            int64_t j = recs[k].i;
                            if (j != i && is_nbr(pos, i, j, rout2)) {
                                if (pass) idx[w++] = (int32_t)j; else ++cnt;
                            }
                        }
                    }
            if (pass == 0) off[i + 1] = cnt;
            else qsort(idx + off[i], (size_t)(off[i + 1] - off[i]), sizeof(int32_t), cmp_i32);
        }
    }
    free(recs);
    return off[n];
}

/* ------------------------------------------------------------------------ */
/* Barnes-Hut octree (Section 2.4 uses a GPU Barnes-Hut tree with opening   */
/* angle theta; theta = 0 reduces it to direct summation).                  */
/*                                                                          */
/* Tree definition shared with the GPU path (written independently there):  */
/*  keys   L = max extent of the cluster's bounding box (1 if 0);           */
/*         i_d = min(floor((x_d - lo_d) * (2^D / L)), 2^D - 1);             */
/*         key = x,y,z bits interleaved, x most significant per level.      */
/*  order  particles sorted by (key, original index).                       */
/*  nodes  the root holds all particles; a node at level l < D with more    */
/*         than n_leaf particles has one child per distinct octant digit    */
/*         at level l+1 (in key order); nodes are numbered breadth first.   */
/*  moments bottom-up: a leaf combines its particles, an inner node its     */
/*         children, in order: M = sum m; COM = sum m x / M;                */
/*         Q_ab = sum [Q_c,ab + m (3 d_a d_b - |d|^2 delta_ab)], d = x-COM; */
/*         tight box lo/hi; l = max extent; delta = |COM - box centre|.     */
/*  groups a node is "big" if it holds more than n_crit particles or its  */
/*         tight box is larger (largest side) than the size limit S. Every  */
/*         big node splits into groups: a big leaf into runs of n_crit      */
/*         particles, or into single particles if its box exceeds S; an     */
/*         inner node packs its consecutive children that are not big,      */
/*         greedily and in order, into groups of at most n_crit particles   */
/*         whose joint box stays within S (a big child interrupts the run). */
/*         A root that is not big is one group. S is 2^5 x 2^e for the     */
/*         octave e (2^e <= x < 2^(e+1)) holding the median box size of the */
/*         groups this rule forms with S = infinity, per cluster; it keeps  */
/*         a sparse-halo group from spanning the dense core. Groups are     */
/*         ordered by their                                                 */
/*         first particle; each has a tight box.                            */
/*  walk   per group and node: dbox2 = squared distance between the group   */
/*         box and the node box; near if dbox2 < r_out^2 or dbox2 == 0;     */
/*         accept (multipole) if not near, theta > 0 and the squared        */
/*         distance from the group box to COM exceeds (l/theta + delta)^2;  */
/*         otherwise open: a leaf gives particle-particle interactions      */
/*         (with the changeover when near), an inner node its children.     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t begin, count;
    int64_t first_child;
    int32_t nchild, level;
    double M, com[3], q[6]; /* q: xx, yy, zz, xy, xz, yz */
    double lo[3], hi[3];
    double rcrit2;
} onode_t;

static uint64_t spread3(uint64_t v, int D)
{
    uint64_t out = 0;
    for (int b = 0; b < D; ++b) out |= ((v >> b) & 1ULL) << (3 * b);
    return out;
}

/* Morton keys of one cluster with D bits per dimension (D <= 21). */
void orc_keys(int64_t n, const double* pos, int D, uint64_t* keys)
{
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = pos[d];
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = pos[3 * i + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double L = 0.0;
    for (int d = 0; d < 3; ++d)
        if (hi[d] - lo[d] > L) L = hi[d] - lo[d];
    if (L == 0.0) L = 1.0;
    double scale = ldexp(1.0, D) / L;
    int64_t maxc = ((int64_t)1 << D) - 1;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t key = 0;
        for (int d = 0; d < 3; ++d) {
            double f = floor((pos[3 * i + d] - lo[d]) * scale);
            int64_t c = (int64_t)f;
            if (c > maxc) c = maxc;
            if (c < 0) c = 0;
            key |= spread3((uint64_t)c, D) << (2 - d);
        }
        keys[i] = key;
    }
}

typedef struct { uint64_t key; int64_t i; } keyrec;

static int key_cmp(const void* pa, const void* pb)
{
    const keyrec* a = (const keyrec*)pa;
    const keyrec* b = (const keyrec*)pb;
    if (a->key != b->key) return (a->key < b->key) ? -1 : 1;
    return (a->i < b->i) ? -1 : (a->i > b->i);
}

/* add child (mass m, centre c, quadrupole qc about c) into a node about com */
static void quad_add(double* q, const double* qc, double m, const double* c, const double* com)
{
    double dx = c[0] - com[0], dy = c[1] - com[1], dz = c[2] - com[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    q[0] = q[0] + (qc[0] + m * (3.0 * dx * dx - r2));
    q[1] = q[1] + (qc[1] + m * (3.0 * dy * dy - r2));
    q[2] = q[2] + (qc[2] + m * (3.0 * dz * dz - r2));
    q[3] = q[3] + (qc[3] + m * (3.0 * dx * dy));
    q[4] = q[4] + (qc[4] + m * (3.0 * dx * dz));
    q[5] = q[5] + (qc[5] + m * (3.0 * dy * dz));
}

typedef struct {
    int64_t n;
    onode_t* nodes;
    int64_t n_nodes, cap_nodes;
    int64_t* order;     /* sorted position -> original index */
    double *x, *y, *z, *m; /* sorted copies */
    uint64_t* keys;     /* sorted keys */
} otree_t;

static int64_t push_node(otree_t* t)
{
    if (t->n_nodes == t->cap_nodes) {
        t->cap_nodes = t->cap_nodes ? 2 * t->cap_nodes : 1024;
        t->nodes = (onode_t*)realloc(t->nodes, sizeof(onode_t) * (size_t)t->cap_nodes);
    }
    memset(&t->nodes[t->n_nodes], 0, sizeof(onode_t));
    return t->n_nodes++;
}

static void tree_build(otree_t* t, int64_t n, const double* pos, const double* mass,
                       int n_leaf, int D)
{
    memset(t, 0, sizeof(*t));
    t->n = n;
    t->keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    orc_keys(n, pos, D, t->keys);
    keyrec* kr = (keyrec*)malloc(sizeof(keyrec) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) { kr[i].key = t->keys[i]; kr[i].i = i; }
    qsort(kr, (size_t)n, sizeof(keyrec), key_cmp);
    t->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    t->x = (double*)malloc(sizeof(double) * (size_t)n);
    t->y = (double*)malloc(sizeof(double) * (size_t)n);
    t->z = (double*)malloc(sizeof(double) * (size_t)n);
    t->m = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = kr[k].i;
        t->order[k] = i;
        t->keys[k] = kr[k].key;
        t->x[k] = pos[3 * i];
        t->y[k] = pos[3 * i + 1];
        t->z[k] = pos[3 * i + 2];
        t->m[k] = mass[i];
    }
    free(kr);

    /* topology, breadth first: children of node k are appended when k is visited */
    int64_t root = push_node(t);
    t->nodes[root].begin = 0;
    t->nodes[root].count = n;
    t->nodes[root].level = 0;
    for (int64_t k = 0; k < t->n_nodes; ++k) {
        onode_t nd = t->nodes[k];
        t->nodes[k].nchild = 0;
        if (!(nd.count > n_leaf && nd.level < D)) continue;
        int shift = 3 * (D - 1 - nd.level);
        int64_t first = t->n_nodes;
        int64_t s = nd.begin;
        while (s < nd.begin + nd.count) {
            unsigned dig = (unsigned)((t->keys[s] >> shift) & 7ULL);
            int64_t e = s;
            while (e < nd.begin + nd.count && (unsigned)((t->keys[e] >> shift) & 7ULL) == dig) ++e;
            int64_t c = push_node(t);
            t->nodes[c].begin = s;
            t->nodes[c].count = e - s;
            t->nodes[c].level = nd.level + 1;
            s = e;
        }
        t->nodes[k].first_child = first;
        t->nodes[k].nchild = (int32_t)(t->n_nodes - first);
    }

    /* moments, children before parents (reverse breadth-first order) */
    for (int64_t k = t->n_nodes - 1; k >= 0; --k) {
        onode_t* nd = &t->nodes[k];
        double M = 0, sx = 0, sy = 0, sz = 0;
        int64_t nsub = nd->nchild ? nd->nchild : nd->count;
        for (int64_t u = 0; u < nsub; ++u) {
            double mu, cu[3];
            if (nd->nchild) {
                const onode_t* c = &t->nodes[nd->first_child + u];
                mu = c->M; cu[0] = c->com[0]; cu[1] = c->com[1]; cu[2] = c->com[2];
            } else {
                int64_t j = nd->begin + u;
                mu = t->m[j]; cu[0] = t->x[j]; cu[1] = t->y[j]; cu[2] = t->z[j];
            }
            M = M + mu;
            sx = sx + mu * cu[0];
            sy = sy + mu * cu[1];
            sz = sz + mu * cu[2];
            for (int d = 0; d < 3; ++d) {
                double lo_u = nd->nchild ? t->nodes[nd->first_child + u].lo[d] : cu[d];
                double hi_u = nd->nchild ? t->nodes[nd->first_child + u].hi[d] : cu[d];
                if (u == 0 || lo_u < nd->lo[d]) nd->lo[d] = lo_u;
                if (u == 0 || hi_u > nd->hi[d]) nd->hi[d] = hi_u;
            }
        }
        nd->M = M;
        if (M > 0.0) {
            nd->com[0] = sx / M; nd->com[1] = sy / M; nd->com[2] = sz / M;
        } else {
            for (int d = 0; d < 3; ++d) nd->com[d] = (nd->lo[d] + nd->hi[d]) * 0.5;
        }
        for (int e = 0; e < 6; ++e) nd->q[e] = 0.0;
        static const double zero6[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t u = 0; u < nsub; ++u) {
            if (nd->nchild) {
                const onode_t* c = &t->nodes[nd->first_child + u];
                quad_add(nd->q, c->q, c->M, c->com, nd->com);
            } else {
                int64_t j = nd->begin + u;
                double cu[3] = {t->x[j], t->y[j], t->z[j]};
                quad_add(nd->q, zero6, t->m[j], cu, nd->com);
            }
        }
    }
}

static void tree_free(otree_t* t)
{
    free(t->nodes); free(t->order); free(t->x); free(t->y); free(t->z); free(t->m); free(t->keys);
}

/* squared distance between boxes [alo, ahi] and [blo, bhi]; per axis gap >= 0 */
static double box_box_d2(const double* alo, const double* ahi, const double* blo, const double* bhi)
{
    double g[3];
    for (int d = 0; d < 3; ++d) {
        double a = blo[d] - ahi[d];
        double b = alo[d] - bhi[d];
        double v = a > b ? a : b;
        g[d] = v > 0.0 ? v : 0.0;
    }
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
}

/* squared distance from point c to box [lo, hi] */
static double box_pt_d2(const double* lo, const double* hi, const double* c)
{
    double g[3];
    for (int d = 0; d < 3; ++d) {
        double a = lo[d] - c[d];
        double b = c[d] - hi[d];
        double v = a > b ? a : b;
        g[d] = v > 0.0 ? v : 0.0;
    }
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
}

typedef struct { int64_t begin, count; } ogroup_t;

static int group_cmp(const void* a, const void* b)
{
    int64_t x = ((const ogroup_t*)a)->begin, y = ((const ogroup_t*)b)->begin;
    return (x > y) - (x < y);
}

#ifndef GROUP_S_LOG2
#define GROUP_S_LOG2 5
#endif

/* largest side of a box */
static double box_extent(const double* lo, const double* hi)
{
    double e = 0.0;
    for (int d = 0; d < 3; ++d)
        if (hi[d] - lo[d] > e) e = hi[d] - lo[d];
    return e;
}

/* octave of a length: index e + 64 for 2^e <= x < 2^(e+1), e clamped to
   [-64, 63]; index 0 for x = 0 */
static int octave_index(double x)
{
    if (!(x > 0.0)) return 0;
    int e;
    frexp(x, &e);   /* x = m 2^e, 1/2 <= m < 1 */
    e -= 1;
    if (e < -64) e = -64;
    if (e > 63) e = 63;
    return e + 64;
}

static void emit_group(ogroup_t* g, int64_t* ng, int64_t begin, int64_t count, double ext,
                       double* ext_out)
{
    g[*ng].begin = begin;
    g[*ng].count = count;
    if (ext_out) ext_out[*ng] = ext;
    ++*ng;
}

/* One pass of the grouping rule with size limit S (see the tree comment). */
static int64_t group_pass(const otree_t* t, int n_crit, double S, ogroup_t* g, double* ext_out)
{
    int64_t ng = 0;
    for (int64_t k = 0; k < t->n_nodes; ++k) {
        const onode_t* nd = &t->nodes[k];
        double ext = box_extent(nd->lo, nd->hi);
        int big = nd->count > n_crit || ext > S;
        if (nd->level == 0 && !big) emit_group(g, &ng, nd->begin, nd->count, ext, ext_out);
        if (!big) continue;
        if (nd->nchild == 0) {
            if (ext > S) {
                for (int64_t j = nd->begin; j < nd->begin + nd->count; ++j)
                    emit_group(g, &ng, j, 1, 0.0, ext_out);
            } else {
                for (int64_t s0 = nd->begin; s0 < nd->begin + nd->count; s0 += n_crit) {
                    int64_t e0 = s0 + n_crit < nd->begin + nd->count ? s0 + n_crit : nd->begin + nd->count;
                    double lo[3], hi[3];
                    for (int64_t j = s0; j < e0; ++j) {
                        double v[3] = {t->x[j], t->y[j], t->z[j]};
                        for (int d = 0; d < 3; ++d) {
                            if (j == s0 || v[d] < lo[d]) lo[d] = v[d];
                            if (j == s0 || v[d] > hi[d]) hi[d] = v[d];
                        }
                    }
                    emit_group(g, &ng, s0, e0 - s0, box_extent(lo, hi), ext_out);
                }
            }
            continue;
        }
        int64_t run_begin = 0, run_count = 0;
        double rlo[3] = {0, 0, 0}, rhi[3] = {0, 0, 0};
        for (int32_t c = 0; c < nd->nchild; ++c) {
            const onode_t* ch = &t->nodes[nd->first_child + c];
            int cbig = ch->count > n_crit || box_extent(ch->lo, ch->hi) > S;
            if (cbig) {
                if (run_count > 0) emit_group(g, &ng, run_begin, run_count, box_extent(rlo, rhi), ext_out);
                run_count = 0;
                continue;
            }
            double ulo[3], uhi[3];
            for (int d = 0; d < 3; ++d) {
                ulo[d] = (run_count > 0 && rlo[d] < ch->lo[d]) ? rlo[d] : ch->lo[d];
                uhi[d] = (run_count > 0 && rhi[d] > ch->hi[d]) ? rhi[d] : ch->hi[d];
            }
            if (run_count > 0 && (run_count + ch->count > n_crit || box_extent(ulo, uhi) > S)) {
                emit_group(g, &ng, run_begin, run_count, box_extent(rlo, rhi), ext_out);
                run_count = 0;
                for (int d = 0; d < 3; ++d) { ulo[d] = ch->lo[d]; uhi[d] = ch->hi[d]; }
            }
            if (run_count == 0) run_begin = ch->begin;
            run_count += ch->count;
            for (int d = 0; d < 3; ++d) { rlo[d] = ulo[d]; rhi[d] = uhi[d]; }
        }
        if (run_count > 0) emit_group(g, &ng, run_begin, run_count, box_extent(rlo, rhi), ext_out);
    }
    return ng;
}

/* Size limit of the walk groups of one cluster: 2^5 x 2^e for the octave e
   holding the median extent of the groups the count rule alone would form. */
static double group_size_limit(const otree_t* t, int n_crit)
{
    ogroup_t* g = (ogroup_t*)malloc(sizeof(ogroup_t) * (size_t)(t->n + 1));
    double* ext = (double*)malloc(sizeof(double) * (size_t)(t->n + 1));
    int64_t ng = group_pass(t, n_crit, INFINITY, g, ext);
    int64_t hist[128] = {0};
    for (int64_t k = 0; k < ng; ++k) hist[octave_index(ext[k])]++;
    int64_t need = (ng + 1) / 2, cum = 0;
    int b = 127;
    for (int i = 0; i < 128; ++i) {
        cum += hist[i];
        if (cum >= need) { b = i; break; }
    }
    free(g);
    free(ext);
    return ldexp(1.0, b - 64 + GROUP_S_LOG2);
}

/* Walk groups of the tree (rule in the comment above); returns the count. */
static int64_t make_groups(const otree_t* t, int n_crit, ogroup_t** out)
{
    double S = group_size_limit(t, n_crit);
    ogroup_t* g = (ogroup_t*)malloc(sizeof(ogroup_t) * (size_t)(t->n + 1));
    int64_t ng = group_pass(t, n_crit, S, g, NULL);
    qsort(g, (size_t)ng, sizeof(ogroup_t), group_cmp);
    *out = g;
    return ng;
}

typedef struct {
    const otree_t* t;
    const phir_t* p;
    double eps2, rlist2, theta;   /* rlist2: square of the list radius r_out + r_buff */
    int64_t gbeg, gcnt;
    double glo[3], ghi[3];
    double* ax; double* ay; double* az; double* ph; /* per group member */
    int64_t n_pn, n_far, n_near;
} walkctx;

/* Monopole + traceless quadrupole of a node acting on the group's members. */
static void eval_pn(walkctx* w, const onode_t* nd)
{
    const otree_t* t = w->t;
    for (int64_t u = 0; u < w->gcnt; ++u) {
        int64_t i = w->gbeg + u;
        /* R = x_i - COM */
        double Rx = t->x[i] - nd->com[0], Ry = t->y[i] - nd->com[1], Rz = t->z[i] - nd->com[2];
        double s2 = Rx * Rx + Ry * Ry + Rz * Rz + w->eps2;
        double s = sqrt(s2);
        double inv = 1.0 / s;
        double inv2 = inv * inv;
        double inv3 = inv * inv2;
        double inv5 = inv3 * inv2;
        double inv7 = inv5 * inv2;
        /* QR and R^T Q R with q = (xx, yy, zz, xy, xz, yz) */
        double qx = nd->q[0] * Rx + nd->q[3] * Ry + nd->q[4] * Rz;
        double qy = nd->q[3] * Rx + nd->q[1] * Ry + nd->q[5] * Rz;
        double qz = nd->q[4] * Rx + nd->q[5] * Ry + nd->q[2] * Rz;
        double rqr = Rx * qx + Ry * qy + Rz * qz;
        /* phi = -M/s - (1/2) R^T Q R / s^5 ; a = -grad phi */
        double cr = -nd->M * inv3 - 2.5 * rqr * inv7;
        w->ax[u] += cr * Rx + qx * inv5;
        w->ay[u] += cr * Ry + qy * inv5;
        w->az[u] += cr * Rz + qz * inv5;
        w->ph[u] += -nd->M * inv - 0.5 * rqr * inv5;
    }
    w->n_pn += w->gcnt;
}

static void eval_pp(walkctx* w, const onode_t* nd, int near)
{
    const otree_t* t = w->t;
    for (int64_t u = 0; u < w->gcnt; ++u) {
        int64_t i = w->gbeg + u;
        for (int64_t j = nd->begin; j < nd->begin + nd->count; ++j) {
            if (j == i) continue;
            if (near) {
                pair_regular(w->p, w->eps2, t->x[i], t->y[i], t->z[i], t->x[j], t->y[j], t->z[j],
                             t->m[j], &w->ax[u], &w->ay[u], &w->az[u], &w->ph[u]);
            } else {
                /* every pair of a far leaf is at r >= r_out + r_buff >= r_out, where W = 1 */
                double dx = t->x[j] - t->x[i], dy = t->y[j] - t->y[i], dz = t->z[j] - t->z[i];
                double s2 = dx * dx + dy * dy + dz * dz + w->eps2;
                double s = sqrt(s2);
                double f = t->m[j] / (s2 * s);
                w->ax[u] += f * dx;
                w->ay[u] += f * dy;
                w->az[u] += f * dz;
                w->ph[u] += -t->m[j] / s;
            }
        }
    }
    if (near) w->n_near += w->gcnt * nd->count; else w->n_far += w->gcnt * nd->count;
}

static void visit(walkctx* w, int64_t k)
{
    const onode_t* nd = &w->t->nodes[k];
    double dbox2 = box_box_d2(w->glo, w->ghi, nd->lo, nd->hi);
    int near = (dbox2 < w->rlist2) || (dbox2 == 0.0);
    if (!near && w->theta > 0.0 && box_pt_d2(w->glo, w->ghi, nd->com) > nd->rcrit2) {
        eval_pn(w, nd);
        return;
    }
    if (nd->nchild == 0) {
        eval_pp(w, nd, near);
        return;
    }
    for (int32_t c = 0; c < nd->nchild; ++c) visit(w, nd->first_child + c);
}

/*
 * Tree walk of one cluster. Outputs acc [n][3], pot [n] in the caller's order.
 * A node is near when its box comes closer than the neighbour-list radius
 * r_out + r_buff to the group box (or touches it); near nodes are opened and
 * their leaf pairs take W(s), which is 1 beyond r_out. With r_buff > 0 the
 * lists hold a buffer beyond the changeover radius (Section 2.3, R_buff, and
 * the rule r_buff = 3 tau sigma of the run parameters), so every list member
 * is found as a particle pair.
 * stats (optional, int64[6]): n_nodes, n_leaves, n_groups, PN, PP-far, PP-near
 * interaction counts (PN counted once per group member, PP once per pair
 * evaluated, the excluded self pair included in PP-near).
 */
void orc_tree(int64_t n, const double* pos, const double* mass,
              double r_in, double r_out, double r_buff, double theta, double eps,
              int n_leaf, int n_crit, int D,
              double* acc, double* pot, int64_t* stats)
{
    otree_t t;
    tree_build(&t, n, pos, mass, n_leaf, D);
    for (int64_t k = 0; k < t.n_nodes; ++k) {
        onode_t* nd = &t.nodes[k];
        double l = 0.0;
        for (int d = 0; d < 3; ++d)
            if (nd->hi[d] - nd->lo[d] > l) l = nd->hi[d] - nd->lo[d];
        double ctr[3], dd[3];
        for (int d = 0; d < 3; ++d) {
            ctr[d] = (nd->lo[d] + nd->hi[d]) * 0.5;
            dd[d] = nd->com[d] - ctr[d];
        }
        double delta = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
        double rc = theta > 0.0 ? l / theta + delta : 0.0;
        nd->rcrit2 = rc * rc;
    }
    phir_t p;
    phir_init(&p, r_in, r_out);
    ogroup_t* groups = NULL;
    int64_t ngroups = make_groups(&t, n_crit, &groups);
    int64_t s_pn = 0, s_far = 0, s_near = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : s_pn, s_far, s_near)
    for (int64_t g = 0; g < ngroups; ++g) {
        walkctx w;
        memset(&w, 0, sizeof(w));
        w.t = &t;
        w.p = &p;
        w.eps2 = eps * eps;
        w.rlist2 = (r_out + r_buff) * (r_out + r_buff);
        w.theta = theta;
        w.gbeg = groups[g].begin;
        w.gcnt = groups[g].count;
        for (int64_t u = 0; u < w.gcnt; ++u) {
            int64_t i = w.gbeg + u;
            double v[3] = {t.x[i], t.y[i], t.z[i]};
            for (int d = 0; d < 3; ++d) {
                if (u == 0 || v[d] < w.glo[d]) w.glo[d] = v[d];
                if (u == 0 || v[d] > w.ghi[d]) w.ghi[d] = v[d];
            }
        }
        double* buf = (double*)calloc((size_t)(4 * w.gcnt), sizeof(double));
        w.ax = buf; w.ay = buf + w.gcnt; w.az = buf + 2 * w.gcnt; w.ph = buf + 3 * w.gcnt;
        visit(&w, 0);
        for (int64_t u = 0; u < w.gcnt; ++u) {
            int64_t i = t.order[w.gbeg + u];
            acc[3 * i] = w.ax[u];
            acc[3 * i + 1] = w.ay[u];
            acc[3 * i + 2] = w.az[u];
            pot[i] = w.ph[u];
        }
        free(buf);
        s_pn += w.n_pn; s_far += w.n_far; s_near += w.n_near;
    }
    if (stats) {
        int64_t leaves = 0;
        for (int64_t k = 0; k < t.n_nodes; ++k) leaves += (t.nodes[k].nchild == 0);
        stats[0] = t.n_nodes; stats[1] = leaves; stats[2] = ngroups;
        stats[3] = s_pn; stats[4] = s_far; stats[5] = s_near;
    }
    free(groups);
    tree_free(&t);
}

/* Size limit S of the walk groups of one cluster. */
double orc_group_limit(int64_t n, const double* pos, const double* mass, int n_leaf, int n_crit, int D)
{
    otree_t t;
    tree_build(&t, n, pos, mass, n_leaf, D);
    double S = group_size_limit(&t, n_crit);
    tree_free(&t);
    return S;
}

/* Walk groups of one cluster: writes up to cap (begin, count) pairs, returns the count. */
int64_t orc_groups(int64_t n, const double* pos, const double* mass, int n_leaf, int n_crit, int D,
                   int64_t cap, int64_t* begin, int64_t* count)
{
    otree_t t;
    tree_build(&t, n, pos, mass, n_leaf, D);
    ogroup_t* groups = NULL;
    int64_t ng = make_groups(&t, n_crit, &groups);
    for (int64_t g = 0; g < ng && g < cap; ++g) {
        begin[g] = groups[g].begin;
        count[g] = groups[g].count;
    }
    free(groups);
    tree_free(&t);
    return ng;
}

/*
 * Tree structure export for stage-level tests: sorted order [n], and for
 * each node (up to cap) begin, count, nchild, level, M, com[3], q[6], lo[3], hi[3].
 * Returns the node count (arrays untouched if it exceeds cap).
 */
int64_t orc_tree_nodes(int64_t n, const double* pos, const double* mass, int n_leaf, int D,
                       int64_t cap, int64_t* order, int64_t* ibuf /* [cap][4] */,
                       double* dbuf /* [cap][16] */)
{
    otree_t t;
    tree_build(&t, n, pos, mass, n_leaf, D);
    int64_t nn = t.n_nodes;
    if (order) memcpy(order, t.order, sizeof(int64_t) * (size_t)n);
    if (nn <= cap) {
        for (int64_t k = 0; k < nn; ++k) {
            const onode_t* nd = &t.nodes[k];
            ibuf[4 * k] = nd->begin;
            ibuf[4 * k + 1] = nd->count;
            ibuf[4 * k + 2] = nd->nchild;
            ibuf[4 * k + 3] = nd->level;
            double* o = dbuf + 16 * k;
            o[0] = nd->M;
            for (int d = 0; d < 3; ++d) { o[1 + d] = nd->com[d]; o[10 + d] = nd->lo[d]; o[13 + d] = nd->hi[d]; }
            for (int e = 0; e < 6; ++e) o[4 + e] = nd->q[e];
        }
    }
    tree_free(&t);
    return nn;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the later parallel loops (timing on fewer cores); no effect
 * on any result, since every parallel loop writes per-index outputs. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
