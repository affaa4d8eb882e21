/*
 * bhmc oracle: a plain, serial, FP64 CPU reference for the Barnes-Hut treecode
 * evaluation of single-particle Metropolis energy changes (Gan & Xu,
 * "Efficient Implementation of the Barnes-Hut Octree Algorithm for Monte Carlo
 * Simulations of Charged Systems").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP library, and the HIP library never
 * calls it.
 *
 * What is here, each routine citing the passage it follows:
 *   - direct O(N^2) energy, energy change, per-ion potential and gradient
 *     (eq. 1.1, eq. 2.1), with Kelvin images of a dielectric sphere written as
 *     the symmetric ion-image pair kernel (the paper names the image model in
 *     Sec. 1 and Sec. 5 without a formula; the kernel is textbook
 *     electrostatics);
 *   - a serial treecode: Morton keys, a stable sort (library qsort), a
 *     recursive octree build (Sec. 3.2), per-cell moments summed directly
 *     from the members of each cell (eq. 3.3), Taylor coefficients by the
 *     recurrence (eq. 3.4), the recursive MAC traversal (Sec. 3.2) and the
 *     local add/delete of an accepted move (Sec. 3.3);
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the Metropolis
 *     driver (Sec. 2, steps 1-3; Sec. 3.3);
 *   - the treecode energy and its exact gradient, summed pair by pair over the
 *     interaction lists the traversal produces;
 *   - the multiple-image model of the dielectric sphere (Sec. 1 and Sec. 5
 *     name it without formulas): besides the Kelvin image, a line image from
 *     the sphere's centre to the Kelvin point, discretised by a Gauss-Jacobi
 *     rule (energies, moves and the gradient).
 *
 * Every floating-point expression whose outcome decides an integer (a key, a
 * MAC decision, a wall or overlap test, a Metropolis decision) is written left
 * to right and built with -ffp-contract=off so that the GPU library, which is
 * written to the same conventions, reaches the same decisions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Parameters                                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    double l_B;          /* Bjerrum length (eq. 2.1); absorbs beta            */
    double theta;        /* MAC parameter, 0 <= theta < 1 (Sec. 3.2)          */
    int32_t p;           /* multipole order (eq. 3.3)                         */
    int32_t leaf_cap;    /* split a cell iff count > leaf_cap                 */
    int32_t n0;          /* minimum expansion number N_0 (Sec. 3.2)           */
    int32_t max_depth;   /* deepest level, <= 21                              */
    int32_t geom;        /* 0: cube [lo, lo+S)^3; 1: shell r_min < |r| < r_max */
    int32_t images;      /* 1: one Kelvin image per ion (shell only)          */
    double box_lo[3];    /* root cube corner                                  */
    double box_side;     /* root cube side S                                  */
    double a;            /* dielectric sphere radius                          */
    double Q_center;     /* central macroion valence Q_M (Sec. 4)             */
    double eps_in, eps_out;
    double r_min, r_max; /* shell confinement (Sec. 4, spherical cell model)  */
    double hard_core;    /* contact distance tau (eq. 2.1)                    */
    int32_t slot_slack;  /* leaf slots = slack * max(count, leaf_cap) + 2 + M */
    int32_t line_images; /* 0, or M line-image points per ion (1..8)          */
} orc_params;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EOUTSIDE = -2, ORC_ECAPACITY = -6 };
enum { REASON_NONE = 0, REASON_WALL = 1, REASON_OVERLAP = 2 };

/* ------------------------------------------------------------------------ */
/* Neumaier compensated summation                                           */
/* ------------------------------------------------------------------------ */

typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Multi-indices, graded order (Sec. 3.1 notation)                          */
/*   for s = 0..p, n1 = s..0, n2 = s-n1..0, n3 = s-n1-n2                    */
/* ------------------------------------------------------------------------ */

static int nterms_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

static int mindex(int n1, int n2, int n3) {
    int s = n1 + n2 + n3;
    return s * (s + 1) * (s + 2) / 6 + (s - n1) * (s - n1 + 1) / 2 + (s - n1 - n2);
}

static void multi_indices(int p, int *mi /* 3*nterms */) {
    int k = 0;
    for (int s = 0; s <= p; ++s)
        for (int n1 = s; n1 >= 0; --n1)
            for (int n2 = s - n1; n2 >= 0; --n2) {
                mi[3 * k] = n1; mi[3 * k + 1] = n2; mi[3 * k + 2] = s - n1 - n2;
                ++k;
            }
}

/* Monomials d^n = dx^n1 dy^n2 dz^n3 by repeated multiplication (eq. 3.3). */
static void monomials(int p, const int *mi, double dx, double dy, double dz, double *out) {
    int nt = nterms_of(p);
    for (int k = 0; k < nt; ++k) {
        double v = 1.0;
        for (int e = 0; e < mi[3 * k]; ++e) v *= dx;
        for (int e = 0; e < mi[3 * k + 1]; ++e) v *= dy;
        for (int e = 0; e < mi[3 * k + 2]; ++e) v *= dz;
        out[k] = v;
    }
}

/* Taylor coefficients T_n(R) = D^n (1/|R|) / n!, |n| <= p, from T_0 = 1/|R|
 * and the recurrence (eq. 3.4):
 *   |n| r^2 T_n + (2|n|-1) sum_i x_i T_{n-e_i} + (|n|-1) sum_i T_{n-2e_i} = 0,
 * with T_n = 0 whenever a component of n is negative. */
static void taylor(int p, const int *mi, double Rx, double Ry, double Rz, double *T) {
    int nt = nterms_of(p);
    double r2 = Rx * Rx + Ry * Ry + Rz * Rz;
    T[0] = 1.0 / sqrt(r2);
    for (int k = 1; k < nt; ++k) {
        int n1 = mi[3 * k], n2 = mi[3 * k + 1], n3 = mi[3 * k + 2];
        int s = n1 + n2 + n3;
        double first = 0.0, second = 0.0;
        if (n1 >= 1) first += Rx * T[mindex(n1 - 1, n2, n3)];
        if (n2 >= 1) first += Ry * T[mindex(n1, n2 - 1, n3)];
        if (n3 >= 1) first += Rz * T[mindex(n1, n2, n3 - 1)];
        if (n1 >= 2) second += T[mindex(n1 - 2, n2, n3)];
        if (n2 >= 2) second += T[mindex(n1, n2 - 2, n3)];
        if (n3 >= 2) second += T[mindex(n1, n2, n3 - 2)];
        T[k] = -((2.0 * s - 1.0) * first + (s - 1.0) * second) / (s * r2);
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11) and the move map                    */
/* ------------------------------------------------------------------------ */

static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out) { philox4x32_10(ctr, key, out); }

/* uniform double in [0,1) from two 32-bit words: 27 + 26 bits over 2^53 */
static double u53(uint32_t wa, uint32_t wb) {
    return ((double)(wa >> 5) * 67108864.0 + (double)(wb >> 6)) * (1.0 / 9007199254740992.0);
}

/* Twelve Philox words for move m of replica r: counter (lo m, hi m, r, t),
 * t = 0, 1, 2; key (lo seed, hi seed).  Ion index from w0, displacement from
 * (w2,w3), (w4,w5), (w6,w7), the Metropolis alpha from (w8,w9). */
void orc_draw_move(uint64_t seed, uint32_t replica, uint64_t m, int64_t n, double step,
                   int64_t *i_out, double *delta /*3*/, double *alpha) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[12];
    for (uint32_t t = 0; t < 3; ++t) {
        uint32_t ctr[4] = {(uint32_t)m, (uint32_t)(m >> 32), replica, t};
        philox4x32_10(ctr, key, w + 4 * t);
    }
    *i_out = (int64_t)(((uint64_t)w[0] * (uint64_t)n) >> 32);
    delta[0] = step * (u53(w[2], w[3]) - 0.5);
    delta[1] = step * (u53(w[4], w[5]) - 0.5);
    delta[2] = step * (u53(w[6], w[7]) - 0.5);
    *alpha = u53(w[8], w[9]);
}

/* ------------------------------------------------------------------------ */
/* Geometry: Kelvin image, confinement, Morton keys                         */
/* ------------------------------------------------------------------------ */

static double gamma_of(const orc_params *P) {
    return (P->eps_out - P->eps_in) / (P->eps_out + P->eps_in);
}

/* Kelvin image of a charge q at r outside a sphere of radius a:
 * charge gamma*a*q/|r| at (a^2/|r|^2) r. */
void orc_kelvin(double a, double gamma, double x, double y, double z, double q, double *out /*4*/) {
    double r2 = x * x + y * y + z * z;
    double s = (a * a) / r2;
    double rn = sqrt(r2);
    out[0] = s * x;
    out[1] = s * y;
    out[2] = s * z;
    out[3] = ((gamma * a) * q) / rn;
}

/* ------------------------------------------------------------------------ */
/* Multiple images                                                          */
/*                                                                          */
/* A unit charge at y outside the sphere (|y| > a, eps_in inside, eps_out   */
/* outside) has the reaction potential, outside,                            */
/*   G_R(x; y) = sum_n b_n a^(2n+1) / (|y|^(n+1) |x|^(n+1)) P_n(cos angle), */
/*   b_n = n (eps_out - eps_in) / (n eps_in + (n + 1) eps_out)              */
/*       = gamma n / (n + sigma),  sigma = eps_out / (eps_in + eps_out).    */
/* With n / (n + sigma) = 1 - sigma int_0^1 t^(n + sigma - 1) dt this is    */
/* the Kelvin image gamma a / |y| at y_K = a^2 y / |y|^2 plus a line of      */
/* charge -sigma (gamma a / |y|) t^(sigma - 1) dt at t y_K, t in [0, 1].      */
/* The line is replaced by M points: the Gauss rule of the weight           */
/* t^(sigma - 1) on [0, 1].                                                  */
/* ------------------------------------------------------------------------ */

/* Jacobi polynomial P_n^(0, b)(x) and its derivative, by the three-term
 * recurrence in n. */
static void jacobi0b(int n, double b, double x, double *p, double *dp) {
    double p0 = 1.0, p1 = 0.5 * (-b + (b + 2.0) * x);
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double c = 2.0 * k + b;
        double a1 = 2.0 * k * (k + b) * (c - 2.0);
        double a2 = (c - 1.0) * (-b * b);
        double a3 = (c - 1.0) * c * (c - 2.0);
        double a4 = 2.0 * (k - 1.0) * (k + b - 1.0) * c;
        double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1; p1 = p2;
    }
    /* (2n + b)(1 - x^2) P_n' = n (-b - (2n + b) x) P_n + 2 n (n + b) P_{n-1} */
    double c = 2.0 * n + b;
    *p = p1;
    *dp = (n * (-b - c * x) * p1 + 2.0 * n * (n + b) * p0) / (c * (1.0 - x * x));
}

/* Nodes t[0..M) and weights w[0..M) with sum_m w_m f(t_m) = int_0^1 t^(sigma-1) f(t) dt
 * for every polynomial f of degree < 2M: Newton's method (with the roots
 * already found divided out) on P_M^(0, sigma - 1)(2t - 1), weights from
 *   w = 2^(-sigma) Gamma(M+1) Gamma(M+sigma) / (Gamma(M+sigma) M!) 2^sigma / ((1 - x^2) P_M'(x)^2)
 *     = 1 / ((1 - x^2) P_M'(x)^2)  in x = 2t - 1.
 * The nodes come out in descending order.  Returns 0, or -1 for M outside 1..8
 * or sigma outside [1/2, 1]. */
int orc_line_rule(double sigma, int M, double *t, double *w) {
    if (M < 1 || M > 8 || !(sigma >= 0.5 && sigma <= 1.0)) return -1;
    double b = sigma - 1.0, x[8];
    for (int m = 0; m < M; ++m) {
        double z = cos(M_PI * (m + 0.75) / (M + 0.5));  /* descending starting points */
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            jacobi0b(M, b, z, &p, &dp);
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += 1.0 / (z - x[k]);
            double dz = p / (dp - p * s);
            z -= dz;
            if (fabs(dz) <= 1e-16 * (1.0 + fabs(z))) break;
        }
        x[m] = z;
    }
    /* nodes and weights rounded to multiples of 2^-40 (about 1e-12, far below the rule's
     * own error), so that an independent computation of the rule gives the same sources */
    for (int m = 0; m < M; ++m) {
        double p, dp;
        jacobi0b(M, b, x[m], &p, &dp);
        t[m] = ldexp(nearbyint(ldexp(0.5 * (1.0 + x[m]), 40)), -40);
        w[m] = ldexp(nearbyint(ldexp(1.0 / ((1.0 - x[m] * x[m]) * dp * dp), 40)), -40);
    }
    return 0;
}

/* sigma = eps_out / (eps_in + eps_out), the exponent of the line image. */
static double sigma_of(const orc_params *P) { return P->eps_out / (P->eps_in + P->eps_out); }

/* Image kernel K(x, y): the potential at x of the images of a unit charge at y
 * (both outside the sphere), symmetric in x and y:
 *   gamma a / sqrt(D_1) - sigma gamma a sum_m w_m / sqrt(D_{t_m}),
 *   D_t = |y|^2 |x - t y_K|^2 = |x|^2 |y|^2 - 2 t a^2 x.y + t^2 a^4. */
typedef struct { int M; double sigma, t[8], w[8]; } orc_lines;

static void lines_of(const orc_params *P, orc_lines *L) {
    L->M = 0;
    L->sigma = sigma_of(P);
    if (P->images && P->line_images > 0 && orc_line_rule(L->sigma, P->line_images, L->t, L->w) == 0)
        L->M = P->line_images;
}

/* the line part alone: - sigma gamma a sum_m w_m / sqrt(D_{t_m}) */
static double line_kernel(const orc_params *P, const orc_lines *L, double xi, double yi, double zi,
                          double xj, double yj, double zj) {
    double a = P->a, a2 = a * a, g = gamma_of(P);
    double ri2 = xi * xi + yi * yi + zi * zi;
    double rj2 = xj * xj + yj * yj + zj * zj;
    double dot = xi * xj + yi * yj + zi * zj;
    double v = 0.0;
    for (int m = 0; m < L->M; ++m) {
        double tt = L->t[m];
        v -= L->sigma * L->w[m] * g * a / sqrt(ri2 * rj2 - 2.0 * tt * a2 * dot + tt * tt * a2 * a2);
    }
    return v;
}

static double image_kernel(const orc_params *P, const orc_lines *L, double xi, double yi, double zi,
                           double xj, double yj, double zj) {
    double a = P->a, a2 = a * a, g = gamma_of(P);
    double ri2 = xi * xi + yi * yi + zi * zi;
    double rj2 = xj * xj + yj * yj + zj * zj;
    double dot = xi * xj + yi * yj + zi * zj;
    return g * a / sqrt(ri2 * rj2 - 2.0 * a2 * dot + a2 * a2) + line_kernel(P, L, xi, yi, zi, xj, yj, zj);
}

/* Self term of the line images of a charge q at squared radius r2:
 * 1/2 q^2 sum_m (-sigma w_m gamma a) / (r2 - t_m a^2), since the line image at
 * t_m r_K lies on the ion's own ray at distance (r2 - t_m a^2) / |r|. */
static double line_self(const orc_params *P, const orc_lines *L, double q, double r2) {
    double a = P->a, g = gamma_of(P), v = 0.0;
    for (int m = 0; m < L->M; ++m) v += -0.5 * L->sigma * L->w[m] * g * a * q * q / (r2 - L->t[m] * a * a);
    return v;
}

/* Hard walls (Sec. 4): a move leaving the cell is rejected. */
static int outside(const orc_params *P, double x, double y, double z) {
    if (P->geom == 0) {
        double hi0 = P->box_lo[0] + P->box_side, hi1 = P->box_lo[1] + P->box_side,
               hi2 = P->box_lo[2] + P->box_side;
        return x < P->box_lo[0] || x >= hi0 || y < P->box_lo[1] || y >= hi1 ||
               z < P->box_lo[2] || z >= hi2;
    }
    double r2 = x * x + y * y + z * z;
    return r2 <= P->r_min * P->r_min || r2 >= P->r_max * P->r_max;
}

static int in_root(const orc_params *P, double x, double y, double z) {
    return x >= P->box_lo[0] && x < P->box_lo[0] + P->box_side &&
           y >= P->box_lo[1] && y < P->box_lo[1] + P->box_side &&
           z >= P->box_lo[2] && z < P->box_lo[2] + P->box_side;
}

/* 21 bits per axis; digit of level l (root = 0) is bits [62-3l, 60-3l] of the
 * key = 4 * x bit + 2 * y bit + z bit (Sec. 3.2: bisection in each direction). */
static uint32_t quantize(double v, double lo, double scale) {
    double f = floor((v - lo) * scale);
    uint32_t k = (uint32_t)f;
    return k > 2097151u ? 2097151u : k;
}

static uint64_t morton(uint32_t kx, uint32_t ky, uint32_t kz) {
    uint64_t key = 0;
    for (int b = 0; b < 21; ++b) {
        key |= (uint64_t)((kx >> b) & 1u) << (3 * b + 2);
        key |= (uint64_t)((ky >> b) & 1u) << (3 * b + 1);
        key |= (uint64_t)((kz >> b) & 1u) << (3 * b);
    }
    return key;
}

static uint64_t key_of(const orc_params *P, double x, double y, double z) {
    double scale = 2097152.0 / P->box_side;
    return morton(quantize(x, P->box_lo[0], scale), quantize(y, P->box_lo[1], scale),
                  quantize(z, P->box_lo[2], scale));
}

void orc_keys(const orc_params *P, int64_t n, const double *x, const double *y, const double *z,
              uint64_t *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = key_of(P, x[i], y[i], z[i]);
}

static int digit_at(uint64_t key, int level /* >= 1 */) {
    return (int)((key >> (63 - 3 * level)) & 7u);
}

/* ------------------------------------------------------------------------ */
/* Direct summation (eq. 1.1, eq. 2.1) with the symmetric image kernel       */
/*   q_i q_Kj / |r_i - r_Kj| = gamma a q_i q_j / sqrt(D_ij),                 */
/*   D_ij = |r_i|^2 |r_j|^2 - 2 a^2 r_i.r_j + a^4.                           */
/* ------------------------------------------------------------------------ */

static double img_D(double a, double xi, double yi, double zi, double xj, double yj, double zj) {
    double ri2 = xi * xi + yi * yi + zi * zi;
    double rj2 = xj * xj + yj * yj + zj * zj;
    double dot = xi * xj + yi * yj + zi * zj;
    return ri2 * rj2 - 2.0 * a * a * dot + a * a * a * a;
}

/* Direct energy: l_B [ sum_{i<j} q_i q_j / r_ij
 *                      + 1/2 sum_i sum_j gamma a q_i q_j / sqrt(D_ij)   (images, incl. j = i)
 *                      + Q_M sum_i q_i / |r_i| ]                        (central charge)     */
double orc_direct_energy(const orc_params *P, int64_t n, const double *x, const double *y,
                         const double *z, const double *q) {
    nsum e = {0, 0};
    int shell = P->geom == 1;
    orc_lines L;
    lines_of(P, &L);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            nadd(&e, q[i] * q[j] / sqrt(dx * dx + dy * dy + dz * dz));
        }
        if (shell && P->images) {
            for (int64_t j = 0; j < n; ++j)
                nadd(&e, 0.5 * q[i] * q[j] * image_kernel(P, &L, x[i], y[i], z[i], x[j], y[j], z[j]));
        }
        if (shell && P->Q_center != 0.0)
            nadd(&e, P->Q_center * q[i] / sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]));
    }
    return P->l_B * nval(&e);
}

/* Direct energy change for moving ion i to rn: the per-j differences are
 * summed (Sec. 1: V_i evaluated at the old and the new position). */
double orc_direct_delta(const orc_params *P, int64_t n, const double *x, const double *y,
                        const double *z, const double *q, int64_t i, const double *rn) {
    nsum e = {0, 0};
    int shell = P->geom == 1;
    double g = gamma_of(P), a = P->a;
    orc_lines L;
    lines_of(P, &L);
    double xo = x[i], yo = y[i], zo = z[i];
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = rn[0] - x[j], dy = rn[1] - y[j], dz = rn[2] - z[j];
        double ex = xo - x[j], ey = yo - y[j], ez = zo - z[j];
        double t = q[j] / sqrt(dx * dx + dy * dy + dz * dz) - q[j] / sqrt(ex * ex + ey * ey + ez * ez);
        if (shell && P->images) {
            double Dn = img_D(a, rn[0], rn[1], rn[2], x[j], y[j], z[j]);
            double Do = img_D(a, xo, yo, zo, x[j], y[j], z[j]);
            t += g * a * q[j] * (1.0 / sqrt(Dn) - 1.0 / sqrt(Do));
            if (L.M)
                t += q[j] * (line_kernel(P, &L, rn[0], rn[1], rn[2], x[j], y[j], z[j]) -
                             line_kernel(P, &L, xo, yo, zo, x[j], y[j], z[j]));
        }
        nadd(&e, q[i] * t);
    }
    if (shell && P->images) {
        double rn2 = rn[0] * rn[0] + rn[1] * rn[1] + rn[2] * rn[2];
        double ro2 = xo * xo + yo * yo + zo * zo;
        nadd(&e, 0.5 * g * a * q[i] * q[i] * (1.0 / (rn2 - a * a) - 1.0 / (ro2 - a * a)));
        if (L.M) nadd(&e, line_self(P, &L, q[i], rn2) - line_self(P, &L, q[i], ro2));
    }
    if (shell && P->Q_center != 0.0) {
        double rn1 = sqrt(rn[0] * rn[0] + rn[1] * rn[1] + rn[2] * rn[2]);
        double ro1 = sqrt(xo * xo + yo * yo + zo * zo);
        nadd(&e, P->Q_center * q[i] * (1.0 / rn1 - 1.0 / ro1));
    }
    return P->l_B * nval(&e);
}

/* Per-ion potential from every other ion and from the images of every other
 * ion (the part the treecode approximates), at the ion's own position:
 * phi_i = sum_{j != i} q_j / r_ij + sum_{j != i} gamma a q_j / sqrt(D_ij). */
void orc_direct_phi(const orc_params *P, int64_t n, const double *x, const double *y,
                    const double *z, const double *q, double *phi) {
    int imgs = P->geom == 1 && P->images;
    orc_lines L;
    lines_of(P, &L);
    for (int64_t i = 0; i < n; ++i) {
        nsum e = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            nadd(&e, q[j] / sqrt(dx * dx + dy * dy + dz * dz));
            if (imgs) nadd(&e, q[j] * image_kernel(P, &L, x[i], y[i], z[i], x[j], y[j], z[j]));
        }
        phi[i] = nval(&e);
    }
}

/* Gradient of the direct energy: dE/dr_i (3 per ion) and dE/dq_i. */
void orc_direct_grad(const orc_params *P, int64_t n, const double *x, const double *y,
                     const double *z, const double *q, double *gx, double *gy, double *gz,
                     double *gq) {
    int shell = P->geom == 1, imgs = shell && P->images;
    double g = gamma_of(P), a = P->a, a2 = a * a;
    orc_lines L;
    lines_of(P, &L);
    for (int64_t i = 0; i < n; ++i) {
        nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0}, sq = {0, 0};
        double ri2 = x[i] * x[i] + y[i] * y[i] + z[i] * z[i];
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2), ir3 = 1.0 / (r2 * r);
            nadd(&sx, -q[i] * q[j] * dx * ir3);
            nadd(&sy, -q[i] * q[j] * dy * ir3);
            nadd(&sz, -q[i] * q[j] * dz * ir3);
            nadd(&sq, q[j] / r);
            if (imgs) {
                double rj2 = x[j] * x[j] + y[j] * y[j] + z[j] * z[j];
                double D = img_D(a, x[i], y[i], z[i], x[j], y[j], z[j]);
                double iD12 = 1.0 / sqrt(D), iD32 = iD12 / D;
                double c = -g * a * q[i] * q[j] * iD32;
                nadd(&sx, c * (rj2 * x[i] - a2 * x[j]));
                nadd(&sy, c * (rj2 * y[i] - a2 * y[j]));
                nadd(&sz, c * (rj2 * z[i] - a2 * z[j]));
                nadd(&sq, g * a * q[j] * iD12);
                /* line image m of either ion: coefficient -sigma w_m on the kernel with
                 * D_t = |r_i|^2 |r_j|^2 - 2 t a^2 r_i.r_j + t^2 a^4 */
                double dot = x[i] * x[j] + y[i] * y[j] + z[i] * z[j];
                for (int m = 0; m < L.M; ++m) {
                    double tt = L.t[m], cm = -L.sigma * L.w[m];
                    double Dt = ri2 * rj2 - 2.0 * tt * a2 * dot + tt * tt * a2 * a2;
                    double iDt12 = 1.0 / sqrt(Dt), iDt32 = iDt12 / Dt;
                    double ct = -cm * g * a * q[i] * q[j] * iDt32;
                    nadd(&sx, ct * (rj2 * x[i] - tt * a2 * x[j]));
                    nadd(&sy, ct * (rj2 * y[i] - tt * a2 * y[j]));
                    nadd(&sz, ct * (rj2 * z[i] - tt * a2 * z[j]));
                    nadd(&sq, cm * g * a * q[j] * iDt12);
                }
            }
        }
        if (imgs) {
            double den = ri2 - a2;
            double c = -g * a * q[i] * q[i] / (den * den);
            nadd(&sx, c * x[i]); nadd(&sy, c * y[i]); nadd(&sz, c * z[i]);
            nadd(&sq, g * a * q[i] / den);
            /* own line images: 1/2 c_m gamma a q^2 / (r^2 - t_m a^2) */
            for (int m = 0; m < L.M; ++m) {
                double cm = -L.sigma * L.w[m], dm = ri2 - L.t[m] * a2;
                double cl = -cm * g * a * q[i] * q[i] / (dm * dm);
                nadd(&sx, cl * x[i]); nadd(&sy, cl * y[i]); nadd(&sz, cl * z[i]);
                nadd(&sq, cm * g * a * q[i] / dm);
            }
        }
        if (shell && P->Q_center != 0.0) {
            double r = sqrt(ri2), ir3 = 1.0 / (ri2 * r);
            nadd(&sx, -P->Q_center * q[i] * x[i] * ir3);
            nadd(&sy, -P->Q_center * q[i] * y[i] * ir3);
            nadd(&sz, -P->Q_center * q[i] * z[i] * ir3);
            nadd(&sq, P->Q_center / r);
        }
        gx[i] = P->l_B * nval(&sx); gy[i] = P->l_B * nval(&sy); gz[i] = P->l_B * nval(&sz);
        gq[i] = P->l_B * nval(&sq);
    }
}

/* ------------------------------------------------------------------------ */
/* Treecode (Sec. 3.2-3.3)                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int level;
    uint32_t ix, iy, iz;     /* integer coordinates at this level           */
    uint64_t kmin;           /* smallest key in the cell                    */
    double cx, cy, cz, h;    /* centre and half side; rho = sqrt(3) h       */
    int count;               /* N_A                                         */
    int child[8];            /* -1 for a leaf                               */
    int parent;
    int leaf;                /* leaf id, -1 for an internal cell            */
    int begin, end;          /* range in the sorted order at build          */
} ocell;

typedef struct {
    int cell, count, cap;
    int *slot;               /* index array of the leaf (Sec. 3.2, item 5)   */
} oleaf;

typedef struct {
    int64_t visited, far, near_src;
} ocount;

typedef struct otree {
    orc_params P;
    double gamma, theta2;
    int n, nsrc, nterms, pmax1;
    double *x, *y, *z, *q;   /* sources: ions 0..n-1, images n..2n-1          */
    uint64_t *skey;          /* keys in sorted order at build               */
    int *perm;               /* sorted order of source indices at build     */
    ocell *cell; int ncell, capcell;
    oleaf *leaf; int nleaf, capleaf;
    double *M;               /* ncell * nterms moments (eq. 3.3)            */
    int *leaf_of, *slot_of;  /* tracking information (Sec. 3.3)             */
    int *mi;                 /* multi-indices up to order p + 1             */
    ocount cnt;              /* interaction counters of the last evaluation */
} otree;

typedef struct { uint64_t key; int idx; } kidx;

static int cmp_kidx(const void *A, const void *B) {
    const kidx *a = (const kidx *)A, *b = (const kidx *)B;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

static int new_cell(otree *t) {
    if (t->ncell == t->capcell) {
        t->capcell = t->capcell ? 2 * t->capcell : 64;
        t->cell = (ocell *)realloc(t->cell, sizeof(ocell) * t->capcell);
    }
    memset(&t->cell[t->ncell], 0, sizeof(ocell));
    return t->ncell++;
}

static int new_leaf(otree *t) {
    if (t->nleaf == t->capleaf) {
        t->capleaf = t->capleaf ? 2 * t->capleaf : 64;
        t->leaf = (oleaf *)realloc(t->leaf, sizeof(oleaf) * t->capleaf);
    }
    memset(&t->leaf[t->nleaf], 0, sizeof(oleaf));
    return t->nleaf++;
}

/* Recursive bisection (Sec. 3.2): a cell is split into its 8 children iff it
 * holds more than leaf_cap sources and is above max_depth; every child is
 * made, empty or not, so that every point of the root lies in one leaf. */
static int build_cell(otree *t, int level, uint32_t ix, uint32_t iy, uint32_t iz, int begin,
                      int end, int parent) {
    int c = new_cell(t);
    ocell *A = &t->cell[c];
    const orc_params *P = &t->P;
    A->level = level; A->ix = ix; A->iy = iy; A->iz = iz;
    A->kmin = level == 0 ? 0 : morton(ix << (21 - level), iy << (21 - level), iz << (21 - level));
    A->h = ldexp(P->box_side, -(level + 1));
    A->cx = P->box_lo[0] + (double)(2u * ix + 1u) * A->h;
    A->cy = P->box_lo[1] + (double)(2u * iy + 1u) * A->h;
    A->cz = P->box_lo[2] + (double)(2u * iz + 1u) * A->h;
    A->count = end - begin;
    A->parent = parent;
    A->begin = begin; A->end = end;
    for (int d = 0; d < 8; ++d) A->child[d] = -1;
    A->leaf = -1;
    if (end - begin > P->leaf_cap && level < P->max_depth) {
        int b = begin;
        for (int d = 0; d < 8; ++d) {
            int e = b;
            while (e < end && digit_at(t->skey[e], level + 1) == d) ++e;
            uint32_t cx = 2u * ix + ((d >> 2) & 1u), cy = 2u * iy + ((d >> 1) & 1u),
                     cz = 2u * iz + (d & 1u);
            int ch = build_cell(t, level + 1, cx, cy, cz, b, e, c);
            t->cell[c].child[d] = ch;
            b = e;
        }
    } else {
        int l = new_leaf(t);
        oleaf *L = &t->leaf[l];
        int cnt = end - begin;
        int base = cnt > P->leaf_cap ? cnt : P->leaf_cap;
        L->cell = c;
        L->count = cnt;
        /* one move inserts at most the ion and its images: 2 + M sources */
        L->cap = P->slot_slack * base + 2 + P->line_images;
        L->slot = (int *)malloc(sizeof(int) * (L->cap > 0 ? L->cap : 1));
        for (int k = 0; k < cnt; ++k) {
            int s = t->perm[begin + k];
            L->slot[k] = s;
            t->leaf_of[s] = l;
            t->slot_of[s] = k;
        }
        t->cell[c].leaf = l;
    }
    return c;
}

/* Moments about the geometric centre, summed directly over the members of
 * each cell (eq. 3.3): M_A^n = sum_{j in A} q_j (r_j - r_A)^n. */
static void cell_moments_direct(otree *t, int c, double *mono) {
    ocell *A = &t->cell[c];
    double *M = t->M + (size_t)c * t->nterms;
    for (int k = 0; k < t->nterms; ++k) M[k] = 0.0;
    for (int r = A->begin; r < A->end; ++r) {
        int j = t->perm[r];
        monomials(t->P.p, t->mi, t->x[j] - A->cx, t->y[j] - A->cy, t->z[j] - A->cz, mono);
        for (int k = 0; k < t->nterms; ++k) M[k] += t->q[j] * mono[k];
    }
}

static int validate(const orc_params *P, int64_t n, const double *x, const double *y,
                    const double *z) {
    if (n <= 0 || !(P->theta >= 0.0 && P->theta < 1.0) || P->p < 0 || P->p > 20 ||
        P->leaf_cap < 0 || P->max_depth < 0 || P->max_depth > 21 || P->slot_slack < 1 ||
        !(P->box_side > 0.0) || P->n0 < 0)
        return ORC_EINVAL;
    if (P->images && P->geom != 1) return ORC_EINVAL;
    if (P->line_images < 0 || P->line_images > 8 || (P->line_images && !P->images)) return ORC_EINVAL;
    if (P->line_images && !(sigma_of(P) >= 0.5 && sigma_of(P) <= 1.0)) return ORC_EINVAL;
    if (P->geom == 1) /* the root cube must contain the shell |r| < r_max */
        for (int d = 0; d < 3; ++d)
            if (!(P->box_lo[d] <= -P->r_max && P->box_lo[d] + P->box_side >= P->r_max)) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) return ORC_EINVAL;
        if (outside(P, x[i], y[i], z[i]) || !in_root(P, x[i], y[i], z[i])) return ORC_EOUTSIDE;
    }
    return ORC_OK;
}

void orc_tree_free(otree *t) {
    if (!t) return;
    for (int l = 0; l < t->nleaf; ++l) free(t->leaf[l].slot);
    free(t->leaf); free(t->cell); free(t->M);
    free(t->x); free(t->y); free(t->z); free(t->q);
    free(t->skey); free(t->perm); free(t->leaf_of); free(t->slot_of); free(t->mi);
    free(t);
}

/* Build the octree and tracking information over the ions and their images
 * (Sec. 3.3: "the octree structure and the tracking information for each
 * particle are built" once, before the Monte Carlo steps). */
int orc_tree_build(const orc_params *P, int64_t n, const double *x, const double *y,
                   const double *z, const double *q, otree **out) {
    *out = NULL;
    int st = validate(P, n, x, y, z);
    if (st) return st;
    otree *t = (otree *)calloc(1, sizeof(otree));
    t->P = *P;
    t->gamma = gamma_of(P);
    t->theta2 = P->theta * P->theta;
    t->n = (int)n;
    t->nsrc = P->images ? (2 + P->line_images) * (int)n : (int)n;
    t->nterms = nterms_of(P->p);
    t->pmax1 = P->p + 1;
    int ns = t->nsrc;
    t->x = (double *)malloc(sizeof(double) * ns); t->y = (double *)malloc(sizeof(double) * ns);
    t->z = (double *)malloc(sizeof(double) * ns); t->q = (double *)malloc(sizeof(double) * ns);
    for (int i = 0; i < n; ++i) { t->x[i] = x[i]; t->y[i] = y[i]; t->z[i] = z[i]; t->q[i] = q[i]; }
    if (P->images) {
        orc_lines L;
        lines_of(P, &L);
        for (int i = 0; i < n; ++i) {
            double im[4];
            orc_kelvin(P->a, t->gamma, x[i], y[i], z[i], q[i], im);
            t->x[n + i] = im[0]; t->y[n + i] = im[1]; t->z[n + i] = im[2]; t->q[n + i] = im[3];
            if (!in_root(P, im[0], im[1], im[2])) { orc_tree_free(t); return ORC_EOUTSIDE; }
            /* line images of ion i: source 2n + m n + i, charge -sigma w_m q_K at t_m r_K */
            for (int m = 0; m < L.M; ++m) {
                int s = 2 * (int)n + m * (int)n + i;
                t->x[s] = L.t[m] * im[0]; t->y[s] = L.t[m] * im[1]; t->z[s] = L.t[m] * im[2];
                t->q[s] = -L.sigma * L.w[m] * im[3];
            }
        }
    }
    t->mi = (int *)malloc(sizeof(int) * 3 * nterms_of(P->p + 1));
    multi_indices(P->p + 1, t->mi);
    /* keys and the stable sort: ascending key, ties by source index */
    kidx *ki = (kidx *)malloc(sizeof(kidx) * ns);
    for (int s = 0; s < ns; ++s) { ki[s].key = key_of(P, t->x[s], t->y[s], t->z[s]); ki[s].idx = s; }
    qsort(ki, ns, sizeof(kidx), cmp_kidx);
    t->skey = (uint64_t *)malloc(sizeof(uint64_t) * ns);
    t->perm = (int *)malloc(sizeof(int) * ns);
    for (int s = 0; s < ns; ++s) { t->skey[s] = ki[s].key; t->perm[s] = ki[s].idx; }
    free(ki);
    t->leaf_of = (int *)malloc(sizeof(int) * ns);
    t->slot_of = (int *)malloc(sizeof(int) * ns);
    build_cell(t, 0, 0, 0, 0, 0, ns, -1);
    t->M = (double *)malloc(sizeof(double) * (size_t)t->ncell * t->nterms);
    double *mono = (double *)malloc(sizeof(double) * t->nterms);
    for (int c = 0; c < t->ncell; ++c) cell_moments_direct(t, c, mono);
    free(mono);
    *out = t;
    return ORC_OK;
}

/* Is source s a member of cell c?  Walk up from the leaf holding s. */
static int contains(const otree *t, int c, int s) {
    for (int a = t->leaf[t->leaf_of[s]].cell; a >= 0; a = t->cell[a].parent)
        if (a == c) return 1;
    return 0;
}

typedef struct {
    const int *ex; int nex;  /* sources removed from the source set           */
    nsum acc;
    int coincide;            /* a near source at distance exactly 0            */
    double *T, *mono, *Mp;
    ocount cnt;
    double farabs;           /* sum over far cells of sum_n |T_n M'_n|            */
} vstate;

static void direct_cell(const otree *t, int c, const double *xt, vstate *v) {
    const ocell *A = &t->cell[c];
    if (A->leaf >= 0) {
        const oleaf *L = &t->leaf[A->leaf];
        for (int k = 0; k < L->count; ++k) {
            int j = L->slot[k];
            int skip = 0;
            for (int e = 0; e < v->nex; ++e) skip |= (j == v->ex[e]);
            if (skip) continue;
            double dx = xt[0] - t->x[j], dy = xt[1] - t->y[j], dz = xt[2] - t->z[j];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 == 0.0) { v->coincide = 1; continue; }
            nadd(&v->acc, t->q[j] / sqrt(d2));
            v->cnt.near_src++;
        }
    } else {
        for (int d = 0; d < 8; ++d) direct_cell(t, A->child[d], xt, v);
    }
}

/* Far value of cell c at the target: sum_n T_n(r_A - x) M'_A^n, where M'
 * removes the excluded members (eq. 3.3 over the remaining sources). */
static double far_value(const otree *t, int c, const double *xt, vstate *v) {
    const ocell *A = &t->cell[c];
    const double *M = t->M + (size_t)c * t->nterms;
    for (int k = 0; k < t->nterms; ++k) v->Mp[k] = M[k];
    for (int e = 0; e < v->nex; ++e) {
        int s = v->ex[e];
        if (!contains(t, c, s)) continue;
        monomials(t->P.p, t->mi, t->x[s] - A->cx, t->y[s] - A->cy, t->z[s] - A->cz, v->mono);
        for (int k = 0; k < t->nterms; ++k) v->Mp[k] = v->Mp[k] - t->q[s] * v->mono[k];
    }
    taylor(t->P.p, t->mi, A->cx - xt[0], A->cy - xt[1], A->cz - xt[2], v->T);
    double val = 0.0;
    for (int k = 0; k < t->nterms; ++k) {
        val += v->T[k] * v->Mp[k];
        v->farabs += fabs(v->T[k] * v->Mp[k]);
    }
    return val;
}

/* Traversal from the root (Sec. 3.2): the multipole approximation is used iff
 * the MAC rho_A / r_{i,A} <= theta holds and N_A >= N_0; otherwise the cell is
 * opened if N_A > N_0 and it is not a leaf; otherwise its sources are summed
 * directly.  rho_A = sqrt(3) h, so the MAC is tested as 3 h^2 <= theta^2 d^2. */
static void visit(const otree *t, int c, const double *xt, vstate *v) {
    const ocell *A = &t->cell[c];
    int nin = 0;
    for (int e = 0; e < v->nex; ++e) nin += contains(t, c, v->ex[e]);
    int np = A->count - nin;
    if (np == 0) return;
    v->cnt.visited++;
    double dx = A->cx - xt[0], dy = A->cy - xt[1], dz = A->cz - xt[2];
    double d2 = dx * dx + dy * dy + dz * dz;
    int mac = 3.0 * (A->h * A->h) <= t->theta2 * d2;
    if (mac && np >= t->P.n0) {
        nadd(&v->acc, far_value(t, c, xt, v));
        v->cnt.far++;
    } else if (np > t->P.n0 && A->leaf < 0) {
        for (int d = 0; d < 8; ++d) visit(t, A->child[d], xt, v);
    } else {
        direct_cell(t, c, xt, v);
    }
}

/* potential at xt from all sources except ex[0..nex); farabs (nullable) receives
 * the sum over far cells of sum_n |T_n M'_n| */
static double tree_phi_abs(otree *t, const double *xt, const int *ex, int nex, int *coincide,
                           double *farabs);
static double tree_phi(otree *t, const double *xt, const int *ex, int nex, int *coincide) {
    return tree_phi_abs(t, xt, ex, nex, coincide, NULL);
}
static double tree_phi_abs(otree *t, const double *xt, const int *ex, int nex, int *coincide,
                           double *farabs) {
    vstate v;
    memset(&v, 0, sizeof(v));
    v.ex = ex; v.nex = nex;
    v.T = (double *)malloc(sizeof(double) * t->nterms);
    v.mono = (double *)malloc(sizeof(double) * t->nterms);
    v.Mp = (double *)malloc(sizeof(double) * t->nterms);
    visit(t, 0, xt, &v);
    free(v.T); free(v.mono); free(v.Mp);
    t->cnt.visited += v.cnt.visited; t->cnt.far += v.cnt.far; t->cnt.near_src += v.cnt.near_src;
    if (coincide) *coincide = v.coincide;
    if (farabs) *farabs = v.farabs;
    return nval(&v.acc);
}

/* Magnitude of the far field at xt: sum over the cells the traversal expands of
 * sum_n |T_n(r_A - x) M'^n_A| (eq. 3.3 term by term), the scale of the rounding of
 * a far-field evaluation in a lower precision. */
double orc_tree_far_magnitude(otree *t, const double *xt, const int *ex, int nex) {
    double fa = 0.0;
    tree_phi_abs(t, xt, ex, nex, NULL, &fa);
    return fa;
}

double orc_tree_phi(otree *t, const double *xt, const int *ex, int nex) {
    return tree_phi(t, xt, ex, nex, NULL);
}

/* The same potential with the traversal's counts of that one target:
 * counts = [cells visited (holding a remaining source), cells taken as far,
 * sources summed directly]. */
double orc_tree_phi_counts(otree *t, const double *xt, const int *ex, int nex, int64_t *counts) {
    memset(&t->cnt, 0, sizeof(t->cnt));
    double v = tree_phi(t, xt, ex, nex, NULL);
    counts[0] = t->cnt.visited; counts[1] = t->cnt.far; counts[2] = t->cnt.near_src;
    return v;
}

static int overlaps(const otree *t, int64_t i, const double *rn) {
    double tau2 = t->P.hard_core * t->P.hard_core;
    for (int j = 0; j < t->n; ++j) {
        if (j == i) continue;
        double dx = rn[0] - t->x[j], dy = rn[1] - t->y[j], dz = rn[2] - t->z[j];
        if (dx * dx + dy * dy + dz * dz <= tau2) return 1;
    }
    return 0;
}

/* Energy change of moving ion i to rn on the committed tree:
 *   l_B q_i [phi_X(rn) - phi_X(r_i)] + exact self-image change + exact
 *   central-charge change, X = {i and all of its images}.
 * A move that leaves the cell (Sec. 4) or overlaps a hard core (eq. 2.1)
 * has dE = +inf and a reason code. */
double orc_tree_delta(otree *t, int64_t i, const double *rn, int *reason, int64_t *counts) {
    *reason = REASON_NONE;
    memset(&t->cnt, 0, sizeof(t->cnt));
    if (outside(&t->P, rn[0], rn[1], rn[2])) { *reason = REASON_WALL; return INFINITY; }
    if (overlaps(t, i, rn)) { *reason = REASON_OVERLAP; return INFINITY; }
    int M = t->P.images ? t->P.line_images : 0;
    int ex[10] = {(int)i, t->n + (int)i};
    for (int m = 0; m < M; ++m) ex[2 + m] = 2 * t->n + m * t->n + (int)i;
    int nex = t->P.images ? 2 + M : 1;
    double ro[3] = {t->x[i], t->y[i], t->z[i]};
    int coin = 0;
    double pn = tree_phi(t, rn, ex, nex, &coin);
    if (coin) { *reason = REASON_OVERLAP; return INFINITY; }
    double po = tree_phi(t, ro, ex, nex, NULL);
    double qi = t->q[i], l = t->P.l_B;
    double dE = l * qi * (pn - po);
    if (t->P.geom == 1) {
        double a = t->P.a;
        double rn2 = rn[0] * rn[0] + rn[1] * rn[1] + rn[2] * rn[2];
        double ro2 = ro[0] * ro[0] + ro[1] * ro[1] + ro[2] * ro[2];
        if (t->P.images)
            dE += 0.5 * l * t->gamma * a * qi * qi * (1.0 / (rn2 - a * a) - 1.0 / (ro2 - a * a));
        if (M) {
            orc_lines L;
            lines_of(&t->P, &L);
            dE += l * (line_self(&t->P, &L, qi, rn2) - line_self(&t->P, &L, qi, ro2));
        }
        if (t->P.Q_center != 0.0)
            dE += l * t->P.Q_center * qi * (1.0 / sqrt(rn2) - 1.0 / sqrt(ro2));
    }
    if (counts) { counts[0] = t->cnt.visited; counts[1] = t->cnt.far; counts[2] = t->cnt.near_src; }
    return dE;
}

/* Leaf that holds a position: descend from the root by the key's digits. */
static int leaf_for(const otree *t, uint64_t key) {
    int c = 0;
    while (t->cell[c].leaf < 0) c = t->cell[c].child[digit_at(key, t->cell[c].level + 1)];
    return t->cell[c].leaf;
}

/* Would the add operations of this move overflow a leaf's index array?  The
 * moved sources (the ion, then its images in source order) are placed one after
 * another, so each one's new leaf is checked with the counts the earlier ones
 * leave behind. */
static int capacity_ok(const otree *t, int ns, const int *src, const double (*pos)[4]) {
    int leaf_o[10], leaf_n[10];
    for (int k = 0; k < ns; ++k) {
        leaf_o[k] = t->leaf_of[src[k]];
        leaf_n[k] = leaf_for(t, key_of(&t->P, pos[k][0], pos[k][1], pos[k][2]));
    }
    for (int k = 0; k < ns; ++k) {
        if (leaf_n[k] == leaf_o[k]) continue;
        int c = t->leaf[leaf_n[k]].count;
        for (int e = 0; e < k; ++e) {
            if (leaf_n[e] == leaf_o[e]) continue;
            if (leaf_n[e] == leaf_n[k]) c += 1;
            if (leaf_o[e] == leaf_n[k]) c -= 1;
        }
        if (c + 1 > t->leaf[leaf_n[k]].cap) return 0;
    }
    return 1;
}

/* Local modification of one source (Sec. 3.3, Fig. 3): if it changes leaf,
 * delete it from the old index array (the last entry fills the hole and its
 * tracking is updated) and append it to the new one; then remove the old
 * contribution from the moments and counts of every ancestor of the old
 * leaf, and add the new contribution along the new leaf's ancestors. */
static void move_source(otree *t, int s, double xn, double yn, double zn, double qn, double *mono) {
    int lo = t->leaf_of[s];
    int ln = leaf_for(t, key_of(&t->P, xn, yn, zn));
    if (ln != lo) {
        oleaf *L = &t->leaf[lo];
        int k = t->slot_of[s], last = L->count - 1;
        int moved = L->slot[last];
        L->slot[k] = moved;
        t->slot_of[moved] = k;
        L->count--;
        oleaf *N = &t->leaf[ln];
        N->slot[N->count] = s;
        t->slot_of[s] = N->count;
        N->count++;
        t->leaf_of[s] = ln;
    }
    double xo = t->x[s], yo = t->y[s], zo = t->z[s], qo = t->q[s];
    for (int c = t->leaf[lo].cell; c >= 0; c = t->cell[c].parent) {
        ocell *A = &t->cell[c];
        double *M = t->M + (size_t)c * t->nterms;
        monomials(t->P.p, t->mi, xo - A->cx, yo - A->cy, zo - A->cz, mono);
        for (int k = 0; k < t->nterms; ++k) M[k] = M[k] - qo * mono[k];
        A->count--;
    }
    for (int c = t->leaf[ln].cell; c >= 0; c = t->cell[c].parent) {
        ocell *A = &t->cell[c];
        double *M = t->M + (size_t)c * t->nterms;
        monomials(t->P.p, t->mi, xn - A->cx, yn - A->cy, zn - A->cz, mono);
        for (int k = 0; k < t->nterms; ++k) M[k] = M[k] + qn * mono[k];
        A->count++;
    }
    t->x[s] = xn; t->y[s] = yn; t->z[s] = zn; t->q[s] = qn;
}

/* Commit an accepted move of ion i to rn: the ion, then its Kelvin image, then
 * its line images m = 0 .. M-1 (placed as the build places them). */
int orc_tree_commit(otree *t, int64_t i, const double *rn) {
    if (i < 0 || i >= t->n) return ORC_EINVAL;
    if (outside(&t->P, rn[0], rn[1], rn[2])) return ORC_EINVAL;
    int src[10], ns = 1;
    double pos[10][4];
    src[0] = (int)i;
    pos[0][0] = rn[0]; pos[0][1] = rn[1]; pos[0][2] = rn[2]; pos[0][3] = t->q[i];
    if (t->P.images) {
        double imn[4];
        orc_kelvin(t->P.a, t->gamma, rn[0], rn[1], rn[2], t->q[i], imn);
        src[1] = t->n + (int)i;
        for (int k = 0; k < 4; ++k) pos[1][k] = imn[k];
        ns = 2;
        orc_lines L;
        lines_of(&t->P, &L);
        for (int m = 0; m < L.M; ++m, ++ns) {
            src[ns] = 2 * t->n + m * t->n + (int)i;
            pos[ns][0] = L.t[m] * imn[0]; pos[ns][1] = L.t[m] * imn[1]; pos[ns][2] = L.t[m] * imn[2];
            pos[ns][3] = -L.sigma * L.w[m] * imn[3];
        }
    }
    if (!capacity_ok(t, ns, src, (const double (*)[4])pos)) return ORC_ECAPACITY;
    double *mono = (double *)malloc(sizeof(double) * t->nterms);
    for (int k = 0; k < ns; ++k) move_source(t, src[k], pos[k][0], pos[k][1], pos[k][2], pos[k][3], mono);
    free(mono);
    return ORC_OK;
}

/* Treecode energy:
 *   E = l_B [ 1/2 sum_i q_i phi_{X_i}(r_i) + 1/2 sum_i gamma a q_i^2 / (|r_i|^2 - a^2)
 *             + Q_M sum_i q_i / |r_i| ],   X_i = {i, image of i}.
 * phi_out (nullable) receives phi_{X_i}(r_i). */
double orc_tree_energy(otree *t, double *phi_out) {
    nsum e = {0, 0};
    int M = t->P.images ? t->P.line_images : 0;
    int nex = t->P.images ? 2 + M : 1;
    double a = t->P.a;
    orc_lines L;
    lines_of(&t->P, &L);
    for (int i = 0; i < t->n; ++i) {
        int ex[10] = {i, t->n + i};  /* the ion and all of its images */
        for (int m = 0; m < M; ++m) ex[2 + m] = 2 * t->n + m * t->n + i;
        double r[3] = {t->x[i], t->y[i], t->z[i]};
        double phi = tree_phi(t, r, ex, nex, NULL);
        if (phi_out) phi_out[i] = phi;
        nadd(&e, 0.5 * t->q[i] * phi);
        if (t->P.geom == 1) {
            double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (t->P.images) nadd(&e, 0.5 * t->gamma * a * t->q[i] * t->q[i] / (r2 - a * a));
            /* own line images: -sigma w_m q_K at t_m r_K, |r - t_m r_K| = (r^2 - t_m a^2) / r */
            for (int m = 0; m < L.M; ++m)
                nadd(&e, -0.5 * L.sigma * L.w[m] * t->gamma * a * t->q[i] * t->q[i] / (r2 - L.t[m] * a * a));
            if (t->P.Q_center != 0.0) nadd(&e, t->P.Q_center * t->q[i] / sqrt(r2));
        }
    }
    return t->P.l_B * nval(&e);
}

/* ------------------------------------------------------------------------ */
/* Exact gradient of the treecode energy                                    */
/*                                                                          */
/* With the interaction lists fixed by the traversal, E_tree is a sum of     */
/* pair terms: for a target t and a far cell A, 1/2 l_B q_t q_j P(r_t; r_j)  */
/* for each remaining member j, with P(x; y) = sum_n T_n(c_A - x)(y - c_A)^n */
/* the truncated expansion of 1/|y - x| (eq. 3.3); for a near source,        */
/* 1/2 l_B q_t q_j / |r_t - r_j|.  Each pair term is differentiated in both  */
/* of its points and charges, using dT_n/dR_k = (n_k + 1) T_{n+e_k}.  The    */
/* image sources are then mapped back to their ions by the chain rule        */
/* through q_K = gamma a q / |r| and r_K = a^2 r / |r|^2.                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *gx, *gy, *gz, *gq;   /* per source                               */
    double *T, *mono;
} gstate;

static void members_of(const otree *t, int c, int **buf, int *nb, int *capb) {
    const ocell *A = &t->cell[c];
    if (A->leaf >= 0) {
        const oleaf *L = &t->leaf[A->leaf];
        for (int k = 0; k < L->count; ++k) {
            if (*nb == *capb) { *capb = *capb ? 2 * *capb : 64; *buf = (int *)realloc(*buf, sizeof(int) * *capb); }
            (*buf)[(*nb)++] = L->slot[k];
        }
    } else {
        for (int d = 0; d < 8; ++d) members_of(t, A->child[d], buf, nb, capb);
    }
}

static void grad_pair_far(const otree *t, int tg, const ocell *A, int j, double w, gstate *g) {
    /* w = 1/2 l_B q_t q_j ; P(x; y) with R = c - x, d = y - c */
    int p = t->P.p;
    double dx = t->x[j] - A->cx, dy = t->y[j] - A->cy, dz = t->z[j] - A->cz;
    /* T up to order p + 1 already in g->T (evaluated at R = c - r_t) */
    double val = 0, gxT = 0, gyT = 0, gzT = 0, gxS = 0, gyS = 0, gzS = 0;
    int nt = nterms_of(p);
    for (int k = 0; k < nt; ++k) {
        int n1 = t->mi[3 * k], n2 = t->mi[3 * k + 1], n3 = t->mi[3 * k + 2];
        double mon = 1.0;
        for (int e = 0; e < n1; ++e) mon *= dx;
        for (int e = 0; e < n2; ++e) mon *= dy;
        for (int e = 0; e < n3; ++e) mon *= dz;
        double Tn = g->T[k];
        val += Tn * mon;
        /* d/dx_t of T_n(c - x_t) = -(n_k + 1) T_{n+e_k} */
        gxT += -(n1 + 1) * g->T[mindex(n1 + 1, n2, n3)] * mon;
        gyT += -(n2 + 1) * g->T[mindex(n1, n2 + 1, n3)] * mon;
        gzT += -(n3 + 1) * g->T[mindex(n1, n2, n3 + 1)] * mon;
        /* d/dy of d^n */
        if (n1 > 0) { double m = n1; for (int e = 0; e < n1 - 1; ++e) m *= dx; for (int e = 0; e < n2; ++e) m *= dy; for (int e = 0; e < n3; ++e) m *= dz; gxS += Tn * m; }
        if (n2 > 0) { double m = n2; for (int e = 0; e < n1; ++e) m *= dx; for (int e = 0; e < n2 - 1; ++e) m *= dy; for (int e = 0; e < n3; ++e) m *= dz; gyS += Tn * m; }
        if (n3 > 0) { double m = n3; for (int e = 0; e < n1; ++e) m *= dx; for (int e = 0; e < n2; ++e) m *= dy; for (int e = 0; e < n3 - 1; ++e) m *= dz; gzS += Tn * m; }
    }
    g->gx[tg] += w * gxT; g->gy[tg] += w * gyT; g->gz[tg] += w * gzT;
    g->gx[j] += w * gxS; g->gy[j] += w * gyS; g->gz[j] += w * gzS;
    /* charges: w / q_j * val for the target's charge, w / q_t * val for j's */
    double half_l = 0.5 * t->P.l_B;
    g->gq[tg] += half_l * t->q[j] * val;
    g->gq[j] += half_l * t->q[tg] * val;
}

static void grad_visit(const otree *t, int c, int tg, const int *ex, int nex, gstate *g,
                       int **buf, int *capb) {
    const ocell *A = &t->cell[c];
    int nin = 0;
    for (int e = 0; e < nex; ++e) nin += contains(t, c, ex[e]);
    int np = A->count - nin;
    if (np == 0) return;
    double xt[3] = {t->x[tg], t->y[tg], t->z[tg]};
    double dx = A->cx - xt[0], dy = A->cy - xt[1], dz = A->cz - xt[2];
    double d2 = dx * dx + dy * dy + dz * dz;
    int mac = 3.0 * (A->h * A->h) <= t->theta2 * d2;
    double half_l = 0.5 * t->P.l_B;
    if (mac && np >= t->P.n0) {
        taylor(t->P.p + 1, t->mi, dx, dy, dz, g->T);
        int nb = 0;
        members_of(t, c, buf, &nb, capb);
        for (int m = 0; m < nb; ++m) {
            int j = (*buf)[m], skip = 0;
            for (int e = 0; e < nex; ++e) skip |= (j == ex[e]);
            if (skip) continue;
            grad_pair_far(t, tg, A, j, half_l * t->q[tg] * t->q[j], g);
        }
    } else if (np > t->P.n0 && A->leaf < 0) {
        for (int d = 0; d < 8; ++d) grad_visit(t, A->child[d], tg, ex, nex, g, buf, capb);
    } else {
        int nb = 0;
        members_of(t, c, buf, &nb, capb);
        for (int m = 0; m < nb; ++m) {
            int j = (*buf)[m], skip = 0;
            for (int e = 0; e < nex; ++e) skip |= (j == ex[e]);
            if (skip) continue;
            double rx = xt[0] - t->x[j], ry = xt[1] - t->y[j], rz = xt[2] - t->z[j];
            double r2 = rx * rx + ry * ry + rz * rz, r = sqrt(r2);
            double w = half_l * t->q[tg] * t->q[j];
            double f = -w / (r2 * r);
            g->gx[tg] += f * rx; g->gy[tg] += f * ry; g->gz[tg] += f * rz;
            g->gx[j] -= f * rx; g->gy[j] -= f * ry; g->gz[j] -= f * rz;
            g->gq[tg] += half_l * t->q[j] / r;
            g->gq[j] += half_l * t->q[tg] / r;
        }
    }
}

/* dE_tree/dr_i and dE_tree/dq_i for every ion; returns E_tree. */
double orc_tree_grad(otree *t, double *gx, double *gy, double *gz, double *gq) {
    int ns = t->nsrc, n = t->n, M = t->P.images ? t->P.line_images : 0;
    int nex = t->P.images ? 2 + M : 1;
    orc_lines L;
    lines_of(&t->P, &L);
    gstate g;
    g.gx = (double *)calloc(ns, sizeof(double)); g.gy = (double *)calloc(ns, sizeof(double));
    g.gz = (double *)calloc(ns, sizeof(double)); g.gq = (double *)calloc(ns, sizeof(double));
    g.T = (double *)malloc(sizeof(double) * nterms_of(t->P.p + 1));
    g.mono = (double *)malloc(sizeof(double) * nterms_of(t->P.p + 1));
    int *buf = NULL, capb = 0;
    for (int i = 0; i < n; ++i) {
        int ex[10] = {i, n + i};  /* the ion and all of its images */
        for (int m = 0; m < M; ++m) ex[2 + m] = 2 * n + m * n + i;
        grad_visit(t, 0, i, ex, nex, &g, &buf, &capb);
    }
    free(buf);
    double l = t->P.l_B, a = t->P.a, gam = t->gamma;
    for (int i = 0; i < n; ++i) {
        double x = t->x[i], y = t->y[i], z = t->z[i], q = t->q[i];
        double r2 = x * x + y * y + z * z, r = sqrt(r2);
        double Gx = g.gx[i], Gy = g.gy[i], Gz = g.gz[i], Gq = g.gq[i];
        if (t->P.images) {
            int s = n + i;
            /* line image m sits at t_m r_K with charge c_m q_K: its gradient joins the
             * Kelvin image's, weighted by t_m (position) and c_m (charge) */
            double hx = g.gx[s], hy = g.gy[s], hz = g.gz[s], dqK = g.gq[s];
            for (int m = 0; m < M; ++m) {
                int sm = 2 * n + m * n + i;
                hx += L.t[m] * g.gx[sm]; hy += L.t[m] * g.gy[sm]; hz += L.t[m] * g.gz[sm];
                dqK += -L.sigma * L.w[m] * g.gq[sm];
            }
            /* r_K = a^2 r / r^2: J = a^2 (I / r^2 - 2 r r^T / r^4), symmetric */
            double a2 = a * a, ir2 = 1.0 / r2, ir4 = ir2 * ir2;
            double rh = x * hx + y * hy + z * hz;
            Gx += a2 * (hx * ir2 - 2.0 * x * rh * ir4);
            Gy += a2 * (hy * ir2 - 2.0 * y * rh * ir4);
            Gz += a2 * (hz * ir2 - 2.0 * z * rh * ir4);
            /* q_K = gamma a q / r */
            double c = -gam * a * q / (r2 * r);
            Gx += dqK * c * x; Gy += dqK * c * y; Gz += dqK * c * z;
            Gq += dqK * gam * a / r;
            /* exact self-image term 1/2 l_B gamma a q^2 / (r^2 - a^2) */
            double den = r2 - a2;
            double cs = -l * gam * a * q * q / (den * den);
            Gx += cs * x; Gy += cs * y; Gz += cs * z;
            Gq += l * gam * a * q / den;
            /* and of the own line images, 1/2 l_B c_m gamma a q^2 / (r^2 - t_m a^2) */
            for (int m = 0; m < M; ++m) {
                double cm = -L.sigma * L.w[m], dm = r2 - L.t[m] * a2;
                double cl = -l * cm * gam * a * q * q / (dm * dm);
                Gx += cl * x; Gy += cl * y; Gz += cl * z;
                Gq += l * cm * gam * a * q / dm;
            }
        }
        if (t->P.geom == 1 && t->P.Q_center != 0.0) {
            double ir3 = 1.0 / (r2 * r), Q = t->P.Q_center;
            Gx += -l * Q * q * x * ir3; Gy += -l * Q * q * y * ir3; Gz += -l * Q * q * z * ir3;
            Gq += l * Q / r;
        }
        gx[i] = Gx; gy[i] = Gy; gz[i] = Gz; gq[i] = Gq;
    }
    free(g.gx); free(g.gy); free(g.gz); free(g.gq); free(g.T); free(g.mono);
    return orc_tree_energy(t, NULL);
}

/* ------------------------------------------------------------------------ */
/* Metropolis drivers (Sec. 2 steps 1-3; Sec. 3.3)                           */
/* ------------------------------------------------------------------------ */

static int rebuild(otree **tp) {
    otree *t = *tp, *nt = NULL;
    int st = orc_tree_build(&t->P, t->n, t->x, t->y, t->z, t->q, &nt);
    if (st) return st;
    orc_tree_free(t);
    *tp = nt;
    return ORC_OK;
}

/* Runs moves move0 .. move0+n_moves-1 of replica `replica`.  Accept iff
 * dE <= 0 or alpha <= exp(-dE) (Sec. 2, step 2).  If an accepted move would
 * overflow a leaf's index array, the tree is rebuilt from the current
 * positions and the same move is evaluated again on the new tree.
 * stats: [accepted, wall, overlap, rebuilds, metropolis_rejected].
 * accept_bits, dE_out and i_out are per move and nullable. */
int orc_mc_run(otree **tp, uint64_t seed, uint32_t replica, uint64_t move0, int64_t n_moves,
               double step, uint8_t *accept_bits, double *dE_out, int64_t *i_out,
               int64_t *stats) {
    memset(stats, 0, sizeof(int64_t) * 5);
    int64_t rebuilt_at = -1;
    for (int64_t k = 0; k < n_moves; ++k) {
        otree *t = *tp;
        uint64_t m = move0 + (uint64_t)k;
        int64_t i; double d[3], alpha;
        orc_draw_move(seed, replica, m, t->n, step, &i, d, &alpha);
        double rn[3] = {t->x[i] + d[0], t->y[i] + d[1], t->z[i] + d[2]};
        int reason;
        double dE = orc_tree_delta(t, i, rn, &reason, NULL);
        int acc = 0;
        if (reason == REASON_WALL) stats[1]++;
        else if (reason == REASON_OVERLAP) stats[2]++;
        else acc = dE <= 0.0 || alpha <= exp(-dE);
        if (acc) {
            int st = orc_tree_commit(t, i, rn);
            if (st == ORC_ECAPACITY) {
                if (rebuilt_at == k) return ORC_ECAPACITY; /* cannot happen: caps hold 2 + M spare */
                rebuilt_at = k;
                st = rebuild(tp);
                if (st) return st;
                stats[3]++;
                --k;
                continue;
            }
            if (st) return st;
            stats[0]++;
        } else if (reason == REASON_NONE) {
            stats[4]++;
        }
        if (accept_bits) accept_bits[k] = (uint8_t)acc;
        if (dE_out) dE_out[k] = dE;
        if (i_out) i_out[k] = i;
    }
    return ORC_OK;
}

/* The same chain with the direct energy change (eq. 1.1) in place of the
 * treecode; positions are updated in place.  Same stats layout (no rebuilds). */
int orc_direct_mc_run(const orc_params *P, int64_t n, double *x, double *y, double *z,
                      const double *q, uint64_t seed, uint32_t replica, uint64_t move0,
                      int64_t n_moves, double step, uint8_t *accept_bits, double *dE_out,
                      int64_t *stats) {
    memset(stats, 0, sizeof(int64_t) * 5);
    double tau2 = P->hard_core * P->hard_core;
    for (int64_t k = 0; k < n_moves; ++k) {
        uint64_t m = move0 + (uint64_t)k;
        int64_t i; double d[3], alpha;
        orc_draw_move(seed, replica, m, n, step, &i, d, &alpha);
        double rn[3] = {x[i] + d[0], y[i] + d[1], z[i] + d[2]};
        double dE = INFINITY;
        int reason = REASON_NONE;
        if (outside(P, rn[0], rn[1], rn[2])) reason = REASON_WALL;
        else {
            for (int64_t j = 0; j < n && reason == REASON_NONE; ++j) {
                if (j == i) continue;
                double dx = rn[0] - x[j], dy = rn[1] - y[j], dz = rn[2] - z[j];
                if (dx * dx + dy * dy + dz * dz <= tau2) reason = REASON_OVERLAP;
            }
        }
        int acc = 0;
        if (reason == REASON_NONE) {
            dE = orc_direct_delta(P, n, x, y, z, q, i, rn);
            acc = dE <= 0.0 || alpha <= exp(-dE);
            if (!acc) stats[4]++;
        } else if (reason == REASON_WALL) stats[1]++;
        else stats[2]++;
        if (acc) { x[i] = rn[0]; y[i] = rn[1]; z[i] = rn[2]; stats[0]++; }
        if (accept_bits) accept_bits[k] = (uint8_t)acc;
        if (dE_out) dE_out[k] = dE;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Introspection for the tests                                              */
/* ------------------------------------------------------------------------ */

/* info: [n, nsrc, ncell, nleaf, nterms, depth] */
void orc_tree_info(const otree *t, int64_t *info) {
    int depth = 0;
    for (int c = 0; c < t->ncell; ++c) if (t->cell[c].level > depth) depth = t->cell[c].level;
    info[0] = t->n; info[1] = t->nsrc; info[2] = t->ncell; info[3] = t->nleaf;
    info[4] = t->nterms; info[5] = depth;
}

void orc_tree_sorted(const otree *t, uint64_t *keys, int32_t *perm) {
    for (int s = 0; s < t->nsrc; ++s) { keys[s] = t->skey[s]; perm[s] = t->perm[s]; }
}

/* per cell: level, kmin, count, is_leaf, parent; geo = (cx, cy, cz, h); M */
void orc_tree_cells(const otree *t, int32_t *level, uint64_t *kmin, int32_t *count,
                    int32_t *is_leaf, int32_t *parent, double *geo, double *M) {
    for (int c = 0; c < t->ncell; ++c) {
        const ocell *A = &t->cell[c];
        level[c] = A->level; kmin[c] = A->kmin; count[c] = A->count;
        is_leaf[c] = A->leaf >= 0; parent[c] = A->parent;
        geo[4 * c] = A->cx; geo[4 * c + 1] = A->cy; geo[4 * c + 2] = A->cz; geo[4 * c + 3] = A->h;
    }
    if (M) memcpy(M, t->M, sizeof(double) * (size_t)t->ncell * t->nterms);
}

/* per leaf: cell, count, cap, begin, end (build range) */
void orc_tree_leaves(const otree *t, int32_t *cell, int32_t *count, int32_t *cap,
                     int32_t *begin, int32_t *end) {
    for (int l = 0; l < t->nleaf; ++l) {
        const oleaf *L = &t->leaf[l];
        cell[l] = L->cell; count[l] = L->count; cap[l] = L->cap;
        begin[l] = t->cell[L->cell].begin; end[l] = t->cell[L->cell].end;
    }
}

int orc_tree_leaf_slots(const otree *t, int l, int32_t *out) {
    const oleaf *L = &t->leaf[l];
    for (int k = 0; k < L->count; ++k) out[k] = L->slot[k];
    return L->count;
}

void orc_tree_tracking(const otree *t, int32_t *leaf_of, int32_t *slot_of) {
    for (int s = 0; s < t->nsrc; ++s) { leaf_of[s] = t->leaf_of[s]; slot_of[s] = t->slot_of[s]; }
}

void orc_tree_sources(const otree *t, double *x, double *y, double *z, double *q) {
    for (int s = 0; s < t->nsrc; ++s) { x[s] = t->x[s]; y[s] = t->y[s]; z[s] = t->z[s]; q[s] = t->q[s]; }
}

/* Recompute every cell's moments from its current members, for the check
 * that incremental repair equals a fresh sum (Sec. 3.3). */
void orc_tree_fresh_moments(const otree *t, double *M) {
    double *mono = (double *)malloc(sizeof(double) * t->nterms);
    int *buf = NULL, nb = 0, capb = 0;
    for (int c = 0; c < t->ncell; ++c) {
        const ocell *A = &t->cell[c];
        double *Mc = M + (size_t)c * t->nterms;
        for (int k = 0; k < t->nterms; ++k) Mc[k] = 0.0;
        nb = 0;
        members_of(t, c, &buf, &nb, &capb);
        for (int m = 0; m < nb; ++m) {
            int j = buf[m];
            monomials(t->P.p, t->mi, t->x[j] - A->cx, t->y[j] - A->cy, t->z[j] - A->cz, mono);
            for (int k = 0; k < t->nterms; ++k) Mc[k] += t->q[j] * mono[k];
        }
    }
    free(buf); free(mono);
}

void orc_taylor(int p, double Rx, double Ry, double Rz, double *T) {
    int *mi = (int *)malloc(sizeof(int) * 3 * nterms_of(p));
    multi_indices(p, mi);
    taylor(p, mi, Rx, Ry, Rz, T);
    free(mi);
}

void orc_multi_indices(int p, int32_t *out) {
    int *mi = (int *)malloc(sizeof(int) * 3 * nterms_of(p));
    multi_indices(p, mi);
    for (int k = 0; k < 3 * nterms_of(p); ++k) out[k] = mi[k];
    free(mi);
}

/* certificate of eq. 3.5 for the target x: sum over far cells of
 * (sum_j |q_j| / R) gamma_A^{p+1} / (1 - gamma_A), gamma_A = rho_A / R. */
static void cert_visit(const otree *t, int c, const double *xt, const int *ex, int nex, double *acc) {
    const ocell *A = &t->cell[c];
    int nin = 0;
    for (int e = 0; e < nex; ++e) nin += contains(t, c, ex[e]);
    int np = A->count - nin;
    if (np == 0) return;
    double dx = A->cx - xt[0], dy = A->cy - xt[1], dz = A->cz - xt[2];
    double d2 = dx * dx + dy * dy + dz * dz;
    int mac = 3.0 * (A->h * A->h) <= t->theta2 * d2;
    if (mac && np >= t->P.n0) {
        double R = sqrt(d2), g = sqrt(3.0) * A->h / R, absq = 0.0;
        int *buf = NULL, nb = 0, capb = 0;
        members_of(t, c, &buf, &nb, &capb);
        for (int m = 0; m < nb; ++m) {
            int j = buf[m], skip = 0;
            for (int e = 0; e < nex; ++e) skip |= (j == ex[e]);
            if (!skip) absq += fabs(t->q[j]);
        }
        free(buf);
        *acc += absq / R * pow(g, t->P.p + 1) / (1.0 - g);
    } else if (np > t->P.n0 && t->cell[c].leaf < 0) {
        for (int d = 0; d < 8; ++d) cert_visit(t, A->child[d], xt, ex, nex, acc);
    }
}

double orc_tree_certificate(const otree *t, const double *xt, const int *ex, int nex) {
    double acc = 0.0;
    cert_visit(t, 0, xt, ex, nex, &acc);
    return acc;
}
