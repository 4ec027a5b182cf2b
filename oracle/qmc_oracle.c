/*
 * qmc_oracle.c -- plain, slow FP64 CPU oracle for particle-by-particle VMC.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the GPU library, and the GPU
 * library never calls it.
 *
 * What it follows (QMCPACK overview paper, arXiv:1802.06922):
 *   - VMC as Metropolis sampling of |Psi_T|^2 with independent walkers
 *     (section "Variational Monte Carlo", the sample-mean energy equation).
 *   - Particle-by-particle moves: electrons visited in order, each proposed
 *     from a Gaussian transition probability without drift (F = 0), accepted
 *     with the Metropolis probability (section "Trial Moves", equations
 *     trans_prob_alle and accept_reject).
 *   - Slater-Jastrow trial function D_up D_dn e^J (equation eq:msdj, one
 *     determinant) with Sherman-Morrison single-row inverse updates (section
 *     "Multi-Determinant Slater-Jastrow Form").
 *   - Periodic tricubic B-spline orbitals, 64 coefficients per orbital per
 *     evaluation (section "B-spline basis sets"); analytic plane-wave
 *     orbitals of the electron gas (section "Orbitals").
 *   - One- and two-body Jastrow with Pade or cubic B-spline radial
 *     functions and the cusp-fixed first control point (section "Jastrow
 *     factors").
 *   - Local energy as kinetic plus Coulomb terms, the periodic Coulomb sum
 *     by Ewald summation (section "Hamiltonian", equation
 *     vmc:electron_ham; section "Long-Range Interactions").
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   Psi = D_up D_dn exp(+J); the B-spline cusp formula read as
 *   p0 = p2 - 2 (rc/M) u'(0); minimum-image distances; positions kept
 *   wrapped into [0, L); Ewald taken to convergence; a counter-based
 *   Philox4x32-10 generator (Salmon et al., SC'11) keyed by the seed and
 *   indexed by (electron, sweep, walker, purpose) for every random number.
 *
 * Every function that is not pinned by a test against something other than
 * itself says so.  (All functions here are pinned; see tests/.)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror,  */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).        */
/* ------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { ORC_INIT = 1, ORC_PROPOSE = 2, ORC_ACCEPT = 3, ORC_BRANCH = 4 };

/* Two uniforms in [0,1) with 53 random bits each, from one Philox block.
 * counter = (electron, sweep, walker, purpose << 16 | sub), key = seed. */
void orc_uniform2(uint64_t seed, uint32_t purpose, uint32_t sub, uint32_t walker,
                  uint32_t sweep, uint32_t electron, double u[2])
{
    uint32_t ctr[4] = {electron, sweep, walker, (purpose << 16) | sub};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    uint64_t x0 = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    uint64_t x1 = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
    u[0] = (double)(x0 >> 11) * 0x1.0p-53;
    u[1] = (double)(x1 >> 11) * 0x1.0p-53;
}

/* Three N(0,1) numbers for the proposal of (walker, sweep, electron):
 * Box-Muller on the two uniform pairs of sub-blocks 0 and 1. */
void orc_gauss3(uint64_t seed, uint32_t walker, uint32_t sweep, uint32_t electron, double xi[3])
{
    double a[2], b[2];
    orc_uniform2(seed, ORC_PROPOSE, 0, walker, sweep, electron, a);
    orc_uniform2(seed, ORC_PROPOSE, 1, walker, sweep, electron, b);
    double ra = sqrt(-2.0 * log(1.0 - a[0]));
    double rb = sqrt(-2.0 * log(1.0 - b[0]));
    xi[0] = ra * cos(2.0 * ORC_PI * a[1]);
    xi[1] = ra * sin(2.0 * ORC_PI * a[1]);
    xi[2] = rb * cos(2.0 * ORC_PI * b[1]);
}

double orc_accept_uniform(uint64_t seed, uint32_t walker, uint32_t sweep, uint32_t electron)
{
    double u[2];
    orc_uniform2(seed, ORC_ACCEPT, 0, walker, sweep, electron, u);
    return u[0];
}

/* The uniform xi of the branching multiplicity of walker slot `slot` at DMC step `step`. */
double orc_branch_uniform(uint64_t seed, uint32_t slot, uint32_t step)
{
    double u[2];
    orc_uniform2(seed, ORC_BRANCH, 0, slot, step, 0u, u);
    return u[0];
}

/* Uniform position of an electron in the cell (the starting distribution of a walker) from
 * the INIT stream of (walker, electron); the counter's sweep slot is 0. */
void orc_init_position(uint64_t seed, uint32_t walker, uint32_t electron, double L, double r[3])
{
    double a[2], b[2];
    orc_uniform2(seed, ORC_INIT, 0, walker, 0u, electron, a);
    orc_uniform2(seed, ORC_INIT, 1, walker, 0u, electron, b);
    r[0] = L * a[0];
    r[1] = L * a[1];
    r[2] = L * b[0];
}

/* ------------------------------------------------------------------ */
/* System description                                                  */
/* ------------------------------------------------------------------ */

enum { ORC_SPO_SPLINE = 0, ORC_SPO_PLANEWAVE = 1 };
enum { ORC_J_NONE = 0, ORC_J_PADE = 1, ORC_J_BSPLINE = 2 };

typedef struct {
    int32_t n_up, n_dn;
    double L;
    int32_t spo_kind;          /* ORC_SPO_SPLINE or ORC_SPO_PLANEWAVE */
    int32_t n_orb;
    int32_t gx, gy, gz;
    const double* coefs;       /* spline: [gx][gy][gz][n_orb] */
    const double* pw_k;        /* plane waves: [n_orb][3] */
    const int32_t* pw_kind;    /* plane waves: 0 cos, 1 sin */
    int32_t n_ions;
    const double* ion_pos;     /* [n_ions][3] */
    const double* ion_Z;       /* [n_ions] */
    int32_t j2_kind;           /* ORC_J_* (same functor form for both spin pairs) */
    double j2_a, j2_b;         /* Pade u = a r / (1 + b r) */
    int32_t j2_M;              /* B-spline: number of free control points */
    double j2_rc;
    const double* j2_p;        /* p_1..p_M */
    double j2_cusp_same, j2_cusp_opp;
    int32_t j1_kind;           /* ORC_J_NONE or ORC_J_BSPLINE */
    int32_t j1_M;
    double j1_rc;
    const double* j1_p;        /* p_1..p_M */
    double j1_cusp;
    double sigma;
    uint64_t seed;
    int32_t coulomb;           /* 0: kinetic only; 1: kinetic + Ewald Coulomb */
    double ewald_kappa;        /* <= 0: 5 / L */
    int32_t all_electron;      /* 0: particle-by-particle sweeps; 1: all-electron moves;
                                  2: all-electron drift-diffusion moves; 3: particle-by-particle
                                  drift-diffusion sweeps */
    int32_t j3_mei, j3_mee;    /* three-body e-e-I term: polynomial orders (0 = term off when
                                  j3_gamma is NULL) */
    double j3_rc;              /* its cutoff r_c: the electron-ion distances stay below r_c/2 */
    const double* j3_gamma;    /* [2][mei+1][mei+1][mee+1] (same spin, opposite spin) or NULL */
} orc_system;

/* ------------------------------------------------------------------ */
/* Periodic tricubic B-spline orbitals (section "B-spline basis sets"). */
/* Uniform cubic B-spline basis with integer knots: the coefficient     */
/* c_j multiplies B(t - j), B the centred cubic B-spline of support     */
/* [-2, 2].  64 coefficients per orbital per evaluation.                */
/* ------------------------------------------------------------------ */

/* Centred cubic B-spline and its first two derivatives. */
static void orc_cubic_bspline(double y, double* b, double* db, double* d2b)
{
    double a = fabs(y), s = (y < 0.0) ? -1.0 : 1.0;
    if (a < 1.0) {
        *b = 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        *db = s * (-2.0 * a + 1.5 * a * a);
        *d2b = -2.0 + 3.0 * a;
    } else if (a < 2.0) {
        double t = 2.0 - a;
        *b = t * t * t / 6.0;
        *db = -s * 0.5 * t * t;
        *d2b = t;
    } else {
        *b = 0.0; *db = 0.0; *d2b = 0.0;
    }
}

static int orc_mod(int i, int n) { int m = i % n; return m < 0 ? m + n : m; }

static double orc_wrap(double x, double L)
{
    double y = x - L * floor(x / L);
    if (y >= L) y = 0.0;
    return y;
}

/* Value, gradient [3][n_orb] and Laplacian of every spline orbital at r. */
static void orc_spline_vgl(const orc_system* s, const double r[3], double* v, double* g, double* lap)
{
    const int n = s->n_orb;
    const int G[3] = {s->gx, s->gy, s->gz};
    double w[3][4], dw[3][4], d2w[3][4];
    int idx[3][4];
    for (int a = 0; a < 3; ++a) {
        double h = (double)G[a] / s->L;          /* knots per bohr */
        double t = orc_wrap(r[a], s->L) * h;
        int i0 = (int)floor(t);
        for (int m = 0; m < 4; ++m) {
            int j = i0 - 1 + m;                  /* the four knots whose support holds t */
            double b, db, d2b;
            orc_cubic_bspline(t - (double)j, &b, &db, &d2b);
            w[a][m] = b;
            dw[a][m] = db * h;
            d2w[a][m] = d2b * h * h;
            idx[a][m] = orc_mod(j, G[a]);
        }
    }
    for (int j = 0; j < n; ++j) { v[j] = 0.0; g[j] = g[n + j] = g[2 * n + j] = 0.0; lap[j] = 0.0; }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                const double* cf = s->coefs + ((size_t)(idx[0][a] * G[1] + idx[1][b]) * G[2] + idx[2][c]) * n;
                double wv = w[0][a] * w[1][b] * w[2][c];
                double wgx = dw[0][a] * w[1][b] * w[2][c];
                double wgy = w[0][a] * dw[1][b] * w[2][c];
                double wgz = w[0][a] * w[1][b] * dw[2][c];
                double wl = d2w[0][a] * w[1][b] * w[2][c] + w[0][a] * d2w[1][b] * w[2][c]
                          + w[0][a] * w[1][b] * d2w[2][c];
                for (int j = 0; j < n; ++j) {
                    v[j] += wv * cf[j];
                    g[j] += wgx * cf[j];
                    g[n + j] += wgy * cf[j];
                    g[2 * n + j] += wgz * cf[j];
                    lap[j] += wl * cf[j];
                }
            }
}

/* Real plane waves cos(k.r) / sin(k.r): the electron-gas orbitals. */
static void orc_planewave_vgl(const orc_system* s, const double r[3], double* v, double* g, double* lap)
{
    const int n = s->n_orb;
    for (int j = 0; j < n; ++j) {
        const double* k = s->pw_k + 3 * j;
        double ph = k[0] * r[0] + k[1] * r[1] + k[2] * r[2];
        double c = cos(ph), sn = sin(ph), k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        double f = s->pw_kind[j] ? sn : c;       /* value */
        double df = s->pw_kind[j] ? c : -sn;     /* d/d(phase) */
        v[j] = f;
        for (int a = 0; a < 3; ++a) g[a * n + j] = k[a] * df;
        lap[j] = -k2 * f;
    }
}

void orc_spo_vgl(const orc_system* s, const double r[3], double* v, double* g, double* lap)
{
    if (s->spo_kind == ORC_SPO_PLANEWAVE) orc_planewave_vgl(s, r, v, g, lap);
    else orc_spline_vgl(s, r, v, g, lap);
}

/* ------------------------------------------------------------------ */
/* Jastrow radial functions (section "Jastrow factors").               */
/* ------------------------------------------------------------------ */

/* u(r) = sum_{m=0}^{M} p_m B3(r / (rc/M) - m), B3 the cardinal cubic
 * B-spline on [-3, 1) centred at -1, i.e. B3(x) = B(x + 1); p_0 fixed by
 * the cusp: u'(0) = (p_2 - p_0) / (2 rc / M).  u = 0 for r >= rc. */
static void orc_bspline_radial(int M, double rc, const double* p1M, double cusp, double r,
                               double* u, double* du, double* d2u)
{
    *u = *du = *d2u = 0.0;
    if (r >= rc) return;
    double delta = rc / (double)M;
    double p0 = p1M[1] - 2.0 * delta * cusp;     /* p_2 is p1M[1] */
    double x = r / delta;
    for (int m = 0; m <= M; ++m) {
        double pm = (m == 0) ? p0 : p1M[m - 1];
        double b, db, d2b;
        orc_cubic_bspline(x - (double)m + 1.0, &b, &db, &d2b);
        *u += pm * b;
        *du += pm * db / delta;
        *d2u += pm * d2b / (delta * delta);
    }
}

/* Two-body radial function between electrons of equal (same=1) or opposite spin. */
static void orc_u2(const orc_system* s, int same, double r, double* u, double* du, double* d2u)
{
    if (s->j2_kind == ORC_J_PADE) {
        double d = 1.0 + s->j2_b * r;
        *u = s->j2_a * r / d;
        *du = s->j2_a / (d * d);
        *d2u = -2.0 * s->j2_a * s->j2_b / (d * d * d);
    } else if (s->j2_kind == ORC_J_BSPLINE) {
        orc_bspline_radial(s->j2_M, s->j2_rc, s->j2_p, same ? s->j2_cusp_same : s->j2_cusp_opp, r, u, du, d2u);
    } else {
        *u = *du = *d2u = 0.0;
    }
}

static void orc_u1(const orc_system* s, double r, double* u, double* du, double* d2u)
{
    if (s->j1_kind == ORC_J_BSPLINE) orc_bspline_radial(s->j1_M, s->j1_rc, s->j1_p, s->j1_cusp, r, u, du, d2u);
    else { *u = *du = *d2u = 0.0; }
}

/*
 * Three-body electron-electron-ion term (section "Jastrow factors", the form of Drummond et
 * al.): for electrons i, j near ion I with a = r_iI, b = r_jI, c = r_ij,
 *   u = sum_{l,m,n} g_lmn a^l b^m c^n (a - h)^3 (b - h)^3,   h = r_c / 2,
 * zero once a >= h or b >= h.  Out: d = (u, du/da, du/dc, d2u/da2, d2u/dc2, d2u/dadc) at
 * fixed b (the partial derivatives the gradient and Laplacian with respect to electron i need).
 */
static void orc_u3(const orc_system* s, int same, double a, double b, double c, double d[6])
{
    const double h = 0.5 * s->j3_rc;
    for (int q = 0; q < 6; ++q) d[q] = 0.0;
    if (!s->j3_gamma || a >= h || b >= h) return;
    const int L = s->j3_mei, M = s->j3_mee;
    const double* g = s->j3_gamma + (same ? 0 : (size_t)(L + 1) * (L + 1) * (M + 1));
    double P = 0.0, Pa = 0.0, Pc = 0.0, Paa = 0.0, Pcc = 0.0, Pac = 0.0;
    for (int l = 0; l <= L; ++l)
        for (int m = 0; m <= L; ++m)
            for (int n = 0; n <= M; ++n) {
                const double gv = g[((size_t)l * (L + 1) + m) * (M + 1) + n];
                const double bm = pow(b, m);
                const double al = pow(a, l), cn = pow(c, n);
                const double al1 = l >= 1 ? l * pow(a, l - 1) : 0.0;
                const double al2 = l >= 2 ? l * (l - 1) * pow(a, l - 2) : 0.0;
                const double cn1 = n >= 1 ? n * pow(c, n - 1) : 0.0;
                const double cn2 = n >= 2 ? n * (n - 1) * pow(c, n - 2) : 0.0;
                P += gv * al * bm * cn;
                Pa += gv * al1 * bm * cn;
                Paa += gv * al2 * bm * cn;
                Pc += gv * al * bm * cn1;
                Pcc += gv * al * bm * cn2;
                Pac += gv * al1 * bm * cn1;
            }
    const double fa = (a - h) * (a - h) * (a - h), fa1 = 3.0 * (a - h) * (a - h), fa2 = 6.0 * (a - h);
    const double fb = (b - h) * (b - h) * (b - h);
    d[0] = P * fa * fb;
    d[1] = (Pa * fa + P * fa1) * fb;
    d[2] = Pc * fa * fb;
    d[3] = (Paa * fa + 2.0 * Pa * fa1 + P * fa2) * fb;
    d[4] = Pcc * fa * fb;
    d[5] = (Pac * fa + Pc * fa1) * fb;
}

/* Exported for the functor pins. kind: 1 = two-body same spin, 2 = two-body
 * opposite spin, 3 = one-body. */
void orc_radial(const orc_system* s, int kind, double r, double out[3])
{
    if (kind == 3) orc_u1(s, r, &out[0], &out[1], &out[2]);
    else orc_u2(s, kind == 1, r, &out[0], &out[1], &out[2]);
}

/* Minimum-image displacement a - b in a cubic cell of side L. */
static void orc_min_image(const double* a, const double* b, double L, double d[3])
{
    for (int k = 0; k < 3; ++k) {
        double x = a[k] - b[k];
        d[k] = x - L * rint(x / L);
    }
}

static double orc_norm3(const double d[3]) { return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]); }

static int orc_spin(const orc_system* s, int i) { return i < s->n_up ? 0 : 1; }

/* Full Jastrow J = sum_{i<j} u2(r_ij) + sum_{i,I} u1(r_iI). */
static double orc_jastrow_total(const orc_system* s, const double* pos)
{
    const int N = s->n_up + s->n_dn;
    double J = 0.0, u, du, d2u, d[3];
    for (int i = 0; i < N; ++i) {
        for (int j = i + 1; j < N; ++j) {
            orc_min_image(pos + 3 * i, pos + 3 * j, s->L, d);
            orc_u2(s, orc_spin(s, i) == orc_spin(s, j), orc_norm3(d), &u, &du, &d2u);
            J += u;
        }
        for (int I = 0; I < s->n_ions; ++I) {
            orc_min_image(pos + 3 * i, s->ion_pos + 3 * I, s->L, d);
            orc_u1(s, orc_norm3(d), &u, &du, &d2u);
            J += u;
        }
    }
    if (s->j3_gamma)
        for (int I = 0; I < s->n_ions; ++I)
            for (int i = 0; i < N; ++i)
                for (int j = i + 1; j < N; ++j) {
                    double da[3], db[3], dc[3], t[6];
                    orc_min_image(pos + 3 * i, s->ion_pos + 3 * I, s->L, da);
                    orc_min_image(pos + 3 * j, s->ion_pos + 3 * I, s->L, db);
                    orc_min_image(pos + 3 * i, pos + 3 * j, s->L, dc);
                    orc_u3(s, orc_spin(s, i) == orc_spin(s, j), orc_norm3(da), orc_norm3(db), orc_norm3(dc), t);
                    J += t[0];
                }
    return J;
}

/* The terms of J that involve electron i when it sits at r. */
static double orc_jastrow_of(const orc_system* s, const double* pos, int i, const double r[3])
{
    const int N = s->n_up + s->n_dn;
    double J = 0.0, u, du, d2u, d[3];
    for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        orc_min_image(r, pos + 3 * j, s->L, d);
        orc_u2(s, orc_spin(s, i) == orc_spin(s, j), orc_norm3(d), &u, &du, &d2u);
        J += u;
    }
    for (int I = 0; I < s->n_ions; ++I) {
        orc_min_image(r, s->ion_pos + 3 * I, s->L, d);
        orc_u1(s, orc_norm3(d), &u, &du, &d2u);
        J += u;
    }
    if (s->j3_gamma)
        for (int I = 0; I < s->n_ions; ++I)
            for (int j = 0; j < N; ++j) {
                if (j == i) continue;
                double da[3], db[3], dc[3], t[6];
                orc_min_image(r, s->ion_pos + 3 * I, s->L, da);
                orc_min_image(pos + 3 * j, s->ion_pos + 3 * I, s->L, db);
                orc_min_image(r, pos + 3 * j, s->L, dc);
                orc_u3(s, orc_spin(s, i) == orc_spin(s, j), orc_norm3(da), orc_norm3(db), orc_norm3(dc), t);
                J += t[0];
            }
    return J;
}

/* Gradient and Laplacian of J with respect to electron i. */
static void orc_jastrow_grad_lap(const orc_system* s, const double* pos, int i, double gJ[3], double* lJ)
{
    const int N = s->n_up + s->n_dn;
    double u, du, d2u, d[3];
    gJ[0] = gJ[1] = gJ[2] = 0.0;
    *lJ = 0.0;
    for (int j = 0; j < N + s->n_ions; ++j) {
        if (j == i) continue;
        double r;
        if (j < N) {
            orc_min_image(pos + 3 * i, pos + 3 * j, s->L, d);
            r = orc_norm3(d);
            orc_u2(s, orc_spin(s, i) == orc_spin(s, j), r, &u, &du, &d2u);
        } else {
            orc_min_image(pos + 3 * i, s->ion_pos + 3 * (j - N), s->L, d);
            r = orc_norm3(d);
            orc_u1(s, r, &u, &du, &d2u);
        }
        for (int k = 0; k < 3; ++k) gJ[k] += du * d[k] / r;
        *lJ += d2u + 2.0 * du / r;
    }
    /* three-body terms: grad_i u = u_a a^ + u_c c^, lap_i u = u_aa + 2 u_a / a + u_cc + 2 u_c / c
     * + 2 u_ac a^.c^ (a = r_iI, c = r_ij, b = r_jI fixed) */
    if (s->j3_gamma)
        for (int I = 0; I < s->n_ions; ++I)
            for (int j = 0; j < N; ++j) {
                if (j == i) continue;
                double da[3], db[3], dc[3], t[6];
                orc_min_image(pos + 3 * i, s->ion_pos + 3 * I, s->L, da);
                orc_min_image(pos + 3 * j, s->ion_pos + 3 * I, s->L, db);
                orc_min_image(pos + 3 * i, pos + 3 * j, s->L, dc);
                const double a = orc_norm3(da), c = orc_norm3(dc);
                orc_u3(s, orc_spin(s, i) == orc_spin(s, j), a, orc_norm3(db), c, t);
                double ac = 0.0;
                for (int k = 0; k < 3; ++k) {
                    gJ[k] += t[1] * da[k] / a + t[2] * dc[k] / c;
                    ac += (da[k] / a) * (dc[k] / c);
                }
                *lJ += t[3] + 2.0 * t[1] / a + t[4] + 2.0 * t[2] / c + 2.0 * t[5] * ac;
            }
}

/* ------------------------------------------------------------------ */
/* Dense linear algebra: LU with partial pivoting (textbook Doolittle). */
/* ------------------------------------------------------------------ */

/* In place: a (row-major n x n) becomes L\U; piv[k] = row swapped with k.
 * Returns 0, or 1 when a pivot is exactly zero. */
static int orc_lu(int n, double* a, int* piv, double* logabs, int* sign)
{
    *logabs = 0.0;
    *sign = 1;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(a[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(a[i * n + k]) > best) { best = fabs(a[i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return 1;
        if (p != k) {
            for (int j = 0; j < n; ++j) { double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t; }
            *sign = -*sign;
        }
        double d = a[k * n + k];
        if (d < 0.0) *sign = -*sign;
        *logabs += log(fabs(d));
        for (int i = k + 1; i < n; ++i) {
            double l = a[i * n + k] / d;
            a[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= l * a[k * n + j];
        }
    }
    return 0;
}

/* log|det a|, sign and the inverse of a (row-major), via LU and n solves. */
int orc_inverse(int n, const double* a, double* ainv, double* logabs, int* sign)
{
    if (n == 0) { *logabs = 0.0; *sign = 1; return 0; }
    double* lu = (double*)malloc(sizeof(double) * n * n);
    int* piv = (int*)malloc(sizeof(int) * n);
    double* x = (double*)malloc(sizeof(double) * n);
    memcpy(lu, a, sizeof(double) * n * n);
    int bad = orc_lu(n, lu, piv, logabs, sign);
    if (!bad) {
        for (int col = 0; col < n; ++col) {
            for (int i = 0; i < n; ++i) x[i] = (i == col) ? 1.0 : 0.0;
            for (int k = 0; k < n; ++k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
            for (int i = 0; i < n; ++i)             /* forward: unit lower */
                for (int j = 0; j < i; ++j) x[i] -= lu[i * n + j] * x[j];
            for (int i = n - 1; i >= 0; --i) {      /* backward: upper */
                for (int j = i + 1; j < n; ++j) x[i] -= lu[i * n + j] * x[j];
                x[i] /= lu[i * n + i];
            }
            for (int i = 0; i < n; ++i) ainv[i * n + col] = x[i];
        }
    }
    free(lu); free(piv); free(x);
    return bad;
}

/* Sherman-Morrison update after row k of A (row = electron, column =
 * orbital, A[k][l] = phi_l(r_k)) is replaced by v, with B = A^{-1}
 * stored row-major as B[l][m]:  B <- B - B[:,k] (v^T B - e_k^T) / R,
 * R = v^T B[:,k] (the determinant ratio).  Textbook rank-one inverse
 * update (the paper cites Fahy et al. 1990 for it). */
void orc_sherman_morrison(int n, double* B, int k, const double* v, double R)
{
    double* t = (double*)malloc(sizeof(double) * n);
    double* colk = (double*)malloc(sizeof(double) * n);
    for (int m = 0; m < n; ++m) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += v[j] * B[j * n + m];
        t[m] = acc - (m == k ? 1.0 : 0.0);
    }
    for (int l = 0; l < n; ++l) colk[l] = B[l * n + k];
    for (int l = 0; l < n; ++l)
        for (int m = 0; m < n; ++m) B[l * n + m] -= colk[l] * t[m] / R;
    free(t); free(colk);
}

/* Woodbury form of m row replacements applied at once (the algebra behind a
 * delayed, rank-m update): rows rows[0..m-1] (distinct) of A replaced by
 * V[0..m-1][:].  With U = B[:, rows], D = V - A[rows,:], C = I + D U:
 * B <- B - U C^{-1} D B.  Used to pin the delayed-update algebra. */
int orc_woodbury(int n, const double* A, double* B, int m, const int* rows, const double* V)
{
    double* U = (double*)malloc(sizeof(double) * n * m);
    double* D = (double*)malloc(sizeof(double) * m * n);
    double* C = (double*)malloc(sizeof(double) * m * m);
    double* Ci = (double*)malloc(sizeof(double) * m * m);
    double* DB = (double*)malloc(sizeof(double) * m * n);
    double* Y = (double*)malloc(sizeof(double) * m * n);
    for (int l = 0; l < n; ++l)
        for (int q = 0; q < m; ++q) U[l * m + q] = B[l * n + rows[q]];
    for (int q = 0; q < m; ++q)
        for (int j = 0; j < n; ++j) D[q * n + j] = V[q * n + j] - A[rows[q] * n + j];
    for (int q = 0; q < m; ++q)
        for (int r = 0; r < m; ++r) {
            double acc = (q == r) ? 1.0 : 0.0;
            for (int j = 0; j < n; ++j) acc += D[q * n + j] * U[j * m + r];
            C[q * m + r] = acc;
        }
    double la; int sg;
    int bad = orc_inverse(m, C, Ci, &la, &sg);
    if (!bad) {
        for (int q = 0; q < m; ++q)
            for (int c = 0; c < n; ++c) {
                double acc = 0.0;
                for (int j = 0; j < n; ++j) acc += D[q * n + j] * B[j * n + c];
                DB[q * n + c] = acc;
            }
        for (int q = 0; q < m; ++q)
            for (int c = 0; c < n; ++c) {
                double acc = 0.0;
                for (int r = 0; r < m; ++r) acc += Ci[q * m + r] * DB[r * n + c];
                Y[q * n + c] = acc;
            }
        for (int l = 0; l < n; ++l)
            for (int c = 0; c < n; ++c) {
                double acc = 0.0;
                for (int q = 0; q < m; ++q) acc += U[l * m + q] * Y[q * n + c];
                B[l * n + c] -= acc;
            }
    }
    free(U); free(D); free(C); free(Ci); free(DB); free(Y);
    return bad;
}

/* ------------------------------------------------------------------ */
/* Ewald sum for point charges in a cubic cell (section "Long-Range    */
/* Interactions"; Ewald 1921).  With a uniform neutralising background  */
/* when the total charge is not zero.  Taken to convergence:            */
/*  E = 1/2 sum_{i!=j} sum_n q_i q_j erfc(k|r_ij+nL|)/|r_ij+nL|         */
/*    + 1/2 sum_i q_i^2 sum_{n!=0} erfc(k|nL|)/|nL|                     */
/*    + (2 pi / V) sum_{G!=0} exp(-G^2/4k^2)/G^2 |sum_i q_i e^{iG.r_i}|^2 */
/*    - (k / sqrt(pi)) sum_i q_i^2 - pi (sum_i q_i)^2 / (2 V k^2)        */
/* ------------------------------------------------------------------ */

double orc_ewald(int n, const double* pos, const double* q, double L, double kappa)
{
    if (kappa <= 0.0) kappa = 5.0 / L;
    const double V = L * L * L;
    int nmax = (int)ceil(6.5 / (kappa * L) - 0.5);
    if (nmax < 1) nmax = 1;
    int mmax = (int)ceil(kappa * L * sqrt(42.0) / ORC_PI) - 1;
    if (mmax < 1) mmax = 1;
    double real = 0.0, self_img = 0.0, recip = 0.0, qsum = 0.0, q2sum = 0.0;
    for (int i = 0; i < n; ++i) { qsum += q[i]; q2sum += q[i] * q[i]; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            double d[3];
            orc_min_image(pos + 3 * i, pos + 3 * j, L, d);
            for (int a = -nmax; a <= nmax; ++a)
                for (int b = -nmax; b <= nmax; ++b)
                    for (int c = -nmax; c <= nmax; ++c) {
                        double x = d[0] + a * L, y = d[1] + b * L, z = d[2] + c * L;
                        double r = sqrt(x * x + y * y + z * z);
                        real += 0.5 * q[i] * q[j] * erfc(kappa * r) / r;
                    }
        }
    for (int a = -nmax; a <= nmax; ++a)
        for (int b = -nmax; b <= nmax; ++b)
            for (int c = -nmax; c <= nmax; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                double r = L * sqrt((double)(a * a + b * b + c * c));
                self_img += 0.5 * q2sum * erfc(kappa * r) / r;
            }
    for (int a = -mmax; a <= mmax; ++a)
        for (int b = -mmax; b <= mmax; ++b)
            for (int c = -mmax; c <= mmax; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                double G[3] = {2.0 * ORC_PI * a / L, 2.0 * ORC_PI * b / L, 2.0 * ORC_PI * c / L};
                double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
                double re = 0.0, im = 0.0;
                for (int i = 0; i < n; ++i) {
                    double ph = G[0] * pos[3 * i] + G[1] * pos[3 * i + 1] + G[2] * pos[3 * i + 2];
                    re += q[i] * cos(ph);
                    im += q[i] * sin(ph);
                }
                recip += (2.0 * ORC_PI / V) * exp(-G2 / (4.0 * kappa * kappa)) / G2 * (re * re + im * im);
            }
    double self = -kappa / sqrt(ORC_PI) * q2sum;
    double bg = -ORC_PI * qsum * qsum / (2.0 * V * kappa * kappa);
    return real + self_img + recip + self + bg;
}

/* Potential components (V_ee, V_eI, V_II): electrons (charge -1) alone with
 * a neutralising background; ions alone likewise; V_eI the remainder of the
 * combined sum, so each part is independent of the splitting parameter. */
static void orc_coulomb(const orc_system* s, const double* pos, double v_ii_cached, double out[3])
{
    const int N = s->n_up + s->n_dn, M = s->n_ions;
    double* q = (double*)malloc(sizeof(double) * (N + M));
    double* all = (double*)malloc(sizeof(double) * 3 * (N + M));
    for (int i = 0; i < N; ++i) q[i] = -1.0;
    for (int I = 0; I < M; ++I) q[N + I] = s->ion_Z[I];
    memcpy(all, pos, sizeof(double) * 3 * N);
    if (M) memcpy(all + 3 * N, s->ion_pos, sizeof(double) * 3 * M);
    double vee = orc_ewald(N, pos, q, s->L, s->ewald_kappa);
    double vii = v_ii_cached, vei = 0.0;
    if (M) {
        if (isnan(vii)) vii = orc_ewald(M, s->ion_pos, q + N, s->L, s->ewald_kappa);
        vei = orc_ewald(N + M, all, q, s->L, s->ewald_kappa) - vee - vii;
    } else {
        vii = 0.0;
    }
    out[0] = vee; out[1] = vei; out[2] = vii;
    free(q); free(all);
}

/* ------------------------------------------------------------------ */
/* Walker state and the trial wavefunction.                            */
/* ------------------------------------------------------------------ */

typedef struct {
    double* pos;          /* [N][3], wrapped into [0, L) */
    double* A[2];         /* Slater matrices, A[k][l] = phi_l(r_k) */
    double* B[2];         /* inverses, B[l][k] */
    double logdet[2];
    int sign[2];
    double logdet_accum[2];
} orc_walker;

static int orc_spin_count(const orc_system* s, int sp) { return sp == 0 ? s->n_up : s->n_dn; }
static int orc_spin_offset(const orc_system* s, int sp) { return sp == 0 ? 0 : s->n_up; }

static void orc_walker_alloc(const orc_system* s, orc_walker* w)
{
    const int N = s->n_up + s->n_dn;
    w->pos = (double*)calloc((size_t)3 * N, sizeof(double));
    for (int sp = 0; sp < 2; ++sp) {
        int n = orc_spin_count(s, sp);
        w->A[sp] = (double*)calloc((size_t)n * n + 1, sizeof(double));
        w->B[sp] = (double*)calloc((size_t)n * n + 1, sizeof(double));
    }
}

static void orc_walker_free(orc_walker* w)
{
    free(w->pos);
    for (int sp = 0; sp < 2; ++sp) { free(w->A[sp]); free(w->B[sp]); }
}

/* Build the Slater matrices from the positions and invert them. */
static int orc_walker_rebuild(const orc_system* s, orc_walker* w)
{
    const int no = s->n_orb;
    double* v = (double*)malloc(sizeof(double) * no);
    double* g = (double*)malloc(sizeof(double) * 3 * no);
    double* l = (double*)malloc(sizeof(double) * no);
    int bad = 0;
    for (int sp = 0; sp < 2; ++sp) {
        int n = orc_spin_count(s, sp), off = orc_spin_offset(s, sp);
        for (int k = 0; k < n; ++k) {
            orc_spo_vgl(s, w->pos + 3 * (off + k), v, g, l);
            for (int j = 0; j < n; ++j) w->A[sp][k * n + j] = v[j];
        }
        bad |= orc_inverse(n, w->A[sp], w->B[sp], &w->logdet[sp], &w->sign[sp]);
        w->logdet_accum[sp] = w->logdet[sp];
    }
    free(v); free(g); free(l);
    return bad;
}

/* log|Psi| with everything recomputed from scratch (for finite differences). */
double orc_log_psi(const orc_system* s, const double* pos, int* sign)
{
    orc_walker w;
    orc_walker_alloc(s, &w);
    const int N = s->n_up + s->n_dn;
    for (int i = 0; i < 3 * N; ++i) w.pos[i] = pos[i];
    int bad = orc_walker_rebuild(s, &w);
    double lp = w.logdet[0] + w.logdet[1] + orc_jastrow_total(s, pos);
    *sign = bad ? 0 : w.sign[0] * w.sign[1];
    orc_walker_free(&w);
    return bad ? -INFINITY : lp;
}

/* Local energy (section "Hamiltonian": E_L = sum_n Psi^{-1} H_n Psi),
 * kinetic part T_L = -1/2 sum_i [lap_i D/D + 2 grad_i ln D . grad_i J
 * + lap_i J + |grad_i J|^2], from the walker's current inverses.
 * out = (T, V_ee, V_eI, V_II). */
static void orc_measure(const orc_system* s, const orc_walker* w, double v_ii_cached, double out[4])
{
    const int no = s->n_orb;
    double* v = (double*)malloc(sizeof(double) * no);
    double* g = (double*)malloc(sizeof(double) * 3 * no);
    double* l = (double*)malloc(sizeof(double) * no);
    double T = 0.0;
    for (int sp = 0; sp < 2; ++sp) {
        int n = orc_spin_count(s, sp), off = orc_spin_offset(s, sp);
        for (int k = 0; k < n; ++k) {
            int i = off + k;
            orc_spo_vgl(s, w->pos + 3 * i, v, g, l);
            double gD[3] = {0.0, 0.0, 0.0}, lD = 0.0;
            for (int j = 0; j < n; ++j) {
                double b = w->B[sp][j * n + k];
                gD[0] += b * g[j]; gD[1] += b * g[no + j]; gD[2] += b * g[2 * no + j];
                lD += b * l[j];
            }
            double gJ[3], lJ;
            orc_jastrow_grad_lap(s, w->pos, i, gJ, &lJ);
            double dot = gD[0] * gJ[0] + gD[1] * gJ[1] + gD[2] * gJ[2];
            double gJ2 = gJ[0] * gJ[0] + gJ[1] * gJ[1] + gJ[2] * gJ[2];
            T += -0.5 * (lD + 2.0 * dot + lJ + gJ2);
        }
    }
    out[0] = T;
    if (s->coulomb) orc_coulomb(s, w->pos, v_ii_cached, out + 1);
    else out[1] = out[2] = out[3] = 0.0;
    free(v); free(g); free(l);
}

/* Local energy at arbitrary positions (fresh inverses). Returns 0 or 1 (singular). */
int orc_local_energy(const orc_system* s, const double* pos, double out[4])
{
    orc_walker w;
    orc_walker_alloc(s, &w);
    const int N = s->n_up + s->n_dn;
    for (int i = 0; i < 3 * N; ++i) w.pos[i] = orc_wrap(pos[i], s->L);
    int bad = orc_walker_rebuild(s, &w);
    if (!bad) orc_measure(s, &w, NAN, out);
    orc_walker_free(&w);
    return bad;
}

/* One particle-by-particle sweep (section "Trial Moves"): every electron
 * i in index order proposes r' = r_i + sigma xi (no drift, so the
 * transition probabilities cancel in the acceptance), the determinant
 * ratio R = sum_l phi_l(r') B[l][k] and Jastrow change dJ give
 * |Psi'/Psi|^2 = R^2 exp(2 dJ), and the move is accepted iff u < that. */
static void orc_sweep(const orc_system* s, orc_walker* w, uint32_t walker_id, uint32_t sweep,
                      uint8_t* accept_bits)
{
    const int N = s->n_up + s->n_dn, no = s->n_orb;
    double* v = (double*)malloc(sizeof(double) * no);
    double* g = (double*)malloc(sizeof(double) * 3 * no);
    double* l = (double*)malloc(sizeof(double) * no);
    for (int i = 0; i < N; ++i) {
        int sp = orc_spin(s, i), n = orc_spin_count(s, sp), k = i - orc_spin_offset(s, sp);
        double xi[3], rp[3];
        orc_gauss3(s->seed, walker_id, sweep, (uint32_t)i, xi);
        for (int a = 0; a < 3; ++a) rp[a] = orc_wrap(w->pos[3 * i + a] + s->sigma * xi[a], s->L);
        orc_spo_vgl(s, rp, v, g, l);
        double R = 0.0;
        for (int j = 0; j < n; ++j) R += v[j] * w->B[sp][j * n + k];
        double dJ = orc_jastrow_of(s, w->pos, i, rp) - orc_jastrow_of(s, w->pos, i, w->pos + 3 * i);
        double u = orc_accept_uniform(s->seed, walker_id, sweep, (uint32_t)i);
        int acc = u < R * R * exp(2.0 * dJ);
        if (acc) {
            orc_sherman_morrison(n, w->B[sp], k, v, R);
            for (int j = 0; j < n; ++j) w->A[sp][k * n + j] = v[j];
            w->logdet_accum[sp] += log(fabs(R));
            if (R < 0.0) w->sign[sp] = -w->sign[sp];
            for (int a = 0; a < 3; ++a) w->pos[3 * i + a] = rp[a];
        }
        if (accept_bits) accept_bits[i] = (uint8_t)acc;
    }
    free(v); free(g); free(l);
}

/*
 * Particle-by-particle drift-diffusion sweep (section "Trial Moves": the transition
 * probability of one electron's move with the wavefunction force F = 2 grad ln Psi and
 * lambda = 1/2, time step tau = sigma^2).  Electron i, in index order, at the current
 * configuration R (the earlier moves of this sweep already applied):
 *   v   = grad_i ln|Psi(R)| = sum_l grad phi_l(r_i) B[l][k] + grad_i J(R)
 *   r'  = r_i + tau v + sigma xi        (xi from the PROPOSE counters of (walker, sweep, i))
 *   R   = sum_l phi_l(r') B[l][k],  dJ = J(R') - J(R)
 *   v'  = grad_i ln|Psi(R')| = sum_l grad phi_l(r') B[l][k] / R + grad_i J(R')
 *         (the k-th column of the updated inverse is B[:,k] / R)
 *   ln T(R'->R) / T(R->R') = [ |sigma xi|^2 - |sigma xi + tau (v + v')|^2 ] / (2 tau)
 * and the move is accepted iff u < R^2 exp(2 dJ + ln T ratio) (eq. accept_reject), u the
 * ACCEPT draw of (walker, sweep, i).  R = 0 rejects; with fixed_node a move with R < 0
 * (a change of the sign of Psi) is rejected too.  Returns the number of such rejections.
 */
static int orc_drift_sweep(const orc_system* s, orc_walker* w, uint32_t walker_id, uint32_t sweep,
                           uint8_t* accept_bits, int fixed_node)
{
    const int N = s->n_up + s->n_dn, no = s->n_orb;
    const double tau = s->sigma * s->sigma;
    double* v = (double*)malloc(sizeof(double) * no);
    double* g = (double*)malloc(sizeof(double) * 3 * no);
    double* l = (double*)malloc(sizeof(double) * no);
    double* trial = (double*)malloc(sizeof(double) * 3 * (N > 0 ? N : 1));
    int crossings = 0;
    for (int i = 0; i < N; ++i) {
        const int sp = orc_spin(s, i), n = orc_spin_count(s, sp), k = i - orc_spin_offset(s, sp);
        const double* B = w->B[sp];
        double vel[3], gJ[3], lJ, xi[3], sx[3], rp[3];
        orc_spo_vgl(s, w->pos + 3 * i, v, g, l);
        orc_jastrow_grad_lap(s, w->pos, i, gJ, &lJ);
        for (int a = 0; a < 3; ++a) {
            double gd = 0.0;
            for (int j = 0; j < n; ++j) gd += g[a * no + j] * B[j * n + k];
            vel[a] = gd + gJ[a];
        }
        orc_gauss3(s->seed, walker_id, sweep, (uint32_t)i, xi);
        for (int a = 0; a < 3; ++a) {
            sx[a] = s->sigma * xi[a];
            rp[a] = orc_wrap(w->pos[3 * i + a] + tau * vel[a] + sx[a], s->L);
        }
        orc_spo_vgl(s, rp, v, g, l);
        double R = 0.0;
        for (int j = 0; j < n; ++j) R += v[j] * B[j * n + k];
        const double dJ = orc_jastrow_of(s, w->pos, i, rp) - orc_jastrow_of(s, w->pos, i, w->pos + 3 * i);
        const double u = orc_accept_uniform(s->seed, walker_id, sweep, (uint32_t)i);
        const int crossed = fixed_node && R < 0.0;
        int acc = 0;
        if (R != 0.0 && !crossed) {
            memcpy(trial, w->pos, sizeof(double) * 3 * N);
            for (int a = 0; a < 3; ++a) trial[3 * i + a] = rp[a];
            orc_jastrow_grad_lap(s, trial, i, gJ, &lJ);
            double logT = 0.0;
            for (int a = 0; a < 3; ++a) {
                double gd = 0.0;
                for (int j = 0; j < n; ++j) gd += g[a * no + j] * B[j * n + k];
                const double back = sx[a] + tau * (vel[a] + gd / R + gJ[a]);
                logT += (sx[a] * sx[a] - back * back) / (2.0 * tau);
            }
            acc = u < R * R * exp(2.0 * dJ + logT);
        }
        crossings += crossed;
        if (acc) {
            orc_sherman_morrison(n, w->B[sp], k, v, R);
            for (int j = 0; j < n; ++j) w->A[sp][k * n + j] = v[j];
            w->logdet_accum[sp] += log(fabs(R));
            if (R < 0.0) w->sign[sp] = -w->sign[sp];
            for (int a = 0; a < 3; ++a) w->pos[3 * i + a] = rp[a];
        }
        if (accept_bits) accept_bits[i] = (uint8_t)acc;
    }
    free(v); free(g); free(l); free(trial);
    return crossings;
}

/*
 * Drift velocity v_i = grad_i ln|Psi| of every electron at configuration pos with
 * inverses B[sp] (B[l][k]): the log-determinant gradient sum_l grad phi_l(r_i) B[l][k]
 * of the electron's spin block plus the Jastrow gradient.  v: [N][3].
 */
static void orc_drift_velocity(const orc_system* s, const double* pos, double* const B[2], double* vel)
{
    const int no = s->n_orb;
    double* v = (double*)malloc(sizeof(double) * no);
    double* g = (double*)malloc(sizeof(double) * 3 * no);
    double* l = (double*)malloc(sizeof(double) * no);
    for (int sp = 0; sp < 2; ++sp) {
        const int n = orc_spin_count(s, sp), off = orc_spin_offset(s, sp);
        for (int k = 0; k < n; ++k) {
            const int i = off + k;
            orc_spo_vgl(s, pos + 3 * i, v, g, l);
            double gD[3] = {0.0, 0.0, 0.0}, gJ[3], lJ;
            for (int j = 0; j < n; ++j) {
                const double b = B[sp][j * n + k];
                gD[0] += b * g[j]; gD[1] += b * g[no + j]; gD[2] += b * g[2 * no + j];
            }
            orc_jastrow_grad_lap(s, pos, i, gJ, &lJ);
            for (int a = 0; a < 3; ++a) vel[3 * i + a] = gD[a] + gJ[a];
        }
    }
    free(v); free(g); free(l);
}

/*
 * All-electron move (section "Trial Moves", all coordinates proposed together):
 * r'_i = r_i + sigma xi_i for every electron from the PROPOSE counters of the
 * particle-by-particle sweep, one uniform per walker (electron 0's ACCEPT
 * counter), accepted with probability min(1, |Psi(R')/Psi(R)|^2), the ratio from
 * fresh LU determinants of both spin blocks at R' and the change of the full
 * Jastrow factor.  A singular matrix at R' rejects the move.  With fixed_node a move to a
 * configuration where Psi has the other sign is rejected too; returns 1 for such a move.
 *
 * With drift (all_electron == 2) the proposal is drawn from the drift-diffusion
 * transition probability T(R -> R') (eq. trans_prob_alle with the wavefunction force
 * F = 2 grad ln Psi and lambda = 1/2): the time step is tau = sigma^2, the Gaussian
 * has variance 2 lambda tau = tau per coordinate and mean R + lambda tau F = R + tau v(R),
 * v = grad ln|Psi|.  The acceptance (eq. accept_reject) gains T(R' -> R) / T(R -> R'),
 * which with R' - R = tau v(R) + sigma xi is
 *   exp( sum_i [ |sigma xi_i|^2 - |sigma xi_i + tau (v_i(R) + v_i(R'))|^2 ] / (2 tau) ).
 */
static int orc_ae_step(const orc_system* s, orc_walker* w, uint32_t walker_id, uint32_t step,
                       uint8_t* accept_bits, int fixed_node)
{
    const int N = s->n_up + s->n_dn, no = s->n_orb;
    double* rp = (double*)malloc(sizeof(double) * 3 * (N > 0 ? N : 1));
    double* v = (double*)malloc(sizeof(double) * no);
    double* g = (double*)malloc(sizeof(double) * 3 * no);
    double* l = (double*)malloc(sizeof(double) * no);
    const int drift = s->all_electron == 2;
    const double tau = s->sigma * s->sigma;
    double* sx = (double*)malloc(sizeof(double) * 3 * (N > 0 ? N : 1));   /* sigma xi */
    double* vR = (double*)malloc(sizeof(double) * 3 * (N > 0 ? N : 1));
    double* vP = (double*)malloc(sizeof(double) * 3 * (N > 0 ? N : 1));
    if (drift) orc_drift_velocity(s, w->pos, w->B, vR);
    for (int i = 0; i < N; ++i) {
        double xi[3];
        orc_gauss3(s->seed, walker_id, step, (uint32_t)i, xi);
        for (int a = 0; a < 3; ++a) {
            sx[3 * i + a] = s->sigma * xi[a];
            rp[3 * i + a] = drift ? orc_wrap(w->pos[3 * i + a] + tau * vR[3 * i + a] + sx[3 * i + a], s->L)
                                  : orc_wrap(w->pos[3 * i + a] + sx[3 * i + a], s->L);
        }
    }
    double* Ap[2];
    double* Bp[2];
    double ldp[2] = {0.0, 0.0};
    int sgp[2] = {1, 1}, bad = 0;
    for (int sp = 0; sp < 2; ++sp) {
        const int n = orc_spin_count(s, sp), off = orc_spin_offset(s, sp);
        Ap[sp] = (double*)calloc((size_t)n * n + 1, sizeof(double));
        Bp[sp] = (double*)calloc((size_t)n * n + 1, sizeof(double));
        for (int k = 0; k < n; ++k) {
            orc_spo_vgl(s, rp + 3 * (off + k), v, g, l);
            for (int j = 0; j < n; ++j) Ap[sp][k * n + j] = v[j];
        }
        bad |= orc_inverse(n, Ap[sp], Bp[sp], &ldp[sp], &sgp[sp]);
    }
    const double dlog = (ldp[0] - w->logdet[0]) + (ldp[1] - w->logdet[1]);
    const double dJ = orc_jastrow_total(s, rp) - orc_jastrow_total(s, w->pos);
    double logT = 0.0;
    if (drift && !bad) {
        orc_drift_velocity(s, rp, Bp, vP);
        for (int q = 0; q < 3 * N; ++q) {
            const double back = sx[q] + tau * (vR[q] + vP[q]);
            logT += (sx[q] * sx[q] - back * back) / (2.0 * tau);
        }
    }
    const double u = orc_accept_uniform(s->seed, walker_id, step, 0u);
    /* fixed node (section "Diffusion Monte Carlo"): a move that changes the sign of the
     * wavefunction (the Jastrow factor is positive, so the sign of D_up D_dn) is rejected */
    const int crossed = fixed_node && !bad && sgp[0] * sgp[1] != w->sign[0] * w->sign[1];
    const int acc = !bad && !crossed && u < exp(2.0 * (dlog + dJ) + logT);
    if (acc) {
        for (int sp = 0; sp < 2; ++sp) {
            double* t = w->A[sp]; w->A[sp] = Ap[sp]; Ap[sp] = t;
            t = w->B[sp]; w->B[sp] = Bp[sp]; Bp[sp] = t;
            w->logdet[sp] = ldp[sp];
            w->logdet_accum[sp] = ldp[sp];
            w->sign[sp] = sgp[sp];
        }
        memcpy(w->pos, rp, sizeof(double) * 3 * N);
    }
    if (accept_bits)
        for (int i = 0; i < N; ++i) accept_bits[i] = (uint8_t)acc;
    for (int sp = 0; sp < 2; ++sp) { free(Ap[sp]); free(Bp[sp]); }
    free(rp); free(v); free(g); free(l); free(sx); free(vR); free(vP);
    return crossed;
}

/*
 * Run independent walkers (section "Variational Monte Carlo": walkers are
 * independent Markov chains).  walker_ids[w] selects the random streams of
 * chain w, so any subset of a large run can be reproduced alone.
 *
 *   init_pos     : [n_walk][N][3] or NULL (positions from the INIT stream)
 *   sweep0       : global index of the first sweep (random-stream index)
 *   measure_every: measure after sweep s when (s+1) % measure_every == 0
 *                  (0 = never); energies[n_walk][n_meas][4]
 *   accept_bits  : [n_walk][n_sweeps][N] or NULL
 *   pos_trace    : [n_walk][n_sweeps][N][3] or NULL (positions after each sweep)
 *   final_pos    : [n_walk][N][3] or NULL
 *   logdet       : [n_walk][2] accumulated log|D| (sum of log|R| from the start)
 *   sign         : [n_walk][2]
 *   logdet_lu    : [n_walk][2] log|D| from a fresh LU of the final positions, or NULL
 * Returns 0, or 1 + walker index of the first walker whose Slater matrix
 * was singular at initialisation.
 */
/* Initial configuration of walker wid: the given positions (wrapped), or uniform draws in
 * the cell from the INIT stream.  Returns nonzero if a Slater matrix is singular. */
static int orc_walker_init(const orc_system* s, orc_walker* w, uint32_t wid, const double* pos)
{
    const int N = s->n_up + s->n_dn;
    if (pos) {
        for (int i = 0; i < 3 * N; ++i) w->pos[i] = orc_wrap(pos[i], s->L);
    } else {
        for (int i = 0; i < N; ++i) orc_init_position(s->seed, wid, (uint32_t)i, s->L, w->pos + 3 * i);
    }
    return orc_walker_rebuild(s, w);
}

int orc_vmc_run(const orc_system* s, int n_walk, const int32_t* walker_ids, const double* init_pos,
                int sweep0, int n_sweeps, int measure_every, double* energies, uint8_t* accept_bits,
                double* pos_trace, double* final_pos, double* logdet, int32_t* sign, double* logdet_lu,
                int n_threads)
{
    const int N = s->n_up + s->n_dn;
    const int n_meas = measure_every > 0 ? n_sweeps / measure_every : 0;
    double v_ii = NAN;
    if (s->coulomb && s->n_ions > 0) {
        double* q = (double*)malloc(sizeof(double) * s->n_ions);
        for (int I = 0; I < s->n_ions; ++I) q[I] = s->ion_Z[I];
        v_ii = orc_ewald(s->n_ions, s->ion_pos, q, s->L, s->ewald_kappa);
        free(q);
    }
    int first_bad = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int wi = 0; wi < n_walk; ++wi) {
        orc_walker w;
        orc_walker_alloc(s, &w);
        uint32_t wid = (uint32_t)walker_ids[wi];
        int bad_init = orc_walker_init(s, &w, wid, init_pos ? init_pos + (size_t)wi * N * 3 : NULL);
        if (bad_init) {
#ifdef _OPENMP
#pragma omp critical
#endif
            { if (!first_bad || wi + 1 < first_bad) first_bad = wi + 1; }
            orc_walker_free(&w);
            continue;
        }
        int im = 0;
        for (int st = 0; st < n_sweeps; ++st) {
            uint8_t* bits = accept_bits ? accept_bits + ((size_t)wi * n_sweeps + st) * N : NULL;
            if (s->all_electron == 3) orc_drift_sweep(s, &w, wid, (uint32_t)(sweep0 + st), bits, 0);
            else if (s->all_electron) orc_ae_step(s, &w, wid, (uint32_t)(sweep0 + st), bits, 0);
            else orc_sweep(s, &w, wid, (uint32_t)(sweep0 + st), bits);
            if (pos_trace) memcpy(pos_trace + ((size_t)wi * n_sweeps + st) * N * 3, w.pos, sizeof(double) * 3 * N);
            if (measure_every > 0 && (st + 1) % measure_every == 0 && im < n_meas) {
                orc_measure(s, &w, v_ii, energies + ((size_t)wi * n_meas + im) * 4);
                ++im;
            }
        }
        if (final_pos) memcpy(final_pos + (size_t)wi * N * 3, w.pos, sizeof(double) * 3 * N);
        if (logdet) { logdet[2 * wi] = w.logdet_accum[0]; logdet[2 * wi + 1] = w.logdet_accum[1]; }
        if (sign) { sign[2 * wi] = w.sign[0]; sign[2 * wi + 1] = w.sign[1]; }
        if (logdet_lu) {
            int bad = orc_walker_rebuild(s, &w);
            logdet_lu[2 * wi] = bad ? NAN : w.logdet[0];
            logdet_lu[2 * wi + 1] = bad ? NAN : w.logdet[1];
        }
        orc_walker_free(&w);
    }
    return first_bad;
}

/* Deep copy of a walker's state: positions, Slater matrices, inverses, log|D| and signs. */
static void orc_walker_copy(const orc_system* s, orc_walker* dst, const orc_walker* src)
{
    const int N = s->n_up + s->n_dn;
    memcpy(dst->pos, src->pos, sizeof(double) * 3 * N);
    for (int sp = 0; sp < 2; ++sp) {
        const int n = orc_spin_count(s, sp);
        memcpy(dst->A[sp], src->A[sp], sizeof(double) * ((size_t)n * n + 1));
        memcpy(dst->B[sp], src->B[sp], sizeof(double) * ((size_t)n * n + 1));
        dst->logdet[sp] = src->logdet[sp];
        dst->sign[sp] = src->sign[sp];
        dst->logdet_accum[sp] = src->logdet_accum[sp];
    }
}

/*
 * Diffusion Monte Carlo (section "Diffusion Monte Carlo") on a population held in n_slots
 * walker slots, of which the first n_target start alive with weight 1 from the INIT stream
 * (walker id = slot).  Step k (moves use sweep index sweep0 + k):
 *   1. every alive walker makes one drift-diffusion all-electron move (eq.
 *      pmc:driftdiffusion_step with the Metropolis acceptance of eq. accept_reject), or one
 *      particle-by-particle drift-diffusion sweep, a move that crosses a node (changes the
 *      sign of Psi) being rejected (fixed node);
 *   2. w <- w G_B with G_B = exp(-tau (E_L(R) + E_L(R_new) - 2 E_T) / 2) (eqs.
 *      pmc:g_growth, pmc:walker_weight), tau = sigma^2, R_new the configuration after the
 *      move (R itself when rejected);
 *   3. the mixed estimate E = sum w E_L / sum w over alive walkers (eq.
 *      pmc:weighted_average);
 *   4. branching: M = INT(w + xi) copies of every alive walker (xi from the BRANCH stream of
 *      (slot, k)), at most n_slots; walkers with M = 0 die; a walker with M >= 1 keeps its
 *      slot and its M - 1 extra copies take the free slots (slots of dead walkers) in
 *      ascending order, the copies of lower slots first; copies beyond the free slots, and
 *      those a multiplicity above n_slots asked for, are dropped (and counted); every
 *      walker alive after branching has weight 1;
 *   5. E_T <- E - feedback ln(population / n_target).
 * Outputs (each nullable): stats[k] = (E, sum w, population after branching, E_T used in
 * step k, dropped copies, moves rejected for crossing a node); weights[k][slot] = w after step 2 (0 for dead slots);
 * mult[k][slot] = M (0 for dead); plan[k][slot] = source slot of a copy placed there, or -1;
 * energies[k][slot] = E_L after the move (alive slots); final_pos[slot][N][3] and
 * final_sign[slot] (sign of D_up D_dn) after the last step (alive slots).
 * Returns 0, 1 + slot of a singular initial walker, -1 if the population dies out, -2 if
 * the system makes no drift-diffusion moves.
 */
int orc_dmc_run(const orc_system* s, int n_slots, int n_target, double e_trial, double feedback, int sweep0,
                int n_steps, double* stats, double* weights, int32_t* mult, int32_t* plan, double* energies,
                double* final_pos, int32_t* final_sign, int n_threads)
{
    if (s->all_electron != 2 && s->all_electron != 3) return -2;
    const int N = s->n_up + s->n_dn;
    const double tau = s->sigma * s->sigma;
    double v_ii = NAN;
    if (s->coulomb && s->n_ions > 0) {
        double* q = (double*)malloc(sizeof(double) * s->n_ions);
        for (int I = 0; I < s->n_ions; ++I) q[I] = s->ion_Z[I];
        v_ii = orc_ewald(s->n_ions, s->ion_pos, q, s->L, s->ewald_kappa);
        free(q);
    }
    orc_walker* W = (orc_walker*)calloc((size_t)n_slots, sizeof(orc_walker));
    double* w = (double*)calloc((size_t)n_slots, sizeof(double));
    double* E = (double*)calloc((size_t)n_slots, sizeof(double));
    int* alive = (int*)calloc((size_t)n_slots, sizeof(int));
    int* M = (int*)calloc((size_t)n_slots, sizeof(int));
    int* pl = (int*)calloc((size_t)n_slots, sizeof(int));
    int* crossed = (int*)calloc((size_t)n_slots, sizeof(int));
    for (int j = 0; j < n_slots; ++j) orc_walker_alloc(s, &W[j]);
    int ret = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    int first_bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int j = 0; j < n_target; ++j) {
        const int bad = orc_walker_init(s, &W[j], (uint32_t)j, NULL);
        double o[4] = {0.0, 0.0, 0.0, 0.0};
        if (!bad) orc_measure(s, &W[j], v_ii, o);
        E[j] = o[0] + o[1] + o[2] + o[3];
#ifdef _OPENMP
#pragma omp critical
#endif
        { if (bad && (!first_bad || j + 1 < first_bad)) first_bad = j + 1; }
    }
    if (first_bad) { ret = first_bad; goto done; }
    for (int j = 0; j < n_target; ++j) { alive[j] = 1; w[j] = 1.0; }
    if (!isfinite(e_trial)) {
        double se = 0.0;
        for (int j = 0; j < n_target; ++j) se += E[j];
        e_trial = se / n_target;
    }
    for (int k = 0; k < n_steps; ++k) {
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
        for (int j = 0; j < n_slots; ++j) {
            if (!alive[j]) continue;
            crossed[j] = s->all_electron == 3 ? orc_drift_sweep(s, &W[j], (uint32_t)j, (uint32_t)(sweep0 + k), NULL, 1)
                                              : orc_ae_step(s, &W[j], (uint32_t)j, (uint32_t)(sweep0 + k), NULL, 1);
            double o[4];
            orc_measure(s, &W[j], v_ii, o);
            const double en = o[0] + o[1] + o[2] + o[3];
            w[j] *= exp(-tau * (E[j] + en - 2.0 * e_trial) / 2.0);
            E[j] = en;
        }
        double sw = 0.0, swe = 0.0;
        int n_crossed = 0;
        for (int j = 0; j < n_slots; ++j)
            if (alive[j]) { sw += w[j]; swe += w[j] * E[j]; n_crossed += crossed[j]; }
        const double emix = swe / sw;
        if (weights) for (int j = 0; j < n_slots; ++j) weights[(size_t)k * n_slots + j] = alive[j] ? w[j] : 0.0;
        if (energies) for (int j = 0; j < n_slots; ++j) energies[(size_t)k * n_slots + j] = alive[j] ? E[j] : NAN;
        /* M = INT(w + xi), at most n_slots: a slot's copies beyond the capacity could never be
         * placed; every copy that is not placed (over the capacity or over the free slots)
         * counts as dropped */
        double raw_extra = 0.0;
        for (int j = 0; j < n_slots; ++j) {
            M[j] = 0;
            if (!alive[j]) continue;
            const double mr = floor(w[j] + orc_branch_uniform(s->seed, (uint32_t)j, (uint32_t)k));
            M[j] = mr < (double)n_slots ? (int)mr : n_slots;
            if (mr >= 1.0) raw_extra += mr - 1.0;
        }
        /* extra copies (source slot ascending) into free slots (ascending) */
        int src = 0, left = 0;   /* the source of the next extra copy and its copies still to place */
        while (src < n_slots && M[src] < 2) ++src;
        if (src < n_slots) left = M[src] - 1;
        long placed = 0;
        for (int f = 0; f < n_slots; ++f) {
            pl[f] = -1;
            if (M[f] != 0) continue;
            if (src < n_slots) {
                pl[f] = src;
                ++placed;
                if (--left == 0) {
                    ++src;
                    while (src < n_slots && M[src] < 2) ++src;
                    if (src < n_slots) left = M[src] - 1;
                }
            }
        }
        const double dropped = raw_extra - (double)placed;
        for (int f = 0; f < n_slots; ++f)
            if (pl[f] >= 0) { orc_walker_copy(s, &W[f], &W[pl[f]]); E[f] = E[pl[f]]; }
        int pop = 0;
        for (int j = 0; j < n_slots; ++j) {
            alive[j] = M[j] >= 1 || pl[j] >= 0;
            w[j] = alive[j] ? 1.0 : 0.0;
            pop += alive[j];
        }
        if (mult) for (int j = 0; j < n_slots; ++j) mult[(size_t)k * n_slots + j] = M[j];
        if (plan) for (int j = 0; j < n_slots; ++j) plan[(size_t)k * n_slots + j] = pl[j];
        if (stats) {
            double* st = stats + (size_t)k * 6;
            st[0] = emix; st[1] = sw; st[2] = pop; st[3] = e_trial; st[4] = (double)dropped;
            st[5] = n_crossed;
        }
        if (pop == 0) { ret = -1; goto done; }
        e_trial = emix - feedback * log((double)pop / n_target);
    }
    for (int j = 0; j < n_slots; ++j) {
        if (final_pos) {
            if (alive[j]) memcpy(final_pos + (size_t)j * N * 3, W[j].pos, sizeof(double) * 3 * N);
            else for (int q = 0; q < 3 * N; ++q) final_pos[(size_t)j * N * 3 + q] = NAN;
        }
        if (final_sign) final_sign[j] = alive[j] ? W[j].sign[0] * W[j].sign[1] : 0;
    }
done:
    for (int j = 0; j < n_slots; ++j) orc_walker_free(&W[j]);
    free(W); free(w); free(E); free(alive); free(M); free(pl); free(crossed);
    return ret;
}

/* Number of threads the OpenMP runtime would use. */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
