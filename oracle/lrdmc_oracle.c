/*
 * CPU oracle for the double-grid lattice-regularized diffusion Monte Carlo
 * (LRDMC) projection step of Nakano, Maezono & Sorella, arXiv:1909.01589.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark load this file.  It shares no code, header or
 * table with the HIP library.
 *
 * Plain, slow, FP64.  Each quantity is computed from its definition:
 *   - Psi(x) = det A_up * det A_dn * exp(J), determinants by LU with partial
 *     pivoting, J summed over all pairs;
 *   - every move ratio Psi(x')/Psi(x) recomputes the moved spin's
 *     determinant from scratch and the whole Jastrow factor (no
 *     Sherman-Morrison, no incremental updates);
 *   - the local energy uses the textbook analytic derivatives;
 *   - cumulative sums are sequential, left to right.
 *
 * Pins: every function here is checked by the CPU tests against what the
 * paper and the mathematics fix (closed forms, brute force on small inputs,
 * the printed values of Table S-I and S-II, statistical limits).  Parity
 * unpinned: the absolute energies of the random-MO workloads (Be-like,
 * Ar-like, Z-sweep, molecule) have no reference value; they are checked only
 * through parity with the GPU path.
 *
 * Method passages (paper numbering):
 *   main text Eq. (1): Laplacian split into a small-spacing part weighted by
 *     p and a large-spacing part weighted by 1-p;
 *   main text Eq. (3): Gaussian switch p(r) around the nearest heavy nucleus;
 *   "Application to large systems": R_c over the heaviest nuclei only.
 * The rest (stencil, regularized potential, fixed-node rule, continuous-time
 * projection, reconfiguration) is the standard LRDMC the paper cites
 * (Casula, Filippi & Sorella 2005).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n_nuc;
    const double *Z;          /* [n_nuc] */
    const double *R;          /* [n_nuc][3] */
    int32_t n_up, n_dn;
    int32_t n_shell;
    const int32_t *shell_nuc; /* [n_shell] */
    const int32_t *shell_l;   /* [n_shell], 0..2 */
    const double *shell_alpha;/* [n_shell] */
    int32_t n_orb;
    const double *mo;         /* [K][n_orb] */
    double b_ee, b_en;
    /* optional learned Jastrow correction (NULL: Pade only): F_ee(r) is added
     * to every electron pair term, Z_I F_en(r) to every electron-nucleus
     * term, for r < ftab_rcut; F is the piecewise quintic Hermite
     * interpolant of the table ftab[2][ftab_n][3] = {F, F', F''} at the
     * nodes r_k = k ftab_rcut / (ftab_n - 1) (type 0: e-e, 1: e-n). */
    const double *ftab;
    int32_t ftab_n;
    double ftab_rcut;
} orc_system;

typedef struct {
    double a, a_prime, r_c, z_heavy, tau;
    uint64_t seed;
    int32_t rotate;
    int32_t switch_form;      /* 0: Gaussian switch, Eq. (3); 1: Pade switch, Eq. (2) */
    int32_t grids;            /* 2: double grid (Eq. (1)); 1: single grid of spacing a */
    int32_t pad;
} orc_params;

/* Moves per electron: two grids x three axes x two signs, or one grid. */
static int moves_per_electron(const orc_params *p) { return p->grids == 1 ? 6 : 12; }

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ESINGULAR = -2, ORC_ENONFINITE = -3, ORC_ENOMEM = -4 };

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11), from its definition. */

static void philox_round(uint64_t c[4], const uint64_t k[2])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    unsigned __int128 p0 = (unsigned __int128)M0 * c[0];
    unsigned __int128 p1 = (unsigned __int128)M1 * c[2];
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c[1] ^ k[0];
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c[3] ^ k[1];
    uint64_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint64_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B97F4A7C15ULL;
            k[1] += 0xBB67AE8584CAA73BULL;
        }
        philox_round(c, k);
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

/* Uniform in (0,1): top 53 bits, centred in their interval. */
double orc_u01(uint64_t x)
{
    return ((double)(x >> 11) + 0.5) * 0x1.0p-53;
}

/* Four uniforms for counter (slot, generation, iteration, purpose). */
void orc_draw(uint64_t seed, uint64_t slot, uint64_t gen, uint64_t iter,
              uint64_t purpose, double u[4])
{
    uint64_t ctr[4] = {slot, gen, iter, purpose}, key[2] = {seed, 0}, o[4];
    orc_philox4x64_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = orc_u01(o[i]);
}

/* Uniform random rotation from three uniforms (Shoemake, Graphics Gems III,
 * "Uniform random rotations").  Rm is row-major; its columns are the three
 * lattice axes e_1, e_2, e_3. */
void orc_rotation(const double u[3], double Rm[9])
{
    const double two_pi = 6.283185307179586476925286766559;
    double r1 = sqrt(1.0 - u[0]), r2 = sqrt(u[0]);
    double t1 = two_pi * u[1], t2 = two_pi * u[2];
    double x = sin(t1) * r1, y = cos(t1) * r1, z = sin(t2) * r2, w = cos(t2) * r2;
    Rm[0] = 1.0 - 2.0 * (y * y + z * z);
    Rm[1] = 2.0 * (x * y - w * z);
    Rm[2] = 2.0 * (x * z + w * y);
    Rm[3] = 2.0 * (x * y + w * z);
    Rm[4] = 1.0 - 2.0 * (x * x + z * z);
    Rm[5] = 2.0 * (y * z - w * x);
    Rm[6] = 2.0 * (x * z - w * y);
    Rm[7] = 2.0 * (y * z + w * x);
    Rm[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* ------------------------------------------------------------------------ */
/* Basis and orbitals                                                         */

int orc_nbasis(const orc_system *s)
{
    int K = 0;
    for (int q = 0; q < s->n_shell; ++q) K += 2 * s->shell_l[q] + 1;
    return K;
}

/* Polynomial parts of one shell at displacement d: values P[c], gradients
 * dP[c][3] and Laplacians lP[c].  l=2 uses the five real harmonic forms
 * xy, yz, zx, x^2-y^2, 2z^2-x^2-y^2. */
static int shell_poly(int l, const double d[3], double *P, double (*dP)[3], double *lP)
{
    double x = d[0], y = d[1], z = d[2];
    if (l == 0) {
        P[0] = 1.0; dP[0][0] = dP[0][1] = dP[0][2] = 0.0; lP[0] = 0.0;
        return 1;
    }
    if (l == 1) {
        for (int c = 0; c < 3; ++c) {
            P[c] = d[c];
            dP[c][0] = dP[c][1] = dP[c][2] = 0.0;
            dP[c][c] = 1.0;
            lP[c] = 0.0;
        }
        return 3;
    }
    /* l == 2 */
    P[0] = x * y;  dP[0][0] = y;   dP[0][1] = x;  dP[0][2] = 0;   lP[0] = 0.0;
    P[1] = y * z;  dP[1][0] = 0;   dP[1][1] = z;  dP[1][2] = y;   lP[1] = 0.0;
    P[2] = z * x;  dP[2][0] = z;   dP[2][1] = 0;  dP[2][2] = x;   lP[2] = 0.0;
    P[3] = x * x - y * y;
    dP[3][0] = 2 * x; dP[3][1] = -2 * y; dP[3][2] = 0;  lP[3] = 2.0 - 2.0;
    P[4] = 2 * z * z - x * x - y * y;
    dP[4][0] = -2 * x; dP[4][1] = -2 * y; dP[4][2] = 4 * z; lP[4] = 4.0 - 2.0 - 2.0;
    return 5;
}

/* g(r) = P(d) e^{-alpha d^2}; grad g = (grad P - 2 alpha d P) e;
 * lap g = (lap P - 4 alpha d.grad P + (4 alpha^2 d^2 - 6 alpha) P) e. */
void orc_basis(const orc_system *s, const double r[3], double *val, double *grad, double *lap)
{
    int mu = 0;
    for (int q = 0; q < s->n_shell; ++q) {
        const double *Rn = s->R + 3 * s->shell_nuc[q];
        double d[3] = {r[0] - Rn[0], r[1] - Rn[1], r[2] - Rn[2]};
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double al = s->shell_alpha[q];
        double e = exp(-al * d2);
        double P[5], dP[5][3], lP[5];
        int nc = shell_poly(s->shell_l[q], d, P, dP, lP);
        for (int c = 0; c < nc; ++c, ++mu) {
            double ddotgP = d[0] * dP[c][0] + d[1] * dP[c][1] + d[2] * dP[c][2];
            if (val) val[mu] = P[c] * e;
            if (grad)
                for (int k = 0; k < 3; ++k) grad[3 * mu + k] = (dP[c][k] - 2.0 * al * d[k] * P[c]) * e;
            if (lap)
                lap[mu] = (lP[c] - 4.0 * al * ddotgP + (4.0 * al * al * d2 - 6.0 * al) * P[c]) * e;
        }
    }
}

/* phi_j(r) = sum_mu C[mu][j] g_mu(r) for j < n; optional gradients and
 * Laplacians. */
static void orbitals_at(const orc_system *s, const double r[3], int n,
                        double *phi, double *dphi, double *lphi, double *work)
{
    int K = orc_nbasis(s);
    double *g = work, *gg = work + K, *lg = work + 4 * K;
    orc_basis(s, r, g, dphi ? gg : NULL, lphi ? lg : NULL);
    for (int j = 0; j < n; ++j) {
        double v = 0, gx = 0, gy = 0, gz = 0, l = 0;
        for (int mu = 0; mu < K; ++mu) {
            double c = s->mo[(size_t)mu * s->n_orb + j];
            v += c * g[mu];
            if (dphi) { gx += c * gg[3 * mu]; gy += c * gg[3 * mu + 1]; gz += c * gg[3 * mu + 2]; }
            if (lphi) l += c * lg[mu];
        }
        phi[j] = v;
        if (dphi) { dphi[3 * j] = gx; dphi[3 * j + 1] = gy; dphi[3 * j + 2] = gz; }
        if (lphi) lphi[j] = l;
    }
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra: LU with partial pivoting (row interchanges).        */

/* In place; returns log|det|, sets *sign (0 if singular). */
static double lu_logdet(double *A, int n, int *sign)
{
    int sg = 1;
    double la = 0.0;
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = fabs(A[c * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > best) { best = fabs(A[r * n + c]); p = r; }
        if (!(best > 0.0)) { *sign = 0; return -INFINITY; }
        if (p != c) {
            for (int k = 0; k < n; ++k) { double t = A[c * n + k]; A[c * n + k] = A[p * n + k]; A[p * n + k] = t; }
            sg = -sg;
        }
        double piv = A[c * n + c];
        if (piv < 0) sg = -sg;
        la += log(fabs(piv));
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / piv;
            A[r * n + c] = f;
            for (int k = c + 1; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
        }
    }
    *sign = sg;
    return la;
}

/* Inverse by LU: solves A X = I column by column.  Returns 0 or -2. */
static int lu_inverse(const double *A, int n, double *X, double *work, int *perm)
{
    double *L = work;
    memcpy(L, A, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = fabs(L[c * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (fabs(L[r * n + c]) > best) { best = fabs(L[r * n + c]); p = r; }
        if (!(best > 0.0) || !isfinite(best)) return ORC_ESINGULAR;
        if (p != c) {
            for (int k = 0; k < n; ++k) { double t = L[c * n + k]; L[c * n + k] = L[p * n + k]; L[p * n + k] = t; }
            int t = perm[c]; perm[c] = perm[p]; perm[p] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            double f = L[r * n + c] / L[c * n + c];
            L[r * n + c] = f;
            for (int k = c + 1; k < n; ++k) L[r * n + k] -= f * L[c * n + k];
        }
    }
    for (int col = 0; col < n; ++col) {
        /* b = P e_col */
        double *x = X; /* solve into column col of X (row-major X[row][col]) */
        double y[64];
        for (int r = 0; r < n; ++r) y[r] = (perm[r] == col) ? 1.0 : 0.0;
        for (int r = 0; r < n; ++r)
            for (int k = 0; k < r; ++k) y[r] -= L[r * n + k] * y[k];
        for (int r = n - 1; r >= 0; --r) {
            double v = y[r];
            for (int k = r + 1; k < n; ++k) v -= L[r * n + k] * x[k * n + col];
            x[r * n + col] = v / L[r * n + r];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Pade Jastrow: J = sum_{i<j} c_ij r/(1+b_ee r) - sum_{i,I} Z_I r/(1+b_en r),
 * c = 1/2 antiparallel, 1/4 parallel (exact cusps).                          */

static int spin_of(const orc_system *s, int i) { return i < s->n_up ? 0 : 1; }

/* The quintic Hermite basis on t in [0, 1] that matches value, first and
 * second derivative at both ends (the interpolant is C^2 across nodes):
 * p(t) = f0 H0 + f0' H1 + f0'' H2 + f1 H3 + f1' H4 + f1'' H5 in units of
 * the interval (derivatives scaled by h, h^2).  Also its first and second
 * t-derivatives. */
static void hermite5(double t, double H[6], double dH[6], double d2H[6])
{
    double t2 = t * t, t3 = t2 * t, t4 = t3 * t, t5 = t4 * t;
    H[0] = 1.0 - 10.0 * t3 + 15.0 * t4 - 6.0 * t5;
    H[1] = t - 6.0 * t3 + 8.0 * t4 - 3.0 * t5;
    H[2] = 0.5 * (t2 - 3.0 * t3 + 3.0 * t4 - t5);
    H[3] = 10.0 * t3 - 15.0 * t4 + 6.0 * t5;
    H[4] = -4.0 * t3 + 7.0 * t4 - 3.0 * t5;
    H[5] = 0.5 * (t3 - 2.0 * t4 + t5);
    dH[0] = -30.0 * t2 + 60.0 * t3 - 30.0 * t4;
    dH[1] = 1.0 - 18.0 * t2 + 32.0 * t3 - 15.0 * t4;
    dH[2] = 0.5 * (2.0 * t - 9.0 * t2 + 12.0 * t3 - 5.0 * t4);
    dH[3] = 30.0 * t2 - 60.0 * t3 + 30.0 * t4;
    dH[4] = -12.0 * t2 + 28.0 * t3 - 15.0 * t4;
    dH[5] = 0.5 * (3.0 * t2 - 8.0 * t3 + 5.0 * t4);
    d2H[0] = -60.0 * t + 180.0 * t2 - 120.0 * t3;
    d2H[1] = -36.0 * t + 96.0 * t2 - 60.0 * t3;
    d2H[2] = 0.5 * (2.0 - 18.0 * t + 36.0 * t2 - 20.0 * t3);
    d2H[3] = 60.0 * t - 180.0 * t2 + 120.0 * t3;
    d2H[4] = -24.0 * t + 84.0 * t2 - 60.0 * t3;
    d2H[5] = 0.5 * (6.0 * t - 24.0 * t2 + 20.0 * t3);
}

/* Learned correction of table type (0: e-e, 1: e-n) at distance r, with its
 * first and second r-derivatives; zero without a table or beyond the cutoff. */
void orc_corr(const orc_system *s, int type, double r, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    if (!s->ftab || s->ftab_n < 2 || !(r < s->ftab_rcut)) return;
    double h = s->ftab_rcut / (s->ftab_n - 1);
    double x = r / h;
    int k = (int)floor(x);
    if (k > s->ftab_n - 2) k = s->ftab_n - 2;
    double t = x - k;
    const double *a = s->ftab + 3 * ((size_t)type * s->ftab_n + k), *b = a + 3;
    double c[6] = {a[0], h * a[1], h * h * a[2], b[0], h * b[1], h * h * b[2]};
    double H[6], dH[6], d2H[6];
    hermite5(t, H, dH, d2H);
    for (int q = 0; q < 6; ++q) {
        out[0] += c[q] * H[q];
        out[1] += c[q] * dH[q] / h;
        out[2] += c[q] * d2H[q] / (h * h);
    }
}

static double dist(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

double orc_jastrow(const orc_system *s, const double *pos)
{
    int N = s->n_up + s->n_dn;
    double J = 0.0;
    for (int i = 0; i < N; ++i) {
        for (int j = i + 1; j < N; ++j) {
            double c = (spin_of(s, i) == spin_of(s, j)) ? 0.25 : 0.5;
            double r = dist(pos + 3 * i, pos + 3 * j);
            double F[3];
            orc_corr(s, 0, r, F);
            J += c * r / (1.0 + s->b_ee * r) + F[0];
        }
        for (int I = 0; I < s->n_nuc; ++I) {
            double r = dist(pos + 3 * i, s->R + 3 * I);
            double F[3];
            orc_corr(s, 1, r, F);
            J -= s->Z[I] * r / (1.0 + s->b_en * r);
            J += s->Z[I] * F[0];
        }
    }
    return J;
}

/* grad_i J and lap_i J. */
static void jastrow_derivs(const orc_system *s, const double *pos, int i, double g[3], double *lap)
{
    int N = s->n_up + s->n_dn;
    g[0] = g[1] = g[2] = 0.0;
    double L = 0.0;
    for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        double c = (spin_of(s, i) == spin_of(s, j)) ? 0.25 : 0.5;
        double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1], pos[3 * i + 2] - pos[3 * j + 2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double q = 1.0 + s->b_ee * r;
        double F[3];
        orc_corr(s, 0, r, F);
        double up = c / (q * q) + F[1];                       /* u'(r)  */
        double upp = -2.0 * c * s->b_ee / (q * q * q) + F[2]; /* u''(r) */
        for (int k = 0; k < 3; ++k) g[k] += up * d[k] / r;
        L += upp + 2.0 * up / r;
    }
    for (int I = 0; I < s->n_nuc; ++I) {
        double d[3] = {pos[3 * i] - s->R[3 * I], pos[3 * i + 1] - s->R[3 * I + 1], pos[3 * i + 2] - s->R[3 * I + 2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double q = 1.0 + s->b_en * r;
        double Z = s->Z[I];
        double F[3];
        orc_corr(s, 1, r, F);
        double up = -Z / (q * q) + Z * F[1];
        double upp = 2.0 * Z * s->b_en / (q * q * q) + Z * F[2];
        for (int k = 0; k < 3; ++k) g[k] += up * d[k] / r;
        L += upp + 2.0 * up / r;
    }
    *lap = L;
}

/* ------------------------------------------------------------------------ */
/* Wave function                                                              */

static int nspin(const orc_system *s, int sg) { return sg == 0 ? s->n_up : s->n_dn; }
static int first_of(const orc_system *s, int sg) { return sg == 0 ? 0 : s->n_up; }

/* Slater matrix of one spin: A[i][j] = phi_j(r_i), i, j < n_sigma. */
static void slater_matrix(const orc_system *s, const double *pos, int sg, double *A, double *work)
{
    int n = nspin(s, sg), i0 = first_of(s, sg);
    for (int i = 0; i < n; ++i) orbitals_at(s, pos + 3 * (i0 + i), n, A + i * n, NULL, NULL, work);
}

/* 5K doubles for orbitals_at, then room for one n_sigma x n_sigma matrix. */
static double *scratch(const orc_system *s)
{
    int K = orc_nbasis(s), N = s->n_up + s->n_dn;
    return (double *)malloc(sizeof(double) * ((size_t)5 * K + (size_t)N * N + 1));
}

/* log|Psi| and sign(Psi). */
int orc_log_psi(const orc_system *s, const double *pos, double *logabs, int *sign)
{
    int N = s->n_up + s->n_dn;
    double *w = scratch(s);
    double *A = w + 5 * orc_nbasis(s);
    if (!w) return ORC_ENOMEM;
    double la = 0.0;
    int sg_total = 1;
    for (int sg = 0; sg < 2; ++sg) {
        int n = nspin(s, sg);
        if (n == 0) continue;
        slater_matrix(s, pos, sg, A, w);
        int sgn;
        la += lu_logdet(A, n, &sgn);
        sg_total *= sgn;
    }
    la += orc_jastrow(s, pos);
    (void)N;
    free(w);
    *logabs = la;
    *sign = sg_total;
    return sg_total == 0 ? ORC_ESINGULAR : ORC_OK;
}

/* Coulomb potential: e-e, e-n and n-n terms. */
double orc_potential(const orc_system *s, const double *pos)
{
    int N = s->n_up + s->n_dn;
    double V = 0.0;
    for (int i = 0; i < N; ++i) {
        for (int j = i + 1; j < N; ++j) V += 1.0 / dist(pos + 3 * i, pos + 3 * j);
        for (int I = 0; I < s->n_nuc; ++I) V -= s->Z[I] / dist(pos + 3 * i, s->R + 3 * I);
    }
    for (int I = 0; I < s->n_nuc; ++I)
        for (int J = I + 1; J < s->n_nuc; ++J) V += s->Z[I] * s->Z[J] / dist(s->R + 3 * I, s->R + 3 * J);
    return V;
}

/* Analytic local energy E_L = -1/2 sum_i lap_i Psi / Psi + V.
 * lap_i Psi/Psi = lap_i D/D + 2 grad_i D/D . grad_i J + lap_i J + |grad_i J|^2,
 * grad_i D/D = sum_j grad phi_j(r_i) Ainv[j][i], lap likewise.
 * Outputs: e_l, lap_psi (sum_i lap_i Psi/Psi), v (potential). */
int orc_local_energy(const orc_system *s, const double *pos, double *e_l, double *lap_psi, double *v)
{
    int K = orc_nbasis(s), nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
    if (nmax > 64) return ORC_EINVAL;
    size_t n2 = (size_t)nmax * nmax;
    double *w = (double *)malloc(sizeof(double) * (5 * (size_t)K + 7 * n2 + 1));
    if (!w) return ORC_ENOMEM;
    double *A = w + 5 * K;   /* [n][n]    phi_j(r_i)      */
    double *Ai = A + n2;     /* [n][n]    inverse         */
    double *LUw = Ai + n2;   /* [n][n]    LU workspace    */
    double *dA = LUw + n2;   /* [n][n][3] grad phi_j(r_i) */
    double *lA = dA + 3 * n2;/* [n][n]    lap phi_j(r_i)  */
    int perm[64];
    double total = 0.0;
    int rc = ORC_OK;
    for (int sg = 0; sg < 2 && rc == ORC_OK; ++sg) {
        int n = nspin(s, sg), i0 = first_of(s, sg);
        if (n == 0) continue;
        for (int i = 0; i < n; ++i)
            orbitals_at(s, pos + 3 * (i0 + i), n, A + i * n, dA + 3 * i * n, lA + i * n, w);
        rc = lu_inverse(A, n, Ai, LUw, perm);
        if (rc) break;
        for (int i = 0; i < n; ++i) {
            double gD[3] = {0, 0, 0}, lD = 0.0;
            for (int j = 0; j < n; ++j) {
                double inv = Ai[j * n + i];
                for (int k = 0; k < 3; ++k) gD[k] += dA[3 * (i * n + j) + k] * inv;
                lD += lA[i * n + j] * inv;
            }
            double gJ[3], lJ;
            jastrow_derivs(s, pos, i0 + i, gJ, &lJ);
            total += lD + 2.0 * (gD[0] * gJ[0] + gD[1] * gJ[1] + gD[2] * gJ[2]) + lJ
                     + gJ[0] * gJ[0] + gJ[1] * gJ[1] + gJ[2] * gJ[2];
        }
    }
    free(w);
    if (rc) return rc;
    double V = orc_potential(s, pos);
    if (lap_psi) *lap_psi = total;
    if (v) *v = V;
    *e_l = -0.5 * total + V;
    return isfinite(*e_l) ? ORC_OK : ORC_ENONFINITE;
}

/* Derivatives of the Jastrow exponent J and of the local energy with respect
 * to the two Pade parameters theta = (b_ee, b_en) at fixed positions (the
 * cusp coefficients stay fixed).  For one pair term u = c r / (1 + b r):
 *   du/db   = -c r^2 / (1 + b r)^2,
 *   du'/db  = -2 c r / (1 + b r)^3,  with u' = c / (1 + b r)^2,
 *   du''/db = -2 c / (1 + b r)^3 + 6 c b r / (1 + b r)^4,  with u'' = -2 c b / (1 + b r)^3;
 * grad_i J collects u'(r) d/r and lap_i J collects u'' + 2 u'/r over the
 * partners of electron i, and E_L = -1/2 sum_i [lap_i D/D + 2 grad_i D/D .
 * grad_i J + lap_i J + |grad_i J|^2] + V, where only the J terms depend on
 * theta.  Outputs dJ[2] and dEL[2] in the order (b_ee, b_en). */
int orc_jastrow_param_grad(const orc_system *s, const double *pos, double dJ[2], double dEL[2])
{
    int N = s->n_up + s->n_dn, K = orc_nbasis(s), nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
    if (nmax > 64) return ORC_EINVAL;
    size_t n2 = (size_t)nmax * nmax;
    double *w = (double *)malloc(sizeof(double) * (5 * (size_t)K + 7 * n2 + 1));
    if (!w) return ORC_ENOMEM;
    double *A = w + 5 * K, *Ai = A + n2, *LUw = Ai + n2, *dA = LUw + n2, *lA = dA + 3 * n2;
    int perm[64];
    dJ[0] = dJ[1] = dEL[0] = dEL[1] = 0.0;
    int rc = ORC_OK;
    for (int sg = 0; sg < 2 && rc == ORC_OK; ++sg) {
        int n = nspin(s, sg), i0 = first_of(s, sg);
        if (n == 0) continue;
        for (int i = 0; i < n; ++i)
            orbitals_at(s, pos + 3 * (i0 + i), n, A + i * n, dA + 3 * i * n, lA + i * n, w);
        rc = lu_inverse(A, n, Ai, LUw, perm);
        if (rc) break;
        for (int il = 0; il < n; ++il) {
            int i = i0 + il;
            double gD[3] = {0, 0, 0};
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < 3; ++k) gD[k] += dA[3 * (il * n + j) + k] * Ai[j * n + il];
            double gJ[3], lJ;
            jastrow_derivs(s, pos, i, gJ, &lJ);
            /* theta-derivatives of grad_i J and lap_i J, one parameter at a time */
            for (int t = 0; t < 2; ++t) {
                double dg[3] = {0, 0, 0}, dl = 0.0;
                int np = t == 0 ? N : s->n_nuc;
                for (int q = 0; q < np; ++q) {
                    const double *other;
                    double c, b;
                    if (t == 0) {
                        if (q == i) continue;
                        other = pos + 3 * q;
                        c = (spin_of(s, i) == spin_of(s, q)) ? 0.25 : 0.5;
                        b = s->b_ee;
                    } else {
                        other = s->R + 3 * q;
                        c = -s->Z[q];
                        b = s->b_en;
                    }
                    double d[3] = {pos[3 * i] - other[0], pos[3 * i + 1] - other[1], pos[3 * i + 2] - other[2]};
                    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    double den = 1.0 + b * r;
                    double dup = -2.0 * c * r / (den * den * den);
                    double dupp = -2.0 * c / (den * den * den) + 6.0 * c * b * r / (den * den * den * den);
                    for (int k = 0; k < 3; ++k) dg[k] += dup * d[k] / r;
                    dl += dupp + 2.0 * dup / r;
                    /* the pair's u once: electron pairs at q > i, every nucleus */
                    if (t == 1 || q > i) dJ[t] += -c * r * r / (den * den);
                }
                double term = 2.0 * ((gD[0] + gJ[0]) * dg[0] + (gD[1] + gJ[1]) * dg[1] + (gD[2] + gJ[2]) * dg[2]) + dl;
                dEL[t] += -0.5 * term;
            }
        }
    }
    free(w);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Lattice moves (main text Eq. (1) and Eq. (3))                              */

/* Switch p at point x as a function of the squared distance d2 to the nearest
 * nucleus with Z_I >= z_heavy (lowest index wins a tie): the Gaussian
 * exp(-d2 / (2 r_c^2)) of Eq. (3), or the Pade form 1 / (1 + r_c^2 d2) of
 * Eq. (2), whose r_c multiplies the distance. */
double orc_p_switch(const orc_system *s, const orc_params *p, const double x[3])
{
    int best = -1;
    double bd2 = 0.0;
    for (int I = 0; I < s->n_nuc; ++I) {
        if (s->Z[I] < p->z_heavy) continue;
        double dx = x[0] - s->R[3 * I], dy = x[1] - s->R[3 * I + 1], dz = x[2] - s->R[3 * I + 2];
        double d2 = dx * dx + dy * dy + dz * dz;
        if (best < 0 || d2 < bd2) { best = I; bd2 = d2; }
    }
    if (best < 0) return 0.0;
    if (p->switch_form == 1) return 1.0 / (1.0 + p->r_c * p->r_c * bd2);
    return exp(-bd2 / (2.0 * p->r_c * p->r_c));
}

/* Move m = 12 i + 6 g + dir of electron i: grid g (0: spacing a weighted by
 * p, 1: spacing a' weighted by 1-p), axis dir/2, sign + for even dir.
 * New position r' = r_i + sign h e_axis; p is taken at the midpoint
 * r_i + sign (h/2) e_axis; coefficient k = p/a^2 or (1-p)/a'^2.
 * Single grid: m = 6 i + dir, spacing a, k = 1/a^2 (p = 1 everywhere). */
static void move_geom(const orc_system *s, const orc_params *p, const double *pos, const double Rm[9], int m,
                      double rp[3], double *k)
{
    const int mpe = moves_per_electron(p);
    int i = m / mpe, g = mpe == 12 ? (m / 6) % 2 : 0, dir = m % 6, ax = dir / 2;
    double sgn = (dir % 2 == 0) ? 1.0 : -1.0;
    double h = (g == 0) ? p->a : p->a_prime;
    double e[3] = {Rm[ax], Rm[3 + ax], Rm[6 + ax]};
    double mid[3];
    for (int c = 0; c < 3; ++c) {
        rp[c] = pos[3 * i + c] + sgn * h * e[c];
        mid[c] = pos[3 * i + c] + sgn * (0.5 * h) * e[c];
    }
    if (mpe == 6) {
        *k = 1.0 / (p->a * p->a);
        return;
    }
    double pv = orc_p_switch(s, p, mid);
    *k = (g == 0) ? pv / (p->a * p->a) : (1.0 - pv) / (p->a_prime * p->a_prime);
}

void orc_move(const orc_system *s, const orc_params *p, const double *pos, const double Rm[9],
              int m, double rp[3], double *k)
{
    move_geom(s, p, pos, Rm, m, rp, k);
}

/* Psi(x')/Psi(x) for x' = x with electron i at rp: the moved spin's
 * determinant recomputed by LU, the whole Jastrow recomputed. */
static int ratio_full(const orc_system *s, const double *pos, int i, const double rp[3],
                      const double *A_cur, double logdet_cur, int sign_cur, double J_cur,
                      double *pos_tmp, double *A_tmp, double *work, double *out)
{
    int sg = spin_of(s, i), n = nspin(s, sg), i0 = first_of(s, sg);
    memcpy(A_tmp, A_cur, sizeof(double) * n * n);
    orbitals_at(s, rp, n, A_tmp + (i - i0) * n, NULL, NULL, work);
    int sgn;
    double ld = lu_logdet(A_tmp, n, &sgn);
    int N = s->n_up + s->n_dn;
    memcpy(pos_tmp, pos, sizeof(double) * 3 * N);
    pos_tmp[3 * i] = rp[0]; pos_tmp[3 * i + 1] = rp[1]; pos_tmp[3 * i + 2] = rp[2];
    double Jn = orc_jastrow(s, pos_tmp);
    if (sgn == 0) { *out = 0.0; return ORC_OK; }
    *out = (double)(sgn * sign_cur) * exp((ld - logdet_cur) + (Jn - J_cur));
    return ORC_OK;
}

/* Table of all M = 12N moves at fixed x: ratios rho[m] and coefficients k[m].
 * diag (optional, 10 doubles):
 *   [0] E_L analytic          [1] e_L lattice-assembled
 *   [2] L^a = sum k (rho-1)   [3] sum_i lap_i Psi/Psi
 *   [4] V^a                   [5] V_sf
 *   [6] Delta = sum T         [7] V
 *   [8] sum k                 [9] unused
 * V^a = V + (L^a - lap Psi/Psi)/2; V_sf = -1/2 sum_{rho<0} k rho;
 * T = k max(rho,0)/2; e_L = sum k/2 + V^a + V_sf -
 * Delta.  T (optional) receives the heat-bath weights. */
static int eval_table(const orc_system *s, const orc_params *p, const double *pos, const double Rm[9],
                      double *rho, double *kout, double *T, double *diag)
{
    int N = s->n_up + s->n_dn, K = orc_nbasis(s), M = moves_per_electron(p) * N;
    int nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
    size_t n2 = (size_t)nmax * nmax;
    double *w = (double *)malloc(sizeof(double) * (5 * (size_t)K + 3 * n2 + 3 * (size_t)N + 1));
    if (!w) return ORC_ENOMEM;
    double *A[2] = {w + 5 * K, w + 5 * K + n2};  /* Slater matrices of x */
    double *Atmp = A[1] + n2;                     /* moved-spin matrix    */
    double *pos_tmp = Atmp + n2;                  /* x'                   */
    double ld[2] = {0, 0};
    int sgn[2] = {1, 1};
    int rc = ORC_OK;
    for (int sg = 0; sg < 2; ++sg) {
        int n = nspin(s, sg);
        if (n == 0) continue;
        slater_matrix(s, pos, sg, A[sg], w);
        memcpy(Atmp, A[sg], sizeof(double) * n * n);
        ld[sg] = lu_logdet(Atmp, n, &sgn[sg]);
        if (sgn[sg] == 0) rc = ORC_ESINGULAR;
    }
    if (rc) { free(w); return rc; }
    double J = orc_jastrow(s, pos);
    double sumk = 0, La = 0, Vsf = 0, Delta = 0;
    for (int m = 0; m < M; ++m) {
        double rp[3], k;
        int i = m / moves_per_electron(p), sg = spin_of(s, i);
        move_geom(s, p, pos, Rm, m, rp, &k);
        double r;
        ratio_full(s, pos, i, rp, A[sg], ld[sg], sgn[sg], J, pos_tmp, Atmp, w, &r);
        rho[m] = r;
        kout[m] = k;
        sumk += k;
        La += k * (r - 1.0);
        if (r < 0) Vsf += -0.5 * k * r;
        double t = 0.5 * k * (r > 0 ? r : 0.0);
        if (T) T[m] = t;
        Delta += t;
    }
    free(w);
    double EL, lap, V;
    rc = orc_local_energy(s, pos, &EL, &lap, &V);
    if (diag) {
        double Va = V + 0.5 * (La - lap);
        diag[0] = EL;
        diag[1] = 0.5 * sumk + Va + Vsf - Delta;
        diag[2] = La;
        diag[3] = lap;
        diag[4] = Va;
        diag[5] = Vsf;
        diag[6] = Delta;
        diag[7] = V;
        diag[8] = sumk;
        diag[9] = 0.0;
    }
    return rc;
}

int orc_eval_moves(const orc_system *s, const orc_params *p, const double *pos, const double Rm[9],
                   double *rho, double *kout, double *diag)
{
    return eval_table(s, p, pos, Rm, rho, kout, NULL, diag);
}

/* Heat-bath choice: first m with C_m > u2 * Delta, C the sequential
 * left-to-right cumulative sum of T and Delta = C_{M-1}.  If rounding leaves
 * no such m, the last m with T_m > 0.  Returns -1 when Delta == 0.
 * margin (optional): the distance of the threshold u2 * Delta to the nearer
 * end of the chosen interval (C_{m-1}, C_m], relative to Delta: how far the
 * cumulative sums may move (another summation order, another rounding of T)
 * before the choice changes.  Only ends shared with another move of positive
 * weight count: the threshold scales with Delta, so it never falls below the
 * first interval or above the last one.  +inf when no end counts (a single
 * move of positive weight) or there is no choice. */
int orc_select_margin(const double *T, int M, double u2, double *margin)
{
    double D = 0.0;
    for (int m = 0; m < M; ++m) D += T[m];
    if (margin) *margin = INFINITY;
    if (!(D > 0.0)) return -1;
    double thr = u2 * D, C = 0.0, lo = 0.0;
    int ms = -1;
    for (int m = 0; m < M; ++m) {
        lo = C;
        C += T[m];
        if (C > thr) { ms = m; break; }
    }
    if (ms < 0) {                       /* rounding fallback */
        for (int m = M - 1; m >= 0 && ms < 0; --m)
            if (T[m] > 0.0) ms = m;
        lo = 0.0;
        for (int m = 0; m < ms; ++m) lo += T[m];
        C = lo + T[ms];
    }
    if (margin) {
        int below = 0, above = 0;
        for (int m = 0; m < ms; ++m) below |= T[m] > 0.0;
        for (int m = ms + 1; m < M; ++m) above |= T[m] > 0.0;
        double mg = INFINITY;
        if (below) mg = fmin(mg, (thr - lo) / D);
        if (above) mg = fmin(mg, (C - thr) / D);
        *margin = mg;
    }
    return ms;
}

int orc_select(const double *T, int M, double u2)
{
    return orc_select_margin(T, M, u2, NULL);
}

/* ------------------------------------------------------------------------ */
/* Continuous-time projection of one walker over one generation.              */
/* Holding time tau_d = -ln(u1)/Delta(x); weight factor exp(-tau_d e_L(x));
 * move chosen with probability T_m/Delta.  E_T = 0.  A tie tau_d == tau_left
 * counts as staying; Delta == 0 stays for the remaining time.
 * Random numbers: iteration t of generation gen of slot s draws the
 * rotation from counter (s, gen, t, 1) and (u1, u2) from (s, gen, t, 0).
 * pos is updated in place; log_w starts at 0.
 * margin (optional): the smallest relative margin of the walker's integer
 * decisions in this generation, each the relative change of the rates that
 * would reverse it: |tau_d - tau_left| / tau_d for move-or-stay, and the
 * heat-bath margin of orc_select_margin for the chosen move.  A GPU path that
 * sums in another order may take another decision only where this margin is
 * at rounding level. */
int orc_generation(const orc_system *s, const orc_params *p, uint64_t slot, uint64_t gen,
                   double *pos, double *log_w, double *e_l, int64_t *n_moves, double *margin)
{
    int N = s->n_up + s->n_dn, M = moves_per_electron(p) * N;
    double *rho = (double *)malloc(sizeof(double) * 3 * M);
    if (!rho) return ORC_ENOMEM;
    double *k = rho + M, *T = k + M;
    double tl = p->tau, lw = 0.0, EL, lap, V, mg = INFINITY;
    int64_t moves = 0;
    int rc = orc_local_energy(s, pos, &EL, &lap, &V);
    for (uint64_t it = 0; rc == ORC_OK; ++it) {
        double Rm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, u[4];
        if (p->rotate) {
            orc_draw(p->seed, slot, gen, it, 1, u);
            orc_rotation(u, Rm);
        }
        rc = eval_table(s, p, pos, Rm, rho, k, T, NULL);
        if (rc) break;
        double D = 0.0;
        for (int m = 0; m < M; ++m) D += T[m];
        orc_draw(p->seed, slot, gen, it, 0, u);
        if (!(D > 0.0)) { lw -= tl * EL; break; }
        double td = -log(u[0]) / D;
        mg = fmin(mg, fabs(td - tl) / td);
        if (td >= tl) { lw -= tl * EL; break; }
        lw -= td * EL;
        tl -= td;
        double ms_margin;
        int ms = orc_select_margin(T, M, u[1], &ms_margin);
        mg = fmin(mg, ms_margin);
        double rp[3], kk;
        orc_move(s, p, pos, Rm, ms, rp, &kk);
        int i = ms / moves_per_electron(p);
        pos[3 * i] = rp[0]; pos[3 * i + 1] = rp[1]; pos[3 * i + 2] = rp[2];
        ++moves;
        rc = orc_local_energy(s, pos, &EL, &lap, &V);
    }
    free(rho);
    if (rc == ORC_OK && !(isfinite(lw) && isfinite(EL))) rc = ORC_ENONFINITE;
    *log_w = lw;
    *e_l = EL;
    *n_moves = moves;
    if (margin) *margin = mg;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Variational Monte Carlo: Metropolis sampling of |Psi|^2 (the variational  */
/* step of the supplement's computational details; Metropolis et al. 1953).  */
/* Step t of generation gen of slot s draws (u0, u1, u2, u3) from counter    */
/* (s, gen, t, 2): electron i = floor(u0 N) moves by step * e with e on the  */
/* unit sphere (cos theta = 2 u1 - 1, phi = 2 pi u2), a proposal symmetric   */
/* in x and x'; it is accepted when u3 < (Psi(x')/Psi(x))^2, the ratio from  */
/* log|Psi| and the sign recomputed in full at both points.  pos is updated  */
/* in place; *n_acc counts accepted steps, *e_l is E_L at the end.           */
int orc_vmc(const orc_system *s, const orc_params *p, uint64_t slot, uint64_t gen, int n_steps, double step,
            double *pos, int64_t *n_acc, double *e_l)
{
    int N = s->n_up + s->n_dn;
    double *trial = (double *)malloc(sizeof(double) * 3 * N);
    if (!trial) return ORC_ENOMEM;
    double l0;
    int sg0;
    int rc = orc_log_psi(s, pos, &l0, &sg0);
    int64_t acc = 0;
    for (int t = 0; t < n_steps && rc == ORC_OK; ++t) {
        double u[4];
        orc_draw(p->seed, slot, gen, (uint64_t)t, 2, u);
        int i = (int)(u[0] * N);
        if (i > N - 1) i = N - 1;
        double ct = 2.0 * u[1] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * M_PI * u[2];
        memcpy(trial, pos, sizeof(double) * 3 * N);
        trial[3 * i] += step * st * cos(ph);
        trial[3 * i + 1] += step * st * sin(ph);
        trial[3 * i + 2] += step * ct;
        double l1;
        int sg1;
        rc = orc_log_psi(s, trial, &l1, &sg1);
        if (rc == ORC_ESINGULAR) {   /* on a node: Psi(x') = 0, never accepted */
            rc = ORC_OK;
            continue;
        }
        if (rc) break;
        double ratio = (double)(sg0 * sg1) * exp(l1 - l0);
        if (u[3] < ratio * ratio) {
            memcpy(pos, trial, sizeof(double) * 3 * N);
            l0 = l1;
            sg0 = sg1;
            ++acc;
        }
    }
    free(trial);
    double lap, v;
    if (rc == ORC_OK) rc = orc_local_energy(s, pos, e_l, &lap, &v);
    *n_acc = acc;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Reconfiguration at fixed population (systematic resampling).              */
/* w_j = exp(log_w_j - max); Ws = sum w; ebar = sum w e / Ws;
 * log_wbar = log(Ws/W) + max; t_s = (s + xi) * (Ws/W);
 * idx_s = first j with CW_j > t_s (CW sequential), clamped to W-1.
 * margin (optional, [W]): for each s the distance of t_s to the nearer end of
 * the chosen interval (CW_{j-1}, CW_j], relative to Ws; the ends 0 and Ws do
 * not count (t_s scales with Ws), +inf for W = 1. */
int orc_reconfigure(const double *log_w, const double *e_l, int W, double xi,
                    int32_t *idx, double *log_wbar, double *ebar, double *margin)
{
    if (W < 1) return ORC_EINVAL;
    double mx = log_w[0];
    for (int j = 1; j < W; ++j) if (log_w[j] > mx) mx = log_w[j];
    double *CW = (double *)malloc(sizeof(double) * W);
    if (!CW) return ORC_ENOMEM;
    double Ws = 0.0, ew = 0.0;
    for (int j = 0; j < W; ++j) {
        double w = exp(log_w[j] - mx);
        Ws += w;
        CW[j] = Ws;
        if (e_l) ew += w * e_l[j];
    }
    if (ebar) *ebar = e_l ? ew / Ws : 0.0;
    if (log_wbar) *log_wbar = log(Ws / (double)W) + mx;
    double q = Ws / (double)W;
    for (int s_ = 0; s_ < W; ++s_) {
        double t = ((double)s_ + xi) * q;
        int j = 0;
        while (j < W - 1 && !(CW[j] > t)) ++j;
        idx[s_] = j;
        if (margin) {
            double mg = INFINITY;
            if (j > 0) mg = fmin(mg, (t - CW[j - 1]) / Ws);
            if (j < W - 1) mg = fmin(mg, (CW[j] - t) / Ws);
            margin[s_] = mg;
        }
    }
    free(CW);
    return isfinite(Ws) && Ws > 0 ? ORC_OK : ORC_ENONFINITE;
}

double orc_xi(uint64_t seed, uint64_t gen)
{
    double u[4];
    orc_draw(seed, ~0ULL, gen, 0, 3, u);
    return u[0];
}

/* One generation of W independent walker slots (no reconfiguration):
 * pos [W][N][3] in/out, per slot log_w, e_L, move count and decision margin
 * (orc_generation), on nthreads host threads (0: the OpenMP default). */
int orc_generations(const orc_system *s, const orc_params *p, int W, double *pos, uint64_t gen,
                    double *log_w, double *e_l, int64_t *n_moves, double *margin, int nthreads)
{
    int N = s->n_up + s->n_dn;
    int err = ORC_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int w = 0; w < W; ++w) {
        int r = orc_generation(s, p, (uint64_t)w, gen, pos + 3 * N * (size_t)w, &log_w[w], &e_l[w], &n_moves[w],
                               margin ? &margin[w] : NULL);
        if (r != ORC_OK) {
#pragma omp critical
            err = r;
        }
    }
    return err;
}

/* Whole projection: n_gen generations of W walkers, each followed by a
 * reconfiguration.  pos [W][N][3] in/out.  Records per generation:
 * log_wbar, ebar, total moves; idx [n_gen][W] if non-NULL; margin
 * [n_gen][2][W] if non-NULL: per slot the smallest decision margin of its
 * projection (orc_generation), then per destination slot the margin of its
 * resampling choice (orc_reconfigure). */
int orc_run(const orc_system *s, const orc_params *p, int W, double *pos, uint64_t gen0, int n_gen,
            double *log_wbar, double *ebar, int64_t *n_moves, int32_t *idx_all, double *margin, int nthreads)
{
    int N = s->n_up + s->n_dn;
    double *lw = (double *)malloc(sizeof(double) * 2 * W);
    int64_t *mv = (int64_t *)malloc(sizeof(int64_t) * W);
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * W);
    double *tmp = (double *)malloc(sizeof(double) * 3 * N * (size_t)W);
    if (!lw || !mv || !idx || !tmp) { free(lw); free(mv); free(idx); free(tmp); return ORC_ENOMEM; }
    double *el = lw + W;
    int rc = ORC_OK;
    for (int g = 0; g < n_gen && rc == ORC_OK; ++g) {
        uint64_t gen = gen0 + (uint64_t)g;
        double *mg = margin ? margin + (size_t)g * 2 * W : NULL;
        rc = orc_generations(s, p, W, pos, gen, lw, el, mv, mg, nthreads);
        if (rc) break;
        int64_t tot = 0;
        for (int w = 0; w < W; ++w) tot += mv[w];
        n_moves[g] = tot;
        rc = orc_reconfigure(lw, el, W, orc_xi(p->seed, gen), idx, &log_wbar[g], &ebar[g], mg ? mg + W : NULL);
        if (rc) break;
        if (idx_all) memcpy(idx_all + (size_t)g * W, idx, sizeof(int32_t) * W);
        for (int w = 0; w < W; ++w)
            memcpy(tmp + 3 * N * (size_t)w, pos + 3 * N * (size_t)idx[w], sizeof(double) * 3 * N);
        memcpy(pos, tmp, sizeof(double) * 3 * N * (size_t)W);
    }
    free(lw); free(mv); free(idx); free(tmp);
    return rc;
}
