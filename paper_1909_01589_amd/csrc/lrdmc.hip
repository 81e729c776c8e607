// Double-grid lattice-regularized DMC projection on AMD Instinct MI355X
// (gfx950): kernels and the C ABI declared in include/lrdmc.h.
//
// Execution model: one workgroup per walker slot for a whole generation.  The
// walker's orbital-projected inverse Y = C * Ainv, its inverse Slater
// matrices, orbital derivative rows and Jastrow sums stay in LDS while the
// workgroup loops over continuous-time moves; HBM sees only the positions at
// the start and end of the generation.  A second, single-workgroup kernel
// does the fixed-population reconfiguration; the next projection gathers the
// selected copies while it loads them.
//
// Method references (arXiv:1909.01589): main text Eq. (1) (double-grid
// Laplacian), Eq. (3) (Gaussian switch around the nearest heavy nucleus),
// "Application to large systems" (R_c over the heaviest nuclei), Eq. (5)-(7)
// and supplement Eq. (S-13) (spacing choice, lrdmc_spacing below).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lrdmc.h"
#include "lrdmc_device.h"

using namespace lrdmc;

namespace {

constexpr int kMaxNs = 32;    // electrons per spin
constexpr int kMaxN = 64;     // electrons
constexpr int kMaxK = 512;    // basis functions
constexpr int kMaxNuc = 64;
constexpr int kMaxThreads = 256;
constexpr int kMaxIter = 1 << 22;  // moves per walker and generation

// Internal kernel error codes (err[0]); err[1] holds the slot.
enum { kErrSingular = 1, kErrNonFinite = 2, kErrIterCap = 3 };

// Offsets (in doubles) of the per-walker LDS arrays.
struct Layout {
    int pos;    // [N][3]            positions
    int Y;      // [N][Kp]           Y[i][mu] = sum_j C[mu][j] Ainv_sigma(i)[j][i_sigma]
    int Ainv;   // [2][ns][ns]       Ainv_sigma[j][i]
    int dphi;   // [N][4][ns]        grad (x,y,z) and Laplacian of phi_j at r_i
    int gD;     // [N][4]            grad D/D (3) and lap D/D of electron i
    int gJ;     // [N][4]            grad J (3) and lap J of electron i
    int Jo;     // [N]               Jastrow terms that contain electron i
    int Vi;     // [N]               sum_{j>i} 1/r_ij - sum_I Z_I/r_iI
    int T;      // [M]               heat-bath weights of the moves
    int bv;     // [5][K]            basis value, gradient, Laplacian at one point
    int vrow;   // [5][ns]           orbital value, gradient, Laplacian at one point
    int wrow;   // [ns]              w_i = phi(r_new) . Ainv[:, i]
    int colk;   // [ns]              column k of Ainv before the update
    int Yk;     // [Kp]              row k of Y before the update
    int G;      // [2][ns][2ns]      Gauss-Jordan workspace
    int piv;    // [2][2][2ns]       pivot row and row c copies
    int fac;    // [2][ns]           elimination factors
    int red;    // [64]              reduction scratch
    int sc;     // [32]              block scalars
    int total;
};

struct KArgs {
    // system
    int N, n_up, n_dn, ns, K, Kp, n_orb, n_nuc, n_grp, n_heavy, M;
    const double *Znuc, *Rnuc;     // [n_nuc], [n_nuc][3]
    const int *heavy;              // [n_heavy] indices of nuclei with Z >= z_heavy
    const int *grp_nuc;            // [n_grp]
    const double *grp_alpha;       // [n_grp]
    const int *grp_off;            // [n_grp][3] first basis index of the s, p, d shell, -1 if none
    const double *mo;              // [K][n_orb]
    double b_ee, b_en, v_nn;
    // lattice
    double a, ap, inv_a2, inv_ap2, inv_2rc2, tau;
    uint64_t seed;
    int rotate;
    // walkers
    int W;
    uint64_t gen;
    const double *pos_in;
    const int *idx_in;             // gather on load, or nullptr
    double *pos_out, *logw, *el;
    int *nmov;
    int *err;
    // evaluation mode
    int eval;
    double *rho_out, *k_out, *diag_out;
    Layout L;
};

// Block scalar slots.
enum {
    SC_R = 0,        // 9 rotation entries
    SC_U1 = 9, SC_U2 = 10, SC_DELTA = 11, SC_EL = 12, SC_TL = 13, SC_LW = 14,
    SC_RP = 15,      // 3 entries: accepted position
    SC_LAP = 18, SC_V = 19
};

__device__ __forceinline__ void report(int *err, int code, int slot)
{
    if (atomicCAS(err, 0, code) == 0) atomicExch(err + 1, slot);
}

__device__ __forceinline__ int spin_of(const KArgs &A, int i) { return i < A.n_up ? 0 : 1; }

// -- basis -------------------------------------------------------------------

// Values, gradients and Laplacians of every function of group g at r into
// bv[5][K].  For a harmonic polynomial P of degree l:
// grad g = (grad P - 2 alpha d P) e, lap g = (4 alpha^2 d^2 - (6 + 4 l) alpha) P e.
__device__ void basis_group_full(const KArgs &A, int g, const double r[3], double *bv)
{
    const int K = A.K;
    const double *Rn = A.Rnuc + 3 * A.grp_nuc[g];
    const double dx = r[0] - Rn[0], dy = r[1] - Rn[1], dz = r[2] - Rn[2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double al = A.grp_alpha[g];
    const double e = exp(-al * d2);
    const double t2a = 2.0 * al;
    const double q = 4.0 * al * al * d2;
    const int *off = A.grp_off + 3 * g;
    if (off[0] >= 0) {
        const int mu = off[0];
        bv[mu] = e;
        bv[K + mu] = -t2a * dx * e;
        bv[2 * K + mu] = -t2a * dy * e;
        bv[3 * K + mu] = -t2a * dz * e;
        bv[4 * K + mu] = (q - 6.0 * al) * e;
    }
    if (off[1] >= 0) {
        const int mu = off[1];
        const double d[3] = {dx, dy, dz};
        const double lf = (q - 10.0 * al) * e;
        for (int c = 0; c < 3; ++c) {
            bv[mu + c] = d[c] * e;
            for (int k = 0; k < 3; ++k)
                bv[(1 + k) * K + mu + c] = ((k == c ? 1.0 : 0.0) - t2a * d[k] * d[c]) * e;
            bv[4 * K + mu + c] = d[c] * lf;
        }
    }
    if (off[2] >= 0) {
        const int mu = off[2];
        const double P[5] = {dx * dy, dy * dz, dz * dx, dx * dx - dy * dy, 2.0 * dz * dz - dx * dx - dy * dy};
        const double dP[5][3] = {{dy, dx, 0.0}, {0.0, dz, dy}, {dz, 0.0, dx},
                                 {2.0 * dx, -2.0 * dy, 0.0}, {-2.0 * dx, -2.0 * dy, 4.0 * dz}};
        const double d[3] = {dx, dy, dz};
        const double lf = (q - 14.0 * al) * e;
        for (int c = 0; c < 5; ++c) {
            bv[mu + c] = P[c] * e;
            for (int k = 0; k < 3; ++k) bv[(1 + k) * K + mu + c] = (dP[c][k] - t2a * d[k] * P[c]) * e;
            bv[4 * K + mu + c] = P[c] * lf;
        }
    }
}

// sum_mu g_mu(r) y[mu]: the determinant ratio of moving an electron whose
// orbital-projected inverse row is y to r.
__device__ __forceinline__ double basis_dot(const KArgs &A, const double r[3], const double *y)
{
    double acc = 0.0;
    for (int g = 0; g < A.n_grp; ++g) {
        const double *Rn = A.Rnuc + 3 * A.grp_nuc[g];
        const double dx = r[0] - Rn[0], dy = r[1] - Rn[1], dz = r[2] - Rn[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        const double e = exp(-A.grp_alpha[g] * d2);
        const int *off = A.grp_off + 3 * g;
        double poly = 0.0;
        if (off[0] >= 0) poly += y[off[0]];
        if (off[1] >= 0) {
            const double *yp = y + off[1];
            poly += dx * yp[0] + dy * yp[1] + dz * yp[2];
        }
        if (off[2] >= 0) {
            const double *yd = y + off[2];
            poly += dx * dy * yd[0] + dy * dz * yd[1] + dz * dx * yd[2] + (dx * dx - dy * dy) * yd[3] +
                    (2.0 * dz * dz - dx * dx - dy * dy) * yd[4];
        }
        acc += e * poly;
    }
    return acc;
}

// Jastrow terms containing electron i when it sits at r (others fixed).
__device__ __forceinline__ double jastrow_point(const KArgs &A, const double *pos, int i, const double r[3])
{
    const int si = spin_of(A, i);
    double acc = 0.0;
    for (int j = 0; j < A.N; ++j) {
        if (j == i) continue;
        const double dx = r[0] - pos[3 * j], dy = r[1] - pos[3 * j + 1], dz = r[2] - pos[3 * j + 2];
        const double rr = sqrt(dx * dx + dy * dy + dz * dz);
        const double c = (spin_of(A, j) == si) ? 0.25 : 0.5;
        acc += c * rr / (1.0 + A.b_ee * rr);
    }
    for (int I = 0; I < A.n_nuc; ++I) {
        const double *R = A.Rnuc + 3 * I;
        const double dx = r[0] - R[0], dy = r[1] - R[1], dz = r[2] - R[2];
        const double rr = sqrt(dx * dx + dy * dy + dz * dz);
        acc -= A.Znuc[I] * rr / (1.0 + A.b_en * rr);
    }
    return acc;
}

// Switch p at x: Gaussian of the distance to the nearest heavy nucleus.
__device__ __forceinline__ double p_switch(const KArgs &A, const double x[3])
{
    double best = 0.0;
    for (int h = 0; h < A.n_heavy; ++h) {
        const double *R = A.Rnuc + 3 * A.heavy[h];
        const double dx = x[0] - R[0], dy = x[1] - R[1], dz = x[2] - R[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (h == 0 || d2 < best) best = d2;
    }
    return exp(-best * A.inv_2rc2);
}

// Displaced position and hopping coefficient of move m.
__device__ __forceinline__ double move_geometry(const KArgs &A, const double *pos, const double *Rm,
                                                int m, double rp[3])
{
    const int i = m / 12, g = (m / 6) & 1, dir = m % 6, ax = dir >> 1;
    const double h = g ? A.ap : A.a;
    const double t = (dir & 1) ? -h : h;
    const double e[3] = {Rm[ax], Rm[3 + ax], Rm[6 + ax]};
    double mid[3];
    for (int c = 0; c < 3; ++c) {
        rp[c] = pos[3 * i + c] + t * e[c];
        mid[c] = pos[3 * i + c] + (0.5 * t) * e[c];
    }
    const double p = p_switch(A, mid);
    return g ? (1.0 - p) * A.inv_ap2 : p * A.inv_a2;
}

// -- per-walker state ------------------------------------------------------

// Orbital rows (value, gradient, Laplacian of phi_j, j < n) at a point whose
// basis block is in bv; threads over (component, orbital).
__device__ __forceinline__ void orbital_rows(const KArgs &A, const double *bv, int n, double *vrow)
{
    const int K = A.K, no = A.n_orb, ns = A.ns;
    for (int t = threadIdx.x; t < 5 * n; t += blockDim.x) {
        const int c = t / n, j = t - c * n;
        const double *b = bv + c * K;
        double acc0 = 0.0, acc1 = 0.0;
        int mu = 0;
        for (; mu + 1 < K; mu += 2) {
            acc0 += b[mu] * A.mo[mu * no + j];
            acc1 += b[mu + 1] * A.mo[(mu + 1) * no + j];
        }
        if (mu < K) acc0 += b[mu] * A.mo[mu * no + j];
        vrow[c * ns + j] = acc0 + acc1;
    }
}

// Jastrow gradient/Laplacian, own sum and potential share of every electron.
// Segments of `seg` lanes (a power of two within a wavefront) per electron.
__device__ void jastrow_all(const KArgs &A, const double *pos, double *gJ, double *Jo, double *Vi)
{
    const int N = A.N;
    int seg = 64;
    while (seg > 1 && seg * N > (int)blockDim.x) seg >>= 1;
    const int per_pass = blockDim.x / seg;
    for (int base = 0; base < N; base += per_pass) {
        const int i = base + threadIdx.x / seg, sub = threadIdx.x % seg;
        double g0 = 0, g1 = 0, g2 = 0, lap = 0, jo = 0, v = 0;
        if (i < N) {
            const int si = spin_of(A, i);
            const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
            for (int j = sub; j < N + A.n_nuc; j += seg) {
                if (j == i) continue;
                double dx, dy, dz, c, b, Zn = 0.0;
                const bool ee = j < N;
                if (ee) {
                    dx = xi - pos[3 * j]; dy = yi - pos[3 * j + 1]; dz = zi - pos[3 * j + 2];
                    c = (spin_of(A, j) == si) ? 0.25 : 0.5;
                    b = A.b_ee;
                } else {
                    const double *R = A.Rnuc + 3 * (j - N);
                    dx = xi - R[0]; dy = yi - R[1]; dz = zi - R[2];
                    Zn = A.Znuc[j - N];
                    c = -Zn;
                    b = A.b_en;
                }
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double r = sqrt(r2);
                const double ir = 1.0 / r;
                const double q = 1.0 / (1.0 + b * r);
                const double up = c * q * q;             // u'(r)
                const double upp = -2.0 * c * b * q * q * q;  // u''(r)
                const double f = up * ir;
                g0 += f * dx; g1 += f * dy; g2 += f * dz;
                lap += upp + 2.0 * f;
                jo += c * r * q;
                if (ee) { if (j > i) v += ir; }
                else v -= Zn * ir;
            }
        }
        for (int off = seg >> 1; off > 0; off >>= 1) {
            g0 += __shfl_xor(g0, off, 64); g1 += __shfl_xor(g1, off, 64); g2 += __shfl_xor(g2, off, 64);
            lap += __shfl_xor(lap, off, 64); jo += __shfl_xor(jo, off, 64); v += __shfl_xor(v, off, 64);
        }
        if (i < N && sub == 0) {
            gJ[4 * i] = g0; gJ[4 * i + 1] = g1; gJ[4 * i + 2] = g2; gJ[4 * i + 3] = lap;
            Jo[i] = jo;
            Vi[i] = v;
        }
    }
}

// grad D/D and lap D/D for the electrons of spin sg (sg < 0: both spins).
__device__ __forceinline__ void det_derivs(const KArgs &A, const double *Ainv, const double *dphi,
                                           double *gD, int sg)
{
    const int ns = A.ns;
    const int i0 = sg == 1 ? A.n_up : 0;
    const int i1 = sg == 0 ? A.n_up : A.N;
    for (int t = threadIdx.x; t < 4 * (i1 - i0); t += blockDim.x) {
        const int i = i0 + t / 4, c = t & 3;
        const int s = spin_of(A, i), n = s ? A.n_dn : A.n_up, il = s ? i - A.n_up : i;
        const double *inv = Ainv + s * ns * ns;
        const double *dp = dphi + (i * 4 + c) * ns;
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += dp[j] * inv[j * ns + il];
        gD[4 * i + c] = acc;
    }
}

// Local energy from the per-electron pieces; every thread gets the result.
__device__ __forceinline__ void local_energy(const KArgs &A, double *lds, double *out_el, double *out_lap,
                                             double *out_v)
{
    const Layout &L = A.L;
    const double *gD = lds + L.gD, *gJ = lds + L.gJ, *Vi = lds + L.Vi;
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < A.N; i += blockDim.x) {
        const double *d = gD + 4 * i, *j = gJ + 4 * i;
        v[0] += d[3] + 2.0 * (d[0] * j[0] + d[1] * j[1] + d[2] * j[2]) + j[3] + j[0] * j[0] + j[1] * j[1] +
                j[2] * j[2];
        v[1] += Vi[i];
    }
    block_sum<2>(v, lds + L.red);
    const double V = v[1] + A.v_nn;
    *out_lap = v[0];
    *out_v = V;
    *out_el = -0.5 * v[0] + V;
}

// Generation start: Slater matrices and derivative rows of every electron,
// Gauss-Jordan inversion with partial pivoting, Y = C Ainv, determinant and
// Jastrow derivatives, local energy.  Returns an error code (uniform).
__device__ int walker_setup(const KArgs &A, double *lds, int *sflag)
{
    const Layout &L = A.L;
    const int N = A.N, ns = A.ns, K = A.K, Kp = A.Kp, tid = threadIdx.x, NT = blockDim.x;
    double *pos = lds + L.pos, *bv = lds + L.bv, *vrow = lds + L.vrow, *G = lds + L.G;
    double *dphi = lds + L.dphi, *Ainv = lds + L.Ainv;
    const int two = 2 * ns;

    // right halves = identity
    for (int t = tid; t < 2 * ns * two; t += NT) {
        const int s = t / (ns * two), r = (t / two) % ns, c = t % two;
        if (c >= ns) G[t] = (c - ns == r) ? 1.0 : 0.0;
    }
    for (int i = 0; i < N; ++i) {
        const int s = spin_of(A, i), n = s ? A.n_dn : A.n_up, il = s ? i - A.n_up : i;
        const double r[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        for (int g = tid; g < A.n_grp; g += NT) basis_group_full(A, g, r, bv);
        __syncthreads();
        orbital_rows(A, bv, n, vrow);
        __syncthreads();
        for (int t = tid; t < 5 * n; t += NT) {
            const int c = t / n, j = t - c * n;
            if (c == 0) G[(s * ns + il) * two + j] = vrow[j];
            else dphi[(i * 4 + c - 1) * ns + j] = vrow[c * ns + j];
        }
    }
    __syncthreads();

    // Gauss-Jordan on [A | I] for both spins at once.
    double *prow = lds + L.piv;   // [2][2][two]: pivot row, row c
    double *fac = lds + L.fac;    // [2][ns]
    for (int c = 0; c < ns; ++c) {
        if (tid < 2) {
            const int s = tid, n = s ? A.n_dn : A.n_up;
            int p = -1;
            if (c < n) {
                double best = -1.0;
                for (int r = c; r < n; ++r) {
                    const double v = fabs(G[(s * ns + r) * two + c]);
                    if (v > best) { best = v; p = r; }
                }
                if (!(best > 0.0) || !isfinite(best)) p = -2;
            }
            sflag[2 + s] = p;
        }
        __syncthreads();
        if (sflag[2] == -2 || sflag[3] == -2) return kErrSingular;
        for (int t = tid; t < 2 * two + 2 * ns; t += NT) {
            // copies: t < 2*two -> pivot row / row c entries; else factors
            if (t < 2 * two) {
                const int s = t / two, col = t % two, p = sflag[2 + s];
                if (p >= 0) {
                    prow[(s * 2 + 0) * two + col] = G[(s * ns + p) * two + col];
                    prow[(s * 2 + 1) * two + col] = G[(s * ns + c) * two + col];
                }
            } else {
                const int u = t - 2 * two, s = u / ns, r = u % ns, p = sflag[2 + s];
                if (p >= 0) {
                    const int src = (r == p) ? c : (r == c ? p : r);
                    fac[s * ns + r] = G[(s * ns + src) * two + c];
                }
            }
        }
        __syncthreads();
        for (int t = tid; t < 2 * ns * two; t += NT) {
            const int s = t / (ns * two), r = (t / two) % ns, col = t % two, p = sflag[2 + s];
            const int n = s ? A.n_dn : A.n_up;
            if (p < 0 || r >= n) continue;
            const double *pr = prow + (s * 2 + 0) * two;
            const double ipiv = 1.0 / pr[c];
            if (r == c) {
                G[t] = pr[col] * ipiv;
            } else {
                const double src = (r == p) ? prow[(s * 2 + 1) * two + col] : G[t];
                G[t] = src - fac[s * ns + r] * (pr[col] * ipiv);
            }
        }
        __syncthreads();
    }
    for (int t = tid; t < 2 * ns * ns; t += NT) {
        const int s = t / (ns * ns), j = (t / ns) % ns, i = t % ns;
        Ainv[t] = G[(s * ns + j) * two + ns + i];
    }
    __syncthreads();

    // Y[i][mu] = sum_j C[mu][j] Ainv_s[j][i_s]
    double *Y = lds + L.Y;
    for (int t = tid; t < N * K; t += NT) {
        const int i = t / K, mu = t - i * K;
        const int s = spin_of(A, i), n = s ? A.n_dn : A.n_up, il = s ? i - A.n_up : i;
        const double *inv = Ainv + s * ns * ns;
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += A.mo[mu * A.n_orb + j] * inv[j * ns + il];
        Y[i * Kp + mu] = acc;
    }
    det_derivs(A, Ainv, dphi, lds + L.gD, -1);
    jastrow_all(A, pos, lds + L.gJ, lds + L.Jo, lds + L.Vi);
    __syncthreads();
    double el, lap, V;
    local_energy(A, lds, &el, &lap, &V);
    if (tid == 0) {
        lds[L.sc + SC_EL] = el;
        lds[L.sc + SC_LAP] = lap;
        lds[L.sc + SC_V] = V;
    }
    __syncthreads();
    return isfinite(el) ? 0 : kErrNonFinite;
}

// Heat-bath weights of every move at the current configuration (S1-S6).
// Optionally stores rho and k, and accumulates sum k, L^a and V_sf.
__device__ __forceinline__ void move_table(const KArgs &A, double *lds, const double *Rm, double *rho_g,
                                           double *k_g, double acc[3], bool diag)
{
    const Layout &L = A.L;
    const double *pos = lds + L.pos, *Y = lds + L.Y, *Jo = lds + L.Jo;
    double *T = lds + L.T;
    for (int m = threadIdx.x; m < A.M; m += blockDim.x) {
        const int i = m / 12;
        double rp[3];
        const double k = move_geometry(A, pos, Rm, m, rp);
        const double rd = basis_dot(A, rp, Y + i * A.Kp);
        const double dJ = jastrow_point(A, pos, i, rp) - Jo[i];
        const double rho = rd * exp(dJ);
        T[m] = 0.5 * k * (rho > 0.0 ? rho : 0.0);
        if (diag) {
            if (rho_g) rho_g[m] = rho;
            if (k_g) k_g[m] = k;
            acc[0] += k;
            acc[1] += k * (rho - 1.0);
            if (rho < 0.0) acc[2] += -0.5 * k * rho;
        }
    }
}

// Sherman-Morrison update after electron k moved to lds[SC_RP].
__device__ void accept_move(const KArgs &A, double *lds, int k)
{
    const Layout &L = A.L;
    const int ns = A.ns, K = A.K, Kp = A.Kp, tid = threadIdx.x, NT = blockDim.x;
    const int s = spin_of(A, k), n = s ? A.n_dn : A.n_up, kl = s ? k - A.n_up : k, i0 = s ? A.n_up : 0;
    double *pos = lds + L.pos, *bv = lds + L.bv, *vrow = lds + L.vrow, *wrow = lds + L.wrow;
    double *colk = lds + L.colk, *Yk = lds + L.Yk, *Y = lds + L.Y, *dphi = lds + L.dphi;
    double *inv = lds + L.Ainv + s * ns * ns;
    const double rp[3] = {lds[L.sc + SC_RP], lds[L.sc + SC_RP + 1], lds[L.sc + SC_RP + 2]};

    for (int g = tid; g < A.n_grp; g += NT) basis_group_full(A, g, rp, bv);
    __syncthreads();
    orbital_rows(A, bv, n, vrow);
    __syncthreads();
    // w_i = phi(r') . Ainv[:, i]; save column k of Ainv and row k of Y
    for (int t = tid; t < n + n + K; t += NT) {
        if (t < n) {
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += vrow[j] * inv[j * ns + t];
            wrow[t] = acc;
        } else if (t < 2 * n) {
            const int j = t - n;
            colk[j] = inv[j * ns + kl];
        } else {
            const int mu = t - 2 * n;
            Yk[mu] = Y[k * Kp + mu];
        }
    }
    __syncthreads();
    const double irho = 1.0 / wrow[kl];
    for (int t = tid; t < n * n + n * K + 4 * n + 3; t += NT) {
        if (t < n * n) {
            const int j = t / n, i = t - j * n;
            const double f = (wrow[i] - (i == kl ? 1.0 : 0.0)) * irho;
            inv[j * ns + i] -= colk[j] * f;
        } else if (t < n * n + n * K) {
            const int u = t - n * n, i = u / K, mu = u - i * K;
            const double f = (wrow[i] - (i == kl ? 1.0 : 0.0)) * irho;
            Y[(i0 + i) * Kp + mu] -= Yk[mu] * f;
        } else if (t < n * n + n * K + 4 * n) {
            const int u = t - n * n - n * K, c = u / n, j = u - c * n;
            dphi[(k * 4 + c) * ns + j] = vrow[(c + 1) * ns + j];
        } else {
            const int c = t - n * n - n * K - 4 * n;
            pos[3 * k + c] = rp[c];
        }
    }
    __syncthreads();
    det_derivs(A, lds + L.Ainv, dphi, lds + L.gD, s);
    jastrow_all(A, pos, lds + L.gJ, lds + L.Jo, lds + L.Vi);
    __syncthreads();
    double el, lap, V;
    local_energy(A, lds, &el, &lap, &V);
    if (tid == 0) lds[L.sc + SC_EL] = el;
    __syncthreads();
}

// One workgroup per walker slot: a generation of continuous-time projection,
// or (eval != 0) the move table at frozen positions.
__global__ void __launch_bounds__(kMaxThreads) project_kernel(KArgs A)
{
    extern __shared__ double lds[];
    __shared__ int sflag[8];  // 0: action, 1: m*, 2-3: pivots, 4: last m with T>0, 5: stop
    const Layout &L = A.L;
    const int tid = threadIdx.x, NT = blockDim.x, slot = blockIdx.x, N = A.N, M = A.M;
    double *pos = lds + L.pos, *sc = lds + L.sc, *T = lds + L.T;

    const int src = A.idx_in ? A.idx_in[slot] : slot;
    for (int t = tid; t < 3 * N; t += NT) pos[t] = A.pos_in[(size_t)src * 3 * N + t];
    if (tid == 0) sflag[5] = (A.err[0] != 0);
    __syncthreads();
    if (sflag[5]) return;

    int rc = walker_setup(A, lds, sflag);
    if (rc) {
        if (tid == 0) report(A.err, rc, slot);
        return;
    }

    if (A.eval) {
        if (tid == 0) {
            double Rm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
            if (A.rotate) {
                double u[4];
                draw4(A.seed, slot, A.gen, 0, 1, u);
                rotation(u, Rm);
            }
            for (int q = 0; q < 9; ++q) sc[SC_R + q] = Rm[q];
        }
        __syncthreads();
        double acc[3] = {0.0, 0.0, 0.0};
        move_table(A, lds, sc + SC_R, A.rho_out ? A.rho_out + (size_t)slot * M : nullptr,
                   A.k_out ? A.k_out + (size_t)slot * M : nullptr, acc, true);
        __syncthreads();
        double dl = 0.0;
        for (int m = tid; m < M; m += NT) dl += T[m];
        double v[4] = {acc[0], acc[1], acc[2], dl};
        block_sum<4>(v, lds + L.red);
        if (tid == 0 && A.diag_out) {
            double *d = A.diag_out + (size_t)slot * LRDMC_NDIAG;
            const double el = sc[SC_EL], lap = sc[SC_LAP], V = sc[SC_V];
            const double Va = V + 0.5 * (v[1] - lap);
            d[0] = el;
            d[1] = 0.5 * v[0] + Va + v[2] - v[3];
            d[2] = v[1];
            d[3] = lap;
            d[4] = Va;
            d[5] = v[2];
            d[6] = v[3];
            d[7] = V;
            d[8] = v[0];
        }
        return;
    }

    if (tid == 0) {
        sc[SC_TL] = A.tau;
        sc[SC_LW] = 0.0;
    }
    int moves = 0;
    const int chunk = (M + NT - 1) / NT;
    const int c0 = min(M, tid * chunk), c1 = min(M, c0 + chunk);
    for (int it = 0;; ++it) {
        if (tid == 0) {
            double Rm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, u[4];
            if (A.rotate) {
                draw4(A.seed, slot, A.gen, (uint64_t)it, 1, u);
                rotation(u, Rm);
            }
            for (int q = 0; q < 9; ++q) sc[SC_R + q] = Rm[q];
            draw4(A.seed, slot, A.gen, (uint64_t)it, 0, u);
            sc[SC_U1] = u[0];
            sc[SC_U2] = u[1];
            sflag[1] = M;
            sflag[4] = -1;
        }
        __syncthreads();
        double dummy[3];
        move_table(A, lds, sc + SC_R, nullptr, nullptr, dummy, false);
        __syncthreads();
        // Delta = sum T and the first m with C_m > u2 Delta (workgroup scan)
        double part = 0.0;
        int last = -1;
        for (int m = c0; m < c1; ++m) {
            part += T[m];
            if (T[m] > 0.0) last = m;
        }
        double Delta;
        const double pre = block_exclusive_scan(part, lds + L.red, &Delta);
        const double thr = sc[SC_U2] * Delta;
        if (pre <= thr) {
            double C = pre;
            for (int m = c0; m < c1; ++m) {
                C += T[m];
                if (C > thr) {
                    atomicMin(&sflag[1], m);
                    break;
                }
            }
        }
        if (last >= 0) atomicMax(&sflag[4], last);
        __syncthreads();
        if (tid == 0) {
            const double EL = sc[SC_EL];
            int action = 0;  // 0 stop, 1 move, 2 error
            if (!(Delta > 0.0)) {
                sc[SC_LW] -= sc[SC_TL] * EL;
            } else if (!isfinite(Delta)) {
                action = 2;
            } else {
                const double td = -log(sc[SC_U1]) / Delta;
                if (td >= sc[SC_TL]) {
                    sc[SC_LW] -= sc[SC_TL] * EL;
                } else {
                    sc[SC_LW] -= td * EL;
                    sc[SC_TL] -= td;
                    int ms = sflag[1];
                    if (ms >= M) ms = sflag[4];
                    if (ms < 0) {
                        action = 2;
                    } else if (it + 1 >= kMaxIter) {
                        action = 3;
                    } else {
                        action = 1;
                        sflag[1] = ms;
                        double rp[3];
                        move_geometry(A, pos, sc + SC_R, ms, rp);
                        sc[SC_RP] = rp[0]; sc[SC_RP + 1] = rp[1]; sc[SC_RP + 2] = rp[2];
                    }
                }
            }
            sflag[0] = action;
        }
        __syncthreads();
        const int action = sflag[0];
        if (action != 1) {
            if (action >= 2) {
                if (tid == 0) report(A.err, action == 2 ? kErrNonFinite : kErrIterCap, slot);
                return;
            }
            break;
        }
        accept_move(A, lds, sflag[1] / 12);
        ++moves;
        if (tid == 0 && !isfinite(sc[SC_EL])) sflag[5] = 1;
        __syncthreads();
        if (sflag[5]) {
            if (tid == 0) report(A.err, kErrNonFinite, slot);
            return;
        }
    }
    for (int t = tid; t < 3 * N; t += NT) A.pos_out[(size_t)slot * 3 * N + t] = pos[t];
    if (tid == 0) {
        const double lw = sc[SC_LW];
        A.logw[slot] = lw;
        A.el[slot] = sc[SC_EL];
        A.nmov[slot] = moves;
        if (!isfinite(lw)) report(A.err, kErrNonFinite, slot);
    }
}

// Fixed-population reconfiguration of W walkers by systematic resampling
// (one workgroup).  cw: W-double scratch for the cumulative weights.
__global__ void __launch_bounds__(1024) reconfigure_kernel(const double *logw, const double *el,
                                                           const int *nmov, int W, double xi_in,
                                                           uint64_t seed, uint64_t gen, double *cw,
                                                           int *idx, double *out_lwb, double *out_eb,
                                                           long long *out_nm, int *err)
{
    __shared__ double red[32];
    __shared__ long long redi[16];
    const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
    double mx = -INFINITY;
    for (int j = tid; j < W; j += NT) mx = fmax(mx, logw[j]);
    mx = wave_max(mx);
    if (lane == 0) red[wv] = mx;
    __syncthreads();
    mx = red[0];
    for (int w = 1; w < nw; ++w) mx = fmax(mx, red[w]);
    __syncthreads();

    const int chunk = (W + NT - 1) / NT;
    const int c0 = min(W, tid * chunk), c1 = min(W, c0 + chunk);
    double ws = 0.0, ew = 0.0;
    long long nm = 0;
    for (int j = c0; j < c1; ++j) {
        const double w = exp(logw[j] - mx);
        cw[j] = w;
        ws += w;
        ew += w * (el ? el[j] : 0.0);
        nm += nmov ? nmov[j] : 0;
    }
    double Ws;
    const double pre = block_exclusive_scan(ws, red, &Ws);
    double run = pre;
    for (int j = c0; j < c1; ++j) {
        run += cw[j];
        cw[j] = run;
    }
    double v[1] = {ew};
    block_sum<1>(v, red + 16);
    for (int off = 32; off > 0; off >>= 1) nm += __shfl_xor(nm, off, 64);
    if (lane == 0) redi[wv] = nm;
    __syncthreads();
    long long nt = 0;
    for (int w = 0; w < nw; ++w) nt += redi[w];

    double xi = xi_in;
    if (!(xi > 0.0)) {
        double u[4];
        draw4(seed, ~0ull, gen, 0, 3, u);
        xi = u[0];
    }
    const double q = Ws / (double)W;
    for (int s = tid; s < W; s += NT) {
        const double t = ((double)s + xi) * q;
        int lo = 0, hi = W - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cw[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        idx[s] = lo;
    }
    if (tid == 0) {
        if (out_lwb) *out_lwb = log(Ws / (double)W) + mx;
        if (out_eb) *out_eb = v[0] / Ws;
        if (out_nm) *out_nm = nt;
        if (!(Ws > 0.0) || !isfinite(Ws) || !isfinite(mx)) report(err, kErrNonFinite, -1);
    }
}

// Copies selected by a reconfiguration into caller buffers.
__global__ void gather_kernel(const double *pos, const double *el, const int *idx, int W, int stride,
                              double *pos_out, double *el_out, double *lw_out, int *nm_out)
{
    const int s = blockIdx.x;
    if (s >= W) return;
    const int j = idx ? idx[s] : s;
    if (pos_out)
        for (int t = threadIdx.x; t < stride; t += blockDim.x)
            pos_out[(size_t)s * stride + t] = pos[(size_t)j * stride + t];
    if (threadIdx.x == 0) {
        if (el_out) el_out[s] = el[j];
        if (lw_out) lw_out[s] = 0.0;
        if (nm_out) nm_out[s] = 0;
    }
}

// ---------------------------------------------------------------------------
// Host side

std::string g_error;  // last failure without a context

}  // namespace

struct lrdmc_ctx {
    int W = 0, N = 0, n_up = 0, n_dn = 0, ns = 0, K = 0, Kp = 0, n_orb = 0, n_nuc = 0, n_grp = 0,
        n_heavy = 0, M = 0;
    double b_ee = 0, b_en = 0, v_nn = 0;
    lrdmc_params prm{};
    double *d_Z = nullptr, *d_R = nullptr, *d_mo = nullptr, *d_galpha = nullptr;
    int *d_heavy = nullptr, *d_gnuc = nullptr, *d_goff = nullptr;
    double *d_pos[2] = {nullptr, nullptr};
    int cur = 0;
    double *d_logw = nullptr, *d_el = nullptr, *d_cw = nullptr;
    int *d_nmov = nullptr, *d_idx = nullptr, *d_err = nullptr;
    bool loaded = false, projected = false, pending = false;
    uint64_t gen = 0;
    int nt = 64;
    size_t lds_bytes = 0;
    Layout L{};
    std::string err;
};

namespace {

int fail(lrdmc_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    else g_error = msg;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                          \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail((ctx), e_ == hipErrorOutOfMemory ? LRDMC_ENOMEM : LRDMC_EDEVICE,            \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                         \
    } while (0)

Layout make_layout(int N, int ns, int K, int Kp, int M)
{
    Layout L{};
    int o = 0;
    auto take = [&](int n) { int r = o; o += n; return r; };
    L.pos = take(3 * N);
    L.Y = take(N * Kp);
    L.Ainv = take(2 * ns * ns);
    L.dphi = take(N * 4 * ns);
    L.gD = take(4 * N);
    L.gJ = take(4 * N);
    L.Jo = take(N);
    L.Vi = take(N);
    L.T = take(M);
    L.bv = take(5 * K);
    L.vrow = take(5 * ns);
    L.wrow = take(ns);
    L.colk = take(ns);
    L.Yk = take(Kp);
    L.G = take(2 * ns * 2 * ns);
    L.piv = take(2 * 2 * 2 * ns);
    L.fac = take(2 * ns);
    L.red = take(64);
    L.sc = take(32);
    L.total = o;
    return L;
}

KArgs base_args(const lrdmc_ctx *c)
{
    KArgs A{};
    A.N = c->N; A.n_up = c->n_up; A.n_dn = c->n_dn; A.ns = c->ns; A.K = c->K; A.Kp = c->Kp;
    A.n_orb = c->n_orb; A.n_nuc = c->n_nuc; A.n_grp = c->n_grp; A.n_heavy = c->n_heavy; A.M = c->M;
    A.Znuc = c->d_Z; A.Rnuc = c->d_R; A.heavy = c->d_heavy; A.grp_nuc = c->d_gnuc;
    A.grp_alpha = c->d_galpha; A.grp_off = c->d_goff; A.mo = c->d_mo;
    A.b_ee = c->b_ee; A.b_en = c->b_en; A.v_nn = c->v_nn;
    A.a = c->prm.a; A.ap = c->prm.a_prime;
    A.inv_a2 = 1.0 / (c->prm.a * c->prm.a);
    A.inv_ap2 = 1.0 / (c->prm.a_prime * c->prm.a_prime);
    A.inv_2rc2 = 1.0 / (2.0 * c->prm.r_c * c->prm.r_c);
    A.tau = c->prm.tau; A.seed = c->prm.seed; A.rotate = c->prm.rotate;
    A.W = c->W; A.gen = c->gen; A.err = c->d_err; A.L = c->L;
    return A;
}

int check_kernel_error(lrdmc_ctx *c, hipStream_t st)
{
    HIP_TRY(c, hipStreamSynchronize(st));
    int e[2] = {0, 0};
    HIP_TRY(c, hipMemcpy(e, c->d_err, sizeof(e), hipMemcpyDeviceToHost));
    if (e[0] == 0) return LRDMC_OK;
    HIP_TRY(c, hipMemset(c->d_err, 0, 2 * sizeof(int)));
    char buf[160];
    switch (e[0]) {
    case kErrSingular:
        snprintf(buf, sizeof buf, "singular Slater matrix in walker slot %d", e[1]);
        return fail(c, LRDMC_ESINGULAR, buf);
    case kErrIterCap:
        snprintf(buf, sizeof buf, "walker slot %d exceeded %d moves in one generation", e[1], kMaxIter);
        return fail(c, LRDMC_ENONFINITE, buf);
    default:
        if (e[1] < 0) snprintf(buf, sizeof buf, "non-finite total weight in reconfiguration");
        else snprintf(buf, sizeof buf, "non-finite local energy, weight or rate in walker slot %d", e[1]);
        return fail(c, LRDMC_ENONFINITE, buf);
    }
}

int launch_project(lrdmc_ctx *c, hipStream_t st, const double *pos_in, const int *idx_in, double *pos_out,
                   int eval, double *rho, double *k, double *diag)
{
    KArgs A = base_args(c);
    A.pos_in = pos_in;
    A.idx_in = idx_in;
    A.pos_out = pos_out;
    A.logw = c->d_logw;
    A.el = c->d_el;
    A.nmov = c->d_nmov;
    A.eval = eval;
    A.rho_out = rho;
    A.k_out = k;
    A.diag_out = diag;
    hipLaunchKernelGGL(project_kernel, dim3(c->W), dim3(c->nt), c->lds_bytes, st, A);
    HIP_TRY(c, hipGetLastError());
    return LRDMC_OK;
}

int launch_branch(lrdmc_ctx *c, hipStream_t st, double *lwb, double *eb, int64_t *nm, int *idx_out)
{
    hipLaunchKernelGGL(reconfigure_kernel, dim3(1), dim3(1024), 0, st, c->d_logw, c->d_el, c->d_nmov, c->W,
                       -1.0, c->prm.seed, c->gen, c->d_cw, c->d_idx, lwb, eb, (long long *)nm, c->d_err);
    HIP_TRY(c, hipGetLastError());
    if (idx_out)
        HIP_TRY(c, hipMemcpyAsync(idx_out, c->d_idx, sizeof(int) * c->W, hipMemcpyDeviceToDevice, st));
    return LRDMC_OK;
}

// Slater's screening rules and the integral of main text Eq. (7).
double slater_n_core(int Z, double r_c)
{
    struct Sub { int n, l; };
    std::vector<Sub> order;
    for (int nl = 1; nl <= 8; ++nl)
        for (int n = 1; n <= 7; ++n) {
            const int l = nl - n;
            if (l >= 0 && l < n) order.push_back({n, l});
        }
    // Madelung order: by n + l, then n
    std::stable_sort(order.begin(), order.end(), [](const Sub &x, const Sub &y) {
        return (x.n + x.l) != (y.n + y.l) ? (x.n + x.l) < (y.n + y.l) : x.n < y.n;
    });
    struct Grp { int n, kind, occ; };  // kind 0 = sp, 1 = d, 2 = f
    std::vector<Grp> g;
    int left = Z;
    for (const Sub &s : order) {
        if (left <= 0) break;
        const int occ = std::min(left, 2 * (2 * s.l + 1));
        left -= occ;
        const int kind = s.l <= 1 ? 0 : s.l - 1;
        bool found = false;
        for (Grp &q : g)
            if (q.n == s.n && q.kind == kind) { q.occ += occ; found = true; }
        if (!found) g.push_back({s.n, kind, occ});
    }
    std::sort(g.begin(), g.end(), [](const Grp &x, const Grp &y) {
        return x.n != y.n ? x.n < y.n : x.kind < y.kind;
    });
    const double nstar_tab[8] = {0, 1.0, 2.0, 3.0, 3.7, 4.0, 4.2, 4.4};
    double total = 0.0;
    for (size_t a = 0; a < g.size(); ++a) {
        double sh = (g[a].occ - 1) * (g[a].n == 1 ? 0.30 : 0.35);
        for (size_t b = 0; b < a; ++b) {
            if (g[a].kind == 0) {
                if (g[b].n == g[a].n - 1) sh += 0.85 * g[b].occ;
                else if (g[b].n <= g[a].n - 2) sh += 1.00 * g[b].occ;
            } else {
                sh += 1.00 * g[b].occ;
            }
        }
        const double ns = nstar_tab[g[a].n];
        const double zeta = (Z - sh) / ns;
        // occ * int_0^inf N^2 r^(2 n*) exp(-2 zeta r - r^2 / 2 r_c^2) dr,
        // N^2 = (2 zeta)^(2n*+1) / Gamma(2n*+1); composite Simpson in log space.
        const double lognorm = (2 * ns + 1) * std::log(2 * zeta) - std::lgamma(2 * ns + 1);
        const double rmax = (2 * ns + 80.0) / (2 * zeta);
        const int n_int = 40000;
        const double h = rmax / n_int;
        double acc = 0.0;
        for (int q = 1; q < n_int; ++q) {
            const double r = q * h;
            const double f = std::exp(lognorm + 2 * ns * std::log(r) - 2 * zeta * r - r * r / (2 * r_c * r_c));
            acc += (q & 1 ? 4.0 : 2.0) * f;
        }
        total += g[a].occ * acc * h / 3.0;
    }
    return total;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int lrdmc_spacing(double Z, double a, double beta, double kappa, double *r_c, double *a_prime, double *n_core)
{
    if (!(Z >= 1.0 && Z <= 86.0) || !(a > 0.0) || !(beta > 0.0) || !(kappa > 0.0) || !r_c || !a_prime)
        return fail(nullptr, LRDMC_EINVAL, "lrdmc_spacing: invalid arguments");
    const double alpha = 1.0 / (a * Z);
    const double x = 1.0 / (alpha * alpha);
    const double rc = beta * (kappa * x + 1.0) / (x + 1.0) * std::pow(Z, -5.0 / 7.0);
    const double nc = slater_n_core((int)std::lround(Z), rc);
    *r_c = rc;
    *a_prime = a * std::sqrt((Z - nc) / nc);
    if (n_core) *n_core = nc;
    return LRDMC_OK;
}

int lrdmc_create(const lrdmc_system *sys, const lrdmc_params *prm, int32_t n_walkers, lrdmc_ctx **out)
{
    if (!sys || !prm || !out) return fail(nullptr, LRDMC_EINVAL, "lrdmc_create: NULL argument");
    *out = nullptr;
    const int N = sys->n_up + sys->n_dn, ns = std::max(sys->n_up, sys->n_dn);
    if (n_walkers < 1 || sys->n_up < 1 || sys->n_dn < 0 || ns > kMaxNs || N > kMaxN || sys->n_orb < ns ||
        sys->n_nuc < 1 || sys->n_nuc > kMaxNuc || sys->n_shell < 1 || !sys->Z || !sys->R || !sys->shell_nuc ||
        !sys->shell_l || !sys->shell_alpha || !sys->mo)
        return fail(nullptr, LRDMC_EINVAL, "lrdmc_create: invalid system sizes or pointers");
    if (!(prm->a > 0.0) || !(prm->a_prime >= prm->a) || !(prm->r_c > 0.0) || !(prm->tau > 0.0) ||
        !std::isfinite(prm->a_prime) || !std::isfinite(prm->tau) || prm->reserved != 0)
        return fail(nullptr, LRDMC_EINVAL, "lrdmc_create: invalid lattice parameters (need a > 0, a' >= a, r_c > 0, tau > 0)");
    int K = 0;
    for (int q = 0; q < sys->n_shell; ++q) {
        const int l = sys->shell_l[q];
        if (l < 0 || l > 2 || sys->shell_nuc[q] < 0 || sys->shell_nuc[q] >= sys->n_nuc ||
            !(sys->shell_alpha[q] >= 0.0) || !std::isfinite(sys->shell_alpha[q]))
            return fail(nullptr, LRDMC_EINVAL, "lrdmc_create: invalid shell");
        K += 2 * l + 1;
    }
    if (K > kMaxK) return fail(nullptr, LRDMC_EINVAL, "lrdmc_create: more than 512 basis functions");
    std::vector<int> heavy;
    for (int I = 0; I < sys->n_nuc; ++I)
        if (sys->Z[I] >= prm->z_heavy) heavy.push_back(I);
    if (heavy.empty()) return fail(nullptr, LRDMC_EINVAL, "lrdmc_create: no nucleus with Z >= z_heavy");

    // Group shells that share nucleus and exponent: one exponential serves them.
    std::vector<int> gnuc, goff;
    std::vector<double> galpha;
    int mu = 0;
    for (int q = 0; q < sys->n_shell; ++q) {
        const int l = sys->shell_l[q], I = sys->shell_nuc[q];
        const double al = sys->shell_alpha[q];
        int gi = -1;
        for (size_t g = 0; g < gnuc.size(); ++g)
            if (gnuc[g] == I && galpha[g] == al && goff[3 * g + l] < 0) { gi = (int)g; break; }
        if (gi < 0) {
            gi = (int)gnuc.size();
            gnuc.push_back(I);
            galpha.push_back(al);
            goff.insert(goff.end(), {-1, -1, -1});
        }
        goff[3 * gi + l] = mu;
        mu += 2 * l + 1;
    }

    lrdmc_ctx *c = new (std::nothrow) lrdmc_ctx();
    if (!c) return fail(nullptr, LRDMC_ENOMEM, "lrdmc_create: host allocation");
    c->W = n_walkers; c->N = N; c->n_up = sys->n_up; c->n_dn = sys->n_dn; c->ns = ns; c->K = K;
    c->Kp = K | 1; c->n_orb = sys->n_orb; c->n_nuc = sys->n_nuc; c->n_grp = (int)gnuc.size();
    c->n_heavy = (int)heavy.size(); c->M = 12 * N; c->b_ee = sys->b_ee; c->b_en = sys->b_en; c->prm = *prm;
    double vnn = 0.0;
    for (int I = 0; I < sys->n_nuc; ++I)
        for (int J = I + 1; J < sys->n_nuc; ++J) {
            const double dx = sys->R[3 * I] - sys->R[3 * J], dy = sys->R[3 * I + 1] - sys->R[3 * J + 1],
                         dz = sys->R[3 * I + 2] - sys->R[3 * J + 2];
            vnn += sys->Z[I] * sys->Z[J] / std::sqrt(dx * dx + dy * dy + dz * dz);
        }
    c->v_nn = vnn;
    c->nt = std::min(kMaxThreads, std::max(64, ((c->M + 63) / 64) * 64));
    c->L = make_layout(N, ns, K, c->Kp, c->M);
    c->lds_bytes = sizeof(double) * (size_t)c->L.total;

    auto cleanup = [&](int code, const std::string &m) {
        lrdmc_destroy(c);
        return fail(nullptr, code, m);
    };
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return cleanup(LRDMC_EDEVICE, "lrdmc_create: no HIP device");
    if (c->lds_bytes > (size_t)prop.sharedMemPerBlock)
        return cleanup(LRDMC_EINVAL, "lrdmc_create: walker state does not fit in LDS");
    if (c->lds_bytes > 65536 &&
        hipFuncSetAttribute((const void *)project_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)c->lds_bytes) != hipSuccess)
        return cleanup(LRDMC_EDEVICE, "lrdmc_create: cannot raise the LDS limit");

    const size_t W = n_walkers, s3 = 3 * (size_t)N;
    auto alloc = [&](void **p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
    bool ok = alloc((void **)&c->d_Z, sizeof(double) * sys->n_nuc) &&
              alloc((void **)&c->d_R, sizeof(double) * 3 * sys->n_nuc) &&
              alloc((void **)&c->d_mo, sizeof(double) * K * sys->n_orb) &&
              alloc((void **)&c->d_galpha, sizeof(double) * gnuc.size()) &&
              alloc((void **)&c->d_gnuc, sizeof(int) * gnuc.size()) &&
              alloc((void **)&c->d_goff, sizeof(int) * goff.size()) &&
              alloc((void **)&c->d_heavy, sizeof(int) * heavy.size()) &&
              alloc((void **)&c->d_pos[0], sizeof(double) * W * s3) &&
              alloc((void **)&c->d_pos[1], sizeof(double) * W * s3) &&
              alloc((void **)&c->d_logw, sizeof(double) * W) && alloc((void **)&c->d_el, sizeof(double) * W) &&
              alloc((void **)&c->d_cw, sizeof(double) * W) && alloc((void **)&c->d_nmov, sizeof(int) * W) &&
              alloc((void **)&c->d_idx, sizeof(int) * W) && alloc((void **)&c->d_err, sizeof(int) * 2);
    if (!ok) return cleanup(LRDMC_ENOMEM, "lrdmc_create: device allocation failed");
    ok = hipMemcpy(c->d_Z, sys->Z, sizeof(double) * sys->n_nuc, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_R, sys->R, sizeof(double) * 3 * sys->n_nuc, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_mo, sys->mo, sizeof(double) * K * sys->n_orb, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_galpha, galpha.data(), sizeof(double) * gnuc.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_gnuc, gnuc.data(), sizeof(int) * gnuc.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_goff, goff.data(), sizeof(int) * goff.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_heavy, heavy.data(), sizeof(int) * heavy.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(c->d_err, 0, 2 * sizeof(int)) == hipSuccess &&
         hipMemset(c->d_logw, 0, sizeof(double) * W) == hipSuccess &&
         hipMemset(c->d_el, 0, sizeof(double) * W) == hipSuccess &&
         hipMemset(c->d_nmov, 0, sizeof(int) * W) == hipSuccess;
    if (!ok) return cleanup(LRDMC_EDEVICE, "lrdmc_create: device copy failed");
    *out = c;
    return LRDMC_OK;
}

int lrdmc_set_walkers(lrdmc_ctx *c, const double *pos, uint64_t generation, void *stream)
{
    if (!c || !pos) return fail(c, LRDMC_EINVAL, "lrdmc_set_walkers: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipMemcpyAsync(c->d_pos[c->cur], pos, sizeof(double) * 3 * (size_t)c->N * c->W,
                              hipMemcpyDeviceToDevice, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    c->gen = generation;
    c->loaded = true;
    c->projected = false;
    c->pending = false;
    return LRDMC_OK;
}

int lrdmc_project(lrdmc_ctx *c, void *stream)
{
    if (!c || !c->loaded) return fail(c, LRDMC_EINVAL, "lrdmc_project: no walkers loaded");
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_project(c, st, c->d_pos[c->cur], c->pending ? c->d_idx : nullptr, c->d_pos[c->cur ^ 1], 0,
                            nullptr, nullptr, nullptr);
    if (rc) return rc;
    c->cur ^= 1;
    c->pending = false;
    c->projected = true;
    return check_kernel_error(c, st);
}

int lrdmc_branch(lrdmc_ctx *c, void *stream, double *log_wbar, double *ebar, int64_t *n_moves, int32_t *idx)
{
    if (!c || !c->projected) return fail(c, LRDMC_EINVAL, "lrdmc_branch: no projection to reconfigure");
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_branch(c, st, log_wbar, ebar, n_moves, idx);
    if (rc) return rc;
    c->pending = true;
    c->projected = false;
    c->gen += 1;
    return check_kernel_error(c, st);
}

int lrdmc_run(lrdmc_ctx *c, int32_t n_gen, void *stream, double *log_wbar, double *ebar, int64_t *n_moves,
              int32_t *idx)
{
    if (!c || !c->loaded || n_gen < 0) return fail(c, LRDMC_EINVAL, "lrdmc_run: no walkers loaded or n_gen < 0");
    hipStream_t st = (hipStream_t)stream;
    for (int g = 0; g < n_gen; ++g) {
        int rc = launch_project(c, st, c->d_pos[c->cur], c->pending ? c->d_idx : nullptr, c->d_pos[c->cur ^ 1],
                                0, nullptr, nullptr, nullptr);
        if (rc) return rc;
        c->cur ^= 1;
        rc = launch_branch(c, st, log_wbar ? log_wbar + g : nullptr, ebar ? ebar + g : nullptr,
                           n_moves ? n_moves + g : nullptr, idx ? idx + (size_t)g * c->W : nullptr);
        if (rc) return rc;
        c->pending = true;
        c->projected = false;
        c->gen += 1;
    }
    return check_kernel_error(c, st);
}

int lrdmc_get_walkers(lrdmc_ctx *c, double *pos, double *log_w, double *e_loc, int32_t *n_moves, void *stream)
{
    if (!c || !c->loaded) return fail(c, LRDMC_EINVAL, "lrdmc_get_walkers: no walkers loaded");
    hipStream_t st = (hipStream_t)stream;
    const size_t W = c->W, s3 = 3 * (size_t)c->N;
    if (c->pending) {
        hipLaunchKernelGGL(gather_kernel, dim3(c->W), dim3(64), 0, st, c->d_pos[c->cur], c->d_el, c->d_idx, c->W,
                           (int)s3, pos, e_loc, log_w, n_moves);
        HIP_TRY(c, hipGetLastError());
    } else {
        if (pos) HIP_TRY(c, hipMemcpyAsync(pos, c->d_pos[c->cur], sizeof(double) * W * s3, hipMemcpyDeviceToDevice, st));
        if (log_w) HIP_TRY(c, hipMemcpyAsync(log_w, c->d_logw, sizeof(double) * W, hipMemcpyDeviceToDevice, st));
        if (e_loc) HIP_TRY(c, hipMemcpyAsync(e_loc, c->d_el, sizeof(double) * W, hipMemcpyDeviceToDevice, st));
        if (n_moves) HIP_TRY(c, hipMemcpyAsync(n_moves, c->d_nmov, sizeof(int) * W, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    return LRDMC_OK;
}

int lrdmc_eval_moves(lrdmc_ctx *c, const double *pos, double *rho, double *k, double *diag, void *stream)
{
    if (!c || !pos) return fail(c, LRDMC_EINVAL, "lrdmc_eval_moves: NULL positions");
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_project(c, st, pos, nullptr, nullptr, 1, rho, k, diag);
    if (rc) return rc;
    return check_kernel_error(c, st);
}

int lrdmc_reconfigure(const double *log_w, const double *e_loc, int32_t W, double xi, int32_t *idx, double *stats,
                      void *stream)
{
    if (!log_w || !idx || W < 1 || !(xi > 0.0 && xi < 1.0))
        return fail(nullptr, LRDMC_EINVAL, "lrdmc_reconfigure: invalid arguments");
    hipStream_t st = (hipStream_t)stream;
    double *cw = nullptr;
    int *err = nullptr;
    if (hipMallocAsync((void **)&cw, sizeof(double) * W, st) != hipSuccess ||
        hipMallocAsync((void **)&err, sizeof(int) * 2, st) != hipSuccess)
        return fail(nullptr, LRDMC_ENOMEM, "lrdmc_reconfigure: scratch allocation failed");
    (void)hipMemsetAsync(err, 0, 2 * sizeof(int), st);
    hipLaunchKernelGGL(reconfigure_kernel, dim3(1), dim3(1024), 0, st, log_w, e_loc, (const int *)nullptr, W, xi,
                       0ull, 0ull, cw, idx, stats, stats ? stats + 1 : nullptr, (long long *)nullptr, err);
    hipError_t le = hipGetLastError();
    int e[2] = {0, 0};
    (void)hipMemcpyAsync(e, err, sizeof(e), hipMemcpyDeviceToHost, st);
    (void)hipFreeAsync(cw, st);
    (void)hipFreeAsync(err, st);
    hipError_t se = hipStreamSynchronize(st);
    if (le != hipSuccess || se != hipSuccess)
        return fail(nullptr, LRDMC_EDEVICE, std::string("lrdmc_reconfigure: ") +
                                                hipGetErrorString(le != hipSuccess ? le : se));
    if (e[0]) return fail(nullptr, LRDMC_ENONFINITE, "lrdmc_reconfigure: non-finite weights");
    return LRDMC_OK;
}

uint64_t lrdmc_generation(const lrdmc_ctx *c) { return c ? c->gen : 0; }

const char *lrdmc_last_error(const lrdmc_ctx *c) { return c ? c->err.c_str() : g_error.c_str(); }

void lrdmc_destroy(lrdmc_ctx *c)
{
    if (!c) return;
    void *ptrs[] = {c->d_Z,    c->d_R,    c->d_mo,   c->d_galpha, c->d_gnuc, c->d_goff, c->d_heavy, c->d_pos[0],
                    c->d_pos[1], c->d_logw, c->d_el, c->d_cw,     c->d_nmov, c->d_idx,  c->d_err};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete c;
}

}  // extern "C"
