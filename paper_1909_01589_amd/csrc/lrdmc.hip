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
#include <mutex>
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
constexpr int kDphLdsBytes = 2048;  // derivative rows up to this size live in LDS (fixed-size kernels)

// Internal kernel error codes (err[0]); err[1] holds the slot.
enum { kErrSingular = 1, kErrNonFinite = 2, kErrIterCap = 3, kErrCollapse = 4 };

// Offsets (in doubles) of the per-walker LDS arrays.  The region starting at
// U is used twice: during the generation start it holds the Gauss-Jordan
// workspace and a batch of basis blocks, during the move loop the heat-bath
// weights and the accepted-move temporaries.
struct Layout {
    int pos;    // [N][3]            positions
    int Y;      // [N][Kp]           Y[i][mu] = sum_j C[mu][j] Ainv_sigma(i)[j][i_sigma]
    int Ainv;   // [2][ns][ns]       Ainv_sigma[j][i]
    int dld;    // row length of the derivative rows (in the walker's HBM state, see KArgs)
    int gD;     // [N][4]            grad D/D (3) and lap D/D of electron i
    int gJ;     // [N][4]            grad J (3) and lap J of electron i
    int Jo;     // [N]               Jastrow terms that contain electron i
    int red;    // [16]              reduction scratch
    int sc;     // [8]               block scalars
    int rng;    // [8][12]           rotations, -ln u1 and u2 of eight iterations
    int dph;    // [N][dld]          derivative rows in LDS (small systems), or -1: in the HBM state blob
    // move-loop view of U: the weights and their prefix sums (table to search),
    // then the accepted-move temporaries
    int xs;     // [NT]              per-thread inclusive prefix of T within its wavefront
    int T;      // [M]               heat-bath weights of the moves
    int bv;     // [5][K]            basis value, gradient, Laplacian at one point
    int vrow;   // [5][ns]           orbital value, gradient, Laplacian at one point
    int wrow;   // [ns]              w_i = phi(r_new) . Ainv[:, i]
    int colk;   // [ns]              column k of Ainv before the update
    int Yk;     // [Kp]              row k of Y before the update
    int dq;     // [4][ns]           dphi_i[c] . Ainv[:, k] of the moved electron's spin
    int kp;     // [6][N + n_nuc]    moved electron's Jastrow terms per partner, potential change
    // generation-start view of U
    int G;      // [2][ns][2ns]      Gauss-Jordan workspace
    int piv;    // [2][2][2ns]       pivot row and row c copies
    int fac;    // [2][ns]           elimination factors
    int bvb;    // [EB][5][K]        basis blocks of a batch of electrons
    int EB;     // electrons per batch
    int yg;     // 1: Y is not in LDS but at the start of the walker's HBM state blob
    int total;
};

constexpr __host__ __device__ int cmax(int a, int b) { return a > b ? a : b; }

// Threads per walker: one per +/- pair of moves, in whole wavefronts, at
// most kMaxThreads (then a thread takes several pairs).
constexpr __host__ __device__ int threads_for(int M)
{
    return cmax(64, ((M / 2 + 63) / 64) * 64) < kMaxThreads ? cmax(64, ((M / 2 + 63) / 64) * 64) : kMaxThreads;
}

// LDS layout of one walker.  The electron batch of the generation start grows until the block reaches
// `target` bytes (or all electrons fit), never below one electron.
constexpr __host__ __device__ Layout make_layout(int N, int ns, int K, int Kp, int M, int n_nuc, int NT,
                                                 size_t target, bool yg = false)
{
    Layout L{};
    int o = 0;
    auto take = [&](int n) { int r = o; o += n; return r; };
    L.pos = take(3 * N);
    L.yg = yg ? 1 : 0;
    L.Y = yg ? 0 : take(N * Kp);
    L.Ainv = take(2 * ns * ns);
    L.dld = 4 * ns + 1;
    L.gD = take(4 * N);
    L.gJ = take(4 * N);
    L.Jo = take(N);
    L.red = take(16);
    L.sc = take(8);
    L.rng = take(8 * 12);
    // small systems keep the derivative rows in LDS during the generation
    // (the accepted move reads and writes them; from HBM its three phases
    // wait on their latency)
    L.dph = (!yg && N * L.dld * (int)sizeof(double) <= kDphLdsBytes) ? take(N * L.dld) : -1;
    const int U = o;
    // move-loop view.  The prefix sums and weights live from the table to
    // the search, which some wavefronts finish while others already write
    // the first-phase temporaries of the accepted move; only the second-phase
    // outputs (vrow, wrow) may share their space.
    int q = U;
    L.xs = q; q += NT;
    L.T = q; q += M;
    const int search_end = q;
    q = U;
    L.vrow = q; q += 5 * ns;
    L.wrow = q; q += ns;
    L.bv = q; q += 5 * Kp;
    L.colk = q; q += ns;
    L.Yk = q; q += Kp;
    L.dq = q; q += 4 * ns;
    L.kp = q; q += 6 * (N + n_nuc);
    const int loop_end = cmax(q, search_end);
    // generation-start view
    q = U;
    L.G = q; q += 2 * ns * 2 * ns;
    L.piv = q; q += 2 * 2 * 2 * ns;
    L.fac = q; q += 2 * ns;
    L.bvb = q;
    const int fixed_end = q;
    int EB = 1;
    const int base_total = cmax(loop_end, fixed_end + 5 * Kp);
    const size_t limit = target > (size_t)base_total * sizeof(double) ? target : (size_t)base_total * sizeof(double);
    while (EB < N && (size_t)cmax(loop_end, fixed_end + (EB + 1) * 5 * Kp) * sizeof(double) <= limit) ++EB;
    L.EB = EB;
    L.total = cmax(loop_end, fixed_end + EB * 5 * Kp);
    return L;
}

// Basis functions are ordered group by group (s, then p x y z, then the five
// d), groups by nucleus and exponent.  A chain is a run of groups on one
// nucleus whose exponents grow by one constant ratio beta (see basis_dot2).
struct ChainDesc {
    double R[3];                 // nucleus
    double alpha0;               // exponent of the first group
    unsigned long long flags;    // 3 bits per group: s, p, d shell present
    int len;                     // groups (at most 21)
    int code;                    // 1, 2, 3: beta = 2, 2.5, 3; 0: single group
    int mu0;                     // first basis function
    int n_spd;                   // leading groups with s, p and d shells
    int n_sp;                    // end of the run of s, p groups that follows
    int tail0;                   // first group of the trailing run of two or more s-only groups (len: none)
};
static_assert(sizeof(ChainDesc) == 64, "chain descriptor size");

// One basis function: exponent, centre, angular momentum and component.
struct FnDesc {
    double alpha;
    double R[3];
    int l, comp;
    int pad[2];
};
static_assert(sizeof(FnDesc) == 48, "basis function descriptor size");

struct KArgs {
    // system
    int N, n_up, n_dn, ns, K, Kp, n_nuc, n_heavy, M;
    int nt;                        // threads per workgroup
    const double *Znuc, *Rnuc;     // [n_nuc], [n_nuc][3]
    const double *Rheavy;          // [n_heavy][3] nuclei with Z >= z_heavy
    const FnDesc *fns;             // [K]
    int n_chain;
    const ChainDesc *chains;       // [n_chain]
    const double *moT;             // [ns][K]: occupied MO coefficients, orbital-major
    double b_ee, b_en, v_nn;
    // learned pair correction (kernels built with CORR): on interval k of
    // width 1 / f_hinv, F = sum_p fcoef[type][k][p] t^p with t in [0, 1)
    const double *fcoef;           // [2][f_nint][6], type 0 e-e, 1 e-n
    int f_nint;
    double f_hinv, f_rcut;
    // lattice
    double a, ap, inv_a2, inv_ap2, tau;
    double sw_c;                   // 1 / (2 r_c^2) (Gaussian switch) or r_c^2 (Pade switch)
    int sw_pade;                   // 1: Pade switch of Eq. (2); 0: Gaussian of Eq. (3)
    int mpe;                       // moves per electron: 12 (double grid) or 6 (single grid, p = 1)
    uint64_t seed;
    int rotate;
    // walkers
    int W;
    int max_iter;                  // moves per walker and generation before LRDMC_EITERCAP
    uint64_t gen;
    const double *pos_in;
    const int *idx_in;             // gather on load, or nullptr
    const double *state_in;        // walker state blobs to resume from, or nullptr (recompute)
    double *state_out;             // walker state blobs: derivative rows during the projection,
                                   // the rest at its end
    int state_len;                 // doubles per blob: LDS [Y, Jo + N), E_L, V, derivative rows
    int dphi_at;                   // offset of the derivative rows in a blob: [N][dld], row i holds
                                   // grad (x, y, z) and Laplacian of phi_j at r_i at c * ns + j
    int save_state;                // store the LDS part, E_L and V at the end
    double *pos_out, *logw, *el;
    int *nmov;
    int *err;
    // Metropolis sampling
    int vmc_steps;
    double vmc_step;
    // evaluation mode
    int eval;
    double *rho_out, *k_out, *diag_out;
    Layout L;
};

// Block scalar slots.
enum { SC_DV = 0 };

__device__ __forceinline__ void report(int *err, int code, int slot)
{
    if (atomicCAS(err, 0, code) == 0) atomicExch(err + 1, slot);
}

__device__ __forceinline__ int spin_of(const KArgs &A, int i) { return i < A.n_up ? 0 : 1; }

// The system tables are read-only during a launch: reading them through the
// constant address space lets uniform indices use scalar loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cst(const T *p)
{
    return (const __attribute__((address_space(4))) T *)p;
}

// Values that every lane of the workgroup holds identically are moved to
// scalar registers (they are read from LDS, so the compiler cannot prove it).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double uni(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// -- basis -------------------------------------------------------------------

// Value, gradient and Laplacian of basis function mu at r into bv[5][Kp].
// For a harmonic polynomial P of degree l: grad g = (grad P - 2 alpha d P) e,
// lap g = (4 alpha^2 d^2 - (6 + 4 l) alpha) P e.
__device__ __forceinline__ void basis_fn_full(const KArgs &A, int mu, const double r[3], double *bv)
{
    const int K = A.Kp;
    const FnDesc F = A.fns[mu];
    const int l = F.l, c = F.comp;
    const double d[3] = {r[0] - F.R[0], r[1] - F.R[1], r[2] - F.R[2]};
    const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double al = F.alpha;
    const double e = exp(-al * d2);
    double P, dP[3];
    if (l == 0) {
        P = 1.0; dP[0] = dP[1] = dP[2] = 0.0;
    } else if (l == 1) {
        P = d[c]; dP[0] = dP[1] = dP[2] = 0.0; dP[c] = 1.0;
    } else {
        const double x = d[0], y = d[1], z = d[2];
        switch (c) {
        case 0: P = x * y; dP[0] = y; dP[1] = x; dP[2] = 0.0; break;
        case 1: P = y * z; dP[0] = 0.0; dP[1] = z; dP[2] = y; break;
        case 2: P = z * x; dP[0] = z; dP[1] = 0.0; dP[2] = x; break;
        case 3: P = x * x - y * y; dP[0] = 2.0 * x; dP[1] = -2.0 * y; dP[2] = 0.0; break;
        default: P = 2.0 * z * z - x * x - y * y; dP[0] = -2.0 * x; dP[1] = -2.0 * y; dP[2] = 4.0 * z; break;
        }
    }
    const double t2a = 2.0 * al;
    bv[mu] = P * e;
    bv[K + mu] = (dP[0] - t2a * d[0] * P) * e;
    bv[2 * K + mu] = (dP[1] - t2a * d[1] * P) * e;
    bv[3 * K + mu] = (dP[2] - t2a * d[2] * P) * e;
    bv[4 * K + mu] = (4.0 * al * al * d2 - (6.0 + 4.0 * l) * al) * P * e;
}

// sqrt(e) for e in [0, 1]: s = e y0 from the hardware reciprocal square-root
// estimate y0 (relative error below 2^-24 on gfx950), then two corrections
// s += (y0 / 2)(e - s^2) with fused residuals, which leave s at rounding
// level.  The estimate is taken at e + 1e-300: that shift changes nothing
// above 1e-284, and below 1e-154 the chain multiplies the result by e^2 = 0.
__device__ __forceinline__ double sqrt_chain(double e)
{
    const double y = __builtin_amdgcn_rsq(e + 1e-300), h = 0.5 * y;
    double s = e * y;
    s = fma(h, fma(-s, s, e), s);
    return fma(h, fma(-s, s, e), s);
}

// Angular factors of a point at (x, y, z) from a nucleus, in the basis
// order of a group: p (x, y, z), then d (xy, yz, zx, x^2 - y^2,
// 2 z^2 - x^2 - y^2).
struct Ang {
    double x, y, z, xy, yz, zx, d3, d4;
};
__device__ __forceinline__ Ang ang_of(double x, double y, double z)
{
    return Ang{x, y, z, x * y, y * z, z * x, x * x - y * y, 2.0 * z * z - x * x - y * y};
}

// sum over one group's functions of angular factor times y (v: slot 0 the s
// function, 1-3 the p, 4-8 the d), accumulated by fused multiply-adds in
// basis order.
__device__ __forceinline__ double shell_dot(const Ang &g, bool s, bool p, bool d, const double v[9])
{
    double t = s ? v[0] : 0.0;
    if (p) {
        t = fma(g.x, v[1], t);
        t = fma(g.y, v[2], t);
        t = fma(g.z, v[3], t);
    }
    if (d) {
        t = fma(g.xy, v[4], t);
        t = fma(g.yz, v[5], t);
        t = fma(g.zx, v[6], t);
        t = fma(g.d3, v[7], t);
        t = fma(g.d4, v[8], t);
    }
    return t;
}

// One group of chain_dot2 with its shells F fixed at compile time: the sums
// of shell_dot, shell by shell, as the generic loop of chain_dot2 forms them.
template <int F, bool TWO>
__device__ __forceinline__ const double *group_lds(const double *yq, double ax, double ay, double az, double bx,
                                                   double by, double bz, double &pa, double &pb)
{
    pa = 0.0;
    pb = 0.0;
    if (F & 1) {
        pa = yq[0];
        if (TWO) pb = pa;
        yq += 1;
    }
    if (F & 2) {
        const double y0 = yq[0], y1 = yq[1], y2 = yq[2];
        pa = fma(ax, y0, pa);
        pa = fma(ay, y1, pa);
        pa = fma(az, y2, pa);
        if (TWO) {
            pb = fma(bx, y0, pb);
            pb = fma(by, y1, pb);
            pb = fma(bz, y2, pb);
        }
        yq += 3;
    }
    if (F & 4) {
        const double y0 = yq[0], y1 = yq[1], y2 = yq[2], y3 = yq[3], y4 = yq[4];
        const Ang ga = ang_of(ax, ay, az);
        pa = fma(ga.xy, y0, pa);
        pa = fma(ga.yz, y1, pa);
        pa = fma(ga.zx, y2, pa);
        pa = fma(ga.d3, y3, pa);
        pa = fma(ga.d4, y4, pa);
        if (TWO) {
            const Ang gb = ang_of(bx, by, bz);
            pb = fma(gb.xy, y0, pb);
            pb = fma(gb.yz, y1, pb);
            pb = fma(gb.zx, y2, pb);
            pb = fma(gb.d3, y3, pb);
            pb = fma(gb.d4, y4, pb);
        }
        yq += 5;
    }
    return yq;
}

// Exponential of the next group of a chain from the current one (TWO false:
// the first point only).
template <int CODE, bool TWO>
__device__ __forceinline__ void chain_step(double &ea, double &eb)
{
    if (CODE == 3) {
        ea = ea * ea * ea;
        if (TWO) eb = eb * eb * eb;
    } else if (CODE == 2) {
        const double sa = sqrt_chain(ea), sb = TWO ? sqrt_chain(eb) : 0.0;
        ea = (ea * ea) * sa;
        if (TWO) eb = (eb * eb) * sb;
    } else if (CODE == 1) {
        ea = ea * ea;
        if (TWO) eb = eb * eb;
    }
}

// One chain of basis_dot2 with its step code fixed at compile time
// (e^2.5 = e^2 sqrt(e)); the chain has no branches on the data.  The runs
// of s,p,d groups, s,p groups and trailing s-only groups that the host found
// in the chain go through loops with the shells fixed; the rest tests each
// group's flags.  TWO false: the first point only (the b results are not
// formed).
template <int CODE, bool TWO, typename DescPtr>
__device__ __forceinline__ void chain_dot2(DescPtr D, const double *yq, double ax, double ay, double az,
                                           double bx, double by, double bz, double ea, double eb, double &acc_a,
                                           double &acc_b)
{
    const unsigned long long fl = D->flags;
    const int len = D->len, n7 = D->n_spd, n3 = D->n_sp, n1 = D->tail0 == n3 ? len : n3;
    int q0 = 0;
    for (; q0 < n7; ++q0) {
        double pa, pb;
        yq = group_lds<7, TWO>(yq, ax, ay, az, bx, by, bz, pa, pb);
        acc_a += ea * pa;
        if (TWO) acc_b += eb * pb;
        if (q0 + 1 == len) return;
        chain_step<CODE, TWO>(ea, eb);
    }
    for (; q0 < n3; ++q0) {
        double pa, pb;
        yq = group_lds<3, TWO>(yq, ax, ay, az, bx, by, bz, pa, pb);
        acc_a += ea * pa;
        if (TWO) acc_b += eb * pb;
        if (q0 + 1 == len) return;
        chain_step<CODE, TWO>(ea, eb);
    }
    for (; q0 < n1; ++q0) {
        double pa, pb;
        yq = group_lds<1, TWO>(yq, ax, ay, az, bx, by, bz, pa, pb);
        acc_a += ea * pa;
        if (TWO) acc_b += eb * pb;
        if (q0 + 1 == len) return;
        chain_step<CODE, TWO>(ea, eb);
    }
    for (int q = q0; q < len; ++q) {
        const int f = (int)(fl >> (3 * q)) & 7;
        // shell_dot's sums, shell by shell as the loads arrive
        double pa = 0.0, pb = 0.0;
        if (f & 1) {
            pa = yq[0];
            if (TWO) pb = pa;
            yq += 1;
        }
        if (f & 2) {
            const double y0 = yq[0], y1 = yq[1], y2 = yq[2];
            pa = fma(ax, y0, pa);
            pa = fma(ay, y1, pa);
            pa = fma(az, y2, pa);
            if (TWO) {
                pb = fma(bx, y0, pb);
                pb = fma(by, y1, pb);
                pb = fma(bz, y2, pb);
            }
            yq += 3;
        }
        if (f & 4) {
            const double y0 = yq[0], y1 = yq[1], y2 = yq[2], y3 = yq[3], y4 = yq[4];
            const Ang ga = ang_of(ax, ay, az);
            pa = fma(ga.xy, y0, pa);
            pa = fma(ga.yz, y1, pa);
            pa = fma(ga.zx, y2, pa);
            pa = fma(ga.d3, y3, pa);
            pa = fma(ga.d4, y4, pa);
            if (TWO) {
                const Ang gb = ang_of(bx, by, bz);
                pb = fma(gb.xy, y0, pb);
                pb = fma(gb.yz, y1, pb);
                pb = fma(gb.zx, y2, pb);
                pb = fma(gb.d3, y3, pb);
                pb = fma(gb.d4, y4, pb);
            }
            yq += 5;
        }
        acc_a += ea * pa;
        if (TWO) acc_b += eb * pb;
        if (q + 1 == len) break;
        chain_step<CODE, TWO>(ea, eb);
    }
}

// One group of chain_dot2_pf with its shell flags F (s, p, d) fixed at
// compile time: all of its loads of y issue together, then the same
// arithmetic in the same order as chain_dot2.  Returns the group's size.
template <int F>
__device__ __forceinline__ int group_dot2(const double *yq, const Ang &ga, const Ang &gb, double &pa, double &pb)
{
    constexpr int os = 0, op = (F & 1), od = op + ((F & 2) ? 3 : 0);
    double v[9];
    if (F & 1) v[0] = yq[os];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        if (F & 2) v[1 + j] = yq[op + j];
#pragma unroll
    for (int j = 0; j < 5; ++j)
        if (F & 4) v[4 + j] = yq[od + j];
    pa = shell_dot(ga, F & 1, F & 2, F & 4, v);
    pb = shell_dot(gb, F & 1, F & 2, F & 4, v);
    return od + ((F & 4) ? 5 : 0);
}

// chain_dot2 with y in device memory: each group's loads issue together at
// its start, in a block of their own for each combination of shells, and
// (TAIL) a trailing run of at least two s-only groups loads four values at
// a time (one wait per block instead of one per shell).  Same arithmetic,
// in the same order, as chain_dot2.
template <int CODE, bool TAIL, typename DescPtr>
__device__ __forceinline__ void chain_dot2_pf(DescPtr D, const double *yq, double ax, double ay,
                                              double az, double bx, double by, double bz, double ea, double eb,
                                              double &acc_a, double &acc_b)
{
    const Ang ga = ang_of(ax, ay, az), gb = ang_of(bx, by, bz);
    const unsigned long long fl = D->flags;
    const int len = D->len;
    // first group of the trailing s-only run
    const int q1 = TAIL ? D->tail0 : len;
    // An even-tempered chain starts with its groups of s, p and d shells,
    // then those of s and p: loops over those runs need no branch on the
    // flags, and the loads of a group are not behind one.
    const int n7 = min(D->n_spd, q1), n3 = min(D->n_sp, q1);
    int q = 0;
    for (; q < n7; ++q) {
        double pa, pb;
        yq += group_dot2<7>(yq, ga, gb, pa, pb);
        acc_a += ea * pa;
        acc_b += eb * pb;
        if (q + 1 == len) return;
        chain_step<CODE, true>(ea, eb);
    }
    for (; q < n3; ++q) {
        double pa, pb;
        yq += group_dot2<3>(yq, ga, gb, pa, pb);
        acc_a += ea * pa;
        acc_b += eb * pb;
        if (q + 1 == len) return;
        chain_step<CODE, true>(ea, eb);
    }
    for (; q < q1; ++q) {
        const int f = (int)(fl >> (3 * q)) & 7;
        double pa = 0.0, pb = 0.0;
        switch (f) {
        case 1: yq += group_dot2<1>(yq, ga, gb, pa, pb); break;
        case 2: yq += group_dot2<2>(yq, ga, gb, pa, pb); break;
        case 3: yq += group_dot2<3>(yq, ga, gb, pa, pb); break;
        case 4: yq += group_dot2<4>(yq, ga, gb, pa, pb); break;
        case 5: yq += group_dot2<5>(yq, ga, gb, pa, pb); break;
        case 6: yq += group_dot2<6>(yq, ga, gb, pa, pb); break;
        case 7: yq += group_dot2<7>(yq, ga, gb, pa, pb); break;
        default: break;
        }
        acc_a += ea * pa;
        acc_b += eb * pb;
        if (q + 1 == len) return;
        chain_step<CODE, true>(ea, eb);
    }
    for (int q = q1; q < len; q += 4) {
        const int nb = min(4, len - q);
        double v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = yq[min(j, nb - 1)];
        yq += nb;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j < nb) {
                acc_a += ea * v[j];
                acc_b += eb * v[j];
                if (q + j + 1 < len) chain_step<CODE, true>(ea, eb);
            }
        }
    }
}

// sum_mu g_mu(r) y[mu] at the two points ra, rb of a +/- move pair of one
// electron (y: its orbital-projected inverse row): the determinant ratios of
// the two moves.  Along a chain the exponential of the next group is a power
// of the current one (e^2, e^2 sqrt(e), e^3 for beta = 2, 2.5, 3), so a chain
// costs one exp per point; both points share the loads of y.  PF: y is in
// device memory, and each group's loads issue together (TAIL: with the
// batched s-only tail; the compacted table, where it measured slower, goes
// without).  TWO false (y in LDS): the first point only, out_b unset.
template <bool PF = false, bool TAIL = true, bool TWO = true>
__device__ __forceinline__ void basis_dot2(const KArgs &A, const double ra[3], const double rb[3],
                                           const double *y, double &out_a, double &out_b)
{
    static_assert(TWO || !PF, "one point only with y in LDS");
    double acc_a = 0.0, acc_b = 0.0;
    const auto *chains = cst(A.chains);
    for (int ch = 0; ch < A.n_chain; ++ch) {
        const auto *D = chains + ch;
        const double ax = ra[0] - D->R[0], ay = ra[1] - D->R[1], az = ra[2] - D->R[2];
        const double bx = rb[0] - D->R[0], by = rb[1] - D->R[1], bz = rb[2] - D->R[2];
        const double a2 = ax * ax + ay * ay + az * az, b2 = bx * bx + by * by + bz * bz;
        const double al0 = D->alpha0;
        const double ea = exp(-al0 * a2), eb = TWO ? exp(-al0 * b2) : 0.0;
        const int code = D->code;
        const double *yq = y + D->mu0;
        if constexpr (PF) {
            if (code == 2)
                chain_dot2_pf<2, TAIL>(D, yq, ax, ay, az, bx, by, bz, ea, eb, acc_a, acc_b);
            else if (code == 1)
                chain_dot2_pf<1, TAIL>(D, yq, ax, ay, az, bx, by, bz, ea, eb, acc_a, acc_b);
            else if (code == 3)
                chain_dot2_pf<3, TAIL>(D, yq, ax, ay, az, bx, by, bz, ea, eb, acc_a, acc_b);
            else
                chain_dot2_pf<0, TAIL>(D, yq, ax, ay, az, bx, by, bz, ea, eb, acc_a, acc_b);
        } else {
            if (code == 2)
                chain_dot2<2, TWO>(D, yq, ax, ay, az, bx, by, bz, ea, eb, acc_a, acc_b);
            else if (code == 1)
                chain_dot2<1, TWO>(D, yq, ax, ay, az, bx, by, bz, ea, eb, acc_a, acc_b);
            else if (code == 3)
                chain_dot2<3, TWO>(D, yq, ax, ay, az, bx, by, bz, ea, eb, acc_a, acc_b);
            else
                chain_dot2<0, TWO>(D, yq, ax, ay, az, bx, by, bz, ea, eb, acc_a, acc_b);
        }
    }
    out_a = acc_a;
    if (TWO) out_b = acc_b;
}

__device__ __forceinline__ double rcp_nr(double a);

// Spacing of grid g (0: a, 1: a').  Both fields are read before the select:
// a select between the two field addresses keeps a modified argument copy
// (the fixed-size kernels) in scratch memory.
__device__ __forceinline__ double grid_spacing(const KArgs &A, int g)
{
    const double a = A.a, ap = A.ap;
    return g ? ap : a;
}

// Switch p at x from the squared distance d2 to the nearest heavy nucleus:
// exp(-d2 / (2 r_c^2)) (Eq. (3)) or 1 / (1 + r_c^2 d2) (Eq. (2)).
__device__ __forceinline__ double p_switch(const KArgs &A, const double x[3])
{
    double best = 0.0;
    const auto *Rh = cst(A.Rheavy);
    for (int h = 0; h < A.n_heavy; ++h) {
        const auto *R = Rh + 3 * h;
        const double dx = x[0] - R[0], dy = x[1] - R[1], dz = x[2] - R[2];
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (h == 0 || d2 < best) best = d2;
    }
    if (A.sw_pade) return rcp_nr(1.0 + A.sw_c * best);
    return exp(-best * A.sw_c);
}

// -- per-walker state ------------------------------------------------------

// Orbital contraction of basis blocks b[e][5][Kp] (value, gradient,
// Laplacian of every basis function at the point of electron e of the
// batch): for each group g = (e, j), e < ne, j < n,
//   out[c] = sum_mu b[e][c][mu] C[mu][j]   (c < 5)
// and with W also out[5] = sum_mu b[e][0][mu] Yrow_j[mu] with Yrow_j at
// yrow + j Kp.  A group is split over P lanes (a power of two, at most 16);
// lane p takes mu = p, p + P, ...  Loads go out four basis functions at a
// time and the P partial sums are combined in registers (DPP).
template <bool W, typename Store>
__device__ __forceinline__ void contract(const KArgs &A, const double *b, int ne, int n, const double *yrow,
                                         Store store)
{
    const int K = A.K, Kp = A.Kp, NT = A.nt, ng = ne * n;
    int lgP = 4;
    while (lgP > 0 && (ng << lgP) > NT) --lgP;
    const int P = 1 << lgP, Q = (K + P - 1) >> lgP;
    for (int base = 0; base < (ng << lgP); base += NT) {
        const int t = base + threadIdx.x, g = t >> lgP, part = t & (P - 1);
        const bool live = g < ng;
        const int e = live ? g / n : 0, j = live ? g - e * n : 0;
        const double *bb = b + e * 5 * Kp, *ct = A.moT + (size_t)j * K, *yr = yrow + j * Kp;
        double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (live) {
            for (int q0 = 0; q0 < Q; q0 += 8) {
                double cv[8], yv[8];
                int mcs[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int mu = part + ((q0 + u) << lgP);
                    const bool ok = mu < K;
                    const int mc = ok ? mu : K - 1;
                    mcs[u] = mc;
                    cv[u] = ok ? ct[mc] : 0.0;
                    if (W) yv[u] = ok ? yr[mc] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    double bq[5];
#pragma unroll
                    for (int c = 0; c < 5; ++c) bq[c] = bb[c * Kp + mcs[u]];
#pragma unroll
                    for (int c = 0; c < 5; ++c) acc[c] = fma(bq[c], cv[u], acc[c]);
                    if (W) acc[5] = fma(bq[0], yv[u], acc[5]);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < (W ? 6 : 5); ++c) acc[c] = group_sum(acc[c], P);
        if (live && part == 0) store(e, j, acc);
    }
}

// -- Pade pair terms -----------------------------------------------------------
// u(r) = c r / (1 + b r) = c / (1/r + b).  With y = 1/r and inv = 1/(y + b):
// u = c inv, q = 1/(1 + b r) = y inv, u' = c q^2, u'' = -2 c b q^3.

// Reciprocal: hardware estimate refined by two Newton-Raphson steps
// x <- x (2 - a x), written as fused multiply-adds.
__device__ __forceinline__ double rcp_nr(double a)
{
    double x = __builtin_amdgcn_rcp(a);
    double e = fma(-a, x, 1.0);
    x = fma(x, e, x);
    e = fma(-a, x, 1.0);
    return fma(x, e, x);
}

// Reciprocal square root: hardware estimate refined by two Newton-Raphson
// steps y <- y (3 - a y^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}


// 1/r for the move table's pair terms: one Newton-Raphson step on the
// hardware estimate (estimates within 2^-24 on gfx950, so about 5e-15
// relative after the step; the same for the shared reciprocals of pair_u2
// and pair_u4), enough for the ratio exp(dJ).
__device__ __forceinline__ double rsqrt_move(double d2)
{
    const double y = __builtin_amdgcn_rsq(d2);
    return fma(y, fma(-0.5 * d2 * y, y, 0.5), y);
}

struct PairD {
    double u;    // u(r)
    double f;    // u'(r) / r
    double lap;  // u''(r) + 2 u'(r) / r
    double y;    // 1 / r
};

__device__ __forceinline__ PairD pade_d(double c, double b, double d2)
{
    const double y = rsqrt_nr(d2);
    const double inv = rcp_nr(y + b);
    const double q = y * inv;
    const double cq2 = c * q * q;
    PairD p;
    p.u = c * inv;
    p.f = cq2 * y;
    p.lap = -2.0 * b * cq2 * q + 2.0 * p.f;
    p.y = y;
    return p;
}

// The learned correction F of pair type `type` at distance r (zero from
// f_rcut on): the quintic of r's interval in Horner form, with F' and F''
// when D asks for them.
template <int D>
__device__ __forceinline__ void corr_eval(const KArgs &A, int type, double r, double F[3])
{
    F[0] = F[1] = F[2] = 0.0;
    if (r < A.f_rcut) {
        const double x = r * A.f_hinv;
        const int k = min((int)x, A.f_nint - 1);
        const double t = x - (double)k;
        const double2 *p = reinterpret_cast<const double2 *>(A.fcoef + 6 * (type * A.f_nint + k));
        const double2 q0 = p[0], q1 = p[1], q2 = p[2];
        const double c0 = q0.x, c1 = q0.y, c2 = q1.x, c3 = q1.y, c4 = q2.x, c5 = q2.y;
        F[0] = fma(t, fma(t, fma(t, fma(t, fma(t, c5, c4), c3), c2), c1), c0);
        if (D >= 1)
            F[1] = fma(t, fma(t, fma(t, fma(t, 5.0 * c5, 4.0 * c4), 3.0 * c3), 2.0 * c2), c1) * A.f_hinv;
        if (D >= 2)
            F[2] = fma(t, fma(t, fma(t, 20.0 * c5, 12.0 * c4), 6.0 * c3), 2.0 * c2) * (A.f_hinv * A.f_hinv);
    }
}

// u = c / (1/r + b) of one pair at the two points a and b of a move pair
// (squared distances d2a, d2b), plus s F(r) with the learned correction
// (s = 1 for electron pairs, Z for an electron and a nucleus, 0 drops the
// pair).  The two denominators share one reciprocal: the hardware estimate
// of 1 / (d_a d_b) with one Newton-Raphson step, times the other factor.
template <bool CORR, bool MX = false>
__device__ __forceinline__ void pair_u2(const KArgs &A, double c, double b, double d2a, double d2b, int type,
                                        double s, double &ua, double &ub)
{
    double ya, yb;
    if constexpr (MX) {
        // mixed precision: 1/r and the shared reciprocal from the FP32
        // hardware estimates (relative error about 2^-22 each), sums in FP64
        const float fa = __builtin_amdgcn_rsqf((float)d2a), fb = __builtin_amdgcn_rsqf((float)d2b);
        const float da = fa + (float)b, db = fb + (float)b;
        const float x = __builtin_amdgcn_rcpf(da * db);
        ua = c * (double)(x * db);
        ub = c * (double)(x * da);
        ya = fa;
        yb = fb;
    } else {
        ya = rsqrt_move(d2a);
        yb = rsqrt_move(d2b);
        const double da = ya + b, db = yb + b, p = da * db;
        double x = __builtin_amdgcn_rcp(p);
        x = fma(x, fma(-p, x, 1.0), x);
        const double cx = c * x;
        ua = cx * db;
        ub = cx * da;
    }
    if constexpr (CORR) {
        double F[3];
        corr_eval<0>(A, type, d2a * ya, F);
        ua = fma(s, F[0], ua);
        corr_eval<0>(A, type, d2b * yb, F);
        ub = fma(s, F[0], ub);
    }
}

// The same for two electron pairs (coefficients c0, c1, correction scales
// s0, s1) at both points: ua, ub are the sums over both pairs, and the four
// denominators share one reciprocal.
template <bool CORR, bool MX = false>
__device__ __forceinline__ void pair_u4(const KArgs &A, double c0, double c1, double b, double qa0, double qb0,
                                        double qa1, double qb1, double s0, double s1, double &ua, double &ub)
{
    double ya0, yb0, ya1, yb1;
    if constexpr (MX) {
        const float fb = (float)b;
        const float fa0 = __builtin_amdgcn_rsqf((float)qa0), fb0 = __builtin_amdgcn_rsqf((float)qb0);
        const float fa1 = __builtin_amdgcn_rsqf((float)qa1), fb1 = __builtin_amdgcn_rsqf((float)qb1);
        const float da0 = fa0 + fb, db0 = fb0 + fb, da1 = fa1 + fb, db1 = fb1 + fb;
        const float p0 = da0 * db0, p1 = da1 * db1;
        const float x = __builtin_amdgcn_rcpf(p0 * p1);
        const float x0 = x * p1, x1 = x * p0;
        ua = c0 * (double)(x0 * db0) + c1 * (double)(x1 * db1);
        ub = c0 * (double)(x0 * da0) + c1 * (double)(x1 * da1);
        ya0 = fa0; yb0 = fb0; ya1 = fa1; yb1 = fb1;
    } else {
        ya0 = rsqrt_move(qa0); yb0 = rsqrt_move(qb0); ya1 = rsqrt_move(qa1); yb1 = rsqrt_move(qb1);
        const double da0 = ya0 + b, db0 = yb0 + b, da1 = ya1 + b, db1 = yb1 + b;
        const double p0 = da0 * db0, p1 = da1 * db1, p = p0 * p1;
        double x = __builtin_amdgcn_rcp(p);
        x = fma(x, fma(-p, x, 1.0), x);
        const double x0 = c0 * (x * p1), x1 = c1 * (x * p0);
        ua = fma(x0, db0, x1 * db1);
        ub = fma(x0, da0, x1 * da1);
    }
    if constexpr (CORR) {
        double F[3];
        corr_eval<0>(A, 0, qa0 * ya0, F);
        ua = fma(s0, F[0], ua);
        corr_eval<0>(A, 0, qb0 * yb0, F);
        ub = fma(s0, F[0], ub);
        corr_eval<0>(A, 0, qa1 * ya1, F);
        ua = fma(s1, F[0], ua);
        corr_eval<0>(A, 0, qb1 * yb1, F);
        ub = fma(s1, F[0], ub);
    }
}

template <bool CORR>
__device__ __forceinline__ PairD pair_d(const KArgs &A, double c, double b, double d2, int type, double s)
{
    PairD p = pade_d(c, b, d2);
    if constexpr (CORR) {
        double F[3];
        corr_eval<2>(A, type, d2 * p.y, F);
        const double f1 = s * F[1] * p.y;
        p.u = fma(s, F[0], p.u);
        p.f += f1;
        p.lap += fma(s, F[2], 2.0 * f1);
    }
    return p;
}

// Jastrow terms containing electron i when it sits at ra and at rb (the two
// points of a +/- move pair; the other electrons fixed).
template <bool CORR, bool MX = false>
__device__ __forceinline__ void jastrow_point2(const KArgs &A, const double *pos, int i, const double ra[3],
                                               const double rb[3], double &out_a, double &out_b)
{
    const bool up = i < A.n_up;
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    int j = 0;
    for (; j + 1 < A.N; j += 2) {
        const double c0 = j == i ? 0.0 : (((j < A.n_up) == up) ? 0.25 : 0.5);
        const double c1 = j + 1 == i ? 0.0 : (((j + 1 < A.n_up) == up) ? 0.25 : 0.5);
        const double s0 = j == i ? 0.0 : 1.0, s1 = j + 1 == i ? 0.0 : 1.0;
        const double x0 = pos[3 * j], y0 = pos[3 * j + 1], z0 = pos[3 * j + 2];
        const double x1 = pos[3 * j + 3], y1 = pos[3 * j + 4], z1 = pos[3 * j + 5];
        double dx = ra[0] - x0, dy = ra[1] - y0, dz = ra[2] - z0;
        const double qa0 = dx * dx + dy * dy + dz * dz;
        dx = rb[0] - x0; dy = rb[1] - y0; dz = rb[2] - z0;
        const double qb0 = dx * dx + dy * dy + dz * dz;
        dx = ra[0] - x1; dy = ra[1] - y1; dz = ra[2] - z1;
        const double qa1 = dx * dx + dy * dy + dz * dz;
        dx = rb[0] - x1; dy = rb[1] - y1; dz = rb[2] - z1;
        const double qb1 = dx * dx + dy * dy + dz * dz;
        double ua, ub;
        pair_u4<CORR, MX>(A, c0, c1, A.b_ee, qa0, qb0, qa1, qb1, s0, s1, ua, ub);
        a0 += ua;
        b0 += ub;
    }
    if (j < A.N) {
        const double c0 = j == i ? 0.0 : (((j < A.n_up) == up) ? 0.25 : 0.5);
        const double s0 = j == i ? 0.0 : 1.0;
        const double x0 = pos[3 * j], y0 = pos[3 * j + 1], z0 = pos[3 * j + 2];
        double dx = ra[0] - x0, dy = ra[1] - y0, dz = ra[2] - z0;
        const double qa0 = dx * dx + dy * dy + dz * dz;
        dx = rb[0] - x0; dy = rb[1] - y0; dz = rb[2] - z0;
        const double qb0 = dx * dx + dy * dy + dz * dz;
        double ua, ub;
        pair_u2<CORR, MX>(A, c0, A.b_ee, qa0, qb0, 0, s0, ua, ub);
        a0 += ua;
        b0 += ub;
    }
    for (int I = 0; I < A.n_nuc; ++I) {
        const auto *R = cst(A.Rnuc) + 3 * I;
        const double c = -cst(A.Znuc)[I];
        double dx = ra[0] - R[0], dy = ra[1] - R[1], dz = ra[2] - R[2];
        const double qa = dx * dx + dy * dy + dz * dz;
        dx = rb[0] - R[0]; dy = rb[1] - R[1]; dz = rb[2] - R[2];
        const double qb = dx * dx + dy * dy + dz * dz;
        double ua, ub;
        pair_u2<CORR, MX>(A, c, A.b_en, qa, qb, 1, -c, ua, ub);
        a1 += ua;
        b1 += ub;
    }
    out_a = a0 + a1;
    out_b = b0 + b1;
}

// Displaced position of move m.
__device__ __forceinline__ void move_position(const KArgs &A, const double *pos, const double *Rm, int m,
                                              double rp[3])
{
    const int i = m / A.mpe, g = A.mpe == 12 ? (m / 6) & 1 : 0, dir = m % 6, ax = dir >> 1;
    const double h = grid_spacing(A, g);
    const double t = (dir & 1) ? -h : h;
    for (int c = 0; c < 3; ++c) rp[c] = pos[3 * i + c] + t * Rm[3 * c + ax];
}

// Jastrow gradient/Laplacian and own sum of every electron; returns the total
// potential to every thread.  Segments of `seg` lanes per electron.
template <bool CORR>
__device__ __forceinline__ double jastrow_setup(const KArgs &A, double *lds)
{
    const Layout &L = A.L;
    const double *pos = lds + L.pos;
    double *gJ = lds + L.gJ, *Jo = lds + L.Jo;
    const int N = A.N;
    int seg = 64;
    while (seg > 1 && seg * N > A.nt) seg >>= 1;
    const int per_pass = A.nt / seg;
    double vsum = 0.0;
    for (int base = 0; base < N; base += per_pass) {
        const int i = base + threadIdx.x / seg, sub = threadIdx.x % seg;
        double g0 = 0, g1 = 0, g2 = 0, lap = 0, jo = 0;
        if (i < N) {
            const int si = spin_of(A, i);
            const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
            for (int j = sub; j < N + A.n_nuc; j += seg) {
                if (j == i) continue;
                double dx, dy, dz, c, b;
                int type;
                if (j < N) {
                    dx = xi - pos[3 * j]; dy = yi - pos[3 * j + 1]; dz = zi - pos[3 * j + 2];
                    c = (spin_of(A, j) == si) ? 0.25 : 0.5;
                    b = A.b_ee;
                    type = 0;
                } else {
                    const double *R = A.Rnuc + 3 * (j - N);
                    dx = xi - R[0]; dy = yi - R[1]; dz = zi - R[2];
                    c = -A.Znuc[j - N];
                    b = A.b_en;
                    type = 1;
                }
                const PairD pr = pair_d<CORR>(A, c, b, dx * dx + dy * dy + dz * dz, type, type ? -c : 1.0);
                g0 += pr.f * dx; g1 += pr.f * dy; g2 += pr.f * dz;
                lap += pr.lap;
                jo += pr.u;
                if (j >= N) vsum += c * pr.y;        // -Z_I / r_iI
                else if (j > i) vsum += pr.y;        // 1 / r_ij, each pair once
            }
        }
        g0 = group_sum(g0, seg); g1 = group_sum(g1, seg); g2 = group_sum(g2, seg);
        lap = group_sum(lap, seg); jo = group_sum(jo, seg);
        if (i < N && sub == 0) {
            gJ[4 * i] = g0; gJ[4 * i + 1] = g1; gJ[4 * i + 2] = g2; gJ[4 * i + 3] = lap;
            Jo[i] = jo;
        }
    }
    double v[1] = {vsum};
    block_sum<1>(v, lds + L.red);
    return v[0] + A.v_nn;
}

// grad D/D and lap D/D of every electron from its derivative rows and Ainv.
__device__ __forceinline__ void det_derivs_all(const KArgs &A, const double *Ainv, const double *dphi,
                                               double *gD)
{
    const int ns = A.ns;
    for (int t = threadIdx.x; t < 4 * A.N; t += A.nt) {
        const int i = t >> 2, c = t & 3;
        const int s = spin_of(A, i), n = s ? A.n_dn : A.n_up, il = s ? i - A.n_up : i;
        const double *inv = Ainv + s * ns * ns;
        const double *dp = dphi + i * A.L.dld + c * ns;
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += dp[j] * inv[j * ns + il];
        gD[4 * i + c] = acc;
    }
}

__device__ __forceinline__ double psi_lap_term(const double *d, const double *j)
{
    return d[3] + 2.0 * (d[0] * j[0] + d[1] * j[1] + d[2] * j[2]) + j[3] + j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
}

// Generation start: Slater matrices and derivative rows of every electron,
// Gauss-Jordan inversion with partial pivoting, Y = C Ainv, determinant and
// Jastrow derivatives, local energy.  Returns an error code (uniform);
// EL, LAP (sum_i lap_i Psi/Psi) and V reach every thread.
// The orbital-projected inverse Y[N][Kp]: in LDS, or (large systems) at the
// start of the walker slot's output state blob in HBM, where it stays for the
// whole generation (L2-resident) and is read and updated in place.
template <bool YG>
__device__ __forceinline__ double *y_base(const KArgs &A, double *lds)
{
    if constexpr (YG) return A.state_out + (size_t)blockIdx.x * A.state_len;
    else return lds + A.L.Y;
}

template <bool CORR, bool YG>
__device__ __forceinline__ int walker_setup(const KArgs &A, double *lds, double *dphi, int *sflag, double &EL, double &LAP,
                            double &V)
{
    const Layout &L = A.L;
    const int N = A.N, ns = A.ns, K = A.K, Kp = A.Kp, tid = threadIdx.x, NT = A.nt;
    double *pos = lds + L.pos, *G = lds + L.G, *bvb = lds + L.bvb;
    double *Ainv = lds + L.Ainv;
    const int two = 2 * ns;

    // right halves = identity
    for (int t = tid; t < 2 * ns * two; t += NT) {
        const int r = (t / two) % ns, c = t % two;
        if (c >= ns) G[t] = (c - ns == r) ? 1.0 : 0.0;
    }
    for (int e0 = 0; e0 < N; e0 += L.EB) {
        const int ne = min(L.EB, N - e0);
        for (int t = tid; t < ne * K; t += NT) {
            const int e = t / K, mu = t - e * K, i = e0 + e;
            const double r[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
            basis_fn_full(A, mu, r, bvb + e * 5 * Kp);
        }
        __syncthreads();
        contract<false>(A, bvb, ne, ns, nullptr, [&](int e, int j, const double *v) {
            const int i = e0 + e, s = spin_of(A, i), n = s ? A.n_dn : A.n_up, il = s ? i - A.n_up : i;
            if (j >= n) return;
            G[(s * ns + il) * two + j] = v[0];
            for (int c = 1; c < 5; ++c) dphi[i * L.dld + (c - 1) * ns + j] = v[c];
        });
        __syncthreads();
    }

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
    double *Y = y_base<YG>(A, lds);
    for (int t = tid; t < N * K; t += NT) {
        const int i = t / K, mu = t - i * K;
        const int s = spin_of(A, i), n = s ? A.n_dn : A.n_up, il = s ? i - A.n_up : i;
        const double *inv = Ainv + s * ns * ns;
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += A.moT[j * K + mu] * inv[j * ns + il];
        Y[i * Kp + mu] = acc;
    }
    det_derivs_all(A, Ainv, dphi, lds + L.gD);
    V = uni(jastrow_setup<CORR>(A, lds));     // ends with workgroup barriers
    double v[1] = {0.0};
    for (int i = tid; i < N; i += NT) v[0] += psi_lap_term(lds + L.gD + 4 * i, lds + L.gJ + 4 * i);
    block_sum<1>(v, lds + L.red);
    LAP = uni(v[0]);
    EL = uni(-0.5 * LAP + V);
    return isfinite(EL) ? 0 : kErrNonFinite;
}

// Random numbers of iterations it .. it+7 (rotation, -ln u1 and u2), computed
// by eight lanes at once into rng[8][12] (it a multiple of 8; every read of
// the previous eight is done when the refill runs).
__device__ __forceinline__ void refill_rng(const KArgs &A, double *rng, int slot, int it)
{
    const int q = threadIdx.x;
    if (q < 8) {
        double Rm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, u[4];
        if (A.rotate) {
            draw4(A.seed, slot, A.gen, (uint64_t)(it + q), 1, u);
            rotation(u, Rm);
        }
        double *o = rng + 12 * q;
        for (int c = 0; c < 9; ++c) o[c] = Rm[c];
        draw4(A.seed, slot, A.gen, (uint64_t)(it + q), 0, u);
        o[9] = -log(u[0]);   // exponential variate of the holding time
        o[10] = u[1];
    }
}

__device__ __forceinline__ const double *rng_slot(const double *rng, int it)
{
    return rng + 12 * (it & 7);
}

// Orders the LDS accesses of one wavefront (its lanes exchange data through
// LDS between the steps of the accepted-move update).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Small-grid moves whose switch p at the midpoint is below 2^-52 are dropped
// from the heat bath (T = 0); their weight p / a^2 is below the rounding of
// the large-grid weights of the same electron.
constexpr double kPDrop = 0x1p-52;

// The heat-bath weights of the table with the dropped pairs skipped (large
// systems with more pairs than threads, where most valence electrons have p
// far below 2^-52, so that the kept pairs fit one round): the pairs
// that keep a move are listed in LDS (wavefront ballots, at most two rounds
// of NT pairs) and shared out over the threads, then every thread sums the
// weights of its own contiguous chunk [c0, c1) in move order, so the search
// sees exactly the sums of the full table.  The list lives in the prefix-sum
// scratch, which is written only after the last barrier here.
template <bool CORR, bool YG, bool MX = false>
__device__ __forceinline__ double move_table_compact(const KArgs &A, double *lds, const double *Rm, int c0,
                                                     int c1, int *last)
{
    const Layout &L = A.L;
    const double *pos = lds + L.pos, *Y = y_base<YG>(A, lds), *Jo = lds + L.Jo;
    double *T = lds + L.T;
    int *list = reinterpret_cast<int *>(lds + L.xs);
    int *cnt = reinterpret_cast<int *>(lds + L.red);
    const int tid = threadIdx.x, NT = A.nt, lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
    const int npairs = A.M / 2;
    const unsigned long long below = (1ull << lane) - 1ull;
    int pre[2] = {0, 0};
    bool act[2] = {false, false};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int q = tid + r * NT;
        bool a = false;
        if (q < npairs) {
            const int m = 2 * q, i = m / A.mpe, g = A.mpe == 12 ? (m / 6) & 1 : 1;
            a = true;
            if (g == 0) {
                const int ax = (m % 6) >> 1;
                const double hh = 0.5 * A.a;
                double ma[3], mb[3];
                for (int c = 0; c < 3; ++c) {
                    const double e = Rm[3 * c + ax], x = pos[3 * i + c];
                    ma[c] = x + hh * e;
                    mb[c] = x + (-hh) * e;
                }
                a = !(p_switch(A, ma) < kPDrop) || !(p_switch(A, mb) < kPDrop);
            }
            if (!a) {
                T[m] = 0.0;
                T[m + 1] = 0.0;
            }
        }
        const unsigned long long mask = __ballot(a);
        if (lane == 0) cnt[r * 4 + wv] = __popcll(mask);
        pre[r] = __popcll(mask & below);
        act[r] = a;
    }
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        int off = 0, rt = 0;
        for (int w = 0; w < nw; ++w) {
            const int n = cnt[r * 4 + w];
            if (w < wv) off += n;
            rt += n;
        }
        if (act[r]) list[base + off + pre[r]] = tid + r * NT;
        base += rt;
        total += rt;
    }
    __syncthreads();
    for (int e = tid; e < total; e += NT) {
        const int m = 2 * list[e];
        const int i = m / A.mpe, g = A.mpe == 12 ? (m / 6) & 1 : 0, ax = (m % 6) >> 1;
        const double h = grid_spacing(A, g);
        const double ev[3] = {Rm[ax], Rm[3 + ax], Rm[6 + ax]};
        double ra[3], rb[3], ma[3], mb[3];
        for (int c = 0; c < 3; ++c) {
            const double r = pos[3 * i + c];
            ra[c] = r + h * ev[c];
            rb[c] = r + (-h) * ev[c];
            ma[c] = r + (0.5 * h) * ev[c];
            mb[c] = r + (-0.5 * h) * ev[c];
        }
        double ka = A.inv_a2, kb = A.inv_a2;
        bool da = false, db = false;
        if (A.mpe == 12) {
            const double pa = p_switch(A, ma), pb = p_switch(A, mb);
            ka = g ? (1.0 - pa) * A.inv_ap2 : pa * A.inv_a2;
            kb = g ? (1.0 - pb) * A.inv_ap2 : pb * A.inv_a2;
            da = !g && pa < kPDrop;
            db = !g && pb < kPDrop;
        }
        double rda, rdb, ja, jb;
        basis_dot2<YG, false>(A, ra, rb, Y + i * A.Kp, rda, rdb);
        jastrow_point2<CORR, MX>(A, pos, i, ra, rb, ja, jb);
        const double jo = Jo[i];
        const double rhoa = rda * exp(ja - jo), rhob = rdb * exp(jb - jo);
        T[m] = da ? 0.0 : 0.5 * ka * (rhoa > 0.0 ? rhoa : 0.0);
        T[m + 1] = db ? 0.0 : 0.5 * kb * (rhob > 0.0 ? rhob : 0.0);
    }
    __syncthreads();
    double part = 0.0;
    for (int m = c0; m < c1; ++m) {
        const double t = T[m];
        part += t;
        if (t > 0.0) *last = m;
    }
    return part;
}

// Heat-bath weights with one move per thread (M <= NT, Y in LDS): every
// lane evaluates its own move m = threadIdx.x at one point, then, after a
// barrier, each thread sums the weights of its chunk [c0, c1) as
// move_table does, so the scan and the search see the same sums.  Small
// systems: a wavefront holds all 12N moves, and one point per lane halves
// the table's latency against one +/- pair per lane.
template <bool CORR, bool MX>
__device__ __forceinline__ double move_table_points(const KArgs &A, double *lds, const double *Rm, int c0, int c1,
                                                    int *last, double *rho_g, double *k_g, double acc[3], bool diag)
{
    const Layout &L = A.L;
    const double *pos = lds + L.pos, *Y = lds + L.Y, *Jo = lds + L.Jo;
    double *T = lds + L.T;
    const int m = threadIdx.x;
    if (m < A.M) {
        const int i = m / A.mpe, g = A.mpe == 12 ? (m / 6) & 1 : 0, d = m % 6, ax = d >> 1;
        const double h = grid_spacing(A, g), sh = (d & 1) ? -h : h;
        const double e[3] = {Rm[ax], Rm[3 + ax], Rm[6 + ax]};
        double r[3], mp[3];
        for (int c = 0; c < 3; ++c) {
            const double x = pos[3 * i + c];
            r[c] = x + sh * e[c];
            mp[c] = x + (0.5 * sh) * e[c];
        }
        double k = A.inv_a2;   // single grid: p = 1
        bool dr = false;
        if (A.mpe == 12) {
            const double pm = p_switch(A, mp);
            k = g ? (1.0 - pm) * A.inv_ap2 : pm * A.inv_a2;
            dr = !g && pm < kPDrop;
        }
        double rd, unused, ja, jb;
        basis_dot2<false, true, false>(A, r, r, Y + i * A.Kp, rd, unused);
        jastrow_point2<CORR, MX>(A, pos, i, r, r, ja, jb);
        const double rho = rd * exp(ja - Jo[i]);
        T[m] = dr ? 0.0 : 0.5 * k * (rho > 0.0 ? rho : 0.0);
        if (diag) {
            if (rho_g) rho_g[m] = rho;
            if (k_g) k_g[m] = k;
            acc[0] += k;
            acc[1] += k * (rho - 1.0);
            if (rho < 0.0) acc[2] += -0.5 * k * rho;
        }
    }
    __syncthreads();
    double part = 0.0;
    for (int mm = c0; mm < c1; ++mm) {
        const double t = T[mm];
        part += t;
        if (t > 0.0) *last = mm;
    }
    return part;
}

// Heat-bath weights (Eq. (1) with the switch of Eq. (3)) of the moves m in
// [c0, c1), c0 and c1 even:
// each step evaluates the +/- pair (m, m + 1) along one axis of one grid of
// one electron.  Returns the sum of the weights; with diag, stores rho and k
// and accumulates sum k, L^a and V_sf.
template <bool CORR, bool YG, bool MX = false>
__device__ __forceinline__ double move_table(const KArgs &A, double *lds, const double *Rm, int c0, int c1,
                                             int *last, double *rho_g, double *k_g, double acc[3], bool diag)
{
    if constexpr (YG) {
        // compaction pays when it saves a second round of pairs per thread
        if (!diag && A.M / 2 > A.nt) return move_table_compact<CORR, YG, MX>(A, lds, Rm, c0, c1, last);
    } else {
        if (A.M <= A.nt) return move_table_points<CORR, MX>(A, lds, Rm, c0, c1, last, rho_g, k_g, acc, diag);
    }
    const Layout &L = A.L;
    const double *pos = lds + L.pos, *Y = y_base<YG>(A, lds), *Jo = lds + L.Jo;
    double *T = lds + L.T;
    double part = 0.0;
    for (int m = c0; m < c1; m += 2) {
        const int i = m / A.mpe, g = A.mpe == 12 ? (m / 6) & 1 : 0, ax = (m % 6) >> 1;
        const double h = grid_spacing(A, g);
        const double e[3] = {Rm[ax], Rm[3 + ax], Rm[6 + ax]};
        double ra[3], rb[3], ma[3], mb[3];
        for (int c = 0; c < 3; ++c) {
            const double r = pos[3 * i + c];
            ra[c] = r + h * e[c];
            rb[c] = r + (-h) * e[c];
            ma[c] = r + (0.5 * h) * e[c];
            mb[c] = r + (-0.5 * h) * e[c];
        }
        double ka = A.inv_a2, kb = A.inv_a2;   // single grid: p = 1
        bool da = false, db = false;
        if (A.mpe == 12) {
            const double pa = p_switch(A, ma), pb = p_switch(A, mb);
            ka = g ? (1.0 - pa) * A.inv_ap2 : pa * A.inv_a2;
            kb = g ? (1.0 - pb) * A.inv_ap2 : pb * A.inv_a2;
            da = !g && pa < kPDrop;
            db = !g && pb < kPDrop;
        }
        double rda, rdb, ja, jb;
        basis_dot2<YG>(A, ra, rb, Y + i * A.Kp, rda, rdb);
        jastrow_point2<CORR, MX>(A, pos, i, ra, rb, ja, jb);
        const double jo = Jo[i];
        const double rhoa = rda * exp(ja - jo), rhob = rdb * exp(jb - jo);
        const double ta = da ? 0.0 : 0.5 * ka * (rhoa > 0.0 ? rhoa : 0.0);
        const double tb = db ? 0.0 : 0.5 * kb * (rhob > 0.0 ? rhob : 0.0);
        T[m] = ta;
        T[m + 1] = tb;
        part += ta;
        part += tb;
        if (ta > 0.0) *last = m;
        if (tb > 0.0) *last = m + 1;
        if (diag) {
            if (rho_g) { rho_g[m] = rhoa; rho_g[m + 1] = rhob; }
            if (k_g) { k_g[m] = ka; k_g[m + 1] = kb; }
            acc[0] += ka + kb;
            acc[1] += ka * (rhoa - 1.0) + kb * (rhob - 1.0);
            if (rhoa < 0.0) acc[2] += -0.5 * ka * rhoa;
            if (rhob < 0.0) acc[2] += -0.5 * kb * rhob;
        }
    }
    return part;
}

// Index of item t in a flat range of rows of length len: t / len for
// t < 2^16, len <= 2^12, through one single-precision multiply (the quotient
// is at least 0.5 / len away from an integer, far above the rounding error).
__device__ __forceinline__ int row_of(int t, float inv_len)
{
    return (int)(((float)t + 0.5f) * inv_len);
}

// Sum of x[0 .. len) in index order, loads issued eight at a time.
__device__ __forceinline__ double seq_sum(const double *x, int len)
{
    double s = 0.0;
    for (int p0 = 0; p0 < len; p0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (p0 + u < len) ? x[min(p0 + u, len - 1)] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    return s;
}

// Dot product of x[0 .. len) and y[0], y[ys], ... in index order, loads
// issued eight at a time.
__device__ __forceinline__ double seq_dot(const double *x, const double *y, int len, int ys)
{
    double s = 0.0;
    for (int p0 = 0; p0 < len; p0 += 8) {
        double u0[8], v0[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = min(p0 + u, len - 1);
            u0[u] = (p0 + u < len) ? x[q] : 0.0;
            v0[u] = y[q * ys];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s = fma(u0[u], v0[u], s);
    }
    return s;
}

// Update of the walker state after electron k moved from rold to rnew, in
// three workgroup-wide phases separated by barriers:
//  1. basis block at r_new; copies of row k of Y and column k of Ainv;
//     dq = dphi_i . Ainv[:, k] of the other electrons of k's spin; the pair
//     terms of every other electron i with k (new minus old) into its Jastrow
//     gradient, Laplacian and own sum, and the terms of k with each partner
//     (electrons and nuclei) with the potential change into kp;
//  2. new orbital row with derivatives (vrow) and w_i = g(r_new) . Y_i;
//  3. rank-1 (Sherman-Morrison) updates of Ainv and of the spin's rows of Y,
//     the new derivative row and position of k, grad/lap D/D of the spin's
//     electrons through Ainv' = Ainv - colk (w - e_k)^T / rho, and the sums
//     of kp (Jastrow gradient, Laplacian and own sum of k; the potential
//     change into the block scalars).
// Item ranges of different cost start on wavefront boundaries.
template <bool CORR, bool YG>
__device__ __forceinline__ void accept_move(const KArgs &A, double *lds, double *dphi, int k, const double rold[3],
                            const double rnew[3])
{
    const Layout &L = A.L;
    const int N = A.N, ns = A.ns, K = A.K, Kp = A.Kp, tid = threadIdx.x, NT = A.nt;
    const int s = spin_of(A, k), n = s ? A.n_dn : A.n_up, kl = s ? k - A.n_up : k, i0 = s ? A.n_up : 0;
    const int np = N + A.n_nuc;
    double *pos = lds + L.pos, *bv = lds + L.bv, *vrow = lds + L.vrow, *wrow = lds + L.wrow;
    double *colk = lds + L.colk, *Yk = lds + L.Yk, *Y = y_base<YG>(A, lds);
    double *gD = lds + L.gD, *gJ = lds + L.gJ, *Jo = lds + L.Jo, *dq = lds + L.dq, *kp = lds + L.kp;
    double *inv = lds + L.Ainv + s * ns * ns;
    auto up64 = [](int x) { return (x + 63) & ~63; };

    // phase 1
    {
        const int r0 = up64(np), r1 = r0 + up64(K), r2 = r1 + up64(4 * n), r3 = r2 + K + n;
        for (int t = tid; t < r3; t += NT) {
            if (t < r0) {
                const int p = t;
                if (p >= np) continue;
                double o[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                if (p < N) {
                    if (p != k) {
                        const double c = (spin_of(A, p) == s) ? 0.25 : 0.5;
                        const double xi = pos[3 * p], yi = pos[3 * p + 1], zi = pos[3 * p + 2];
                        const double ax = xi - rnew[0], ay = yi - rnew[1], az = zi - rnew[2];
                        const double bx = xi - rold[0], by = yi - rold[1], bz = zi - rold[2];
                        const PairD pn = pair_d<CORR>(A, c, A.b_ee, ax * ax + ay * ay + az * az, 0, 1.0);
                        const PairD po = pair_d<CORR>(A, c, A.b_ee, bx * bx + by * by + bz * bz, 0, 1.0);
                        gJ[4 * p] += pn.f * ax - po.f * bx;
                        gJ[4 * p + 1] += pn.f * ay - po.f * by;
                        gJ[4 * p + 2] += pn.f * az - po.f * bz;
                        gJ[4 * p + 3] += pn.lap - po.lap;
                        Jo[p] += pn.u - po.u;
                        o[0] = -(pn.f * ax); o[1] = -(pn.f * ay); o[2] = -(pn.f * az);
                        o[3] = pn.lap; o[4] = pn.u; o[5] = pn.y - po.y;
                    }
                } else {
                    const double *R = A.Rnuc + 3 * (p - N);
                    const double c = -A.Znuc[p - N];
                    const double dx = rnew[0] - R[0], dy = rnew[1] - R[1], dz = rnew[2] - R[2];
                    const double ex = rold[0] - R[0], ey = rold[1] - R[1], ez = rold[2] - R[2];
                    const PairD pr = pair_d<CORR>(A, c, A.b_en, dx * dx + dy * dy + dz * dz, 1, -c);
                    o[0] = pr.f * dx; o[1] = pr.f * dy; o[2] = pr.f * dz;
                    o[3] = pr.lap; o[4] = pr.u; o[5] = c * (pr.y - rsqrt_nr(ex * ex + ey * ey + ez * ez));
                }
#pragma unroll
                for (int c = 0; c < 6; ++c) kp[c * np + p] = o[c];
            } else if (t < r1) {
                const int mu = t - r0;
                if (mu < K) basis_fn_full(A, mu, rnew, bv);
            } else if (t < r2) {
                const int u = t - r1;
                if (u >= 4 * n) continue;
                const int c4 = u & 3, il = u >> 2;
                if (il != kl) dq[c4 * ns + il] = seq_dot(dphi + (i0 + il) * L.dld + c4 * ns, inv + kl, n, ns);
            } else {
                const int u = t - r2;
                if (u < K) Yk[u] = Y[k * Kp + u];
                else colk[u - K] = inv[(u - K) * ns + kl];
            }
        }
    }
    __syncthreads();

    // phase 2
    contract<true>(A, bv, 1, n, Y + i0 * Kp, [&](int, int j, const double *v) {
#pragma unroll
        for (int c = 0; c < 5; ++c) vrow[c * ns + j] = v[c];
        wrow[j] = v[5];
    });
    __syncthreads();

    // phase 3
    const double irho = uni(1.0 / wrow[kl]);
    {
        const int r0 = up64(6 + 4 * n);
        const int q0 = r0 + 4 * n, q1 = q0 + 3, q2 = q1 + n * n;
        const float inv_n = 1.0f / (float)n, inv_K = 1.0f / (float)K;
        for (int t = tid; t < q2; t += NT) {
            if (t < r0) {
                if (t < 6) {
                    const double v = seq_sum(kp + t * np, np);
                    if (t < 4) gJ[4 * k + t] = v;
                    else if (t == 4) Jo[k] = v;
                    else lds[L.sc + SC_DV] = v;
                } else if (t < 6 + 4 * n) {
                    const int u = t - 6, c4 = u & 3, il = u >> 2;
                    if (il != kl) {
                        gD[4 * (i0 + il) + c4] -= (wrow[il] * irho) * dq[c4 * ns + il];
                    } else {
                        gD[4 * k + c4] = seq_dot(vrow + (c4 + 1) * ns, colk, n, 1) * irho;
                    }
                }
            } else if (t < q0) {
                const int u = t - r0, c = row_of(u, inv_n), j = u - c * n;
                dphi[k * L.dld + c * ns + j] = vrow[(c + 1) * ns + j];
            } else if (t < q1) {
                pos[3 * k + t - q0] = rnew[t - q0];
            } else {
                const int u = t - q1, j = row_of(u, inv_n), i = u - j * n;
                const double f = (wrow[i] - (i == kl ? 1.0 : 0.0)) * irho;
                inv[j * ns + i] -= colk[j] * f;
            }
        }
        // the spin's rows of Y, eight elements per thread in flight
        const int nY = n * K;
        for (int u0 = tid; u0 < nY; u0 += 8 * NT) {
            double y[8], yk[8], f[8];
            int at[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int u = min(u0 + v * NT, nY - 1), i = row_of(u, inv_K), mu = u - i * K;
                at[v] = (i0 + i) * Kp + mu;
                y[v] = Y[at[v]];
                yk[v] = Yk[mu];
                f[v] = (wrow[i] - (i == kl ? 1.0 : 0.0)) * irho;
            }
#pragma unroll
            for (int v = 0; v < 8; ++v)
                if (u0 + v * NT < nY) Y[at[v]] = y[v] - yk[v] * f[v];
        }
    }
}

// Local energy from the determinant and Jastrow derivatives of every
// electron: E_L = -1/2 sum_i (lap Psi / Psi)_i + V, summed by each wavefront
// (identical in all of them).
__device__ __forceinline__ double local_energy(const KArgs &A, const double *lds, double V)
{
    const int lane = threadIdx.x & 63;
    double t = 0.0;
    for (int i = lane; i < A.N; i += 64) t += psi_lap_term(lds + A.L.gD + 4 * i, lds + A.L.gJ + 4 * i);
    return -0.5 * wave_sum(t) + V;
}

// One workgroup per walker slot: a generation of continuous-time projection,
// or (eval != 0) the move table at frozen positions.
template <bool CORR, bool YG, bool MX = false, bool DL = false>
__device__ __forceinline__ void project_body(const KArgs &A)
{
    extern __shared__ double lds[];
    __shared__ int sflag[8];   // 2-3: pivots of the generation start, 5: stop, 6: bad input, 7: last move
    const Layout &L = A.L;
    const int tid = threadIdx.x, NT = A.nt, slot = blockIdx.x, N = A.N, M = A.M;
    const int lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
    double *pos = lds + L.pos, *T = lds + L.T, *rng = lds + L.rng, *red = lds + L.red, *xs = lds + L.xs;

    const int src = A.idx_in ? A.idx_in[slot] : slot;
    if (tid == 0) {
        sflag[5] = (A.err[0] != 0);
        sflag[6] = 0;
    }
    __syncthreads();
    for (int t = tid; t < 3 * N; t += NT) {
        const double v = A.pos_in[(size_t)src * 3 * N + t];
        pos[t] = v;
        if (!isfinite(v)) sflag[6] = 1;
    }
    refill_rng(A, rng, slot, 0);
    __syncthreads();
    if (sflag[5]) return;
    if (sflag[6]) {
        if (tid == 0) report(A.err, kErrNonFinite, slot);
        return;
    }

    double EL, LAP = 0.0, V;
    const int blob = A.dphi_at - 2;  // Y and the LDS part of the state blob
    // LDS part: [Ainv, Jo + N) at blob offset N Kp (with Y in LDS, Y precedes
    // Ainv and is copied with it)
    const int lds0 = YG ? L.Ainv : L.Y, blob0 = YG ? N * A.Kp : 0;
    // derivative rows: in the state blob, or (DL) in LDS and copied to the
    // blob at the end of the generation
    double *dphi_blob = A.state_out + (size_t)slot * A.state_len + A.dphi_at;
    double *dphi = DL ? lds + L.dph : dphi_blob;
    if (A.state_in && !A.eval) {
        const double *sb = A.state_in + (size_t)src * A.state_len;
        if (YG) {
            double *yo = A.state_out + (size_t)slot * A.state_len;
            for (int t = tid; t < blob0; t += NT) yo[t] = sb[t];
        }
        for (int t = tid; t < blob - blob0; t += NT) lds[lds0 + t] = sb[blob0 + t];
        for (int t = tid; t < N * L.dld; t += NT) dphi[t] = sb[A.dphi_at + t];
        EL = uni(sb[blob]);
        V = uni(sb[blob + 1]);
        __syncthreads();
    } else {
        int rc = walker_setup<CORR, YG>(A, lds, dphi, sflag, EL, LAP, V);
        if (rc) {
            if (tid == 0) report(A.err, rc, slot);
            return;
        }
    }

    // contiguous chunk of +/- move pairs per thread (moves [c0, c1))
    const int chunk = 2 * ((M / 2 + NT - 1) / NT);
    const int c0 = min(M, tid * chunk), c1 = min(M, c0 + chunk);

    if (A.eval) {
        double acc[3] = {0.0, 0.0, 0.0};
        int last = -1;
        const double part = move_table<CORR, YG, MX>(A, lds, rng_slot(rng, 0), c0, c1, &last,
                                       A.rho_out ? A.rho_out + (size_t)slot * M : nullptr,
                                       A.k_out ? A.k_out + (size_t)slot * M : nullptr, acc, true);
        double v[4] = {acc[0], acc[1], acc[2], part};
        block_sum<4>(v, xs);
        if (tid == 0 && A.diag_out) {
            double *d = A.diag_out + (size_t)slot * LRDMC_NDIAG;
            const double Va = V + 0.5 * (v[1] - LAP);
            d[0] = EL;
            d[1] = 0.5 * v[0] + Va + v[2] - v[3];
            d[2] = v[1];
            d[3] = LAP;
            d[4] = Va;
            d[5] = v[2];
            d[6] = v[3];
            d[7] = V;
            d[8] = v[0];
        }
        return;
    }

    double tl = A.tau, lw = 0.0;
    int moves = 0;
    for (int it = 0;; ++it) {
        const double *R = rng_slot(rng, it);
        int last = -1;
        double dummy[3];
        const double part = move_table<CORR, YG, MX>(A, lds, R, c0, c1, &last, nullptr, nullptr, dummy, false);

        // inclusive prefix of the per-thread sums within each wavefront; the
        // wavefront totals go to LDS
        const double x = wave_inclusive_scan(part);
        xs[tid] = x;
        if (lane == 63) red[wv] = x;
        __syncthreads();

        double Delta = 0.0;
        for (int w = 0; w < nw; ++w) Delta += red[w];
        Delta = uni(Delta);
        // every thread takes the same decision
        int action = 0;  // 0 stop, 1 move, 2 error
        double thr = 0.0;
        if (!(Delta > 0.0)) {
            lw -= tl * EL;
        } else if (!isfinite(Delta)) {
            action = 2;
        } else {
            const double td = R[9] / Delta;
            if (td >= tl) {
                lw -= tl * EL;
            } else {
                lw -= td * EL;
                tl -= td;
                action = it + 1 >= A.max_iter ? 3 : 1;
                thr = R[10] * Delta;
            }
        }
        if (action != 1) {
            if (action >= 2) {
                if (tid == 0) report(A.err, action == 2 ? kErrNonFinite : kErrIterCap, slot);
                return;
            }
            break;
        }
        // m* = first m with C_m > thr, found by every wavefront from the LDS
        // prefix sums: the wavefront, then the lane (ballot), then the move
        // inside that lane's chunk; the last move with T > 0 if rounding
        // leaves none.
        int ms = -1;
        {
            double cum = 0.0;
            int ws = -1;
            for (int w = 0; w < nw; ++w) {
                const double r = red[w];
                if (cum + r > thr) { ws = w; break; }
                cum += r;
            }
            if (ws >= 0) {
                const double incl = cum + xs[ws * 64 + lane];
                const unsigned long long hit = __ballot(incl > thr);
                if (hit) {
                    const int ls = __ffsll((long long)hit) - 1;
                    const int ts = ws * 64 + ls;
                    double C = cum + (ls ? xs[ts - 1] : 0.0);
                    const int m0 = min(M, ts * chunk), m1 = min(M, m0 + chunk);
                    for (int m = m0; m < m1; ++m) {
                        C += T[m];
                        if (C > thr) { ms = m; break; }
                    }
                }
            }
        }
        ms = uni(ms);
        if (ms < 0) {
            // rounding left no C_m above the threshold: the last move with T > 0
            if (tid == 0) sflag[7] = -1;
            __syncthreads();
            if (last >= 0) atomicMax(&sflag[7], last);
            __syncthreads();
            ms = uni(sflag[7]);
        }
        if (ms < 0) {
            if (tid == 0) report(A.err, kErrNonFinite, slot);
            return;
        }
        {
            const int k = ms / A.mpe;
            double rnew[3];
            move_position(A, pos, R, ms, rnew);
            for (int c = 0; c < 3; ++c) rnew[c] = uni(rnew[c]);
            const double rold[3] = {uni(pos[3 * k]), uni(pos[3 * k + 1]), uni(pos[3 * k + 2])};
            __syncthreads();   // every wavefront is done with T and xs
            accept_move<CORR, YG>(A, lds, dphi, k, rold, rnew);
            if (((it + 1) & 7) == 0) refill_rng(A, rng, slot, it + 1);
        }
        __syncthreads();
        V = uni(V + lds[L.sc + SC_DV]);
        EL = uni(local_energy(A, lds, V));
        ++moves;
        if (!isfinite(EL)) {
            if (tid == 0) report(A.err, kErrNonFinite, slot);
            return;
        }
    }
    for (int t = tid; t < 3 * N; t += NT) A.pos_out[(size_t)slot * 3 * N + t] = pos[t];
    if (A.save_state) {
        double *sb = A.state_out + (size_t)slot * A.state_len;
        for (int t = tid; t < blob - blob0; t += NT) sb[blob0 + t] = lds[lds0 + t];
        if (DL)
            for (int t = tid; t < N * L.dld; t += NT) dphi_blob[t] = dphi[t];
        if (tid == 0) {
            sb[blob] = EL;
            sb[blob + 1] = V;
        }
    }
    if (tid == 0) {
        A.logw[slot] = lw;
        A.el[slot] = EL;
        A.nmov[slot] = moves;
        if (!isfinite(lw)) report(A.err, kErrNonFinite, slot);
    }
}

// The projection kernel for any system: sizes and LDS offsets come from the
// arguments.
template <bool CORR, bool YG>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(4))) project_kernel(KArgs A)
{
    project_body<CORR, YG>(A);
}

// The same with the move table's Jastrow pair terms in mixed precision.
template <bool CORR, bool YG>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(4))) project_kernel_mx(KArgs A)
{
    project_body<CORR, YG, true>(A);
}

// The same kernel built for one system size: electron counts, basis size and
// nucleus count (hence thread count and every LDS offset) are compile-time
// constants, so loops over electrons and basis functions have fixed trip
// counts and addresses fold into immediates.  The host takes it only when its
// own layout for the context is this one.
template <int NUP, int NDN, int KB, int NNUC>
struct FixedShape {
    static constexpr int N = NUP + NDN, ns = NUP > NDN ? NUP : NDN, M = 12 * N, Kp = KB | 1;
    static constexpr int NT = threads_for(M);
};

template <int NUP, int NDN, int KB, int NNUC, bool CORR>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(4)))
project_kernel_fixed(KArgs A)
{
    using S = FixedShape<NUP, NDN, KB, NNUC>;
    constexpr Layout L = make_layout(S::N, S::ns, KB, S::Kp, S::M, NNUC, S::NT, 0);
    A.N = S::N; A.n_up = NUP; A.n_dn = NDN; A.ns = S::ns; A.K = KB; A.Kp = S::Kp; A.M = S::M;
    A.n_nuc = NNUC; A.nt = S::NT; A.mpe = 12; A.L = L;
    project_body<CORR, false, false, (L.dph >= 0)>(A);
}

template <int NUP, int NDN, int KB, int NNUC, bool CORR>
__global__ void __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(4)))
project_kernel_fixed_mx(KArgs A)
{
    using S = FixedShape<NUP, NDN, KB, NNUC>;
    constexpr Layout L = make_layout(S::N, S::ns, KB, S::Kp, S::M, NNUC, S::NT, 0);
    A.N = S::N; A.n_up = NUP; A.n_dn = NDN; A.ns = S::ns; A.K = KB; A.Kp = S::Kp; A.M = S::M;
    A.n_nuc = NNUC; A.nt = S::NT; A.mpe = 12; A.L = L;
    project_body<CORR, false, true, (L.dph >= 0)>(A);
}

// Derivatives with respect to the Pade parameters theta = (b_ee, b_en) of
// the Jastrow exponent J and of the local energy, for the walkers at pos_in
// (one workgroup per walker; the cusp coefficients c stay fixed).  With
// q = 1 / (1 + b r) a pair term u = c r q has du/db = -c r^2 q^2; its part
// u'(r) d / r of grad_i J changes by -2 c q^3 d and its part u'' + 2 u'/r of
// lap_i J by -6 c q^4.  E_L depends on theta through
// -1/2 sum_i [2 (grad_i D/D + grad_i J) . d grad_i J + d lap_i J].
// out[slot][6] = {E_L, J, dJ/db_ee, dJ/db_en, dE_L/db_ee, dE_L/db_en}.  With
// CORR, J and E_L include the learned correction (which does not depend on
// theta).
template <bool CORR, bool YG>
__global__ void __launch_bounds__(kMaxThreads) jastrow_grad_kernel(KArgs A, double *out)
{
    extern __shared__ double lds[];
    __shared__ int sflag[8];
    const Layout &L = A.L;
    const int tid = threadIdx.x, NT = A.nt, slot = blockIdx.x, N = A.N;
    double *pos = lds + L.pos;
    if (tid == 0) sflag[6] = 0;
    __syncthreads();
    for (int t = tid; t < 3 * N; t += NT) {
        const double v = A.pos_in[(size_t)slot * 3 * N + t];
        pos[t] = v;
        if (!isfinite(v)) sflag[6] = 1;
    }
    __syncthreads();
    if (sflag[6]) {
        if (tid == 0) report(A.err, kErrNonFinite, slot);
        return;
    }
    double EL, LAP = 0.0, V;
    double *dphi = A.state_out + (size_t)slot * A.state_len + A.dphi_at;
    const int rc = walker_setup<CORR, YG>(A, lds, dphi, sflag, EL, LAP, V);
    if (rc) {
        if (tid == 0) report(A.err, rc, slot);
        return;
    }
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // J, dJ/db_ee, dJ/db_en, dE/db_ee, dE/db_en
    for (int i = tid; i < N; i += NT) {
        const double *gD = lds + L.gD + 4 * i, *gJ = lds + L.gJ + 4 * i;
        const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
        const bool up = i < A.n_up;
        for (int t = 0; t < 2; ++t) {
            double dg[3] = {0.0, 0.0, 0.0}, dl = 0.0, dj = 0.0, jv = 0.0;
            const int np = t == 0 ? N : A.n_nuc;
            for (int q = 0; q < np; ++q) {
                double dx, dy, dz, c, b;
                if (t == 0) {
                    if (q == i) continue;
                    dx = xi - pos[3 * q]; dy = yi - pos[3 * q + 1]; dz = zi - pos[3 * q + 2];
                    c = ((q < A.n_up) == up) ? 0.25 : 0.5;
                    b = A.b_ee;
                } else {
                    const auto *R = cst(A.Rnuc) + 3 * q;
                    dx = xi - R[0]; dy = yi - R[1]; dz = zi - R[2];
                    c = -cst(A.Znuc)[q];
                    b = A.b_en;
                }
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                const double qq = 1.0 / (1.0 + b * r), q2 = qq * qq, q3 = q2 * qq;
                dg[0] += -2.0 * c * q3 * dx;
                dg[1] += -2.0 * c * q3 * dy;
                dg[2] += -2.0 * c * q3 * dz;
                dl += -6.0 * c * q2 * q2;
                if (t == 1 || q > i) {
                    dj += -c * r * r * q2;
                    jv += c * r * qq;
                    if constexpr (CORR) {
                        double F[3];
                        corr_eval<0>(A, t, r, F);
                        jv += (t ? -c : 1.0) * F[0];
                    }
                }
            }
            acc[0] += jv;
            acc[1 + t] += dj;
            acc[3 + t] += -0.5 * (2.0 * ((gD[0] + gJ[0]) * dg[0] + (gD[1] + gJ[1]) * dg[1] +
                                         (gD[2] + gJ[2]) * dg[2]) + dl);
        }
    }
    // the table region is free after the walker setup (at least 76 doubles:
    // 16 per summed value)
    double s3[3] = {acc[0], acc[1], acc[2]}, s2[2] = {acc[3], acc[4]};
    block_sum<3>(s3, lds + L.xs);
    block_sum<2>(s2, lds + L.xs);   // its first barrier ends the reads of the first sum
    if (tid == 0) {
        double *o = out + (size_t)slot * 6;
        o[0] = EL;
        o[1] = s3[0];
        o[2] = s3[1];
        o[3] = s3[2];
        o[4] = s2[0];
        o[5] = s2[1];
        if (!isfinite(EL)) report(A.err, kErrNonFinite, slot);
    }
}

// Gradient of sum_w (cJ[w] J_w + cE[w] E_L,w) with respect to the node
// table {F, F', F''} of the learned correction (adjoint of the Hermite data
// to interval-polynomial conversion of corr_coef_kernel), accumulated into
// gtab[2][f_nint + 1][3] with atomic adds.  J is linear in the table: a pair
// of scale s at distance r adds s F(r).  E_L depends on it through
// -1/2 sum_i [2 G_i . d grad_i J + d lap_i J] with G_i = grad_i D/D +
// grad_i J: an electron pair (i, j) along d = (r_i - r_j) / r carries
// -[(G_i - G_j) . d + 2 / r] dF' - dF'', an electron and a nucleus of charge
// Z carry -Z [(G_i . d + 1 / r) dF' + dF'' / 2].
__device__ __forceinline__ void corr_adjoint(const KArgs &A, int type, double r, double wv, double w1, double w2,
                                             double *gtab)
{
    if (!(r < A.f_rcut)) return;
    const double hinv = A.f_hinv, h = 1.0 / hinv;
    const double x = r * hinv;
    const int k = min((int)x, A.f_nint - 1);
    const double t = x - (double)k;
    // dL/dm_p for F = sum_p m_p t^p, F' = hinv sum_p p m_p t^(p-1), F'' = hinv^2 ...
    double tp[6];
    tp[0] = 1.0;
    for (int q = 1; q < 6; ++q) tp[q] = tp[q - 1] * t;
    const double u1 = w1 * hinv, u2 = w2 * hinv * hinv;
    double mb[6];
    mb[0] = wv;
    mb[1] = wv * t + u1;
    for (int q = 2; q < 6; ++q) mb[q] = wv * tp[q] + u1 * q * tp[q - 1] + u2 * q * (q - 1) * tp[q - 2];
    const double e0 = 10.0 * mb[3] - 15.0 * mb[4] + 6.0 * mb[5];
    const double e1 = -4.0 * mb[3] + 7.0 * mb[4] - 3.0 * mb[5];
    const double e2 = 0.5 * mb[3] - mb[4] + 0.5 * mb[5];
    double *g = gtab + 3 * (type * (A.f_nint + 1) + k);
    unsafeAtomicAdd(g + 0, mb[0] - e0);
    unsafeAtomicAdd(g + 1, (mb[1] - e0 - e1) * h);
    unsafeAtomicAdd(g + 2, (0.5 * mb[2] - 0.5 * e0 - e1 - e2) * h * h);
    unsafeAtomicAdd(g + 3, e0);
    unsafeAtomicAdd(g + 4, e1 * h);
    unsafeAtomicAdd(g + 5, e2 * h * h);
}

template <bool YG>
__global__ void __launch_bounds__(kMaxThreads) jastrow_table_grad_kernel(KArgs A, const double *cJ,
                                                                         const double *cE, double *gtab)
{
    extern __shared__ double lds[];
    __shared__ int sflag[8];
    const Layout &L = A.L;
    const int tid = threadIdx.x, NT = A.nt, slot = blockIdx.x, N = A.N;
    double *pos = lds + L.pos;
    if (tid == 0) sflag[6] = 0;
    __syncthreads();
    for (int t = tid; t < 3 * N; t += NT) {
        const double v = A.pos_in[(size_t)slot * 3 * N + t];
        pos[t] = v;
        if (!isfinite(v)) sflag[6] = 1;
    }
    __syncthreads();
    if (sflag[6]) {
        if (tid == 0) report(A.err, kErrNonFinite, slot);
        return;
    }
    double EL, LAP = 0.0, V;
    double *dphi = A.state_out + (size_t)slot * A.state_len + A.dphi_at;
    const int rc = walker_setup<true, YG>(A, lds, dphi, sflag, EL, LAP, V);
    if (rc) {
        if (tid == 0) report(A.err, rc, slot);
        return;
    }
    const double aj = cJ ? cJ[slot] : 0.0, ae = cE ? cE[slot] : 0.0;
    const double *gD = lds + L.gD, *gJ = lds + L.gJ;
    // items: electron pairs i < j (row-major over the strict upper triangle), then (i, I)
    const int n_ee = N * (N - 1) / 2, n_items = n_ee + N * A.n_nuc;
    for (int u = tid; u < n_items; u += NT) {
        int i, j = -1, I = -1;
        if (u < n_ee) {
            i = 0;
            int rem = u;
            while (rem >= N - 1 - i) { rem -= N - 1 - i; ++i; }
            j = i + 1 + rem;
        } else {
            i = (u - n_ee) / A.n_nuc;
            I = (u - n_ee) - i * A.n_nuc;
        }
        const double *pj = j >= 0 ? pos + 3 * j : A.Rnuc + 3 * I;
        const double d0 = pos[3 * i] - pj[0], d1 = pos[3 * i + 1] - pj[1], d2 = pos[3 * i + 2] - pj[2];
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2), ir = 1.0 / r;
        const double Gi0 = gD[4 * i] + gJ[4 * i], Gi1 = gD[4 * i + 1] + gJ[4 * i + 1], Gi2 = gD[4 * i + 2] + gJ[4 * i + 2];
        if (j >= 0) {
            const double G0 = Gi0 - gD[4 * j] - gJ[4 * j], G1 = Gi1 - gD[4 * j + 1] - gJ[4 * j + 1],
                         G2 = Gi2 - gD[4 * j + 2] - gJ[4 * j + 2];
            const double gd = (G0 * d0 + G1 * d1 + G2 * d2) * ir;
            corr_adjoint(A, 0, r, aj, -ae * (gd + 2.0 * ir), -ae, gtab);
        } else {
            const double Z = A.Znuc[I];
            const double gd = (Gi0 * d0 + Gi1 * d1 + Gi2 * d2) * ir;
            corr_adjoint(A, 1, r, aj * Z, -ae * Z * (gd + ir), -0.5 * ae * Z, gtab);
        }
    }
    if (tid == 0 && !isfinite(EL)) report(A.err, kErrNonFinite, slot);
}

// Metropolis sampling of |Psi|^2, one walker per workgroup: vmc_steps
// single-electron moves.  Step t of generation gen of slot s draws
// (u0, u1, u2, u3) from counter (s, gen, t, 2): electron i = floor(u0 N)
// moves by vmc_step * e, e on the unit sphere (cos theta = 2 u1 - 1,
// phi = 2 pi u2); the proposal is symmetric, so accepting with probability
// min(1, rho^2), rho = Psi(x') / Psi(x) (one thread evaluates it from the
// orbital-projected inverse and the Jastrow sums), leaves |Psi|^2
// invariant.  An accepted step updates the state as an accepted projection
// move.  Writes positions, E_L at the end and the accepted count; log w = 0.
template <bool CORR, bool YG>
__global__ void __launch_bounds__(kMaxThreads) vmc_kernel(KArgs A)
{
    extern __shared__ double lds[];
    __shared__ int sflag[8];
    __shared__ double rho_s;
    const Layout &L = A.L;
    const int tid = threadIdx.x, NT = A.nt, slot = blockIdx.x, N = A.N;
    double *pos = lds + L.pos;
    const int src = A.idx_in ? A.idx_in[slot] : slot;
    if (tid == 0) {
        sflag[5] = (A.err[0] != 0);
        sflag[6] = 0;
    }
    __syncthreads();
    for (int t = tid; t < 3 * N; t += NT) {
        const double v = A.pos_in[(size_t)src * 3 * N + t];
        pos[t] = v;
        if (!isfinite(v)) sflag[6] = 1;
    }
    __syncthreads();
    if (sflag[5]) return;
    if (sflag[6]) {
        if (tid == 0) report(A.err, kErrNonFinite, slot);
        return;
    }
    double EL, LAP = 0.0, V;
    double *dphi = A.state_out + (size_t)slot * A.state_len + A.dphi_at;
    const int rc = walker_setup<CORR, YG>(A, lds, dphi, sflag, EL, LAP, V);
    if (rc) {
        if (tid == 0) report(A.err, rc, slot);
        return;
    }
    const double *Jo = lds + L.Jo, *Y = y_base<YG>(A, lds);
    int acc = 0;
    for (int it = 0; it < A.vmc_steps; ++it) {
        double u[4];
        draw4(A.seed, slot, A.gen, (uint64_t)it, 2, u);
        const int i = min((int)(u[0] * N), N - 1);
        const double ct = 2.0 * u[1] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double sn, cs;
        sincos(2.0 * M_PI * u[2], &sn, &cs);
        const double rold[3] = {uni(pos[3 * i]), uni(pos[3 * i + 1]), uni(pos[3 * i + 2])};
        const double h = A.vmc_step;
        const double rnew[3] = {uni(rold[0] + h * (st * cs)), uni(rold[1] + h * (st * sn)), uni(rold[2] + h * ct)};
        if (tid == 0) {
            double rd, rd2, ja, jb;
            basis_dot2(A, rnew, rnew, Y + i * A.Kp, rd, rd2);
            jastrow_point2<CORR>(A, pos, i, rnew, rnew, ja, jb);
            rho_s = rd * exp(ja - Jo[i]);
        }
        __syncthreads();
        const double rho = uni(rho_s);
        if (!isfinite(rho)) {
            if (tid == 0) report(A.err, kErrNonFinite, slot);
            return;
        }
        if (u[3] < rho * rho) {
            accept_move<CORR, YG>(A, lds, dphi, i, rold, rnew);
            __syncthreads();
            V = uni(V + lds[L.sc + SC_DV]);
            ++acc;
        }
        __syncthreads();   // this step's reads of rho_s and pos are done
    }
    EL = uni(local_energy(A, lds, V));
    for (int t = tid; t < 3 * N; t += NT) A.pos_out[(size_t)slot * 3 * N + t] = pos[t];
    if (tid == 0) {
        A.logw[slot] = 0.0;
        A.el[slot] = EL;
        A.nmov[slot] = acc;
        if (!isfinite(EL)) report(A.err, kErrNonFinite, slot);
    }
}

// Interval polynomials of the learned correction from its node table
// tab[2][G][3] = {F, F', F''} at r_k = k h: on [r_k, r_k+1] the quintic in
// t = (r - r_k) / h that matches value, first and second derivative at both
// ends (so F is C^2 across nodes).  With the t-derivatives A1 = h F'_k,
// A2 = h^2 F''_k (B1, B2 at k + 1) the low coefficients are F_k, A1, A2 / 2,
// and the top three solve the end conditions
//   m3 + m4 + m5 = e0,  3 m3 + 4 m4 + 5 m5 = e1,  6 m3 + 12 m4 + 20 m5 = e2
// with e0 = F_k+1 - F_k - A1 - A2 / 2, e1 = B1 - A1 - A2, e2 = B2 - A2.
__global__ void corr_coef_kernel(const double *tab, int G, double h, double *coef, int *bad)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= 2 * (G - 1)) return;
    const int type = u / (G - 1), k = u - type * (G - 1);
    const double *a = tab + 3 * (type * G + k), *b = a + 3;
    const double A1 = h * a[1], A2 = h * h * a[2], B1 = h * b[1], B2 = h * h * b[2];
    const double e0 = b[0] - a[0] - A1 - 0.5 * A2, e1 = B1 - A1 - A2, e2 = B2 - A2;
    double *m = coef + 6 * u;
    m[0] = a[0];
    m[1] = A1;
    m[2] = 0.5 * A2;
    m[3] = 10.0 * e0 - 4.0 * e1 + 0.5 * e2;
    m[4] = -15.0 * e0 + 7.0 * e1 - e2;
    m[5] = 6.0 * e0 - 3.0 * e1 + 0.5 * e2;
    bool ok = true;
    for (int q = 0; q < 6; ++q) ok = ok && isfinite(m[q]);
    if (!ok) atomicExch(bad, 1);
}

__global__ void fill_kernel(double *p, size_t n, double v)
{
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        p[t] = v;
}

// ---------------------------------------------------------------------------
// The network behind the learned correction.  Per pair type a network
// 1 -> H -> H -> 1 with SiLU activations, silu(z) = z / (1 + e^-z), gives
// g(x) = w3 . silu(W2 silu(W1 x + b1) + b2) + b3 at x = r / r_cut, and the
// correction is f(r) = r^2 (1 - r / r_cut)^3 g(r / r_cut): f and f' vanish at
// r = 0 (the Pade cusps stay exact), f, f', f'' at r_cut.  Parameters of one
// network, packed: W1[H], b1[H], W2[H][H] (row = output unit), b2[H], w3[H],
// b3.  The node table {f, f', f''} is built with the r-derivatives carried
// through every layer (first and second order forward mode); its reverse pass
// gives the parameter gradient of a loss on the table.

constexpr int kNetMaxHidden = 256;

__host__ __device__ constexpr int net_param_count(int H) { return H * H + 4 * H + 1; }

// silu and its first three derivatives.
__device__ __forceinline__ void silu_d3(double z, double &a, double &d1, double &d2, double &d3)
{
    const double sg = 1.0 / (1.0 + exp(-z));
    const double p = sg * (1.0 - sg), om = 1.0 - 2.0 * sg;
    a = z * sg;
    d1 = sg + z * p;
    d2 = p * (2.0 + z * om);
    d3 = p * (3.0 * om + z * (1.0 - 6.0 * sg + 6.0 * sg * sg));
}

// w(r) = r^2 (1 - r / rc)^3 and its first two derivatives.
__device__ __forceinline__ void envelope3(double r, double rc, double &w, double &w1, double &w2)
{
    const double q = 1.0 - r / rc, q2 = q * q;
    w = r * r * q2 * q;
    w1 = r * q2 * (2.0 * q - 3.0 * r / rc);
    w2 = q * (2.0 * q2 - 12.0 * r * q / rc + 6.0 * r * r / (rc * rc));
}

struct NetFwd {
    double x;                   // input r / rc
    double s1, s2, s3;          // first to third derivative of silu at this unit's z2
    double z2[3];               // z2 and its first two r-derivatives
    double h2[3];               // h2 and its first two r-derivatives
};

// Forward pass of one node for the unit of this thread (u < H); leaves the
// first-layer streams in hs[3][H] and returns the second-layer quantities.
__device__ __forceinline__ NetFwd net_forward(const double *P, int H, double r, double rc, double *hs)
{
    const int u = threadIdx.x;
    const double *W1 = P, *b1 = P + H, *W2 = P + 2 * H, *b2 = P + 2 * H + H * H;
    NetFwd o{};
    o.x = r / rc;
    if (u < H) {
        double a, d1, d2, d3;
        const double dz = W1[u] / rc;
        silu_d3(fma(W1[u], o.x, b1[u]), a, d1, d2, d3);
        hs[u] = a;
        hs[H + u] = d1 * dz;
        hs[2 * H + u] = d2 * dz * dz;
    }
    __syncthreads();
    if (u < H) {
        double z = b2[u], dz = 0.0, ddz = 0.0;
        const double *row = W2 + (size_t)u * H;
        for (int v = 0; v < H; ++v) {
            const double wv = row[v];
            z = fma(wv, hs[v], z);
            dz = fma(wv, hs[H + v], dz);
            ddz = fma(wv, hs[2 * H + v], ddz);
        }
        double a;
        silu_d3(z, a, o.s1, o.s2, o.s3);
        o.z2[0] = z; o.z2[1] = dz; o.z2[2] = ddz;
        o.h2[0] = a;
        o.h2[1] = o.s1 * dz;
        o.h2[2] = o.s2 * dz * dz + o.s1 * ddz;
    }
    return o;
}

// Node position r_k = k rc / (G - 1), the last node exactly rc.
__device__ __forceinline__ double net_node(int k, int G, double rc)
{
    return (k == G - 1) ? rc : k * (rc / (G - 1));
}

// tab[type][k][3] = {f, f', f''} at the nodes; grid (G, 2).
__global__ void __launch_bounds__(kNetMaxHidden) net_table_kernel(const double *params, int H, int G, double rc,
                                                                  double *tab)
{
    __shared__ double hs[3 * kNetMaxHidden];
    __shared__ double red[3 * 16];
    const int k = blockIdx.x, type = blockIdx.y, u = threadIdx.x;
    const double *P = params + (size_t)type * net_param_count(H);
    const double r = net_node(k, G, rc);
    const NetFwd o = net_forward(P, H, r, rc, hs);
    const double *w3 = P + 3 * H + H * H;
    double v[3] = {0.0, 0.0, 0.0};
    if (u < H)
        for (int c = 0; c < 3; ++c) v[c] = w3[u] * o.h2[c];
    block_sum<3>(v, red);
    if (u == 0) {
        const double g = v[0] + P[4 * H + H * H], dg = v[1], ddg = v[2];
        double w, w1, w2;
        envelope3(r, rc, w, w1, w2);
        double *t = tab + 3 * ((size_t)type * G + k);
        t[0] = w * g;
        t[1] = w1 * g + w * dg;
        t[2] = w2 * g + 2.0 * w1 * dg + w * ddg;
    }
}

// Reverse pass, per node: given the table gradient gtab, the node's share of
// every parameter gradient, in work[type][k][9H + 1]:
//   [0, 3H)   z2 adjoints (value, d/dr, d2/dr2 streams) of each unit
//   [3H, 6H)  the first-layer streams h1, dh1, d2h1
//   [6H, 7H)  W1 share, [7H, 8H) b1 share, [8H, 9H) w3 share, [9H] b3 share
// (W2 = sum over nodes and streams of z2 adjoint times h1 stream, b2 = sum of
// the value-stream z2 adjoints).  Grid (G, 2).
__global__ void __launch_bounds__(kNetMaxHidden) net_table_back_kernel(const double *params, int H, int G, double rc,
                                                                       const double *gtab, double *work)
{
    __shared__ double hs[3 * kNetMaxHidden], zb[3 * kNetMaxHidden];
    const int k = blockIdx.x, type = blockIdx.y, u = threadIdx.x;
    const double *P = params + (size_t)type * net_param_count(H);
    const double *W1 = P, *b1 = P + H, *W2 = P + 2 * H, *w3 = P + 3 * H + H * H;
    const double r = net_node(k, G, rc);
    const NetFwd o = net_forward(P, H, r, rc, hs);
    double w, w1, w2;
    envelope3(r, rc, w, w1, w2);
    const double *gt = gtab + 3 * ((size_t)type * G + k);
    const double gb = w * gt[0] + w1 * gt[1] + w2 * gt[2];   // dL/dg
    const double dgb = w * gt[1] + 2.0 * w1 * gt[2];          // dL/dg'
    const double ddgb = w * gt[2];                            // dL/dg''
    double *out = work + ((size_t)type * G + k) * (9 * H + 1);
    if (u < H) {
        const double hb = gb * w3[u], dhb = dgb * w3[u], ddhb = ddgb * w3[u];
        const double dz = o.z2[1], ddz = o.z2[2];
        const double zb0 = hb * o.s1 + dhb * o.s2 * dz + ddhb * (o.s3 * dz * dz + o.s2 * ddz);
        const double zb1 = dhb * o.s1 + 2.0 * ddhb * o.s2 * dz;
        const double zb2 = ddhb * o.s1;
        zb[u] = zb0; zb[H + u] = zb1; zb[2 * H + u] = zb2;
        out[u] = zb0; out[H + u] = zb1; out[2 * H + u] = zb2;
        out[3 * H + u] = hs[u]; out[4 * H + u] = hs[H + u]; out[5 * H + u] = hs[2 * H + u];
        out[8 * H + u] = gb * o.h2[0] + dgb * o.h2[1] + ddgb * o.h2[2];
    }
    if (u == 0) out[9 * H] = gb;
    __syncthreads();
    if (u < H) {
        // adjoints of the first-layer streams of unit u: W2^T times the z2 adjoints
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int q = 0; q < H; ++q) {
            const double wq = W2[(size_t)q * H + u];
            a0 = fma(wq, zb[q], a0);
            a1 = fma(wq, zb[H + q], a1);
            a2 = fma(wq, zb[2 * H + q], a2);
        }
        double s, t1, t2, t3;
        const double dz1 = W1[u] / rc;
        silu_d3(fma(W1[u], o.x, b1[u]), s, t1, t2, t3);
        const double z1b = a0 * t1 + a1 * t2 * dz1 + a2 * t3 * dz1 * dz1;
        const double dz1b = a1 * t1 + 2.0 * a2 * t2 * dz1;
        out[6 * H + u] = z1b * o.x + dz1b / rc;
        out[7 * H + u] = z1b;
    }
}

// Sum of the per-node shares into gparams[type][P]; grid (ceil(P / 256), 2),
// node order fixed (deterministic).
__global__ void net_table_reduce_kernel(int H, int G, const double *work, double *gparams)
{
    const int PC = net_param_count(H), type = blockIdx.y;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= PC) return;
    const size_t S = 9 * (size_t)H + 1;
    const double *base = work + (size_t)type * G * S;
    double acc = 0.0;
    if (p < H) {                                   // W1
        for (int k = 0; k < G; ++k) acc += base[k * S + 6 * H + p];
    } else if (p < 2 * H) {                        // b1
        for (int k = 0; k < G; ++k) acc += base[k * S + 7 * H + (p - H)];
    } else if (p < 2 * H + H * H) {                // W2[u][v]
        const int u = (p - 2 * H) / H, v = (p - 2 * H) % H;
        for (int k = 0; k < G; ++k) {
            const double *o = base + k * S;
            acc += o[u] * o[3 * H + v] + o[H + u] * o[4 * H + v] + o[2 * H + u] * o[5 * H + v];
        }
    } else if (p < 3 * H + H * H) {                // b2
        const int u = p - 2 * H - H * H;
        for (int k = 0; k < G; ++k) acc += base[k * S + u];
    } else if (p < 4 * H + H * H) {                // w3
        const int u = p - 3 * H - H * H;
        for (int k = 0; k < G; ++k) acc += base[k * S + 8 * H + u];
    } else {                                       // b3
        for (int k = 0; k < G; ++k) acc += base[k * S + 9 * H];
    }
    gparams[(size_t)type * PC + p] = acc;
}

// Fixed-population reconfiguration of W walkers by systematic resampling
// (one workgroup).  cw: W-double scratch for the cumulative weights.
// out_ess (optional): the effective sample size (sum w)^2 / sum w^2.
// min_ess > 0: report a population collapse (generation gen in err[1]) when
// the effective sample size falls below it.
__global__ void __launch_bounds__(1024) reconfigure_kernel(const double *logw, const double *el,
                                                           const int *nmov, int W, double xi_in,
                                                           uint64_t seed, uint64_t gen, double *cw,
                                                           int *idx, double *out_lwb, double *out_eb,
                                                           long long *out_nm, double *out_ess, int *err,
                                                           double min_ess)
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
    double ws = 0.0, ew = 0.0, w2 = 0.0;
    long long nm = 0;
    for (int j = c0; j < c1; ++j) {
        const double w = exp(logw[j] - mx);
        cw[j] = w;
        ws += w;
        ew += w * (el ? el[j] : 0.0);
        w2 += w * w;
        nm += nmov ? nmov[j] : 0;
    }
    double Ws;
    const double pre = block_exclusive_scan(ws, red, &Ws);
    double run = pre;
    for (int j = c0; j < c1; ++j) {
        run += cw[j];
        cw[j] = run;
    }
    double v[2] = {ew, w2};
    block_sum<2>(v, red + 16);
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
        if (out_ess) *out_ess = Ws * Ws / v[1];
        if (!(Ws > 0.0) || !isfinite(Ws) || !isfinite(mx)) report(err, kErrNonFinite, -1);
        else if (min_ess > 0.0 && Ws * Ws < min_ess * v[1]) report(err, kErrCollapse, (int)gen);
    }
}

// Residual of the inverse Slater matrices carried in the walker state: for
// walker slot s (its source src[s] after a reconfiguration), A is recomputed
// from the positions (A[i][j] = phi_j(r_i), phi_j = sum_mu C[mu][j] g_mu)
// and res[s] = max |(A Ainv - I)_ik| over both spins, with Ainv the one the
// Sherman-Morrison updates have carried since the last refresh.  One
// workgroup of 64 threads per slot; LDS: g[K] and phi[N][ns].
__global__ void __launch_bounds__(64) inverse_residual_kernel(const double *pos, const double *state,
                                                              const int *src, int W, int N, int n_up,
                                                              int ns, int K, int state_len, int ainv_at,
                                                              const FnDesc *fns, const double *moT,
                                                              double *res)
{
    extern __shared__ double sm[];
    double *g = sm, *phi = sm + K;
    const int s = blockIdx.x, tid = threadIdx.x;
    if (s >= W) return;
    const int j0 = src ? src[s] : s;
    const double *p = pos + (size_t)j0 * 3 * N;
    for (int i = 0; i < N; ++i) {
        const double r0 = p[3 * i], r1 = p[3 * i + 1], r2 = p[3 * i + 2];
        for (int mu = tid; mu < K; mu += 64) {
            const FnDesc F = fns[mu];
            const double dx = r0 - F.R[0], dy = r1 - F.R[1], dz = r2 - F.R[2];
            double P = 1.0;
            if (F.l == 1) P = F.comp == 0 ? dx : (F.comp == 1 ? dy : dz);
            else if (F.l == 2)
                P = F.comp == 0 ? dx * dy : F.comp == 1 ? dy * dz : F.comp == 2 ? dz * dx
                  : F.comp == 3 ? dx * dx - dy * dy : 2.0 * dz * dz - dx * dx - dy * dy;
            g[mu] = P * exp(-F.alpha * (dx * dx + dy * dy + dz * dz));
        }
        __syncthreads();
        for (int j = tid; j < ns; j += 64) {
            double acc = 0.0;
            for (int mu = 0; mu < K; ++mu) acc += moT[j * K + mu] * g[mu];
            phi[i * ns + j] = acc;
        }
        __syncthreads();
    }
    const double *ainv = state + (size_t)j0 * state_len + ainv_at;
    double worst = 0.0;
    for (int t = tid; t < 2 * ns * ns; t += 64) {
        const int sg = t / (ns * ns), i = (t / ns) % ns, k = t % ns;
        const int n = sg ? N - n_up : n_up;
        if (i >= n || k >= n) continue;
        const double *ai = ainv + sg * ns * ns;
        const int e = (sg ? n_up : 0) + i;
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += phi[e * ns + j] * ai[j * ns + k];
        worst = fmax(worst, fabs(acc - (i == k ? 1.0 : 0.0)));
    }
    for (int off = 32; off > 0; off >>= 1) worst = fmax(worst, __shfl_xor(worst, off, 64));
    if (tid == 0) res[s] = worst;
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

// Projection kernels built for fixed system sizes (n_up, n_dn, basis
// functions, nuclei).  The list can be set at build time through
// LRDMC_FIXED_SHAPES.  By default it holds the Ar-like (18 electrons, 64
// functions) and Be-like (4 electrons, 8 functions) atoms; for the 40-electron
// molecule with 256 functions the fully unrolled kernel spills registers and
// runs slower than the general one, so it is left out.
#define LRDMC_SHAPE(u, d, k, z) \
    {u, d, k, z, {(const void *)project_kernel_fixed<u, d, k, z, false>, (const void *)project_kernel_fixed<u, d, k, z, true>}, \
     {(const void *)project_kernel_fixed_mx<u, d, k, z, false>, (const void *)project_kernel_fixed_mx<u, d, k, z, true>}},
#ifndef LRDMC_FIXED_SHAPES
#define LRDMC_FIXED_SHAPES LRDMC_SHAPE(9, 9, 64, 1) LRDMC_SHAPE(2, 2, 8, 1)
#endif
struct FixedKernel {
    int n_up, n_dn, K, n_nuc;
    const void *fn[2];      // without, with the learned correction
    const void *fn_mx[2];   // the same in mixed precision
};
const FixedKernel kFixedKernels[] = {LRDMC_FIXED_SHAPES};

}  // namespace

struct lrdmc_ctx {
    int W = 0, N = 0, n_up = 0, n_dn = 0, ns = 0, K = 0, Kp = 0, n_nuc = 0, n_heavy = 0, M = 0;
    double b_ee = 0, b_en = 0, v_nn = 0;
    double min_ess_frac = 0.0;    // population-collapse threshold (0: off)
    int max_iter = kMaxIter;      // move cap per walker and generation
    lrdmc_params prm{};
    double *d_Z = nullptr, *d_R = nullptr, *d_mo = nullptr, *d_Rheavy = nullptr;
    FnDesc *d_fn = nullptr;
    ChainDesc *d_chain = nullptr;
    int n_chain = 0;
    double *d_pos[2] = {nullptr, nullptr};
    int cur = 0;
    // walker state blobs (double-buffered, follow d_pos through reconfiguration)
    double *d_state[2] = {nullptr, nullptr};
    int state_len = 0, dphi_at = 0;
    bool state_ok = false;  // d_state[cur] holds the state of d_pos[cur]
    double *d_logw = nullptr, *d_el = nullptr, *d_cw = nullptr;
    int *d_nmov = nullptr, *d_idx = nullptr, *d_err = nullptr;
    bool loaded = false, projected = false, pending = false;
    uint64_t gen = 0;
    int nt = 64;
    size_t lds_bytes = 0;
    Layout L{};
    const void *fixed_fn[2] = {nullptr, nullptr};  // kernels built for this system's sizes, if any
    const void *fixed_fn_mx[2] = {nullptr, nullptr};
    int precision = 0;   // 0 FP64; 1 mixed precision in the move table's Jastrow pair terms
    // LDS layouts with Y in LDS and with Y in the HBM state blob (same blob
    // format); the second is taken automatically when the first would leave
    // fewer than four walkers per CU
    Layout L_lds{}, L_yg{};
    bool yg_auto = false;
    int kmode = 0;   // 0 automatic, 1 general kernel, 2 general kernel with Y in HBM
    // learned Jastrow correction
    bool corr = false;
    int f_G = 0;
    double f_rcut = 0.0;
    double *d_fcoef = nullptr, *d_ftab = nullptr;   // [2][kMaxNodes - 1][6], staging [2][kMaxNodes][3]
    int *d_fbad = nullptr;
    std::string err;
    // event timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_pending;  // (kind 0 project / 1 branch, first event index)
    int ev_used = 0;
    double t_ms[2] = {0.0, 0.0};
    long long t_n[2] = {0, 0};
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

void apply_kernel_mode(lrdmc_ctx *c)
{
    c->L = (c->kmode == 2 || c->yg_auto) ? c->L_yg : c->L_lds;
    c->lds_bytes = sizeof(double) * (size_t)c->L.total;
}

bool use_fixed(const lrdmc_ctx *c) { return c->kmode == 0 && !c->L.yg && c->fixed_fn[c->corr]; }

const void *project_fn(const lrdmc_ctx *c)
{
    if (c->precision == 1) {
        if (use_fixed(c) && c->fixed_fn_mx[c->corr]) return c->fixed_fn_mx[c->corr];
        const void *f[4] = {(const void *)project_kernel_mx<false, false>, (const void *)project_kernel_mx<false, true>,
                            (const void *)project_kernel_mx<true, false>, (const void *)project_kernel_mx<true, true>};
        return f[2 * (int)c->corr + c->L.yg];
    }
    if (use_fixed(c)) return c->fixed_fn[c->corr];
    const void *f[4] = {(const void *)project_kernel<false, false>, (const void *)project_kernel<false, true>,
                        (const void *)project_kernel<true, false>, (const void *)project_kernel<true, true>};
    return f[2 * (int)c->corr + c->L.yg];
}

const void *jastrow_grad_fn(const lrdmc_ctx *c)
{
    const void *f[4] = {(const void *)jastrow_grad_kernel<false, false>, (const void *)jastrow_grad_kernel<false, true>,
                        (const void *)jastrow_grad_kernel<true, false>, (const void *)jastrow_grad_kernel<true, true>};
    return f[2 * (int)c->corr + c->L.yg];
}

const void *vmc_fn(const lrdmc_ctx *c)
{
    const void *f[4] = {(const void *)vmc_kernel<false, false>, (const void *)vmc_kernel<false, true>,
                        (const void *)vmc_kernel<true, false>, (const void *)vmc_kernel<true, true>};
    return f[2 * (int)c->corr + c->L.yg];
}

const void *table_grad_fn(const lrdmc_ctx *c)
{
    return c->L.yg ? (const void *)jastrow_table_grad_kernel<true> : (const void *)jastrow_table_grad_kernel<false>;
}

KArgs base_args(const lrdmc_ctx *c)
{
    KArgs A{};
    A.N = c->N; A.n_up = c->n_up; A.n_dn = c->n_dn; A.ns = c->ns; A.K = c->K; A.Kp = c->Kp;
    A.n_nuc = c->n_nuc; A.n_heavy = c->n_heavy; A.M = c->M; A.nt = c->nt;
    A.Znuc = c->d_Z; A.Rnuc = c->d_R; A.Rheavy = c->d_Rheavy; A.moT = c->d_mo;
    A.n_chain = c->n_chain; A.chains = c->d_chain; A.fns = c->d_fn;
    A.b_ee = c->b_ee; A.b_en = c->b_en; A.v_nn = c->v_nn;
    A.a = c->prm.a; A.ap = c->prm.a_prime;
    A.inv_a2 = 1.0 / (c->prm.a * c->prm.a);
    A.inv_ap2 = 1.0 / (c->prm.a_prime * c->prm.a_prime);
    A.sw_pade = c->prm.switch_form == 1;
    A.sw_c = A.sw_pade ? c->prm.r_c * c->prm.r_c : 1.0 / (2.0 * c->prm.r_c * c->prm.r_c);
    A.mpe = c->M / c->N;
    A.tau = c->prm.tau; A.seed = c->prm.seed; A.rotate = c->prm.rotate;
    A.W = c->W; A.gen = c->gen; A.err = c->d_err; A.L = c->L; A.max_iter = c->max_iter;
    if (c->corr) {
        A.fcoef = c->d_fcoef;
        A.f_nint = c->f_G - 1;
        A.f_hinv = (c->f_G - 1) / c->f_rcut;
        A.f_rcut = c->f_rcut;
    }
    return A;
}

void timing_collect(lrdmc_ctx *c);

int check_kernel_error(lrdmc_ctx *c, hipStream_t st)
{
    HIP_TRY(c, hipStreamSynchronize(st));
    timing_collect(c);
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
        snprintf(buf, sizeof buf, "walker slot %d reached the cap of %d moves in one generation", e[1], c->max_iter);
        return fail(c, LRDMC_EITERCAP, buf);
    case kErrCollapse:
        snprintf(buf, sizeof buf,
                 "population collapse at generation %d: effective sample size (sum w)^2 / sum w^2 below %g of "
                 "the %d walkers", e[1], c->min_ess_frac, c->W);
        return fail(c, LRDMC_ECOLLAPSE, buf);
    default:
        if (e[1] < 0) snprintf(buf, sizeof buf, "non-finite total weight in reconfiguration");
        else snprintf(buf, sizeof buf, "non-finite local energy, weight or rate in walker slot %d", e[1]);
        return fail(c, LRDMC_ENONFINITE, buf);
    }
}

// Record a start event for a kernel of the given kind; returns the index of
// the event pair or -1 when timing is off.
int timing_begin(lrdmc_ctx *c, hipStream_t st, int kind)
{
    if (!c->timing) return -1;
    if (c->ev_used + 2 > (int)c->ev_pool.size()) {
        for (int q = 0; q < 64; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            c->ev_pool.push_back(e);
        }
    }
    const int i = c->ev_used;
    c->ev_used += 2;
    if (hipEventRecord(c->ev_pool[i], st) != hipSuccess) return -1;
    c->ev_pending.push_back({kind, i});
    return i;
}

void timing_end(lrdmc_ctx *c, hipStream_t st, int i)
{
    if (i >= 0) (void)hipEventRecord(c->ev_pool[i + 1], st);
}

// After the stream has been synchronized: fold the recorded pairs into the totals.
void timing_collect(lrdmc_ctx *c)
{
    for (const auto &p : c->ev_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev_pool[p.second], c->ev_pool[p.second + 1]) == hipSuccess) {
            c->t_ms[p.first] += ms;
            c->t_n[p.first] += 1;
        }
    }
    c->ev_pending.clear();
    c->ev_used = 0;
}

int launch_project(lrdmc_ctx *c, hipStream_t st, const double *pos_in, const int *idx_in, double *pos_out,
                   int eval, double *rho, double *k, double *diag)
{
    KArgs A = base_args(c);
    A.pos_in = pos_in;
    A.idx_in = idx_in;
    A.pos_out = pos_out;
    A.state_len = c->state_len;
    A.dphi_at = c->dphi_at;
    // the derivative rows live in the output blobs (also as evaluation scratch)
    A.state_out = c->d_state[c->cur ^ 1];
    if (!eval) {
        // resume from the stored state except on refresh generations
        const int R = std::max(1, (int)c->prm.refresh);
        const bool resume = c->state_ok && R > 1 && (c->gen % (uint64_t)R) != 0;
        A.state_in = resume ? c->d_state[c->cur] : nullptr;
        A.save_state = R > 1;
    }
    A.logw = c->d_logw;
    A.el = c->d_el;
    A.nmov = c->d_nmov;
    A.eval = eval;
    A.rho_out = rho;
    A.k_out = k;
    A.diag_out = diag;
    const int ev = eval ? -1 : timing_begin(c, st, 0);
    const void *fn = project_fn(c);
    void *args[] = {&A};
    HIP_TRY(c, hipLaunchKernel(fn, dim3(c->W), dim3(c->nt), args, c->lds_bytes, st));
    timing_end(c, st, ev);
    return LRDMC_OK;
}

int launch_branch(lrdmc_ctx *c, hipStream_t st, double *lwb, double *eb, int64_t *nm, int *idx_out, double *ess)
{
    const int ev = timing_begin(c, st, 1);
    hipLaunchKernelGGL(reconfigure_kernel, dim3(1), dim3(1024), 0, st, c->d_logw, c->d_el, c->d_nmov, c->W,
                       -1.0, c->prm.seed, c->gen, c->d_cw, c->d_idx, lwb, eb, (long long *)nm, ess, c->d_err,
                       c->min_ess_frac * (double)c->W);
    HIP_TRY(c, hipGetLastError());
    timing_end(c, st, ev);
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

int lrdmc_spacing_pade(double Z, double a, double *r_c, double *a_prime)
{
    if (!(Z > 0.0) || !(a > 0.0) || !r_c || !a_prime)
        return fail(nullptr, LRDMC_EINVAL, "lrdmc_spacing_pade: need Z > 0, a > 0 and output pointers");
    *r_c = 0.5 * Z;
    *a_prime = a * std::sqrt(0.25 * Z * Z + 1.0);
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
        !std::isfinite(prm->a_prime) || !std::isfinite(prm->tau) || prm->refresh < 0 ||
        prm->switch_form < 0 || prm->switch_form > 1 || prm->grids < 0 || prm->grids > 2)
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

    // Group shells that share nucleus and exponent (one s, p and d shell at
    // most): one exponential serves the group.  Groups are sorted by nucleus
    // and exponent and cut into chains whose exponent ratio is one constant
    // beta (step code 1, 2, 3 for beta = 2, 2.5, 3; other groups stand alone),
    // and the basis functions are renumbered group by group (s, p x y z, the
    // five d) so that a chain reads its coefficients in one sweep.
    struct Grp { int nuc; double alpha; int shell[3]; };
    std::vector<Grp> groups;
    std::vector<int> shell_mu(sys->n_shell);   // first function of each shell, input numbering
    {
        int mu = 0;
        for (int q = 0; q < sys->n_shell; ++q) {
            const int l = sys->shell_l[q], I = sys->shell_nuc[q];
            const double al = sys->shell_alpha[q];
            shell_mu[q] = mu;
            mu += 2 * l + 1;
            int gi = -1;
            for (size_t g = 0; g < groups.size(); ++g)
                if (groups[g].nuc == I && groups[g].alpha == al && groups[g].shell[l] < 0) { gi = (int)g; break; }
            if (gi < 0) {
                gi = (int)groups.size();
                groups.push_back({I, al, {-1, -1, -1}});
            }
            groups[gi].shell[l] = q;
        }
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Grp &x, const Grp &y) {
        return x.nuc != y.nuc ? x.nuc < y.nuc : x.alpha < y.alpha;
    });
    std::vector<int> perm(K);            // input function -> renumbered function
    std::vector<FnDesc> fns(K);
    std::vector<int> grp_mu(groups.size());
    {
        int mu = 0;
        for (size_t g = 0; g < groups.size(); ++g) {
            grp_mu[g] = mu;
            for (int l = 0; l < 3; ++l) {
                const int q = groups[g].shell[l];
                if (q < 0) continue;
                for (int cmp = 0; cmp < 2 * l + 1; ++cmp, ++mu) {
                    perm[shell_mu[q] + cmp] = mu;
                    FnDesc &F = fns[mu];
                    F = FnDesc{};
                    F.alpha = groups[g].alpha;
                    for (int x = 0; x < 3; ++x) F.R[x] = sys->R[3 * groups[g].nuc + x];
                    F.l = l;
                    F.comp = cmp;
                }
            }
        }
    }
    std::vector<ChainDesc> chains;
    {
        auto code_of = [](double ratio) {
            const double betas[3] = {2.0, 2.5, 3.0};
            for (int q = 0; q < 3; ++q)
                if (std::fabs(ratio - betas[q]) <= 1e-12 * betas[q]) return q + 1;
            return 0;
        };
        size_t g = 0;
        while (g < groups.size()) {
            size_t e = g + 1;
            int code = 0;
            if (e < groups.size() && groups[e].nuc == groups[g].nuc && groups[g].alpha > 0.0)
                code = code_of(groups[e].alpha / groups[g].alpha);
            if (code)
                while (e < groups.size() && e - g < 21 && groups[e].nuc == groups[g].nuc &&
                       code_of(groups[e].alpha / groups[e - 1].alpha) == code)
                    ++e;
            if (e - g == 1) code = 0;
            ChainDesc D{};
            for (int x = 0; x < 3; ++x) D.R[x] = sys->R[3 * groups[g].nuc + x];
            D.alpha0 = groups[g].alpha;
            for (size_t q = g; q < e; ++q)
                for (int l = 0; l < 3; ++l)
                    if (groups[q].shell[l] >= 0) D.flags |= 1ull << (3 * (q - g) + l);
            D.len = (int)(e - g);
            D.code = code;
            D.mu0 = grp_mu[g];
            auto shells = [&](int q) { return (int)(D.flags >> (3 * q)) & 7; };
            int t = D.len;
            while (t > 0 && shells(t - 1) == 1) --t;
            D.tail0 = D.len - t >= 2 ? t : D.len;
            int a7 = 0;
            while (a7 < D.len && shells(a7) == 7) ++a7;
            int a3 = a7;
            while (a3 < D.len && shells(a3) == 3) ++a3;
            D.n_spd = a7;
            D.n_sp = a3;
            chains.push_back(D);
            g = e;
        }
    }
    std::vector<double> Rheavy;
    for (int I : heavy)
        for (int x = 0; x < 3; ++x) Rheavy.push_back(sys->R[3 * I + x]);

    lrdmc_ctx *c = new (std::nothrow) lrdmc_ctx();
    if (!c) return fail(nullptr, LRDMC_ENOMEM, "lrdmc_create: host allocation");
    c->W = n_walkers; c->N = N; c->n_up = sys->n_up; c->n_dn = sys->n_dn; c->ns = ns; c->K = K;
    c->Kp = K | 1; c->n_nuc = sys->n_nuc;
    c->n_heavy = (int)heavy.size(); c->M = (prm->grids == 1 ? 6 : 12) * N; c->n_chain = (int)chains.size(); c->b_ee = sys->b_ee; c->b_en = sys->b_en; c->prm = *prm;
    double vnn = 0.0;
    for (int I = 0; I < sys->n_nuc; ++I)
        for (int J = I + 1; J < sys->n_nuc; ++J) {
            const double dx = sys->R[3 * I] - sys->R[3 * J], dy = sys->R[3 * I + 1] - sys->R[3 * J + 1],
                         dz = sys->R[3 * I + 2] - sys->R[3 * J + 2];
            vnn += sys->Z[I] * sys->Z[J] / std::sqrt(dx * dx + dy * dy + dz * dz);
        }
    c->v_nn = vnn;
    c->nt = threads_for(c->M);
    const size_t target = prm->refresh > 1 ? 0 : 38 * 1024;
    c->L_lds = make_layout(N, ns, K, c->Kp, c->M, sys->n_nuc, c->nt, target, false);
    c->L_yg = make_layout(N, ns, K, c->Kp, c->M, sys->n_nuc, c->nt, target, true);
    c->yg_auto = sizeof(double) * (size_t)c->L_lds.total > 40 * 1024;
    apply_kernel_mode(c);
    // a kernel built for these sizes serves the context if its layout is this one
    for (const FixedKernel &F : kFixedKernels) {
        if (F.n_up != sys->n_up || F.n_dn != sys->n_dn || F.K != K || F.n_nuc != sys->n_nuc || c->M != 12 * N)
            continue;
        const Layout Lf = make_layout(N, ns, K, c->Kp, c->M, sys->n_nuc, c->nt, 0);
        if (!c->yg_auto && std::memcmp(&Lf, &c->L_lds, sizeof(Layout)) == 0) {
            c->fixed_fn[0] = F.fn[0];
            c->fixed_fn[1] = F.fn[1];
            c->fixed_fn_mx[0] = F.fn_mx[0];
            c->fixed_fn_mx[1] = F.fn_mx[1];
        }
    }
    // state blob: Y [N][Kp], the LDS part [Ainv, Jo + N), E_L, V, derivative rows
    c->dphi_at = N * c->Kp + (c->L_lds.Jo + N - c->L_lds.Ainv) + 2;
    c->state_len = c->dphi_at + N * c->L.dld;

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
    {
        // the LDS limit of every kernel (the current layout is the larger one
        // that can run: the HBM-Y layout is never larger)
        const size_t lim = c->lds_bytes;
        if (lim > 65536) {
            for (const void *fn :
                 {(const void *)project_kernel<false, false>, (const void *)project_kernel<false, true>,
                  (const void *)project_kernel<true, false>, (const void *)project_kernel<true, true>, c->fixed_fn[0],
                  c->fixed_fn[1], (const void *)project_kernel_mx<false, false>, (const void *)project_kernel_mx<false, true>,
                  (const void *)project_kernel_mx<true, false>, (const void *)project_kernel_mx<true, true>,
                  c->fixed_fn_mx[0], c->fixed_fn_mx[1], (const void *)jastrow_grad_kernel<false, false>,
                  (const void *)jastrow_grad_kernel<false, true>, (const void *)jastrow_grad_kernel<true, false>,
                  (const void *)jastrow_grad_kernel<true, true>, (const void *)jastrow_table_grad_kernel<false>,
                  (const void *)jastrow_table_grad_kernel<true>, (const void *)vmc_kernel<false, false>,
                  (const void *)vmc_kernel<false, true>, (const void *)vmc_kernel<true, false>,
                  (const void *)vmc_kernel<true, true>})
                if (fn && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) !=
                              hipSuccess)
                    return cleanup(LRDMC_EDEVICE, "lrdmc_create: cannot raise the LDS limit");
        }
    }

    const size_t W = n_walkers, s3 = 3 * (size_t)N;
    std::vector<double> moT((size_t)ns * K);   // occupied block, orbital-major, renumbered functions
    for (int j = 0; j < ns; ++j)
        for (int mu = 0; mu < K; ++mu) moT[(size_t)j * K + perm[mu]] = sys->mo[(size_t)mu * sys->n_orb + j];
    auto alloc = [&](void **p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; };
    bool ok = alloc((void **)&c->d_Z, sizeof(double) * sys->n_nuc) &&
              alloc((void **)&c->d_R, sizeof(double) * 3 * sys->n_nuc) &&
              alloc((void **)&c->d_mo, sizeof(double) * K * ns) &&
              alloc((void **)&c->d_chain, sizeof(ChainDesc) * chains.size()) &&
              alloc((void **)&c->d_fn, sizeof(FnDesc) * K) &&
              alloc((void **)&c->d_Rheavy, sizeof(double) * Rheavy.size()) &&
              alloc((void **)&c->d_pos[0], sizeof(double) * W * s3) &&
              alloc((void **)&c->d_pos[1], sizeof(double) * W * s3) &&
              alloc((void **)&c->d_state[0], sizeof(double) * W * c->state_len) &&
              alloc((void **)&c->d_state[1], sizeof(double) * W * c->state_len) &&
              alloc((void **)&c->d_logw, sizeof(double) * W) && alloc((void **)&c->d_el, sizeof(double) * W) &&
              alloc((void **)&c->d_cw, sizeof(double) * W) && alloc((void **)&c->d_nmov, sizeof(int) * W) &&
              alloc((void **)&c->d_idx, sizeof(int) * W) && alloc((void **)&c->d_err, sizeof(int) * 2);
    if (!ok) return cleanup(LRDMC_ENOMEM, "lrdmc_create: device allocation failed");
    ok = hipMemcpy(c->d_Z, sys->Z, sizeof(double) * sys->n_nuc, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_R, sys->R, sizeof(double) * 3 * sys->n_nuc, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_mo, moT.data(), sizeof(double) * K * ns, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_chain, chains.data(), sizeof(ChainDesc) * chains.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_fn, fns.data(), sizeof(FnDesc) * K, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->d_Rheavy, Rheavy.data(), sizeof(double) * Rheavy.size(), hipMemcpyHostToDevice) == hipSuccess &&
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
    c->state_ok = false;
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
    c->state_ok = c->prm.refresh > 1;
    c->pending = false;
    c->projected = true;
    return check_kernel_error(c, st);
}

int lrdmc_branch(lrdmc_ctx *c, void *stream, double *log_wbar, double *ebar, int64_t *n_moves, int32_t *idx,
                 double *ess)
{
    if (!c || !c->projected) return fail(c, LRDMC_EINVAL, "lrdmc_branch: no projection to reconfigure");
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_branch(c, st, log_wbar, ebar, n_moves, idx, ess);
    if (rc) return rc;
    c->pending = true;
    c->projected = false;
    c->gen += 1;
    return check_kernel_error(c, st);
}

int lrdmc_run(lrdmc_ctx *c, int32_t n_gen, void *stream, double *log_wbar, double *ebar, int64_t *n_moves,
              int32_t *idx, double *ess)
{
    if (!c || !c->loaded || n_gen < 0) return fail(c, LRDMC_EINVAL, "lrdmc_run: no walkers loaded or n_gen < 0");
    hipStream_t st = (hipStream_t)stream;
    for (int g = 0; g < n_gen; ++g) {
        int rc = launch_project(c, st, c->d_pos[c->cur], c->pending ? c->d_idx : nullptr, c->d_pos[c->cur ^ 1],
                                0, nullptr, nullptr, nullptr);
        if (rc) return rc;
        c->cur ^= 1;
        c->state_ok = c->prm.refresh > 1;
        rc = launch_branch(c, st, log_wbar ? log_wbar + g : nullptr, ebar ? ebar + g : nullptr,
                           n_moves ? n_moves + g : nullptr, idx ? idx + (size_t)g * c->W : nullptr,
                           ess ? ess + g : nullptr);
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

int lrdmc_inverse_residual(lrdmc_ctx *c, double *res, void *stream)
{
    if (!c || !res) return fail(c, LRDMC_EINVAL, "lrdmc_inverse_residual: NULL argument");
    if (!c->loaded || !c->state_ok || c->prm.refresh <= 1)
        return fail(c, LRDMC_EINVAL, "lrdmc_inverse_residual: no stored walker state (needs refresh > 1 and a "
                                     "projection since the walkers were set)");
    hipStream_t st = (hipStream_t)stream;
    const size_t lds = sizeof(double) * ((size_t)c->K + (size_t)c->N * c->ns);
    // Ainv sits after Y in the state blob (the blob format of every layout)
    const int ainv_at = c->N * c->Kp;
    hipLaunchKernelGGL(inverse_residual_kernel, dim3(c->W), dim3(64), lds, st, c->d_pos[c->cur], c->d_state[c->cur],
                       c->pending ? c->d_idx : nullptr, c->W, c->N, c->n_up, c->ns, c->K, c->state_len, ainv_at,
                       c->d_fn, c->d_mo, res);
    HIP_TRY(c, hipGetLastError());
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

int lrdmc_jastrow_grad(lrdmc_ctx *c, const double *pos, double *out, void *stream)
{
    if (!c || !pos || !out) return fail(c, LRDMC_EINVAL, "lrdmc_jastrow_grad: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    KArgs A = base_args(c);
    A.pos_in = pos;
    A.state_len = c->state_len;
    A.dphi_at = c->dphi_at;
    A.state_out = c->d_state[c->cur ^ 1];   // derivative rows as scratch, as in lrdmc_eval_moves
    {
        void *args[] = {&A, &out};
        HIP_TRY(c, hipLaunchKernel(jastrow_grad_fn(c), dim3(c->W), dim3(c->nt), args, c->lds_bytes, st));
    }
    return check_kernel_error(c, st);
}

int lrdmc_set_jastrow_table(lrdmc_ctx *c, const double *tab, int32_t n_nodes, double r_cut, int32_t on_device,
                            void *stream)
{
    if (!c) return fail(nullptr, LRDMC_EINVAL, "lrdmc_set_jastrow_table: NULL context");
    hipStream_t st = (hipStream_t)stream;
    if (!tab || n_nodes == 0) {
        c->corr = false;
        c->state_ok = false;
        return LRDMC_OK;
    }
    if (n_nodes < 2 || n_nodes > LRDMC_MAX_TABLE_NODES || !(r_cut > 0.0) || !std::isfinite(r_cut))
        return fail(c, LRDMC_EINVAL, "lrdmc_set_jastrow_table: need 2 <= n_nodes <= LRDMC_MAX_TABLE_NODES and "
                                     "finite r_cut > 0");
    if (!c->d_fcoef) {
        const size_t nc = 2 * (size_t)(LRDMC_MAX_TABLE_NODES - 1) * 6, nt = 2 * (size_t)LRDMC_MAX_TABLE_NODES * 3;
        HIP_TRY(c, hipMalloc((void **)&c->d_fcoef, sizeof(double) * nc));
        HIP_TRY(c, hipMalloc((void **)&c->d_ftab, sizeof(double) * nt));
        HIP_TRY(c, hipMalloc((void **)&c->d_fbad, sizeof(int)));
    }
    const size_t bytes = sizeof(double) * 2 * (size_t)n_nodes * 3;
    const double *src = tab;
    if (!on_device) {
        HIP_TRY(c, hipMemcpyAsync(c->d_ftab, tab, bytes, hipMemcpyHostToDevice, st));
        src = c->d_ftab;
    }
    HIP_TRY(c, hipMemsetAsync(c->d_fbad, 0, sizeof(int), st));
    const int n_int = 2 * (n_nodes - 1);
    hipLaunchKernelGGL(corr_coef_kernel, dim3((n_int + 255) / 256), dim3(256), 0, st, src, (int)n_nodes,
                       r_cut / (n_nodes - 1), c->d_fcoef, c->d_fbad);
    HIP_TRY(c, hipGetLastError());
    int bad = 0;
    HIP_TRY(c, hipMemcpyAsync(&bad, c->d_fbad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (bad) {
        c->corr = false;
        c->state_ok = false;
        return fail(c, LRDMC_EINVAL, "lrdmc_set_jastrow_table: non-finite table entry (correction removed)");
    }
    c->corr = true;
    c->f_G = n_nodes;
    c->f_rcut = r_cut;
    c->state_ok = false;   // stored Jastrow sums belong to the old trial function
    return LRDMC_OK;
}

int lrdmc_jastrow_table_grad(lrdmc_ctx *c, const double *pos, const double *c_j, const double *c_e, double *gtab,
                             void *stream)
{
    if (!c || !pos || !gtab) return fail(c, LRDMC_EINVAL, "lrdmc_jastrow_table_grad: NULL argument");
    if (!c->corr) return fail(c, LRDMC_EINVAL, "lrdmc_jastrow_table_grad: no correction table is set");
    hipStream_t st = (hipStream_t)stream;
    KArgs A = base_args(c);
    A.pos_in = pos;
    A.state_len = c->state_len;
    A.dphi_at = c->dphi_at;
    A.state_out = c->d_state[c->cur ^ 1];
    const size_t n = 2 * (size_t)c->f_G * 3;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gtab, n, 0.0);
    {
        void *args[] = {&A, &c_j, &c_e, &gtab};
        HIP_TRY(c, hipLaunchKernel(table_grad_fn(c), dim3(c->W), dim3(c->nt), args, c->lds_bytes, st));
    }
    return check_kernel_error(c, st);
}

int lrdmc_set_jastrow(lrdmc_ctx *c, double b_ee, double b_en)
{
    if (!c) return fail(nullptr, LRDMC_EINVAL, "lrdmc_set_jastrow: NULL context");
    if (!(b_ee >= 0.0) || !(b_en >= 0.0) || !std::isfinite(b_ee) || !std::isfinite(b_en))
        return fail(c, LRDMC_EINVAL, "lrdmc_set_jastrow: need finite b_ee >= 0 and b_en >= 0");
    c->b_ee = b_ee;
    c->b_en = b_en;
    c->state_ok = false;   // stored Jastrow sums belong to the old parameters
    return LRDMC_OK;
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
                       0ull, 0ull, cw, idx, stats, stats ? stats + 1 : nullptr, (long long *)nullptr, nullptr, err,
                       0.0);
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

// ---------------------------------------------------------------------------
// Reconfiguration without allocation.  The cumulative weights and the error
// flag live in a fixed device array (one per GPU, held until the process
// ends), so the call allocates nothing.  Calls on one GPU share the array:
// calls that overlap on one GPU (other streams, other host threads) race.

constexpr int kNoAllocMaxWalkers = LRDMC_NOALLOC_MAX_WALKERS;
constexpr int kMaxDevices = 64;
// cumulative weights [kNoAllocMaxWalkers], then the two error ints
static __device__ __align__(256) double scratch[kNoAllocMaxWalkers + 32];

__global__ void clear_flags_kernel(int *flags, int n)
{
    if ((int)threadIdx.x < n) flags[threadIdx.x] = 0;
}

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's scratch array, looked up once per device
// (with the device current); nullptr with the message set on failure.
static double *scratch_address(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            g_error = std::string("lrdmc_reconfigure_noalloc: scratch address: ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

int lrdmc_reconfigure_noalloc(const double *log_w, const double *e_loc, int32_t W, double xi, int32_t *idx,
                              double *stats, void *stream)
{
    if (!log_w || !idx || W < 1 || !(xi > 0.0 && xi < 1.0))
        return fail(nullptr, LRDMC_EINVAL, "lrdmc_reconfigure_noalloc: invalid arguments");
    if (W > kNoAllocMaxWalkers)
        return fail(nullptr, LRDMC_EINVAL, "lrdmc_reconfigure_noalloc: W exceeds LRDMC_NOALLOC_MAX_WALKERS");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, LRDMC_EDEVICE, "lrdmc_reconfigure_noalloc: no current device");
    double *cw = scratch_address(dev);
    if (!cw) return LRDMC_EDEVICE;
    int *err = (int *)(cw + kNoAllocMaxWalkers);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(32), 0, st, err, 2);
    hipLaunchKernelGGL(reconfigure_kernel, dim3(1), dim3(1024), 0, st, log_w, e_loc, (const int *)nullptr, W, xi,
                       0ull, 0ull, cw, idx, stats, stats ? stats + 1 : nullptr, (long long *)nullptr, nullptr, err,
                       0.0);
    hipError_t le = hipGetLastError();
    int e[2] = {0, 0};
    hipError_t ce = hipMemcpyAsync(e, err, sizeof(e), hipMemcpyDeviceToHost, st);
    hipError_t se = hipStreamSynchronize(st);
    if (le != hipSuccess || ce != hipSuccess || se != hipSuccess)
        return fail(nullptr, LRDMC_EDEVICE, std::string("lrdmc_reconfigure_noalloc: ") +
                                                hipGetErrorString(le != hipSuccess ? le : ce != hipSuccess ? ce : se));
    if (e[0]) return fail(nullptr, LRDMC_ENONFINITE, "lrdmc_reconfigure_noalloc: non-finite weights");
    return LRDMC_OK;
}

int32_t lrdmc_net_param_count(int32_t hidden)
{
    return (hidden >= 1 && hidden <= kNetMaxHidden) ? net_param_count(hidden) : 0;
}

int64_t lrdmc_net_workspace_size(int32_t hidden, int32_t n_nodes)
{
    if (hidden < 1 || hidden > kNetMaxHidden || n_nodes < 2 || n_nodes > LRDMC_MAX_TABLE_NODES) return 0;
    return 2 * (int64_t)n_nodes * (9 * (int64_t)hidden + 1);
}

static int net_check(int32_t hidden, int32_t n_nodes, double r_cut, const char *who)
{
    if (hidden < 1 || hidden > kNetMaxHidden || n_nodes < 2 || n_nodes > LRDMC_MAX_TABLE_NODES || !(r_cut > 0.0) ||
        !std::isfinite(r_cut))
        return fail(nullptr, LRDMC_EINVAL, std::string(who) + ": need 1 <= hidden <= 256, 2 <= n_nodes <= "
                                                              "LRDMC_MAX_TABLE_NODES and finite r_cut > 0");
    return LRDMC_OK;
}

int lrdmc_net_tabulate(const double *params, int32_t hidden, int32_t n_nodes, double r_cut, double *tab, void *stream)
{
    if (!params || !tab) return fail(nullptr, LRDMC_EINVAL, "lrdmc_net_tabulate: NULL argument");
    if (int rc = net_check(hidden, n_nodes, r_cut, "lrdmc_net_tabulate")) return rc;
    const int nt = ((hidden + 63) / 64) * 64;
    hipLaunchKernelGGL(net_table_kernel, dim3(n_nodes, 2), dim3(nt), 0, (hipStream_t)stream, params, (int)hidden,
                       (int)n_nodes, r_cut, tab);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(nullptr, LRDMC_EDEVICE, std::string("lrdmc_net_tabulate: ") + hipGetErrorString(e));
    return LRDMC_OK;
}

int lrdmc_net_tabulate_backward(const double *params, int32_t hidden, int32_t n_nodes, double r_cut,
                                const double *gtab, double *gparams, double *work, void *stream)
{
    if (!params || !gtab || !gparams || !work)
        return fail(nullptr, LRDMC_EINVAL, "lrdmc_net_tabulate_backward: NULL argument");
    if (int rc = net_check(hidden, n_nodes, r_cut, "lrdmc_net_tabulate_backward")) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int nt = ((hidden + 63) / 64) * 64, PC = net_param_count(hidden);
    hipLaunchKernelGGL(net_table_back_kernel, dim3(n_nodes, 2), dim3(nt), 0, st, params, (int)hidden, (int)n_nodes,
                       r_cut, gtab, work);
    hipLaunchKernelGGL(net_table_reduce_kernel, dim3((PC + 255) / 256, 2), dim3(256), 0, st, (int)hidden,
                       (int)n_nodes, (const double *)work, gparams);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(nullptr, LRDMC_EDEVICE, std::string("lrdmc_net_tabulate_backward: ") + hipGetErrorString(e));
    return LRDMC_OK;
}

int lrdmc_vmc(lrdmc_ctx *c, int32_t n_steps, double step, void *stream)
{
    if (!c || !c->loaded) return fail(c, LRDMC_EINVAL, "lrdmc_vmc: no walkers loaded");
    if (n_steps < 0 || !(step > 0.0) || !std::isfinite(step))
        return fail(c, LRDMC_EINVAL, "lrdmc_vmc: need n_steps >= 0 and finite step > 0");
    hipStream_t st = (hipStream_t)stream;
    KArgs A = base_args(c);
    A.pos_in = c->d_pos[c->cur];
    A.idx_in = c->pending ? c->d_idx : nullptr;
    A.pos_out = c->d_pos[c->cur ^ 1];
    A.state_out = c->d_state[c->cur ^ 1];
    A.state_len = c->state_len;
    A.dphi_at = c->dphi_at;
    A.logw = c->d_logw;
    A.el = c->d_el;
    A.nmov = c->d_nmov;
    A.vmc_steps = n_steps;
    A.vmc_step = step;
    {
        void *args[] = {&A};
        HIP_TRY(c, hipLaunchKernel(vmc_fn(c), dim3(c->W), dim3(c->nt), args, c->lds_bytes, st));
    }
    c->cur ^= 1;
    c->pending = false;
    c->projected = false;
    c->state_ok = false;
    c->gen += 1;
    return check_kernel_error(c, st);
}

int lrdmc_use_generic(lrdmc_ctx *c, int32_t enable)
{
    if (!c) return fail(nullptr, LRDMC_EINVAL, "lrdmc_use_generic: NULL context");
    if (enable < 0 || enable > 2) return fail(c, LRDMC_EINVAL, "lrdmc_use_generic: mode must be 0, 1 or 2");
    c->kmode = enable;
    apply_kernel_mode(c);   // the state blob format is the same for every mode
    return LRDMC_OK;
}

int lrdmc_set_precision(lrdmc_ctx *c, int32_t mode)
{
    if (!c) return fail(nullptr, LRDMC_EINVAL, "lrdmc_set_precision: NULL context");
    if (mode < 0 || mode > 1) return fail(c, LRDMC_EINVAL, "lrdmc_set_precision: mode must be 0 or 1");
    c->precision = mode;
    return LRDMC_OK;
}

int lrdmc_set_collapse_threshold(lrdmc_ctx *c, double min_fraction)
{
    if (!c) return fail(nullptr, LRDMC_EINVAL, "lrdmc_set_collapse_threshold: NULL context");
    if (!(min_fraction >= 0.0 && min_fraction <= 1.0))
        return fail(c, LRDMC_EINVAL, "lrdmc_set_collapse_threshold: need 0 <= min_fraction <= 1");
    c->min_ess_frac = min_fraction;
    return LRDMC_OK;
}

int lrdmc_set_move_cap(lrdmc_ctx *c, int32_t max_moves)
{
    if (!c) return fail(nullptr, LRDMC_EINVAL, "lrdmc_set_move_cap: NULL context");
    if (max_moves < 1 || max_moves > kMaxIter)
        return fail(c, LRDMC_EINVAL, "lrdmc_set_move_cap: need 1 <= max_moves <= 2^22");
    c->max_iter = max_moves;
    return LRDMC_OK;
}

int32_t lrdmc_is_specialized(const lrdmc_ctx *c)
{
    return (c && use_fixed(c)) ? 1 : 0;
}

int lrdmc_set_timing(lrdmc_ctx *c, int32_t enable)
{
    if (!c) return fail(nullptr, LRDMC_EINVAL, "lrdmc_set_timing: NULL context");
    c->timing = enable != 0;
    c->t_ms[0] = c->t_ms[1] = 0.0;
    c->t_n[0] = c->t_n[1] = 0;
    c->ev_pending.clear();
    c->ev_used = 0;
    return LRDMC_OK;
}

int lrdmc_timing(const lrdmc_ctx *c, double *out)
{
    if (!c || !out) return fail(nullptr, LRDMC_EINVAL, "lrdmc_timing: NULL argument");
    out[0] = c->t_ms[0];
    out[1] = (double)c->t_n[0];
    out[2] = c->t_ms[1];
    out[3] = (double)c->t_n[1];
    return LRDMC_OK;
}

uint64_t lrdmc_generation(const lrdmc_ctx *c) { return c ? c->gen : 0; }

const char *lrdmc_last_error(const lrdmc_ctx *c) { return c ? c->err.c_str() : g_error.c_str(); }

void lrdmc_destroy(lrdmc_ctx *c)
{
    if (!c) return;
    void *ptrs[] = {c->d_Z,      c->d_R,        c->d_mo,       c->d_chain,    c->d_fn,   c->d_Rheavy, c->d_pos[0], c->d_state[0], c->d_state[1],
                    c->d_pos[1], c->d_logw, c->d_el, c->d_cw,     c->d_nmov, c->d_idx,  c->d_err,
                    c->d_fcoef, c->d_ftab, c->d_fbad};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
