// Measurement prototype: the determinant ratios of the move table computed
// two ways, to decide whether the orbital contraction belongs on the matrix
// cores of gfx950.
//
// For every walker and every lattice move m of the table (electron i, grid,
// axis, sign; fixed axes) the determinant ratio of the moved spin is
//   rho_D(m) = sum_j phi_j(r'_m) Ainv[j][i] = sum_mu g_mu(r'_m) Y[i][mu],
//   phi_j = sum_mu g_mu C[mu][j],  Y[i][mu] = sum_j C[mu][j] Ainv[j][i]
// (the matrix determinant lemma for a replaced row).
//
// variant 0 (FP64 Y-dot, the formulation of the projection kernels): each
//   move point's basis values are dotted in FP64 with the electron's row of
//   Y (walker state in device memory).
// variant 1 (BF16x3 on MFMA): the basis values of 16 points x 32 functions
//   are split into two BF16 terms (hi = truncated x, lo = truncated x - hi),
//   multiplied with the two-term split of C (shared by every walker) on
//   v_mfma_f32_16x16x32_bf16 as hi.hi + hi.lo + lo.hi with FP32
//   accumulation, giving Phi' = B' C for 32 orbital columns; rho_D is then
//   the FP64 dot of each row of Phi' with the column of the inverse Slater
//   matrix of the moved electron.
//
// Both variants evaluate the basis functions with the same code (one exp
// per function, no exponent chains), so that the difference of their times
// is the difference of the two contractions.  One workgroup of four waves
// per walker; each wave takes blocks of 16 move points; lane l evaluates
// the functions 8 (l / 16) .. 8 (l / 16) + 7 of every 32-function chunk at
// point l % 16 of the block (the A-operand layout of the 16x16x32 MFMA).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct ProbeFn {            // one basis function
    double R[3];
    double alpha;
    int l, comp, pad0, pad1;
};

struct ProbeArgs {
    int W, N, n_up, K, Kpad;          // Kpad: K rounded up to 32
    double a, ap;                     // grid spacings
    const double *pos;                // [W][N][3]
    const ProbeFn *fns;               // [K]
    const double *Y;                  // [W][N][Kpad]        (variant 0)
    const uint4 *Cb;                  // [Kpad/32][2 tiles][2 hi/lo][64 lanes] x 8 bf16 (variant 1)
    const double *Ainv;               // [W][2][32][32] Ainv[s][j][c], zero padded (variant 1)
    double *rho;                      // [W][12 N]
};

__device__ __forceinline__ double basis_value(const ProbeFn &F, const double r[3])
{
    const double dx = r[0] - F.R[0], dy = r[1] - F.R[1], dz = r[2] - F.R[2];
    const double e = exp(-F.alpha * (dx * dx + dy * dy + dz * dz));
    double P = 1.0;
    if (F.l == 1) {
        P = F.comp == 0 ? dx : (F.comp == 1 ? dy : dz);
    } else if (F.l == 2) {
        switch (F.comp) {
        case 0: P = dx * dy; break;
        case 1: P = dy * dz; break;
        case 2: P = dz * dx; break;
        case 3: P = dx * dx - dy * dy; break;
        default: P = 2.0 * dz * dz - dx * dx - dy * dy; break;
        }
    }
    return P * e;
}

// Displaced point of move m (m = 12 i + 6 g + d; fixed axes).
__device__ __forceinline__ void move_point(const ProbeArgs &A, const double *pw, int m, double r[3])
{
    const int i = m / 12, g = (m / 6) & 1, d = m % 6, ax = d >> 1;
    const double h = (g ? A.ap : A.a) * ((d & 1) ? -1.0 : 1.0);
    r[0] = pw[3 * i];
    r[1] = pw[3 * i + 1];
    r[2] = pw[3 * i + 2];
    r[ax] += h;
}

// Upper 16 bits of two floats packed into one word (two BF16 by truncation).
__device__ __forceinline__ unsigned pack_hi16(float x0, float x1)
{
    return __builtin_amdgcn_perm(__float_as_uint(x1), __float_as_uint(x0), 0x07060302u);
}

template <int VARIANT>
__global__ void __launch_bounds__(256) probe_kernel(ProbeArgs A)
{
    const int w = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int M = 12 * A.N, n_blk = (M + 15) / 16;
    const int row = lane & 15, q = lane >> 4;
    const double *pw = A.pos + (size_t)w * A.N * 3;
    const int n_kc = A.Kpad / 32;
    for (int blk = wave; blk < n_blk; blk += 4) {
        const int m = blk * 16 + row;
        const bool live = m < M;
        const int mm = live ? m : M - 1;
        const int i = mm / 12;
        double r[3];
        move_point(A, pw, mm, r);
        if (VARIANT == 0) {
            const double *y = A.Y + ((size_t)w * A.N + i) * A.Kpad;
            double part[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int kc = 0; kc < n_kc; ++kc) {
                const int k0 = kc * 32 + 8 * q;
                double yv[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) yv[j] = y[k0 + j];      // Y is zero padded to Kpad
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = k0 + j;
                    if (k < A.K) part[j] += basis_value(A.fns[k], r) * yv[j];
                }
            }
            double acc = ((part[0] + part[1]) + (part[2] + part[3])) + ((part[4] + part[5]) + (part[6] + part[7]));
            acc += __shfl_xor(acc, 16, 64);
            acc += __shfl_xor(acc, 32, 64);
            if (live && q == 0) A.rho[(size_t)w * M + m] = acc;
        } else {
            f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
            for (int kc = 0; kc < n_kc; ++kc) {
                const int k0 = kc * 32 + 8 * q;
                float x[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = k0 + j;
                    x[j] = k < A.K ? (float)basis_value(A.fns[k], r) : 0.0f;
                }
                unsigned hi[4], lo[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float h0 = __uint_as_float(__float_as_uint(x[2 * j]) & 0xffff0000u);
                    const float h1 = __uint_as_float(__float_as_uint(x[2 * j + 1]) & 0xffff0000u);
                    hi[j] = pack_hi16(h0, h1);
                    lo[j] = pack_hi16(x[2 * j] - h0, x[2 * j + 1] - h1);
                }
                bf16x8 ah, al;
                __builtin_memcpy(&ah, hi, 16);
                __builtin_memcpy(&al, lo, 16);
                const uint4 *cb = A.Cb + (size_t)kc * 4 * 64 + lane;
                bf16x8 b0h, b0l, b1h, b1l;
                const uint4 v0 = cb[0], v1 = cb[64], v2 = cb[128], v3 = cb[192];
                __builtin_memcpy(&b0h, &v0, 16);
                __builtin_memcpy(&b0l, &v1, 16);
                __builtin_memcpy(&b1h, &v2, 16);
                __builtin_memcpy(&b1l, &v3, 16);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b0h, acc0, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b0l, acc0, 0, 0, 0);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b0h, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b1h, acc1, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b1l, acc1, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b1h, acc1, 0, 0, 0);
            }
            // lane holds Phi'[4 q + rr][row + 16 t]; contract with the inverse
            // column of each row's moved electron in FP64
            const double *ai = A.Ainv + (size_t)w * 2 * 32 * 32;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int mr = blk * 16 + 4 * q + rr;
                const int mc = mr < M ? mr : M - 1;
                const int ie = mc / 12, s = ie < A.n_up ? 0 : 1, col = ie - (s ? A.n_up : 0);
                const double *as = ai + (size_t)s * 32 * 32;
                double p = (double)acc0[rr] * as[row * 32 + col] + (double)acc1[rr] * as[(row + 16) * 32 + col];
                p += __shfl_xor(p, 1, 64);
                p += __shfl_xor(p, 2, 64);
                p += __shfl_xor(p, 4, 64);
                p += __shfl_xor(p, 8, 64);
                if (row == 0 && mr < M) A.rho[(size_t)w * M + mr] = p;
            }
        }
    }
}

}  // namespace

extern "C" {

// Determinant ratios of the fixed-axis move table of W walkers, by variant
// 0 (FP64 Y-dot) or 1 (BF16x3 MFMA contraction with C, then FP64 with the
// inverse).  Device pointers; layouts as in ProbeArgs.  Returns 0, or -1 for
// bad sizes (N > 64, K > 512, n_sigma > 32), -5 for a launch error.
int mfma_probe_ratios(int variant, int W, int N, int n_up, int K, double a, double ap, const double *pos,
                      const void *fns, const double *Y, const void *Cb, const double *Ainv, double *rho,
                      void *stream)
{
    if (W < 1 || N < 1 || N > 64 || K < 1 || K > 512 || n_up > 32 || N - n_up > 32 || n_up < 0 ||
        (variant != 0 && variant != 1))
        return -1;
    ProbeArgs A{};
    A.W = W;
    A.N = N;
    A.n_up = n_up;
    A.K = K;
    A.Kpad = (K + 31) / 32 * 32;
    A.a = a;
    A.ap = ap;
    A.pos = pos;
    A.fns = (const ProbeFn *)fns;
    A.Y = Y;
    A.Cb = (const uint4 *)Cb;
    A.Ainv = Ainv;
    A.rho = rho;
    hipStream_t st = (hipStream_t)stream;
    if (variant == 0)
        hipLaunchKernelGGL(probe_kernel<0>, dim3(W), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL(probe_kernel<1>, dim3(W), dim3(256), 0, st, A);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int mfma_probe_fn_bytes(void) { return (int)sizeof(ProbeFn); }

}  // extern "C"
