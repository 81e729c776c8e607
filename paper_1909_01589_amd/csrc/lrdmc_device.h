// Device-side building blocks of the double-grid LRDMC projection for gfx950:
// counter-based random numbers, lattice rotations, wavefront and workgroup
// reductions.  Included by lrdmc.hip only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lrdmc {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with the published multipliers and Weyl key bumps.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        uint64_t n0 = hi1 ^ c[1] ^ k0;
        uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// Top 53 bits, centred: a double in the open interval (0, 1).
__device__ __forceinline__ double u01(uint64_t x)
{
    return ((double)(x >> 11) + 0.5) * 0x1.0p-53;
}

// Four uniforms for counter (slot, generation, iteration, purpose), key (seed, 0).
__device__ __forceinline__ void draw4(uint64_t seed, uint64_t slot, uint64_t gen,
                                      uint64_t it, uint64_t purpose, double u[4])
{
    uint64_t c[4] = {slot, gen, it, purpose};
    philox4x64_10(c, seed, 0ull);
    u[0] = u01(c[0]); u[1] = u01(c[1]); u[2] = u01(c[2]); u[3] = u01(c[3]);
}

// Uniform random rotation from three uniforms (Shoemake's quaternion method);
// Rm is row-major and its columns are the lattice axes.
__device__ __forceinline__ void rotation(const double u[3], double Rm[9])
{
    const double two_pi = 6.283185307179586476925286766559;
    double r1 = sqrt(1.0 - u[0]), r2 = sqrt(u[0]);
    double s1, c1, s2, c2;
    sincos(two_pi * u[1], &s1, &c1);
    sincos(two_pi * u[2], &s2, &c2);
    double x = s1 * r1, y = c1 * r1, z = s2 * r2, w = c2 * r2;
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

// ---------------------------------------------------------------------------
// Cross-lane moves that stay in the VALU: DPP row operations and the gfx950
// permlane swaps.  They read every lane of the wavefront, so callers keep the
// whole wavefront active.

// Value of the lane selected by the DPP control; 0 where there is none (row
// shifts at the row edge) and in rows left out by row_mask.
template <int ctrl, int row_mask = 0xf>
__device__ __forceinline__ double dpp(double v)
{
    return __builtin_amdgcn_update_dpp(0.0, v, ctrl, row_mask, 0xf, false);
}

constexpr int kDppQuad1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppQuad2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane 7 - i within 8
constexpr int kDppMirror = 0x140;      // lane 15 - i within 16
constexpr int kDppShr = 0x110;         // + n: row_shr:n
constexpr int kDppBcast15 = 0x142;     // lane 15 of the previous row
constexpr int kDppBcast31 = 0x143;     // lane 31

// v plus the value of the same lane in the neighbouring group of 16 (rows
// 0 <-> 1, 2 <-> 3) or 32 (halves); both lanes of a pair get the same sum.
__device__ __forceinline__ double add_swap16(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)b, hi = (unsigned)((unsigned long long)b >> 32);
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double a = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
    const double c = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
    return a + c;
}

__device__ __forceinline__ double add_swap32(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)b, hi = (unsigned)((unsigned long long)b >> 32);
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const double a = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
    const double c = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
    return a + c;
}

// Sum over aligned groups of P lanes (P a power of two, at most 64, uniform).
// A butterfly: every lane of a group ends with the same bits.
__device__ __forceinline__ double group_sum(double v, int P)
{
    if (P >= 2) v += dpp<kDppQuad1>(v);
    if (P >= 4) v += dpp<kDppQuad2>(v);
    if (P >= 8) v += dpp<kDppHalfMirror>(v);
    if (P >= 16) v += dpp<kDppMirror>(v);
    if (P >= 32) v = add_swap16(v);
    if (P >= 64) v = add_swap32(v);
    return v;
}

// Inclusive prefix sum over the 64 lanes (Hillis-Steele inside rows of 16,
// then the row totals by broadcast).
__device__ __forceinline__ double wave_inclusive_scan(double x)
{
    x += dpp<kDppShr + 1>(x);
    x += dpp<kDppShr + 2>(x);
    x += dpp<kDppShr + 4>(x);
    x += dpp<kDppShr + 8>(x);
    x += dpp<kDppBcast15, 0xa>(x);
    x += dpp<kDppBcast31, 0xc>(x);
    return x;
}

// ---------------------------------------------------------------------------
// Reductions over 64-lane wavefronts and over the workgroup.

__device__ __forceinline__ double wave_sum(double v)
{
    return group_sum(v, 64);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum of `n` values per thread over the workgroup; every thread receives the
// totals (summed in the same order, hence identical).  red needs 16*n doubles
// (up to 16 wavefronts).
template <int n>
__device__ __forceinline__ void block_sum(double (&v)[n], double *red)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < n; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if (lane == 0)
        for (int q = 0; q < n; ++q) red[q * 16 + wv] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < n; ++q) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += red[q * 16 + w];
        v[q] = t;
    }
}

// Exclusive prefix sum of one value per thread in thread order; *total gets
// the workgroup sum.  red needs 16 doubles (up to 16 wavefronts).
__device__ __forceinline__ double block_exclusive_scan(double v, double *red, double *total)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        double y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    double excl = __shfl_up(x, 1, 64);
    if (lane == 0) excl = 0.0;
    __syncthreads();
    if (lane == 63) red[wv] = x;
    __syncthreads();
    double pre = 0.0, tot = 0.0;
    for (int w = 0; w < nw; ++w) {
        if (w < wv) pre += red[w];
        tot += red[w];
    }
    *total = tot;
    return pre + excl;
}

}  // namespace lrdmc
