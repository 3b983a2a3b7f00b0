// Device arithmetic of the MPCD+MD path for gfx950.  Every formula here is
// evaluated with contraction off (the library is built with
// -ffp-contract=off); fused multiply-adds are written as fma() where the
// method uses them, so each result is a defined sequence of IEEE operations.
#pragma once
#include "rmp_internal.h"

namespace rmp {

// A pointer typed as pointing into global memory.  Pointers read from a
// descriptor are generic, and a generic access compiles to a flat
// instruction, which also counts against the LDS counter: every later LDS
// wait, and every workgroup barrier, would then wait for the memory access
// to complete.  Accesses through a gptr compile to global instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> G(T* p)
{
    return (gptr<T>)p;
}

// relaxed device-scope add on global memory (the result unused: no return)
__device__ __forceinline__ void g_add(gptr<uint32_t> p, uint32_t v)
{
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Philox4x64-10 (Salmon et al., SC'11): counter (a, b, c, 0), key (seed, tag).
// ROLL keeps the ten rounds as a loop: unrolled, the key schedule is hoisted
// into scalar registers, which the collision kernels cannot spare; the
// MD chain keeps the unrolled form (same values either way).
template <bool ROLL = false>
__device__ __forceinline__ void philox(uint64_t a, uint64_t b, uint64_t c,
                                       uint64_t seed, uint64_t tag, uint64_t w[4])
{
    uint64_t c0 = a, c1 = b, c2 = c, c3 = 0, k0 = seed, k1 = tag;
    auto round = [&]() {
        const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
        uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
        uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    };
    if constexpr (ROLL) {
#pragma unroll 1
        for (int r = 0; r < 10; ++r) round();
    } else {
#pragma unroll
        for (int r = 0; r < 10; ++r) round();
    }
    w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
}

// top 53 bits -> [0,1), and the (0,1] variant for logarithms
__device__ __forceinline__ double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
__device__ __forceinline__ double u01o(uint64_t w) { return ((double)(w >> 11) + 1.0) * 0x1.0p-53; }

__device__ __forceinline__ double tfma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float tfma(float a, float b, float c) { return fmaf(a, b, c); }

// periodic wrap of a solvent coordinate after a drift
template <class T>
__device__ __forceinline__ T wrap_coord(T x, T L)
{
    if (x >= L) {
        x -= L;
    } else if (x < (T)0) {
        x += L;
        if (x >= L) x -= L;
    }
    return x;
}

// minimum image of a difference of two coordinates in [0, L)
__device__ __forceinline__ double min_image(double d, double L, double halfL)
{
    if (d > halfL) d -= L;
    else if (d < -halfL) d += L;
    return d;
}

// image in [0, L) of an unwrapped colloid coordinate
__device__ __forceinline__ double colloid_image(double X, double L)
{
    double k = floor(X / L);
    double w = X - k * L;
    if (w >= L) {
        w -= L;
    } else if (w < 0.0) {
        w += L;
        if (w >= L) w -= L;
    }
    return w;
}

__device__ __forceinline__ double dot3(double ax, double ay, double az, double bx, double by, double bz)
{
    return ((ax * bx) + (ay * by)) + (az * bz);
}

// WCA (cut-off repulsive 12-6 LJ): coef = -(dV/dr)/r, pot = V(r), for r2 < rc2.
__device__ __forceinline__ void wca(double r2, double sig2, double eps, double& coef, double& pot)
{
    double ir2 = 1.0 / r2;
    double s2 = sig2 * ir2;
    double s6 = (s2 * s2) * s2;
    coef = (((24.0 * eps) * ir2) * s6) * ((2.0 * s6) - 1.0);
    pot = (4.0 * eps) * (((s6 * s6) - s6) + 0.25);
}

// Marsaglia point on the unit sphere, two tries per Philox block.
template <bool ROLL = false>
__device__ __forceinline__ void marsaglia_axis(uint64_t seed, uint64_t coll, uint64_t cell, double n[3])
{
    for (uint64_t sub = 0; sub < 64; ++sub) {
        uint64_t w[4];
        philox<ROLL>(coll, cell, sub, seed, TAG_ROT, w);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            double a = (2.0 * u01(w[2 * t])) - 1.0;
            double b = (2.0 * u01(w[2 * t + 1])) - 1.0;
            double ss = (a * a) + (b * b);
            if (ss < 1.0) {
                double q = sqrt(1.0 - ss);
                n[0] = (2.0 * a) * q;
                n[1] = (2.0 * b) * q;
                n[2] = 1.0 - (2.0 * ss);
                return;
            }
        }
    }
    n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
}

// Rodrigues rotation of w by alpha about the unit axis n.
__device__ __forceinline__ void rotate(const double n[3], double ca, double sa, double oma,
                                       double w0, double w1, double w2, double out[3])
{
    double nw = ((n[0] * w0) + (n[1] * w1)) + (n[2] * w2);
    double cx = (n[1] * w2) - (n[2] * w1);
    double cy = (n[2] * w0) - (n[0] * w2);
    double cz = (n[0] * w1) - (n[1] * w0);
    double k = oma * nw;
    out[0] = ((ca * w0) + (sa * cx)) + (k * n[0]);
    out[1] = ((ca * w1) + (sa * cy)) + (k * n[1]);
    out[2] = ((ca * w2) + (sa * cz)) + (k * n[2]);
}

// three standard normals (Box-Muller) from one Philox block
__device__ __forceinline__ void normals3(const uint64_t w[4], double z[3])
{
    const double two_pi = 6.283185307179586;
    double r0 = sqrt(-2.0 * log(u01o(w[0])));
    double t0 = two_pi * u01(w[1]);
    double r1 = sqrt(-2.0 * log(u01o(w[2])));
    double t1 = two_pi * u01(w[3]);
    z[0] = r0 * cos(t0);
    z[1] = r0 * sin(t0);
    z[2] = r1 * cos(t1);
}

// replica owning work item `item`: largest r with prefix[r] <= item
// Position of cell (x, y, z) along the Hilbert curve of the 2^bits cube
// (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707 (2004)
// 381): undo the excess work level by level from the top (invert the low
// bits of the first axis where an axis has the level's bit set, otherwise
// exchange the low bits of the first axis and that axis), Gray-encode, then
// read the bits level by level, first axis most significant.
__device__ __forceinline__ uint32_t hilbert_index(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint32_t a[3] = {x, y, z};
    for (int lv = bits - 1; lv >= 1; --lv) {
        const uint32_t Q = 1u << lv, low = Q - 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const uint32_t sw = (a[0] ^ a[i]) & low;
            const bool set = (a[i] & Q) != 0;
            a[0] ^= set ? low : sw;
            if (!set) a[i] ^= sw;
        }
    }
    a[1] ^= a[0];
    a[2] ^= a[1];
    uint32_t g = 0;
    for (int lv = bits - 1; lv >= 1; --lv)
        if (a[2] & (1u << lv)) g ^= (1u << lv) - 1;
    a[0] ^= g; a[1] ^= g; a[2] ^= g;
    uint32_t h = 0;
    for (int lv = bits - 1; lv >= 0; --lv)
        h = (h << 3) | (((a[0] >> lv) & 1u) << 2) | (((a[1] >> lv) & 1u) << 1) | ((a[2] >> lv) & 1u);
    return h;
}

__device__ __forceinline__ int find_rep(const int32_t* prefix, int nrep, int item)
{
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace rmp
