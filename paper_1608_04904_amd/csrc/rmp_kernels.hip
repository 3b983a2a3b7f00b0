// gfx950 kernels of the MPCD+MD solvent path.
//
// One interval (paper, "Algorithms"): n_md velocity-Verlet steps with WCA
// colloid-solvent forces over a Verlet list built from the cell sort, exact
// RATTLE for dimers and catalytic conversion, then one MPCD collision on a
// randomly shifted grid with the RMPCD bulk reaction.  Kernels of one
// interval, in stream order:
//
//   k_stream_bin   particles outside the Verlet list: n_md drifts held in
//                  registers, then the cell key of the next collision and an
//                  atomic rank (HBM-bound, one pass over x, v)
//   k_chain        Verlet-list particles and colloids: n_md MD steps in
//                  persistent workgroups; colloid forces reduced with a fixed
//                  binary tree over list positions; inter-workgroup barrier
//                  per step when the list spans several workgroups
//   k_scan_*       exclusive scan of the cell counts -> cell_start
//   k_scatter      each particle's record (x, v, id, old index, state) to
//                  slot cell_start[key] + rank of the staging array
//   k_collide      per tile of cells: read the tile's records (contiguous),
//                  restore the stable (old-index) order inside each cell,
//                  FP64 centre-of-mass sums,
//                  rotation about a random axis (or Anderson thermostat),
//                  bulk B->A reaction, Verlet-list flags for the next
//                  interval, coalesced write of the cell-ordered arrays
//   k_chunk_scan   list compaction offsets, per-interval bookkeeping
//   k_cand_write   compacted Verlet list
//
// Data layout in HBM: structure-of-arrays, x[3][N] and v[3][N] in the
// storage precision (double or float), double-buffered across collisions.
#include "rmp_device.h"

namespace rmp {

// ------------------------------------------------------------------ utils

// Pairwise binary tree over the 64 lanes of a wave with DPP moves:
// xor 1 and xor 2 (quad permutes), 4-blocks (half-row mirror), 8-blocks (row
// mirror), 16-blocks (row broadcast of lane 15 into rows 1 and 3), and the
// two 32-blocks combined from lanes 31 and 63.  Each level adds the value of
// the adjacent block of the same size, so the result is the tree
// node(l, j) = node(l-1, 2j) + node(l-1, 2j+1) over lanes; it is returned in
// every lane.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_tree_sum(double v)
{
    v = v + dpp_d<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
    v = v + dpp_d<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
    v = v + dpp_d<0x141, 0xF>(v);    // row_half_mirror
    v = v + dpp_d<0x140, 0xF>(v);    // row_mirror
    v = v + dpp_d<0x142, 0xA>(v);    // row_bcast15 into rows 1 and 3
    const double a = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 31),
                                      __builtin_amdgcn_readlane(__double2loint(v), 31));
    const double b = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                                      __builtin_amdgcn_readlane(__double2loint(v), 63));
    return a + b;
}

// wave_tree_sum of N independent values, level by level so that the N
// dependent chains overlap (each value's additions are the same as above)
template <int N>
__device__ __forceinline__ void wave_tree_sum_n(double (&v)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<0xB1, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<0x4E, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<0x141, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<0x140, 0xF>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = v[i] + dpp_d<0x142, 0xA>(v[i]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double a = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[i]), 31),
                                          __builtin_amdgcn_readlane(__double2loint(v[i]), 31));
        const double b = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[i]), 63),
                                          __builtin_amdgcn_readlane(__double2loint(v[i]), 63));
        v[i] = a + b;
    }
}

// minimum of lo and maximum of hi over the 64 lanes (DPP within rows of 16,
// then the four rows' results read from lanes 15, 31, 47, 63); exact, in
// every lane
__device__ __forceinline__ void wave_min_max(double& lo, double& hi)
{
#define RMP_MM_STEP(CTRL)                                                       \
    {                                                                           \
        const double ol = dpp_d<CTRL, 0xF>(lo), oh = dpp_d<CTRL, 0xF>(hi);      \
        lo = ol < lo ? ol : lo;                                                 \
        hi = oh > hi ? oh : hi;                                                 \
    }
    RMP_MM_STEP(0xB1)       // quad_perm [1,0,3,2]
    RMP_MM_STEP(0x4E)       // quad_perm [2,3,0,1]
    RMP_MM_STEP(0x141)      // row_half_mirror
    RMP_MM_STEP(0x140)      // row_mirror
#undef RMP_MM_STEP
    double l = lo, h = hi;
#pragma unroll
    for (int r = 15; r < 64; r += 16) {
        const double rl = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(lo), r),
                                           __builtin_amdgcn_readlane(__double2loint(lo), r));
        const double rh = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(hi), r),
                                           __builtin_amdgcn_readlane(__double2loint(hi), r));
        l = rl < l ? rl : l;
        h = rh > h ? rh : h;
    }
    lo = l;
    hi = h;
}

// minimum of lo and maximum of hi over the 64 lanes, for integers (same
// pattern as wave_min_max)
__device__ __forceinline__ void wave_min_max_i(int& lo, int& hi)
{
#define RMP_MMI_STEP(CTRL)                                                      \
    {                                                                           \
        const int ol = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);  \
        const int oh = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);  \
        lo = ol < lo ? ol : lo;                                                 \
        hi = oh > hi ? oh : hi;                                                 \
    }
    RMP_MMI_STEP(0xB1)
    RMP_MMI_STEP(0x4E)
    RMP_MMI_STEP(0x141)
    RMP_MMI_STEP(0x140)
#undef RMP_MMI_STEP
    int l = lo, h = hi;
#pragma unroll
    for (int r = 15; r < 64; r += 16) {
        const int rl = __builtin_amdgcn_readlane(lo, r), rh = __builtin_amdgcn_readlane(hi, r);
        l = rl < l ? rl : l;
        h = rh > h ? rh : h;
    }
    lo = l;
    hi = h;
}

// maximum of v over the 64 lanes (exact), in every lane
__device__ __forceinline__ double wave_max_d(double v)
{
#define RMP_MX_STEP(CTRL)                                                       \
    {                                                                           \
        const double o = dpp_d<CTRL, 0xF>(v);                                   \
        v = o > v ? o : v;                                                      \
    }
    RMP_MX_STEP(0xB1)
    RMP_MX_STEP(0x4E)
    RMP_MX_STEP(0x141)
    RMP_MX_STEP(0x140)
#undef RMP_MX_STEP
    double m = v;
#pragma unroll
    for (int r = 15; r < 64; r += 16) {
        const double o = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), r),
                                          __builtin_amdgcn_readlane(__double2loint(v), r));
        m = o > m ? o : m;
    }
    return m;
}

// deterministic block sum: wave butterfly, then a pairwise tree over the
// wave sums (xor butterfly over the first NT/64 lanes of wave 0)
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sbuf)
{
    v = wave_tree_sum(v);
    constexpr int NW = NT / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sbuf[wave] = v;
    __syncthreads();
    if (NW > 1) {
        if (wave == 0) {
            double a = lane < NW ? sbuf[lane] : 0.0;
#pragma unroll
            for (int m = 1; m < NW; m <<= 1) a = a + __shfl_xor(a, m, 64);
            if (lane == 0) sbuf[NW] = a;
        }
        __syncthreads();
    }
    double r = sbuf[NW > 1 ? NW : 0];
    __syncthreads();
    return r;
}

// N sums over the workgroup; sbuf holds (NT / 64 + 1) * N doubles.  Every
// thread receives the totals.
template <int NT, int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double* sbuf)
{
    constexpr int NW = NT / 64;
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = wave_tree_sum(v[q]);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) sbuf[wave * N + q] = v[q];
    __syncthreads();
    if (threadIdx.x < N) {
        double a = 0.0;
#pragma unroll 4
        for (int w = 0; w < NW; ++w) a = a + sbuf[w * N + threadIdx.x];
        sbuf[NW * N + threadIdx.x] = a;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = sbuf[NW * N + q];
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, uint32_t* sbuf)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sbuf[wave] = v;
    __syncthreads();
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) r += sbuf[k];
    __syncthreads();
    return r;
}

// exclusive block scan of u32, returns the prefix of this thread; *total set
template <int NT>
__device__ __forceinline__ uint32_t block_exscan_u32(uint32_t v, uint32_t* sbuf, uint32_t* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        uint32_t o = __shfl_up(inc, m, 64);
        if (lane >= m) inc += o;
    }
    __syncthreads();
    if (lane == 63) sbuf[wave] = inc;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        if (k < wave) wpre += sbuf[k];
        tot += sbuf[k];
    }
    __syncthreads();
    *total = tot;
    return wpre + inc - v;
}

__device__ __forceinline__ void shift_of(uint64_t seed, int64_t coll, double s[3])
{
    uint64_t w[4];
    philox((uint64_t)coll, 0, 0, seed, TAG_SHIFT, w);
    s[0] = u01(w[0]);
    s[1] = u01(w[1]);
    s[2] = u01(w[2]);
}

// Sort key of the shifted cell holding (x0, x1, x2): its linear index
// x + Lx (y + Ly z) in the row-major order; in the compact-Hilbert order its
// rank along the curve, computed for a cubic power-of-two box and otherwise
// looked up by the linear index.
__device__ __forceinline__ uint32_t cell_key(const RepDesc& D, double x0, double x1, double x2,
                                             const double s[3])
{
    int64_t c[3];
    const double xs[3] = {x0, x1, x2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double fq = floor(xs[d] - s[d]);
        if (d == 2 && D.walls) {
            // plates: layers floor(z - s) + 1 in [0, L_z], not periodic
            c[d] = (fq >= -1.0 && fq < (double)(D.L[d] - 1)) ? (int64_t)fq + 1 : 0;
            continue;
        }
        int64_t q = (fq >= -1.0 && fq < (double)D.L[d]) ? (int64_t)fq : 0;   // NaN-safe
        if (q < 0) q += D.L[d];
        c[d] = q;
    }
    const uint32_t lin = (uint32_t)(c[0] + (int64_t)D.L[0] * (c[1] + (int64_t)D.L[1] * c[2]));
    if (D.hbits == KEY_ROW) return lin;
    if (D.hbits >= 0) return hilbert_index((uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2], D.hbits);
    return D.rank_of[lin];
}

// Verlet-list membership for the coming interval of length tau: flagged
// particles, or r_ic^2 < (r_cut,c + skin + |v| tau)^2 for some colloid c.
__device__ __forceinline__ bool is_candidate(const RepDesc& D, const ColloidParams* cp, int nc,
                                             const double (*Xw)[3], uint8_t st,
                                             double x0, double x1, double x2,
                                             double v0, double v1, double v2)
{
    if (D.flow) return false;     // flows: no colloids, every particle streams
    if (st & 2) return true;
    if (nc == 0) return false;
    double vv = dot3(v0, v1, v2, v0, v1, v2);
    double reach = sqrt(vv) * D.tau;
    for (int c = 0; c < nc; ++c) {
        double dx = min_image(x0 - Xw[c][0], D.Ld[0], D.halfL[0]);
        double dy = min_image(x1 - Xw[c][1], D.Ld[1], D.halfL[1]);
        double dz = min_image(x2 - Xw[c][2], D.Ld[2], D.halfL[2]);
        double r2 = dot3(dx, dy, dz, dx, dy, dz);
        double tt = cp->reachR[c] + reach;
        if (r2 < tt * tt) return true;
    }
    return false;
}

// potential change of a solvent particle whose species changes (bookkeeping)
__device__ __forceinline__ double species_dU(const RepDesc& D, const ColloidParams* cp, int nc,
                                             const double (*Xw)[3], double x0, double x1,
                                             double x2, int from, int to)
{
    double du = 0.0;
    for (int c = 0; c < nc; ++c) {
        double dx = min_image(x0 - Xw[c][0], D.Ld[0], D.halfL[0]);
        double dy = min_image(x1 - Xw[c][1], D.Ld[1], D.halfL[1]);
        double dz = min_image(x2 - Xw[c][2], D.Ld[2], D.halfL[2]);
        double r2 = dot3(dx, dy, dz, dx, dy, dz);
        if (r2 < cp->rc2[c]) {
            double cf, p0, p1;
            wca(r2, cp->sig2[c], from ? cp->epsB[c] : cp->epsA[c], cf, p0);
            wca(r2, cp->sig2[c], to ? cp->epsB[c] : cp->epsA[c], cf, p1);
            du += p1 - p0;
        }
    }
    return du;
}

template <class T>
__device__ __forceinline__ T* comp(void* base, int64_t n, int d)
{
    return reinterpret_cast<T*>(base) + (int64_t)d * n;
}

// ------------------------------------------------------------------- init

// Solvent initial state: uniform positions rejected inside colloid cores,
// Maxwellian velocities; per-chunk velocity sums for the mean removal.
template <class T>
__global__ __launch_bounds__(256) void k_init(const RepDesc* Dp)
{
    const RepDesc& D = *Dp;
    const ColloidParams* cp = D.cp;
    RepState* rs = D.rs;
    __shared__ double sXw[MAXC][3];
    __shared__ double sred[8];
    const int nc = cp->nc;
    const int t = threadIdx.x;
    if (t < nc)
        for (int d = 0; d < 3; ++d) sXw[t][d] = colloid_image(rs->X[t][d], D.Ld[d]);
    __syncthreads();
    const int64_t n = D.n;
    const int64_t base = (int64_t)blockIdx.x * CHUNK;
    double sum[3] = {0.0, 0.0, 0.0};
    bool bad = false;
    for (int j = t; j < CHUNK; j += 256) {
        int64_t i = base + j;
        if (i >= n) break;
        double xi[3] = {0.0, 0.0, 0.0};
        bool ok = false;
        for (uint64_t att = 0; att < 4096 && !ok; ++att) {
            uint64_t w[4];
            philox(att, (uint64_t)i, 0, D.seed, TAG_INIT_POS, w);
            for (int d = 0; d < 3; ++d) xi[d] = u01(w[d]) * D.Ld[d];
            ok = true;
            for (int c = 0; c < nc && ok; ++c) {
                double dx = min_image(xi[0] - sXw[c][0], D.Ld[0], D.halfL[0]);
                double dy = min_image(xi[1] - sXw[c][1], D.Ld[1], D.halfL[1]);
                double dz = min_image(xi[2] - sXw[c][2], D.Ld[2], D.halfL[2]);
                if (dot3(dx, dy, dz, dx, dy, dz) < cp->sig2[c]) ok = false;
            }
        }
        bad |= !ok;
        uint64_t w[4];
        double z[3];
        philox(0, (uint64_t)i, 0, D.seed, TAG_INIT_VEL, w);
        normals3(w, z);
        for (int d = 0; d < 3; ++d) {
            T xv = (T)xi[d];
            if (xv >= (T)D.Ld[d]) xv = (T)0;    // FP32 rounding up to L
            comp<T>(D.x[0], n, d)[i] = xv;
            T vv = (T)(D.vscale * z[d]);
            comp<T>(D.v[0], n, d)[i] = vv;
            sum[d] += (double)vv;
        }
        D.id[0][i] = (uint32_t)i;
        D.st[0][i] = 0;
    }
    if (bad) atomicOr(&rs->flags, RMP_FLAG_INIT);
    for (int d = 0; d < 3; ++d) {
        double s = block_sum<256>(sum[d], sred);
        if (t == 0) D.obs_part[(int64_t)blockIdx.x * 8 + d] = s;
    }
}

// mean velocity from the chunk sums (one workgroup)
__global__ __launch_bounds__(256) void k_init_mean(const RepDesc* Dp, double* mean_out)
{
    const RepDesc& D = *Dp;
    __shared__ double sred[8];
    for (int d = 0; d < 3; ++d) {
        double s = 0.0;
        for (int k = threadIdx.x; k < D.n_chunks; k += 256) s += D.obs_part[(int64_t)k * 8 + d];
        s = block_sum<256>(s, sred);
        if (threadIdx.x == 0) mean_out[d] = D.n > 0 ? s / (double)D.n : 0.0;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_init_sub(const RepDesc* Dp, const double* mean)
{
    const RepDesc& D = *Dp;
    const int64_t n = D.n;
    const int64_t base = (int64_t)blockIdx.x * CHUNK;
    for (int j = threadIdx.x; j < CHUNK; j += 256) {
        int64_t i = base + j;
        if (i >= n) break;
        for (int d = 0; d < 3; ++d) {
            T* v = comp<T>(D.v[0], n, d);
            v[i] = (T)((double)v[i] - mean[d]);
        }
    }
}

// ------------------------------------------------------- Verlet list build

// Stand-alone list flags (first interval, or a change of n_md).
template <class T>
__global__ __launch_bounds__(256) void k_list(Work w)
{
    const int item = blockIdx.x;
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int chunk = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active) return;
    const ColloidParams* cp = D.cp;
    RepState* rs = D.rs;
    __shared__ double sXw[MAXC][3];
    __shared__ uint32_t sred[4];
    const int nc = cp->nc;
    const int t = threadIdx.x;
    if (t < nc)
        for (int d = 0; d < 3; ++d) sXw[t][d] = colloid_image(rs->X[t][d], D.Ld[d]);
    __syncthreads();
    const int cur = (int)(rs->coll_step & 1);
    const int64_t n = D.n;
    const int64_t base = (int64_t)chunk * CHUNK;
    uint32_t cnt = 0;
    for (int j = t; j < CHUNK; j += 256) {
        int64_t i = base + j;
        if (i >= n) break;
        double x0 = comp<T>(D.x[cur], n, 0)[i], x1 = comp<T>(D.x[cur], n, 1)[i],
               x2 = comp<T>(D.x[cur], n, 2)[i];
        double v0 = comp<T>(D.v[cur], n, 0)[i], v1 = comp<T>(D.v[cur], n, 1)[i],
               v2 = comp<T>(D.v[cur], n, 2)[i];
        bool c = is_candidate(D, cp, nc, sXw, D.st[cur][i], x0, x1, x2, v0, v1, v2);
        D.cflag[i] = c ? 1 : 0;
        cnt += c ? 1u : 0u;
    }
    uint32_t tot = block_sum_u32<256>(cnt, sred);
    if (t == 0) D.chunk_cnt[chunk] = tot;
}

// Per replica (one workgroup each): exclusive scan of the chunk counts of
// Verlet-list members, list length and capacity check, barrier reset.  When
// `after_collision` is set it also closes the interval: collision-step
// counter, temperature of the collision, reaction bookkeeping.
__global__ __launch_bounds__(1024) void k_chunk_scan(Work w, int after_collision)
{
    const int rep = blockIdx.x;
    const RepDesc& D = w.desc[rep];
    if (!D.active) return;
    RepState* rs = D.rs;
    __shared__ uint32_t sbuf[16];
    __shared__ double dbuf[17 * 6];
    const int t = threadIdx.x;
    const int nch = D.n_chunks;
    const int per = (nch + 1023) / 1024;
    const gptr<const uint32_t> cnt = G(D.chunk_cnt);
    const gptr<uint32_t> off = G(D.chunk_off);
    // a single workgroup walks all chunks: latency, not bandwidth, bounds
    // this, so each thread's counts (up to CS_REG of them) are loaded at
    // once and kept for the second pass; more are read in batches, twice
    constexpr int CS_REG = 32, UB = 4;
    const int q0 = t * per;
    uint32_t c[CS_REG];
    uint32_t local = 0;
    if (per <= CS_REG) {
#pragma unroll
        for (int u = 0; u < CS_REG; ++u) c[u] = (u < per && q0 + u < nch) ? cnt[q0 + u] : 0u;
#pragma unroll
        for (int u = 0; u < CS_REG; ++u) local += c[u];
    } else {
        int kk = 0;
        for (; kk + UB <= per; kk += UB) {
            uint32_t b[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) b[u] = q0 + kk + u < nch ? cnt[q0 + kk + u] : 0u;
#pragma unroll
            for (int u = 0; u < UB; ++u) local += b[u];
        }
        for (; kk < per; ++kk)
            if (q0 + kk < nch) local += cnt[q0 + kk];
    }
    uint32_t total;
    uint32_t pre = block_exscan_u32<1024>(local, sbuf, &total);
    if (per <= CS_REG) {
#pragma unroll
        for (int u = 0; u < CS_REG; ++u) {
            if (u < per && q0 + u < nch) off[q0 + u] = pre;
            pre += c[u];
        }
    } else {
        int kk = 0;
        for (; kk + UB <= per; kk += UB) {
            uint32_t b[UB];
#pragma unroll
            for (int u = 0; u < UB; ++u) b[u] = q0 + kk + u < nch ? cnt[q0 + kk + u] : 0u;
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                if (q0 + kk + u < nch) off[q0 + kk + u] = pre;
                pre += b[u];
            }
        }
        for (; kk < per; ++kk) {
            const int q = q0 + kk;
            if (q < nch) {
                off[q] = pre;
                pre += cnt[q];
            }
        }
    }
    if (after_collision) {
        // tile partials (temperature sum and cells, reaction energy, bulk
        // flips): eight 32-byte loads in flight per round into two
        // accumulators; the order is fixed for a given tile count
        double a[2][4] = {};
        const gptr<const double> tp = G(D.tpart);
        constexpr int TL = 8;
        int k = t;
        for (; k + (TL - 1) * 1024 < D.n_tiles; k += TL * 1024) {
            double q[TL][4];
#pragma unroll
            for (int j = 0; j < TL; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) q[j][e] = tp[(int64_t)(k + j * 1024) * 4 + e];
#pragma unroll
            for (int j = 0; j < TL; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) a[j & 1][e] += q[j][e];
        }
        for (; k < D.n_tiles; k += 1024)
#pragma unroll
            for (int e = 0; e < 4; ++e) a[0][e] += tp[(int64_t)k * 4 + e];
        double v[6];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = a[0][j] + a[1][j];
        v[4] = 0.0;
        v[5] = 0.0;
        for (int g = t; g < D.G; g += 1024) {
            v[4] += D.epart[(int64_t)g * 2 + 0];
            v[5] += D.epart[(int64_t)g * 2 + 1];
            D.epart[(int64_t)g * 2 + 0] = 0.0;
            D.epart[(int64_t)g * 2 + 1] = 0.0;
        }
        block_sum_n<1024, 6>(v, dbuf);
        if (t == 0) {
            rs->T_sum = v[0];
            rs->T_cells = v[1];
            rs->e_rxn += v[2] + v[4];
            rs->n_bulk += (int64_t)v[3];
            rs->n_cat += (int64_t)v[5];
            rs->coll_step += 1;
        }
    }
    if (!after_collision) {
        // a stand-alone list build follows init or set_state, where the step
        // counters may have moved backwards: clear the exchange words so no
        // stale epoch can match
        uint64_t* part = reinterpret_cast<uint64_t*>(D.partials);
        for (int64_t k = t; k < 2 * ((int64_t)D.G * ROWW + BCW); k += 1024) part[k] = 0ull;
    }
    if (t == 0) {
        rs->n_cand = total;
        if ((int64_t)total > (int64_t)D.cand_cap) rs->flags |= RMP_FLAG_LIST_OVERFLOW;
        rs->bar = 0;
        rs->list_nmd = D.n_md;
    }
}

// Compacted Verlet list in array order.
__global__ __launch_bounds__(256) void k_cand_write(Work w)
{
    const int item = blockIdx.x;
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int chunk = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active) return;
    // most chunks hold no list member (the list gathers around the
    // colloids): their flags are not read at all, and their count is zero
    // already
    if (D.chunk_cnt[chunk] == 0u) return;
    __shared__ uint32_t sbuf[4];
    const int64_t n = D.n;
    const int64_t base = (int64_t)chunk * CHUNK;
    constexpr int PER = CHUNK / 256;
    const int t = threadIdx.x;
    uint32_t f[PER];
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int64_t i = base + (int64_t)t * PER + k;
        f[k] = (i < n) ? (uint32_t)D.cflag[i] : 0u;
        cnt += f[k];
    }
    uint32_t total;
    uint32_t pre = block_exscan_u32<256>(cnt, sbuf, &total) + D.chunk_off[chunk];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (f[k]) {
            const int64_t i = base + (int64_t)t * PER + k;
            if ((int64_t)pre < (int64_t)D.cand_cap) {
                D.cand_idx[pre] = (uint32_t)i;
            } else {
                // beyond the list capacity (RMP_FLAG_LIST_OVERFLOW is set):
                // the particle is streamed freely so that every particle is
                // still binned exactly once
                D.cflag[i] = 0;
            }
            pre++;
        }
    }
    if (t == 0) D.chunk_cnt[chunk] = 0;
}

// ------------------------------------------------- free streaming + binning

// Rank of this lane's particle within its cell, with one atomic per run of
// equal keys in consecutive lanes (particles arrive sorted by the previous
// collision's cells, so runs are common).  All 64 lanes must call it.
struct RankIssue {
    uint32_t base;             // the run head's atomic result (head lanes only)
    int h;                     // lane of this lane's run head
};

__device__ __forceinline__ RankIssue wave_rank_issue(gptr<uint32_t> count, uint32_t key, bool valid)
{
    const int lane = threadIdx.x & 63;
    const uint32_t k = valid ? key : 0xffffffffu;
    const uint32_t prev = __shfl_up(k, 1, 64);
    const bool head = (lane == 0) || (k != prev);
    const uint64_t H = __ballot(head);
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int h = 63 - __clzll(H & upto);
    const uint64_t above = (h == 63) ? 0ull : (H & (~0ull << (h + 1)));
    const int nexth = above ? (__ffsll((long long)above) - 1) : 64;
    RankIssue r;
    r.base = 0;
    r.h = h;
    if (head && valid)
        r.base = __hip_atomic_fetch_add(count + key, (uint32_t)(nexth - h), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return r;
}

__device__ __forceinline__ uint32_t wave_rank_finish(const RankIssue& r)
{
    const int lane = threadIdx.x & 63;
    return __shfl(r.base, r.h, 64) + (uint32_t)(lane - r.h);
}

__device__ __forceinline__ uint32_t wave_rank(gptr<uint32_t> count, uint32_t key, bool valid)
{
    return wave_rank_finish(wave_rank_issue(count, key, valid));
}

// One streaming step under the constant acceleration g, with the plates at
// z = 0 and z = L_z when present: half kick, drift, half kick; a drift that
// crosses a plate is cut at the crossing time, the velocity reversed
// (bounce-back) and the rest of the step travelled back.
template <class T>
__device__ __forceinline__ T below(T L);
template <>
__device__ __forceinline__ double below<double>(double L) { return nextafter(L, 0.0); }
template <>
__device__ __forceinline__ float below<float>(float L) { return nextafterf(L, 0.0f); }

template <class T>
__device__ __forceinline__ void flow_step(T (&x)[3], T (&v)[3], const T (&g)[3], T dt, T hdt,
                                          const T (&L)[3], bool walls)
{
    T y[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v[d] = tfma(hdt, g[d], v[d]);
        y[d] = tfma(dt, v[d], x[d]);
    }
    if (walls) {
        if (y[2] < (T)0 || y[2] >= L[2]) {
            const T wz = y[2] < (T)0 ? (T)0 : L[2];
            const T ts = (wz - x[2]) / v[2];
            const T rem = dt - ts;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const T xc = tfma(ts, v[d], x[d]);
                v[d] = -v[d];
                y[d] = tfma(rem, v[d], xc);
            }
            if (y[2] >= L[2]) y[2] = below<T>(L[2]);
            if (y[2] < (T)0) y[2] = (T)0;
        }
        x[0] = wrap_coord<T>(y[0], L[0]);
        x[1] = wrap_coord<T>(y[1], L[1]);
        x[2] = y[2];
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] = wrap_coord<T>(y[d], L[d]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] = tfma(hdt, g[d], v[d]);
}

// Flows (constant acceleration, plates) stream every particle with flow_step
// and write back positions and velocities.  Otherwise:
// particles outside the Verlet list feel no force during the interval: n_md
// drifts x <- fma(dt, v, x) with a periodic wrap after each.  The drift of a
// coordinate is monotone, so if its final value is still inside the box no
// wrap occurred and the per-step wrap can be skipped; otherwise the drifts
// are replayed with the wrap.  Then the key of the shifted cell of the coming
// collision and a rank within the cell.  Workgroup `sub` of a chunk covers
// particles [sub*span, (sub+1)*span) of it, span = blockDim.x * PPT; thread t
// holds particles t, t + blockDim.x, ... of its span: every load is issued
// before the drifts, every rank atomic before the first of them is waited
// for.
template <class T, int PPT>
__global__ __launch_bounds__(256) void k_stream_bin(Work w, int wg_per_chunk)
{
    const int item = blockIdx.x / wg_per_chunk;
    const int sub = blockIdx.x - item * wg_per_chunk;
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int chunk = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active) return;
    RepState* rs = D.rs;
    __shared__ double sshift[3];
    const int64_t coll = rs->coll_step;
    if (threadIdx.x == 0) shift_of(D.seed, coll, sshift);
    __syncthreads();
    const double s[3] = {sshift[0], sshift[1], sshift[2]};
    const int cur = (int)(coll & 1);
    const int64_t n = D.n;
    const int nmd = D.n_md;
    const T dt = (T)D.dt;
    const T Lt[3] = {(T)D.Ld[0], (T)D.Ld[1], (T)D.Ld[2]};
    const gptr<T> xs[3] = {G(comp<T>(D.x[cur], n, 0)), G(comp<T>(D.x[cur], n, 1)), G(comp<T>(D.x[cur], n, 2))};
    const gptr<T> vs[3] = {G(comp<T>(D.v[cur], n, 0)), G(comp<T>(D.v[cur], n, 1)), G(comp<T>(D.v[cur], n, 2))};
    const gptr<const uint8_t> cflag = G(D.cflag);
    const gptr<uint64_t> keyrank = G(D.keyrank);
    const gptr<uint32_t> count = G(D.count);
    const int span = CHUNK / wg_per_chunk;
    const int64_t base = (int64_t)chunk * CHUNK + (int64_t)sub * span;
    if (D.flow) {
        const T g[3] = {(T)D.g[0], (T)D.g[1], (T)D.g[2]};
        const T hdt = (T)(0.5 * D.dt);
        for (int j0 = 0; j0 < span; j0 += blockDim.x) {
            const int64_t i = base + j0 + threadIdx.x;
            bool valid = (j0 + (int)threadIdx.x < span) && (i < n);
            if (valid) valid = cflag[i] == 0;
            uint32_t key = 0;
            if (valid) {
                T x[3], v[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) { x[d] = xs[d][i]; v[d] = vs[d][i]; }
                for (int k = 0; k < nmd; ++k) flow_step<T>(x, v, g, dt, hdt, Lt, D.walls != 0);
#pragma unroll
                for (int d = 0; d < 3; ++d) { xs[d][i] = x[d]; vs[d][i] = v[d]; }
                key = cell_key(D, (double)x[0], (double)x[1], (double)x[2], s);
            }
            const uint32_t rank = wave_rank(count, key, valid);
            if (valid) keyrank[i] = ((uint64_t)key << 32) | rank;
        }
        return;
    }
    bool valid[PPT];
    int64_t ii[PPT];
    T x[PPT][3], v[PPT][3];
    const int bs = (int)blockDim.x;
    // the flag and the state are loaded side by side, so one memory latency
    // precedes the drifts (a list entry's state, which the MD chain on the
    // side stream may be writing meanwhile, is loaded and never used)
    uint8_t fl[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        ii[u] = base + u * bs + threadIdx.x;
        valid[u] = (u * bs + (int)threadIdx.x < span) && (ii[u] < n);
        fl[u] = valid[u] ? cflag[ii[u]] : (uint8_t)1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[u][d] = valid[u] ? xs[d][ii[u]] : (T)0;
            v[u][d] = valid[u] ? vs[d][ii[u]] : (T)0;
        }
    }
#pragma unroll
    for (int u = 0; u < PPT; ++u) valid[u] = valid[u] && fl[u] == 0;
    uint32_t key[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            T y = x[u][d];
            for (int k = 0; k < nmd; ++k) y = tfma(dt, v[u][d], y);
            const bool inside = (v[u][d] >= (T)0) ? (y < Lt[d]) : (y >= (T)0);
            if (!inside) {
                y = x[u][d];
                for (int k = 0; k < nmd; ++k) y = wrap_coord<T>(tfma(dt, v[u][d], y), Lt[d]);
            }
            x[u][d] = y;
        }
        key[u] = valid[u] ? cell_key(D, (double)x[u][0], (double)x[u][1], (double)x[u][2], s) : 0u;
    }
    RankIssue ri[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) ri[u] = wave_rank_issue(count, key[u], valid[u]);
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        const uint32_t rank = wave_rank_finish(ri[u]);
        if (valid[u]) {
#pragma unroll
            for (int d = 0; d < 3; ++d) xs[d][ii[u]] = x[u][d];
            keyrank[ii[u]] = ((uint64_t)key[u] << 32) | rank;
        }
    }
}

// ------------------------------------------------------------- MD chain

// ordering of LDS accesses between lanes of one wave (no workgroup barrier)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double shfl_d(double v, int src)
{
    const int lo = __shfl(__double2loint(v), src, 64);
    const int hi = __shfl(__double2hiint(v), src, 64);
    return __hiloint2double(hi, lo);
}

// Bond of the colloid of lane t (t < nc), loaded once per interval
struct BondLane {
    int other;                 // lane of the bond partner (t itself if none)
    bool has, ia;              // has a bond; is its first colloid a
    double dd, ima, imb, mu;   // bond length, inverse masses of a and b, sum
};

__device__ __forceinline__ BondLane bond_lane(const ColloidParams* cp, int nc)
{
    const int t = threadIdx.x & 63;
    BondLane L;
    const int k = t < nc ? cp->bond_of[t] : -1;
    L.has = k >= 0;
    const int a = L.has ? cp->bond_a[k] : t, b = L.has ? cp->bond_b[k] : t;
    L.ia = t == a;
    L.other = L.ia ? b : a;
    L.dd = L.has ? cp->bond_d[k] : 0.0;
    L.ima = L.has ? cp->imass[a] : 0.0;
    L.imb = L.has ? cp->imass[b] : 0.0;
    L.mu = L.ima + L.imb;
    return L;
}

// RATTLE position stage for the colloid of lane t (t < nc, all 64 lanes of
// the wave call it).  Both colloids of a bond evaluate the bond's
// correction from the same operands in the bond's (a, b) order, so they
// agree exactly; Xo are the positions before the drift.
__device__ __forceinline__ void rattle_pos_lane(const BondLane& L, double dt, double (&X)[3], double (&V)[3],
                                                const double (&Xo)[3], uint32_t& flags)
{
    double pXo[3], pX[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pXo[d] = shfl_d(Xo[d], L.other);
        pX[d] = shfl_d(X[d], L.other);
    }
    if (!L.has) return;
    const bool ia = L.ia;
    double r0[3], sv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r0[d] = ia ? Xo[d] - pXo[d] : pXo[d] - Xo[d];
        sv[d] = ia ? X[d] - pX[d] : pX[d] - X[d];
    }
    const double mu = L.mu;
    const double r0r0 = dot3(r0[0], r0[1], r0[2], r0[0], r0[1], r0[2]);
    const double sr0 = dot3(sv[0], sv[1], sv[2], r0[0], r0[1], r0[2]);
    const double ss = dot3(sv[0], sv[1], sv[2], sv[0], sv[1], sv[2]);
    const double A = (mu * mu) * r0r0;
    const double Bh = mu * sr0;
    const double C = ss - (L.dd * L.dd);
    double disc = (Bh * Bh) - (A * C);
    if (disc < 0.0) {
        flags |= RMP_FLAG_RATTLE;
        disc = 0.0;
    }
    const double gq = C / (Bh + sqrt(disc));
    if (ia) {
        const double ga = gq * L.ima;
        const double gad = ga / dt;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            X[d] = X[d] - (ga * r0[d]);
            V[d] = V[d] - (gad * r0[d]);
        }
    } else {
        const double gb = gq * L.imb;
        const double gbd = gb / dt;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            X[d] = X[d] + (gb * r0[d]);
            V[d] = V[d] + (gbd * r0[d]);
        }
    }
}

// Iterative RATTLE (Andersen 1983) for bond networks, by the 64 lanes of
// wave 0 on the colloid state staged in LDS.  Position stage: sweeps over
// the bonds in order; a bond whose squared length s.s misses d^2 by more than
// 2 tol d^2 is corrected along its direction before the drift, r0: both
// colloids move by g r0 / m, g = (d^2 - s.s) / (2 mu s.r0), mu = 1/m_a +
// 1/m_b, and their velocities by the same displacement over dt; until a
// sweep changes nothing, at most rattle_maxit sweeps (else the RATTLE flag).
// A sweep runs layer by layer, a layer being consecutive bonds with no
// colloid in common, one lane per bond: the corrections within a layer
// commute exactly, so the result is that of the bonds one after another.
//
// A layer's lane reads both ends of its bond, their velocities and the
// bond's constants (LDS tables filled once per interval and per stage) in
// one round trip, and writes the results back together; the ends of the
// next layer's bonds are read a layer ahead.
template <class Ctx>
__device__ __forceinline__ uint32_t rattle_pos_iter(Ctx& S, const ColloidParams* cp, double dt)
{
    const int lane = threadIdx.x & 63;
    const int nl = cp->n_layers, nbond = cp->nbonds;
    for (int q = lane; q < nbond; q += 64) {
        const int a = S.sBa[q], b = S.sBb[q];
        for (int d = 0; d < 3; ++d) S.sBr[q][d] = S.sXoc[a][d] - S.sXoc[b][d];
    }
    wave_sync();
    bool moved = true;
    for (int sweep = 0; sweep < cp->rattle_maxit && moved; ++sweep) {
        bool m = false;
        int s0 = S.sLay[0], s1 = nl > 0 ? S.sLay[1] : s0;
        int a = 0, b = 0;
        if (s0 + lane < s1) {
            a = S.sBa[s0 + lane];
            b = S.sBb[s0 + lane];
        }
        for (int L = 0; L < nl; ++L) {
            const int q = s0 + lane;
            const bool act = q < s1;
            // both ends read at once (a != b) with the bond's constants,
            // written back at once
            double xa[3], xb[3], va[3], vb[3], r0[3];
            double dd2 = 0.0, thr = 0.0, mu2 = 0.0, ima = 0.0, imb = 0.0;
            if (act) {
                for (int d = 0; d < 3; ++d) {
                    xa[d] = S.sXc[a][d];
                    xb[d] = S.sXc[b][d];
                    r0[d] = S.sBr[q][d];
                }
                dd2 = S.sBd2[q];
                thr = S.sBthr[q];
                mu2 = S.sBmu2[q];
                ima = S.sBia[q];
                imb = S.sBib[q];
                for (int d = 0; d < 3; ++d) {
                    va[d] = S.sVc[a][d];
                    vb[d] = S.sVc[b][d];
                }
            }
            // ends of the next layer's bonds (unused past its end)
            const int s2 = S.sLay[min(L + 2, nl)];
            const int qn = s1 + lane;
            int na = 0, nb = 0;
            if (qn < nbond) {
                na = S.sBa[qn];
                nb = S.sBb[qn];
            }
            if (act) {
                double sv[3];
                for (int d = 0; d < 3; ++d) sv[d] = xa[d] - xb[d];
                const double ss = dot3(sv[0], sv[1], sv[2], sv[0], sv[1], sv[2]);
                const double diff = dd2 - ss;
                if (fabs(diff) > thr) {
                    const double sr0 = dot3(sv[0], sv[1], sv[2], r0[0], r0[1], r0[2]);
                    const double g = diff / (mu2 * sr0);
                    const double ga = g * ima, gb = g * imb;
                    for (int d = 0; d < 3; ++d) {
                        S.sXc[a][d] = xa[d] + (ga * r0[d]);
                        S.sXc[b][d] = xb[d] - (gb * r0[d]);
                    }
                    const double gad = ga / dt, gbd = gb / dt;
                    for (int d = 0; d < 3; ++d) {
                        S.sVc[a][d] = va[d] + (gad * r0[d]);
                        S.sVc[b][d] = vb[d] - (gbd * r0[d]);
                    }
                    m = true;
                }
            }
            wave_sync();
            s0 = s1;
            s1 = s2;
            a = na;
            b = nb;
        }
        moved = __ballot(m) != 0ull;
    }
    return moved ? RMP_FLAG_RATTLE : 0u;
}

// Iterative RATTLE, velocity stage: sweeps removing the relative velocity
// along each bond, k = (r.v) / (mu d^2), while |r.v| exceeds tol d^2 / dt
// (layer by layer, as above; the bond vectors r are fixed for the stage).
template <class Ctx>
__device__ __forceinline__ uint32_t rattle_vel_iter(Ctx& S, const ColloidParams* cp, double dt)
{
    (void)dt;
    const int lane = threadIdx.x & 63;
    const int nl = cp->n_layers, nbond = cp->nbonds;
    for (int q = lane; q < nbond; q += 64) {
        const int a = S.sBa[q], b = S.sBb[q];
        for (int d = 0; d < 3; ++d) S.sBr[q][d] = S.sXc[a][d] - S.sXc[b][d];
    }
    wave_sync();
    bool moved = true;
    for (int sweep = 0; sweep < cp->rattle_maxit && moved; ++sweep) {
        bool m = false;
        int s0 = S.sLay[0], s1 = nl > 0 ? S.sLay[1] : s0;
        int a = 0, b = 0;
        if (s0 + lane < s1) {
            a = S.sBa[s0 + lane];
            b = S.sBb[s0 + lane];
        }
        for (int L = 0; L < nl; ++L) {
            const int q = s0 + lane;
            const bool act = q < s1;
            double va[3], vb[3], r[3];
            double thv = 0.0, mud = 0.0, ima = 0.0, imb = 0.0;
            if (act) {
                for (int d = 0; d < 3; ++d) {
                    va[d] = S.sVc[a][d];
                    vb[d] = S.sVc[b][d];
                    r[d] = S.sBr[q][d];
                }
                thv = S.sBthv[q];
                mud = S.sBmud[q];
                ima = S.sBia[q];
                imb = S.sBib[q];
            }
            const int s2 = S.sLay[min(L + 2, nl)];
            const int qn = s1 + lane;
            int na = 0, nb = 0;
            if (qn < nbond) {
                na = S.sBa[qn];
                nb = S.sBb[qn];
            }
            if (act) {
                double vr[3];
                for (int d = 0; d < 3; ++d) vr[d] = va[d] - vb[d];
                const double rv = dot3(r[0], r[1], r[2], vr[0], vr[1], vr[2]);
                if (fabs(rv) > thv) {
                    const double k = rv / mud;
                    const double ka = k * ima, kb = k * imb;
                    for (int d = 0; d < 3; ++d) {
                        S.sVc[a][d] = va[d] - (ka * r[d]);
                        S.sVc[b][d] = vb[d] + (kb * r[d]);
                    }
                    m = true;
                }
            }
            wave_sync();
            s0 = s1;
            s1 = s2;
            a = na;
            b = nb;
        }
        moved = __ballot(m) != 0ull;
    }
    return moved ? RMP_FLAG_RATTLE : 0u;
}

// RATTLE velocity stage for the colloid of lane t (same conventions)
__device__ __forceinline__ void rattle_vel_lane(const BondLane& L, const double (&X)[3], double (&V)[3])
{
    double pX[3], pV[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pX[d] = shfl_d(X[d], L.other);
        pV[d] = shfl_d(V[d], L.other);
    }
    if (!L.has) return;
    const bool ia = L.ia;
    double r[3], vr[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r[d] = ia ? X[d] - pX[d] : pX[d] - X[d];
        vr[d] = ia ? V[d] - pV[d] : pV[d] - V[d];
    }
    const double rr = dot3(r[0], r[1], r[2], r[0], r[1], r[2]);
    const double vrr = dot3(vr[0], vr[1], vr[2], r[0], r[1], r[2]);
    const double kk = vrr / (L.mu * rr);
    if (ia) {
        const double ka = kk * L.ima;
#pragma unroll
        for (int d = 0; d < 3; ++d) V[d] = V[d] - (ka * r[d]);
    } else {
        const double kb = kk * L.imb;
#pragma unroll
        for (int d = 0; d < 3; ++d) V[d] = V[d] + (kb * r[d]);
    }
}

// Chain workgroup g of a replica holds Verlet-list positions
// [g*B, (g+1)*B), B = NT*K (NT = 256 or 512 threads), K consecutive
// positions per thread, in registers for the whole interval.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double uniform_d(double v)
{
    return __longlong_as_double((long long)uniform_u64((uint64_t)__double_as_longlong(v)));
}

// Descriptor fields used in every MD step, copied to scalar registers once:
// read through the descriptor they are fetched again after each fence of
// the exchange.
struct ChainConst {
    double Lv[3], hv[3];       // box lengths and half lengths
    uint64_t* partv;           // exchange buffers, two of stridev words
    int64_t stridev;           // G * ROWW + BCW
    int Gv;                    // workgroups of the replica's exchange buffers
    double catv;
    uint64_t seedv;
    uint64_t budgetv;          // longest wait for the other workgroups (ticks)
    __device__ double L(int d) const { return Lv[d]; }
    __device__ double h(int d) const { return hv[d]; }
    __device__ gptr<uint64_t> part() const { return (gptr<uint64_t>)partv; }
    __device__ int G() const { return Gv; }
    __device__ int64_t stride() const { return stridev; }
    __device__ double cat_prob() const { return catv; }
    __device__ uint64_t seed() const { return seedv; }
    __device__ uint64_t budget() const { return budgetv; }
};

__device__ __forceinline__ ChainConst chain_const(const RepDesc& D, uint64_t budget)
{
    ChainConst c;
    for (int d = 0; d < 3; ++d) {
        c.Lv[d] = uniform_d(D.Ld[d]);
        c.hv[d] = uniform_d(D.halfL[d]);
    }
    c.partv = reinterpret_cast<uint64_t*>(uniform_u64((uint64_t)(uintptr_t)D.partials));
    c.Gv = __builtin_amdgcn_readfirstlane(D.G);
    c.stridev = (int64_t)c.Gv * ROWW + BCW;
    c.catv = uniform_d(D.cat_prob);
    c.seedv = uniform_u64(D.seed);
    c.budgetv = uniform_u64(budget);
    return c;
}

// NB: bond capacity of the iterative-RATTLE tables (1 in the variants
// unrolled for one or two colloids, which never run it).
template <int NT, int NB>
struct ChainCtx {
    double sXw[MAXC][3];       // periodic images of the colloid positions
    // colloid constants read in every MD step, staged once per interval
    double cRc2[MAXC], cSig2[MAXC], cEpsA[MAXC], cEpsB[MAXC], cSigma[MAXC];
    double cCull2[MAXC];       // (cut-off + reach margin)^2 of the interval's cull
    int32_t cCat[MAXC], cType[MAXC], cBody[MAXC];
    double cEcc[2][2];
    double sRed[NT / 64][NVAL_MAX];
    double sNode[NVAL_MAX];
    uint32_t sWhit[NT / 64];   // colloids that some entry of the wave is within cut-off of
    // master of the multi-workgroup exchange: the colloids each row listed
    // at the last look, a chunk of XV values by row and value, and the
    // trees' partial sums of each wave (the variants for one or two colloids
    // have at most 7 values)
    static constexpr int XV = NB > 1 ? XTAB_V : 8;
    uint32_t sE[MAX_CHAIN_G];
    double sTab[XTAB_R][XV];
    double sPart[NT / 64][XV];
    uint32_t sPairMask[MAXC];  // colloid c: bit a set when the pair (c, a) interacts
    uint32_t sFull;            // a colloid left its interval-start reach margin: no cull
    // colloid-colloid pairs (a < b) of the current positions: force on the
    // lower colloid and potential, and whether the pair interacts
    static constexpr int NPAIR = NB > 1 ? MAXC * (MAXC - 1) / 2 : 1;
    double sPairF[NPAIR][4];
    uint8_t sPairOn[NPAIR];
    double sU;
    uint32_t sflags;
    // colloid state and bonds staged for the iterative RATTLE (bond networks)
    static constexpr int NCI = NB > 1 ? MAXC : 1;
    double sXc[NCI][3], sVc[NCI][3], sXoc[NCI][3];
    int32_t sBa[NB], sBb[NB], sLay[NB + 1];
    // per bond, for the interval: d^2, the two thresholds, the two mass
    // factors and the inverse masses of its ends; for the stage under way:
    // the bond vector that the stage holds fixed
    double sBd2[NB], sBthr[NB], sBthv[NB];
    double sBmu2[NB], sBmud[NB], sBia[NB], sBib[NB];
    double sBr[NB][3];
};

// species_dU for an A -> B flip inside the MD chain, with the colloid
// constants from LDS (same arithmetic)
template <class Ctx>
__device__ __forceinline__ double species_dU_lds(const Ctx& S, const ChainConst& cc, int nc, double x0, double x1,
                                                 double x2)
{
    double du = 0.0;
    for (int c = 0; c < nc; ++c) {
        double dx = min_image(x0 - S.sXw[c][0], cc.L(0), cc.h(0));
        double dy = min_image(x1 - S.sXw[c][1], cc.L(1), cc.h(1));
        double dz = min_image(x2 - S.sXw[c][2], cc.L(2), cc.h(2));
        double r2 = dot3(dx, dy, dz, dx, dy, dz);
        if (r2 < S.cRc2[c]) {
            double cf, p0, p1;
            wca(r2, S.cSig2[c], S.cEpsA[c], cf, p0);
            wca(r2, S.cSig2[c], S.cEpsB[c], cf, p1);
            du += p1 - p0;
        }
    }
    return du;
}

// WCA force of colloid b on colloid a (a < b, sigma_ab = sigma_a + sigma_b,
// epsilon by the pair's types) and its potential, for the current colloid
// images; `on` is 0 when the two are of one rigid body or beyond the cut-off
// (then the values are not used)
template <class Ctx>
__device__ __forceinline__ void pair_force(const Ctx& S, const ChainConst& cc, const ColloidParams* cp, int a,
                                           int b, double (&out)[4], uint8_t& on)
{
    on = 0;
    out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = 0.0;
    if (S.cBody[a] == S.cBody[b]) return;
    const double dx = min_image(S.sXw[a][0] - S.sXw[b][0], cc.L(0), cc.h(0));
    const double dy = min_image(S.sXw[a][1] - S.sXw[b][1], cc.L(1), cc.h(1));
    const double dz = min_image(S.sXw[a][2] - S.sXw[b][2], cc.L(2), cc.h(2));
    const double r2 = dot3(dx, dy, dz, dx, dy, dz);
    const double sab = S.cSigma[a] + S.cSigma[b];
    const double rc = 0x1.1f59ac3c7d6c0p+0 * sab;
    if (r2 < rc * rc) {
        double coef, pot;
        wca(r2, sab * sab, S.cEcc[S.cType[a]][S.cType[b]], coef, pot);
        out[0] = coef * dx; out[1] = coef * dy; out[2] = coef * dz; out[3] = pot;
        on = 1;
    }
}

// First half of a force evaluation: forces on this workgroup's list
// entries from all colloids, and the per-colloid force sums and the
// potential reduced over this workgroup's list positions with the fixed
// binary tree (within a thread over K, over the lanes of a wave, over the
// waves).  With several workgroups the node values are then published for
// the others (chain_collect completes the tree over workgroups).
template <class T, int K, int NT, int NB>
__device__ __forceinline__ void chain_compute(ChainCtx<NT, NB>& S, const ChainConst& cc, const ColloidParams* cp,
                              int nc, const bool* valid, const T (*x)[3], const T (*x0)[3], const uint8_t* st,
                              double (*f)[3], bool* inside, int g, int Gact, bool solo,
                              uint32_t& wmask, double me2, uint32_t& nbar, uint32_t epoch0)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double u[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        f[j][0] = 0.0; f[j][1] = 0.0; f[j][2] = 0.0;
        u[j] = 0.0;
        inside[j] = false;
    }
    // Colloids within reach of this wave: wmask, set at the start of the
    // interval from the box of the wave's entries (reach_box).  It holds
    // while every entry stays within the margin me of its position at the
    // start and every colloid within half the skin of its own; once either
    // fails the wave tests every colloid for the rest of the interval.  A
    // colloid out of reach contributes exactly zero to every entry of the
    // wave, so its distances are not computed.
    const uint32_t all_mask = nc >= 32 ? 0xffffffffu : ((1u << nc) - 1u);
    if (wmask != all_mask) {
        bool moved = false;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (valid[j]) {
                const double dx = min_image((double)x[j][0] - (double)x0[j][0], cc.L(0), cc.h(0));
                const double dy = min_image((double)x[j][1] - (double)x0[j][1], cc.L(1), cc.h(1));
                const double dz = min_image((double)x[j][2] - (double)x0[j][2], cc.L(2), cc.h(2));
                moved = moved || !(dot3(dx, dy, dz, dx, dy, dz) < me2);
            }
        if (__ballot(moved) != 0 || S.sFull != 0) wmask = all_mask;
    }
    const uint32_t reach_mask = wmask;
    uint32_t whit = 0;           // colloids some entry of the wave is within cut-off of
    // colloids two at a time: forces and the reduction over the K entries
    // of each thread, then the wave trees of the six components (and, after
    // the last pair, of the potential) side by side
    constexpr int CB = 2;
    bool hit_any = false;        // some entry of this wave hit some colloid so far
    for (int c0 = 0; c0 < nc; c0 += CB) {
        double tv[3 * CB + 1];
        bool hit_chunk = false;  // ... one of this pair of colloids
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int c = c0 + cb;
            tv[3 * cb + 0] = 0.0; tv[3 * cb + 1] = 0.0; tv[3 * cb + 2] = 0.0;
            if (c >= nc || !((reach_mask >> c) & 1u)) continue;
            const double Xc0 = S.sXw[c][0], Xc1 = S.sXw[c][1], Xc2 = S.sXw[c][2];
            const double rc2 = S.cRc2[c], sig2 = S.cSig2[c];
            const double eA = S.cEpsA[c], eB = S.cEpsB[c];
            const bool cat = S.cCat[c] != 0;
            double gx[K], gy[K], gz[K];
            bool any = false;
            // distances for the K entries, then the WCA terms only if some
            // lane of the wave is inside this colloid's cut-off (wave-uniform
            // test); within it the K entries are evaluated branch-free with
            // selects, the untaken case at the cut-off radius (discarded)
            double dxs[K], dys[K], dzs[K], r2s[K];
            bool hit[K];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                dxs[j] = min_image((double)x[j][0] - Xc0, cc.L(0), cc.h(0));
                dys[j] = min_image((double)x[j][1] - Xc1, cc.L(1), cc.h(1));
                dzs[j] = min_image((double)x[j][2] - Xc2, cc.L(2), cc.h(2));
                r2s[j] = dot3(dxs[j], dys[j], dzs[j], dxs[j], dys[j], dzs[j]);
                hit[j] = valid[j] && (r2s[j] < rc2);
                any = any || hit[j];
                gx[j] = 0.0; gy[j] = 0.0; gz[j] = 0.0;
            }
            if (__ballot(any) != 0) {
                hit_chunk = true;
                whit |= 1u << c;
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    double coef, pot;
                    wca(hit[j] ? r2s[j] : rc2, sig2, (st[j] & 1) ? eB : eA, coef, pot);
                    const double ax = coef * dxs[j], ay = coef * dys[j], az = coef * dzs[j];
                    gx[j] = hit[j] ? ax : 0.0;
                    gy[j] = hit[j] ? ay : 0.0;
                    gz[j] = hit[j] ? az : 0.0;
                    f[j][0] = hit[j] ? f[j][0] + ax : f[j][0];
                    f[j][1] = hit[j] ? f[j][1] + ay : f[j][1];
                    f[j][2] = hit[j] ? f[j][2] + az : f[j][2];
                    u[j] = hit[j] ? u[j] + pot : u[j];
                    inside[j] = inside[j] || (hit[j] && cat);
                }
            }
            // the three components over this thread's K list positions
#pragma unroll
            for (int s2 = 1; s2 < K; s2 <<= 1)
#pragma unroll
                for (int j = 0; j + s2 < K; j += 2 * s2) {
                    gx[j] = gx[j] + gx[j + s2];
                    gy[j] = gy[j] + gy[j + s2];
                    gz[j] = gz[j] + gz[j + s2];
                }
            tv[3 * cb + 0] = gx[0]; tv[3 * cb + 1] = gy[0]; tv[3 * cb + 2] = gz[0];
        }
        const bool last = c0 + CB >= nc;
        tv[3 * CB] = 0.0;
        if (last) {
            double a[K];
#pragma unroll
            for (int j = 0; j < K; ++j) a[j] = u[j];
#pragma unroll
            for (int s2 = 1; s2 < K; s2 <<= 1)
#pragma unroll
                for (int j = 0; j + s2 < K; j += 2 * s2) a[j] = a[j] + a[j + s2];
            tv[3 * CB] = a[0];
        }
        hit_any = hit_any || hit_chunk;
        // no entry of the wave inside either colloid's cut-off (and, for the
        // potential, inside any): every value is +0.0, and so is its tree
        if (hit_chunk || (last && hit_any)) wave_tree_sum_n<3 * CB + 1>(tv);
        if (lane == 0) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int c = c0 + cb;
                if (c < nc) {
                    S.sRed[wave][3 * c + 0] = tv[3 * cb + 0];
                    S.sRed[wave][3 * c + 1] = tv[3 * cb + 1];
                    S.sRed[wave][3 * c + 2] = tv[3 * cb + 2];
                }
            }
            if (last) S.sRed[wave][3 * nc] = tv[3 * CB];
        }
    }
    if (nc == 0) {
        // no colloid: the potential of the list is zero (tree of zeros)
        if (lane == 0) S.sRed[wave][0] = 0.0;
    }
    if (lane == 0) S.sWhit[wave] = whit;
    __syncthreads();
    const int nv = 3 * nc + 1;
    constexpr int NW = NT / 64;
    if (t < nv) {
        double a[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) a[k] = S.sRed[k][t];
#pragma unroll
        for (int s = 1; s < NW; s <<= 1)
#pragma unroll
            for (int k = 0; k + s < NW; k += 2 * s) a[k] = a[k] + a[k + s];
        S.sNode[t] = a[0];
    }
    if (Gact > 1) {
        // Publish this workgroup's node values, each double as two 64-bit
        // words (low and high half, each with the barrier's epoch in its low
        // 32 bits), so that a reader accepts a word only when its epoch
        // matches and needs no separate flag or fence.  Epochs are unique per
        // barrier of the replica; the two buffers alternate between barriers.
        // Solo form: value v in planes 2v and 2v + 1, column g (every value).
        // Otherwise the packed row g of the master exchange (exchange_master).
        nbar++;
        const uint32_t epoch = epoch0 + nbar;
        const int64_t Gs = cc.G();
        const gptr<uint64_t> P = cc.part() + (int64_t)(nbar & 1) * cc.stride();
        uint32_t m = 0;
        if (t < nv || t == 0)
#pragma unroll
            for (int w2 = 0; w2 < NW; ++w2) m |= S.sWhit[w2];
        if (t < nv) {
            const double val = S.sNode[t];
            const uint64_t lo = ((uint64_t)(uint32_t)__double2loint(val) << 32) | epoch;
            const uint64_t hi = ((uint64_t)(uint32_t)__double2hiint(val) << 32) | epoch;
            int64_t o = -1;
            if (solo) {
                o = (int64_t)(2 * t) * Gs + g;          // planes 2t, 2t + 1 (all values)
            } else if (t == 3 * nc) {
                o = (int64_t)g * ROWW + 2;               // potential: slot 1
            } else if ((m >> (t / 3)) & 1u) {
                const int c = t / 3;
                o = (int64_t)g * ROWW + 2 * (2 + 3 * __popc(m & ((1u << c) - 1u)) + (t - 3 * c));
            }
            if (o >= 0) {
                __hip_atomic_store(&P[o], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&P[solo ? o + Gs : o + 1], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (t == 0 && !solo)
            __hip_atomic_store(&P[(int64_t)g * ROWW], ((uint64_t)m << 32) | epoch, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Colloids within reach of this wave for an interval: the bounding box of
// the wave's entries at its start (minimum-image offsets from its first
// entry, which is valid whenever any is) against each colloid's sphere of
// the cut-off plus the reach margin (me plus half the skin, cCull2), one lane
// per colloid.  Systems of one or two colloids test them all.
template <class T, int K, int NT, int NB>
__device__ __forceinline__ uint32_t reach_box(const ChainCtx<NT, NB>& S, const ChainConst& cc, int nc,
                                              const bool* valid, const T (*x)[3])
{
    const int lane = threadIdx.x & 63;
    uint32_t mask = nc >= 32 ? 0xffffffffu : ((1u << nc) - 1u);
    if (nc <= 2) return mask;
    double ref[3], lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ref[d] = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint((double)x[0][d])),
                                  __builtin_amdgcn_readfirstlane(__double2loint((double)x[0][d])));
        lo[d] = 1e300; hi[d] = -1e300;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (valid[j]) {
                const double o = min_image((double)x[j][d] - ref[d], cc.L(d), cc.h(d));
                lo[d] = o < lo[d] ? o : lo[d];
                hi[d] = o > hi[d] ? o : hi[d];
            }
        wave_min_max(lo[d], hi[d]);
    }
    bool near = true;
    if (lane < nc) {
        double r2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (!(hi[d] - lo[d] < cc.h(d))) continue;          // wide (or no entry): no bound
            const double oc = min_image(S.sXw[lane][d] - ref[d], cc.L(d), cc.h(d));
            double dd = 1e300;
#pragma unroll
            for (int img = -1; img <= 1; ++img) {
                const double ci = oc + (double)img * cc.L(d);
                double e = lo[d] - ci > ci - hi[d] ? lo[d] - ci : ci - hi[d];
                e = e > 0.0 ? e : 0.0;
                dd = e < dd ? e : dd;
            }
            r2 += dd * dd;
        }
        // margin far above the rounding of the entries' own r^2
        near = r2 <= S.cCull2[lane] * (1.0 + 1e-9) + 1e-9;
    }
    return mask & (uint32_t)__ballot(near);
}

// Exchange through a master workgroup (workgroup 0), used when the solo
// form does not apply.  Every workgroup publishes a packed row: the header
// (the mask of the colloids some entry of the workgroup was within cut-off
// of, and the barrier's epoch), the potential, then the three components
// of each listed colloid in ascending order, each double as two 64-bit
// words tagged with the epoch.  The node value of an unlisted colloid is
// exactly +0.0 (a tree of zeros), so it is not sent.  The master reads the
// rows in slots of two words (slot 0 the header, 1 the potential, 2 + 3j + d
// component d of the j-th listed colloid), a fixed group of NT / XTAB_R
// threads per row, expecting the colloids each row listed at the last look
// (sE); a round is repeated until every header is current and lists what
// was expected and every slot read is current.  The values go into a table
// by row and value; each value is then summed over the rows in the balanced
// binary tree (the wave w of NW takes a block of rows, the blocks pairwise),
// an entry the final round did not list counting as +0.0.  The master alone
// then updates the colloids and broadcasts their positions (broadcast_images
// / await_images).
constexpr int XSLOTS = 4;      // slots per thread and batch of the master's reads

__device__ __forceinline__ int nth_bit(uint32_t m, int j)
{
    for (int i = 0; i < j; ++i) m &= m - 1u;
    return __ffs(m) - 1;
}

// Balanced binary tree over N (a power of two) values get(0..N-1), formed
// in one pass as a binary counter: the partial sum of each complete block of
// 2^k values is kept until its sibling block is complete.
template <int N, class F>
__device__ __forceinline__ double tree_sum(F get)
{
    constexpr int LG = N <= 1 ? 0 : N <= 2 ? 1 : N <= 4 ? 2 : N <= 8 ? 3 : N <= 16 ? 4 : N <= 32 ? 5 : N <= 64 ? 6 : 7;
    static_assert((1 << LG) == N, "a power of two up to 128");
    double st[LG + 1];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double c = get(r);
        int lvl = 0;
#pragma unroll
        for (int b = 1; b < N; b <<= 1) {
            if (!(r & b)) break;
            c = st[lvl] + c;
            ++lvl;
        }
        st[lvl] = c;
    }
    return st[LG];
}

template <int NT, int NB>
__device__ __forceinline__ void exchange_master(ChainCtx<NT, NB>& S, const ChainConst& cc, int nc, int Gact,
                                                uint32_t nbar, uint32_t epoch0)
{
    constexpr int NW = NT / 64;
    constexpr int TPR = NT / XTAB_R;          // threads per row
    constexpr int RB = XTAB_R / NW;           // rows per wave in the trees
    constexpr int XV = ChainCtx<NT, NB>::XV;  // values per table chunk
    static_assert(TPR >= 1 && (64 % TPR) == 0 && RB >= 1, "row groups within a wave");
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t epoch = epoch0 + nbar;
    const gptr<const uint64_t> P = cc.part() + (int64_t)(nbar & 1) * cc.stride();
    const int nv = 3 * nc + 1;
    const uint64_t t_start = wall_clock64();
    const int rt = t / TPR, sub = t - rt * TPR;   // this thread's row of the chunk, place in its group
    // passes over chunks of XV values and of XTAB_R rows of the table
    for (int v0 = 0; v0 < nv; v0 += XV)
        for (int r0 = 0; r0 < Gact; r0 += XTAB_R) {
            const int nr = Gact - r0 < XTAB_R ? Gact - r0 : XTAB_R;
            const bool rv = rt < nr;
            const gptr<const uint64_t> row = P + (int64_t)(r0 + (rv ? rt : 0)) * ROWW;
            int nap = 0;
            while (true) {
                __asm__ __volatile__("" ::: "memory");
                const uint32_t e = rv ? S.sE[r0 + rt] : 0u;
                const int ns = rv ? 2 + 3 * __popc(e) : 0;       // slots of the row
                int ok = 1;
                uint32_t mnew = e;
                for (int s0 = sub; s0 < ns; s0 += XSLOTS * TPR) {
                    uint64_t wl[XSLOTS], wh[XSLOTS];
#pragma unroll
                    for (int k = 0; k < XSLOTS; ++k) {
                        const int sl = s0 + k * TPR;
                        wl[k] = wh[k] = 0ull;
                        if (sl < ns) {
                            // slot 0: the header word; slot s > 0: words 2s, 2s + 1
                            wl[k] = __hip_atomic_load(&row[sl == 0 ? 0 : 2 * sl], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                            if (sl > 0)
                                wh[k] = __hip_atomic_load(&row[2 * sl + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < XSLOTS; ++k) {
                        const int sl = s0 + k * TPR;
                        if (sl >= ns) continue;
                        if (sl == 0) {
                            const bool cur = (uint32_t)wl[k] == epoch;
                            const uint32_t m = (uint32_t)(wl[k] >> 32);
                            ok &= (cur && m == e) ? 1 : 0;
                            if (cur) mnew = m;
                            continue;
                        }
                        ok &= ((uint32_t)wl[k] == epoch && (uint32_t)wh[k] == epoch) ? 1 : 0;
                        // value index of the slot
                        int v = 3 * nc;
                        if (sl >= 2) {
                            const int j = (sl - 2) / 3, d = (sl - 2) - 3 * j;
                            v = 3 * nth_bit(e, j) + d;
                        }
                        if (v >= v0 && v < v0 + XV)
                            S.sTab[rt][v - v0] = __hiloint2double((int)(wh[k] >> 32), (int)(wl[k] >> 32));
                    }
                }
                // the row's header thread: look for the listed colloids next
                // round (the row's threads share a wave, so every one of them
                // read e above)
                if (rv && sub == 0 && mnew != e) S.sE[r0 + rt] = mnew;
                if (__syncthreads_and(ok)) break;
                // the time budget, decided for the workgroup by thread 0; once
                // given up (RMP_FLAG_BARRIER) later barriers do not wait
                if (t == 0 && !(S.sflags & RMP_FLAG_BARRIER) && wall_clock64() - t_start > cc.budget())
                    atomicOr(&S.sflags, RMP_FLAG_BARRIER);
                __syncthreads();
                if (S.sflags & RMP_FLAG_BARRIER) break;
                if (++nap > 16) __builtin_amdgcn_s_sleep(2);
            }
            // trees: lane l the value v0 + l; wave w the rows [w RB, (w + 1) RB)
            // of the chunk, then wave 0 the NW blocks pairwise.  An entry of a
            // row past Gact, or of a colloid the row did not list, is +0.0.
            const int nvc = nv - v0 < XV ? nv - v0 : XV;
            if (lane < nvc) {
                const int v = v0 + lane;
                const bool isU = v == 3 * nc;
                const int c = v / 3;
                const int rb = wave * RB;
                const double part = tree_sum<RB>([&](int q) {
                    const int r = rb + q;
                    const bool listed = r < nr && (isU || ((S.sE[r0 + r] >> c) & 1u) != 0u);
                    return listed ? S.sTab[r][lane] : 0.0;
                });
                S.sPart[wave][lane] = part;
            }
            __syncthreads();
            if (wave == 0 && lane < nvc) {
                const double tot = tree_sum<NW>([&](int w) { return S.sPart[w][lane]; });
                S.sNode[v0 + lane] = r0 == 0 ? tot : S.sNode[v0 + lane] + tot;
            }
            // the next chunk rewrites the table only after every wave has read it
            __syncthreads();
        }
}

// Master: the colloid positions of the coming MD step (their images, as in
// sXw) for the other workgroups, each double as two words tagged with the
// barrier's epoch, then the flag word (sFull << 32 | epoch).  Wave 0.
template <int NT, int NB>
__device__ __forceinline__ void broadcast_images(ChainCtx<NT, NB>& S, const ChainConst& cc, int nc, uint32_t nbar,
                                                 uint32_t epoch0)
{
    const int lane = threadIdx.x & 63;
    const uint32_t epoch = epoch0 + nbar;
    const gptr<uint64_t> B = cc.part() + (int64_t)(nbar & 1) * cc.stride() + cc.G() * (int64_t)ROWW;
    for (int k = lane; k < 3 * nc; k += 64) {
        const double val = S.sXw[k / 3][k % 3];
        const uint64_t lo = ((uint64_t)(uint32_t)__double2loint(val) << 32) | epoch;
        const uint64_t hi = ((uint64_t)(uint32_t)__double2hiint(val) << 32) | epoch;
        __hip_atomic_store(&B[2 * k], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&B[2 * k + 1], hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0)
        __hip_atomic_store(&B[6 * nc], ((uint64_t)S.sFull << 32) | epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Other workgroups: wait (bounded) for the master's positions of the coming
// MD step into sXw and sFull.  Wave 0: lane 0 polls the flag word, then the
// wave reads the positions (read again if a word is not yet current).
template <int NT, int NB>
__device__ __forceinline__ void await_images(ChainCtx<NT, NB>& S, const ChainConst& cc, int nc, uint32_t nbar,
                                             uint32_t epoch0)
{
    const int lane = threadIdx.x & 63;
    const uint32_t epoch = epoch0 + nbar;
    const gptr<const uint64_t> B = cc.part() + (int64_t)(nbar & 1) * cc.stride() + cc.G() * (int64_t)ROWW;
    const uint64_t t_start = wall_clock64();
    int nap = 0;
    uint64_t fw = 0;
    bool gave_up = (__hip_atomic_load(&S.sflags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) &
                    RMP_FLAG_BARRIER) != 0;
    while (!gave_up) {
        __asm__ __volatile__("" ::: "memory");
        uint64_t f = 0;
        if (lane == 0) f = __hip_atomic_load(&B[6 * nc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        fw = __shfl(f, 0, 64);
        if ((uint32_t)fw == epoch) break;
        if (wall_clock64() - t_start > cc.budget()) {
            if (lane == 0) atomicOr(&S.sflags, RMP_FLAG_BARRIER);
            gave_up = true;
            break;
        }
        if (++nap > 16) __builtin_amdgcn_s_sleep(2);
    }
    while (!gave_up) {
        // every round loads anew (no load of the words may be carried over
        // from an earlier round)
        __asm__ __volatile__("" ::: "memory");
        bool good = true;
        for (int k = lane; k < 3 * nc; k += 64) {
            const uint64_t lo = __hip_atomic_load(&B[2 * k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t hi = __hip_atomic_load(&B[2 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            good = good && (uint32_t)lo == epoch && (uint32_t)hi == epoch;
            S.sXw[k / 3][k % 3] = __hiloint2double((int)(hi >> 32), (int)(lo >> 32));
        }
        if (__ballot(!good) == 0) break;
        if (wall_clock64() - t_start > cc.budget()) {
            if (lane == 0) atomicOr(&S.sflags, RMP_FLAG_BARRIER);
            break;
        }
    }
    if (lane == 0 && (fw >> 32) != 0) S.sFull = 1u;
}

// Wait (bounded) for the exchange words of values v = v0 + vb*vs (vb < VB,
// v < nv) of workgroups [0, Gact) at this barrier, then reduce each value
// over the workgroups with the fixed tree: lane l holds workgroups
// [l*Q, l*Q+Q) (Q <= QM), summed pairwise, then the wave tree, padded with
// zeros to a power of two.  out[vb] is the same in every lane.  Only slots
// that exist are loaded (wave-uniform guards): a co-resident workgroup that
// is still computing must not be starved by polling traffic.
template <int VB, int QM, class Ctx>
__device__ __forceinline__ void poll_reduce(Ctx& S, gptr<const uint64_t> part, int64_t Gs, int v0, int vs, int nv,
                                            int Gact, int Q, uint32_t epoch, uint64_t budget, double (&out)[VB])
{
    const int lane = threadIdx.x & 63;
    double b4[VB][QM];
    // once this workgroup has given up on one barrier (RMP_FLAG_BARRIER) it
    // does not wait on later ones, so a kernel whose peers cannot all run
    // ends within about one time budget (wall_clock64 counts at 100 MHz)
    const uint64_t t_start = wall_clock64();
    int nap = 0;
    while (true) {
        // every round loads anew
        __asm__ __volatile__("" ::: "memory");
        uint64_t wl[VB][QM], wh[VB][QM];
#pragma unroll
        for (int vb = 0; vb < VB; ++vb) {
            const int v = v0 + vb * vs;
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int gg = lane * Q + q;
                const int gc = gg < Gact ? gg : 0;
                const int64_t o = (int64_t)(2 * v) * Gs + gc;
                if (v < nv && q < Q) {
                    wl[vb][q] = __hip_atomic_load(&part[o], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    wh[vb][q] = __hip_atomic_load(&part[o + Gs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    wl[vb][q] = 0;
                    wh[vb][q] = 0;
                }
            }
        }
        bool ok = true;
#pragma unroll
        for (int vb = 0; vb < VB; ++vb) {
            const int v = v0 + vb * vs;
#pragma unroll
            for (int q = 0; q < QM; ++q) {
                const int gg = lane * Q + q;
                const bool use = v < nv && q < Q && gg < Gact;
                const bool good = ((uint32_t)wl[vb][q] == epoch) & ((uint32_t)wh[vb][q] == epoch);
                ok = ok & (!use | good);
                b4[vb][q] = use ? __hiloint2double((int)(wh[vb][q] >> 32), (int)(wl[vb][q] >> 32)) : 0.0;
            }
        }
        if (__ballot(!ok) == 0) break;
        if (__hip_atomic_load(&S.sflags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) & RMP_FLAG_BARRIER)
            break;
        if (wall_clock64() - t_start > budget) {
            if (lane == 0) atomicOr(&S.sflags, RMP_FLAG_BARRIER);
            break;
        }
        // a long wait backs off (128 clocks a round after the first 16)
        if (++nap > 16) __builtin_amdgcn_s_sleep(2);
    }
#pragma unroll
    for (int vb = 0; vb < VB; ++vb) {
        double a2 = b4[vb][0];
        if (QM >= 2 && Q == 2) a2 = b4[vb][0] + b4[vb][QM >= 2 ? 1 : 0];
        if (QM >= 4 && Q == 4)
            a2 = (b4[vb][0] + b4[vb][QM >= 4 ? 1 : 0]) + (b4[vb][QM >= 4 ? 2 : 0] + b4[vb][QM >= 4 ? 3 : 0]);
        out[vb] = a2;
    }
    wave_tree_sum_n<VB>(out);
}

// Second half: wait for the other workgroups' node values of this
// evaluation, finish the tree over workgroups, then the colloid forces
// (solvent part, then colloid-colloid pairs in (a<b) order) into cF of
// thread c (c < nc) and, when requested, the potential into sU.  With at
// most 8 values and 64 workgroups (one workgroup per lane) wave 0 does all
// of it alone (the solo form: it reads every value of every row) and the
// other waves go straight on; otherwise the whole workgroup takes part in
// the sparse exchange.
// Constants of the colloid of lane c (c < nc) used by the pair forces,
// loaded once per interval
struct PairLane {
    uint32_t same;             // bit a set: colloid a is in this colloid's rigid body (no force)
    int ctype;
    double sigma;
};

template <class T, int K, int NT, int NB>
__device__ __forceinline__ void chain_collect(ChainCtx<NT, NB>& S, const ChainConst& cc, const ColloidParams* cp,
                              int nc, int g, int Gact, int Gpad, uint32_t nbar, uint32_t epoch0,
                              bool want_potential, double (&cF)[3], const PairLane& PL)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nv = 3 * nc + 1;
    const int Q = Gpad > 64 ? Gpad / 64 : 1;
    const bool solo = Q == 1 && nv <= 8;
    if (solo && wave != 0) return;
    if constexpr (NB > 1) {
        // colloid-colloid pair forces (a < b, enumerated row by row), one
        // thread per pair, and the mask of the interacting pairs of each
        // colloid (cleared with the colloid position update)
        const int np = nc * (nc - 1) / 2;
        const int ps = solo ? 64 : NT;
        for (int p = t; p < np; p += ps) {
            int a = 0, rem = p;
            while (rem >= nc - 1 - a) { rem -= nc - 1 - a; ++a; }
            const int b = a + 1 + rem;
            pair_force(S, cc, cp, a, b, S.sPairF[p], S.sPairOn[p]);
            if (S.sPairOn[p]) {
                atomicOr(&S.sPairMask[a], 1u << b);
                atomicOr(&S.sPairMask[b], 1u << a);
            }
        }
    }
    if (Gact > 1) {
        if (solo) {
            const uint32_t epoch = epoch0 + nbar;
            const gptr<const uint64_t> part = cc.part() + (int64_t)(nbar & 1) * cc.stride();
            double out[8];
            poll_reduce<8, 1>(S, part, cc.G(), 0, 1, nv, Gact, 1, epoch, cc.budget(), out);
            if (lane == 0)
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    if (v < nv) S.sNode[v] = out[v];
        } else {
            exchange_master(S, cc, nc, Gact, nbar, epoch0);
        }
    }
    if (solo) wave_sync();
    else __syncthreads();
    // colloid forces: solvent part, then colloid-colloid pairs in (a<b) order
    if constexpr (NB > 1) {
        // pairs from LDS: colloid c adds those that interact in the order of
        // the other colloid, + for the lower index
        if (t < nc) {
            const int c = t;
            double F[3] = {-S.sNode[3 * c + 0], -S.sNode[3 * c + 1], -S.sNode[3 * c + 2]};
            uint32_t m = S.sPairMask[c];
            while (m) {
                const int a = __ffs(m) - 1;
                m &= m - 1u;
                const bool c_lo = c < a;
                const int lo = c_lo ? c : a, hi = c_lo ? a : c;
                const int p = lo * nc - (lo * (lo + 1)) / 2 + (hi - lo - 1);
                for (int d = 0; d < 3; ++d) F[d] = c_lo ? F[d] + S.sPairF[p][d] : F[d] - S.sPairF[p][d];
            }
            for (int d = 0; d < 3; ++d) cF[d] = F[d];
        }
        if (t == 0 && want_potential) {
            double ucc = 0.0;
            const int np = nc * (nc - 1) / 2;
            for (int p = 0; p < np; ++p)
                if (S.sPairOn[p]) ucc = ucc + S.sPairF[p][3];
            S.sU = S.sNode[3 * nc] + ucc;
        }
        return;
    }
    if (t < nc) {
        const int c = t;
        double F[3] = {-S.sNode[3 * c + 0], -S.sNode[3 * c + 1], -S.sNode[3 * c + 2]};
        for (int a = 0; a < nc; ++a) {
            if ((PL.same >> a) & 1u) continue;      // itself or its own rigid body
            // colloid a's constants by its (uniform) index, this lane's from
            // registers; operands in the pair's (lo, hi) order
            const double sig_a = S.cSigma[a];
            const int ct_a = S.cType[a];
            const bool c_lo = c < a;
            const int lo = c_lo ? c : a, hi = c_lo ? a : c;
            double dx = min_image(S.sXw[lo][0] - S.sXw[hi][0], cc.L(0), cc.h(0));
            double dy = min_image(S.sXw[lo][1] - S.sXw[hi][1], cc.L(1), cc.h(1));
            double dz = min_image(S.sXw[lo][2] - S.sXw[hi][2], cc.L(2), cc.h(2));
            double r2 = dot3(dx, dy, dz, dx, dy, dz);
            double sab = c_lo ? PL.sigma + sig_a : sig_a + PL.sigma;
            double rc = 0x1.1f59ac3c7d6c0p+0 * sab;
            if (r2 < rc * rc) {
                const int t_lo = c_lo ? PL.ctype : ct_a, t_hi = c_lo ? ct_a : PL.ctype;
                const double e_lo0 = t_lo == 0 ? cp->eps_cc[0][0] : cp->eps_cc[1][0];
                const double e_lo1 = t_lo == 0 ? cp->eps_cc[0][1] : cp->eps_cc[1][1];
                double coef, pot;
                wca(r2, sab * sab, t_hi == 0 ? e_lo0 : e_lo1, coef, pot);
                double g3[3] = {coef * dx, coef * dy, coef * dz};
                for (int d = 0; d < 3; ++d) F[d] = c_lo ? F[d] + g3[d] : F[d] - g3[d];
            }
        }
        for (int d = 0; d < 3; ++d) cF[d] = F[d];
    }
    if (t == 0 && want_potential) {
        double ucc = 0.0;
        for (int a = 0; a < nc; ++a)
            for (int b = a + 1; b < nc; ++b) {
                if (cp->body[a] == cp->body[b]) continue;
                double dx = min_image(S.sXw[a][0] - S.sXw[b][0], cc.L(0), cc.h(0));
                double dy = min_image(S.sXw[a][1] - S.sXw[b][1], cc.L(1), cc.h(1));
                double dz = min_image(S.sXw[a][2] - S.sXw[b][2], cc.L(2), cc.h(2));
                double r2 = dot3(dx, dy, dz, dx, dy, dz);
                double sab = cp->sigma[a] + cp->sigma[b];
                double rc = 0x1.1f59ac3c7d6c0p+0 * sab;
                if (r2 < rc * rc) {
                    double coef, pot;
                    wca(r2, sab * sab, cp->eps_cc[cp->ctype[a]][cp->ctype[b]], coef, pot);
                    ucc = ucc + pot;
                }
            }
        S.sU = S.sNode[3 * nc] + ucc;
    }
    // no barrier here: the node values and colloid images are next written
    // after the workgroup barrier that follows the colloid position update
}

template <class T, int K, int NC, int NT>
__device__ __forceinline__ void chain_body(Work w, int g, const RepDesc& D, const ChainConst& cc)
{
    if (!D.active) return;
    RepState* rs = D.rs;
    const ColloidParams* cp = D.cp;
    // NC > 0: every system of the launch has NC colloids (loops over the
    // colloids unrolled at compile time); NC == 0: read per system
    const int nc = NC > 0 ? NC : cp->nc;
    constexpr int B = NT * K;
    int64_t ncand = rs->n_cand;
    if (ncand > D.cand_cap) ncand = D.cand_cap;
    int Gact = (int)((ncand + B - 1) / B);
    if (Gact < 1) Gact = 1;
    if (Gact > D.G) Gact = D.G;
    if (g >= Gact) return;
    if (nc == 0 && ncand == 0) {
        // no colloid and an empty list (flows, bare solvent): nothing moves
        // in the chain; close the interval's counters as the full path would
        if (g == 0 && threadIdx.x == 0) {
            D.epart[0] = 0.0;
            D.epart[1] = 0.0;
            rs->U = 0.0;
            rs->md_step = rs->md_step + D.n_md;
            rs->n_cand_used = 0;
        }
        return;
    }
    int Gpad = 1;
    while (Gpad < Gact) Gpad <<= 1;

    __shared__ ChainCtx<NT, NC == 0 ? RMP_MAX_BONDS : 1> S;
    const int t = threadIdx.x;
    if (t == 0) {
        S.sflags = 0;
        S.sFull = 0;
    }
    if (t < MAXC) S.sPairMask[t] = 0u;
    for (int r = t; r < MAX_CHAIN_G; r += NT) S.sE[r] = 0u;
    if (t < 4) S.cEcc[t >> 1][t & 1] = cp->eps_cc[t >> 1][t & 1];
    // colloid c lives in registers of thread c (c < nc, wave 0): position,
    // velocity, force, position at the start of the interval
    double cX[3] = {0.0, 0.0, 0.0}, cV[3] = {0.0, 0.0, 0.0}, cF[3] = {0.0, 0.0, 0.0};
    double cX0[3] = {0.0, 0.0, 0.0};
    const BondLane BL = bond_lane(cp, nc);
    // iterative RATTLE (bond networks, or asked for): generic variant only,
    // the host launches it whenever a system of the launch needs it
    const bool iter = NC == 0 && cp->iterative != 0;
    PairLane PL;
    PL.same = 0u;
    if (t < nc)
        for (int a = 0; a < nc; ++a)
            if (cp->body[a] == cp->body[t]) PL.same |= 1u << a;
    PL.ctype = t < nc ? cp->ctype[t] : 0;
    PL.sigma = t < nc ? cp->sigma[t] : 0.0;
    const double chc = t < nc ? cp->hc[t] : 0.0;
    if (t < nc) {
        for (int d = 0; d < 3; ++d) {
            cX[d] = rs->X[t][d];
            cV[d] = rs->V[t][d];
            cX0[d] = cX[d];
            S.sXw[t][d] = colloid_image(cX[d], cc.L(d));
        }
        S.cRc2[t] = cp->rc2[t];
        {
            const double rr = sqrt(cp->rc2[t]) + D.cull_margin;
            S.cCull2[t] = rr * rr;
        }
        S.cSig2[t] = cp->sig2[t];
        S.cEpsA[t] = cp->epsA[t];
        S.cEpsB[t] = cp->epsB[t];
        S.cSigma[t] = cp->sigma[t];
        S.cCat[t] = cp->catalytic[t];
        S.cType[t] = cp->ctype[t];
        S.cBody[t] = cp->body[t];
    }
    if (iter) {
        // bonds of the iterative RATTLE in LDS for the interval
        const double tol = cp->rattle_tol;
        for (int q = t; q < cp->nbonds; q += NT) {
            const int a = cp->bond_a[q], b = cp->bond_b[q];
            const double dd2 = cp->bond_d[q] * cp->bond_d[q];
            const double ima = cp->imass[a], imb = cp->imass[b];
            const double mu = ima + imb;
            S.sBa[q] = a;
            S.sBb[q] = b;
            S.sBd2[q] = dd2;
            S.sBthr[q] = (2.0 * tol) * dd2;
            S.sBthv[q] = (tol * dd2) / D.dt;
            S.sBmu2[q] = 2.0 * mu;
            S.sBmud[q] = mu * dd2;
            S.sBia[q] = ima;
            S.sBib[q] = imb;
        }
        for (int L = t; L <= cp->n_layers; L += NT) S.sLay[L] = cp->layer_start[L];
    }
    const int64_t coll = rs->coll_step;
    const int cur = (int)(coll & 1);
    const int64_t md0 = rs->md_step;
    const int nmd = D.n_md;
    const int64_t n = D.n;
    const gptr<T> xb[3] = {G(comp<T>(D.x[cur], n, 0)), G(comp<T>(D.x[cur], n, 1)), G(comp<T>(D.x[cur], n, 2))};
    const gptr<T> vb[3] = {G(comp<T>(D.v[cur], n, 0)), G(comp<T>(D.v[cur], n, 1)), G(comp<T>(D.v[cur], n, 2))};
    const gptr<uint8_t> stb = G(D.st[cur]);
    const gptr<const uint32_t> idb = G(D.id[cur]);
    const gptr<const uint32_t> cand = G(D.cand_idx);

    bool valid[K];
    int64_t idx[K];
    T x[K][3], v[K][3], x0[K][3];
    double f[K][3];
    uint8_t st[K];
    uint32_t pid[K];
    bool inside[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        int64_t pos = (int64_t)g * B + (int64_t)t * K + j;
        valid[j] = pos < ncand;
        idx[j] = valid[j] ? (int64_t)cand[pos] : 0;
        for (int d = 0; d < 3; ++d) {
            x[j][d] = valid[j] ? xb[d][idx[j]] : (T)0;
            v[j][d] = valid[j] ? vb[d][idx[j]] : (T)0;
        }
        st[j] = valid[j] ? stb[idx[j]] : 0;
        pid[j] = valid[j] ? idb[idx[j]] : 0;
        for (int d = 0; d < 3; ++d) x0[j][d] = x[j][d];
    }
    __syncthreads();
    // this wave's colloids within reach for the interval
    uint32_t wmask = reach_box<T, K>(S, cc, nc, valid, x);
    const double me2 = D.cull_me * D.cull_me;
    // Roles: with one workgroup, or in the solo form, every workgroup
    // completes the exchange and updates the colloids itself; otherwise
    // workgroup 0 (the master) does, and the others take the colloid
    // positions of each MD step from its broadcast.
    const int Qx = Gpad > 64 ? Gpad / 64 : 1;
    const bool solo = Qx == 1 && 3 * nc + 1 <= 8;
    const bool worker = Gact > 1 && !solo && g != 0;
    const bool updates = !worker;
    uint32_t nbar = 0;
    // barrier epochs: unique per barrier of the replica between list
    // rebuilds (md_step + coll_step grows by n_md + 1 per interval)
    const uint32_t epoch0 = (uint32_t)(md0 + coll);
    const double dt = D.dt;
    const T dtT = (T)dt, hT = (T)D.h;
    const T Lt[3] = {(T)cc.L(0), (T)cc.L(1), (T)cc.L(2)};
    const bool colloid_wave = t < 64;

    // forces at the start of the interval
    chain_compute<T, K, NT>(S, cc, cp, nc, valid, x, x0, st, f, inside, g, Gact, solo, wmask, me2, nbar, epoch0);
    if (updates) chain_collect<T, K, NT>(S, cc, cp, nc, g, Gact, Gpad, nbar, epoch0, false, cF, PL);
    // list entries: first half kick and drift of step 0
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            v[j][d] = tfma(hT, (T)f[j][d], v[j][d]);
            x[j][d] = wrap_coord<T>(tfma(dtT, v[j][d], x[j][d]), Lt[d]);
        }

    double eu = 0.0, ef = 0.0;
    for (int step = 0; step < nmd; ++step) {
        const int64_t md = md0 + step;
        // colloids (wave 0, in registers): half kick, drift, RATTLE
        // position stage, periodic images for the force evaluation
        if (worker) {
            if (colloid_wave) await_images(S, cc, nc, nbar, epoch0);
        } else if (colloid_wave) {
            double cXo[3];
            if (t < nc) {
                for (int d = 0; d < 3; ++d) {
                    cV[d] = fma(chc, cF[d], cV[d]);
                    cXo[d] = cX[d];
                    cX[d] = fma(dt, cV[d], cX[d]);
                }
            } else {
                for (int d = 0; d < 3; ++d) cXo[d] = cX[d];
            }
            uint32_t lflags = 0;
            if (iter) {
                // bond network: wave 0 sweeps over the bonds on the
                // colloid state staged in LDS
                if (t < nc)
                    for (int d = 0; d < 3; ++d) {
                        S.sXc[t][d] = cX[d];
                        S.sVc[t][d] = cV[d];
                        S.sXoc[t][d] = cXo[d];
                    }
                wave_sync();
                {
                    const uint32_t f = rattle_pos_iter(S, cp, dt);   // all lanes of wave 0
                    if (t == 0) lflags |= f;
                }
                wave_sync();
                if (t < nc)
                    for (int d = 0; d < 3; ++d) {
                        cX[d] = S.sXc[t][d];
                        cV[d] = S.sVc[t][d];
                    }
            } else {
                rattle_pos_lane(BL, dt, cX, cV, cXo, lflags);
            }
            if (lflags) atomicOr(&S.sflags, lflags);
            if (t < nc) {
                for (int d = 0; d < 3; ++d) S.sXw[t][d] = colloid_image(cX[d], cc.L(d));
                // a colloid beyond half the skin from its interval-start
                // position voids the reach masks of the interval
                const double dx = cX[0] - cX0[0], dy = cX[1] - cX0[1], dz = cX[2] - cX0[2];
                if (dot3(dx, dy, dz, dx, dy, dz) >= D.skin_half2) S.sFull = 1u;
                S.sPairMask[t] = 0u;
            }
            if (Gact > 1 && !solo) {
                wave_sync();
                broadcast_images(S, cc, nc, nbar, epoch0);
            }
        }
        __syncthreads();
        chain_compute<T, K, NT>(S, cc, cp, nc, valid, x, x0, st, f, inside, g, Gact, solo, wmask, me2, nbar,
                                epoch0);
        // while the other workgroups' sums arrive: the list entries' second
        // half kick, catalysis, and (except after the last step) the next
        // step's first half kick and drift -- each entry's own arithmetic,
        // in the same order as a step-by-step update
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int d = 0; d < 3; ++d) v[j][d] = tfma(hT, (T)f[j][d], v[j][d]);
        // catalysis: A inside a catalytic sphere is flagged; a flagged A
        // outside all of them converts to B with probability cat_prob
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!valid[j]) continue;
            uint8_t s = st[j];
            if (s & 1) continue;
            if (inside[j]) {
                st[j] = (uint8_t)(s | 2);
            } else if (s & 2) {
                bool flip = true;
                if (cc.cat_prob() < 1.0) {
                    uint64_t wv[4];
                    philox((uint64_t)md, pid[j], 0, cc.seed(), TAG_CAT, wv);
                    flip = u01(wv[0]) < cc.cat_prob();
                }
                if (flip) {
                    st[j] = 1;
                    ef += 1.0;
                    eu += species_dU_lds(S, cc, nc, (double)x[j][0], (double)x[j][1], (double)x[j][2]);
                } else {
                    st[j] = 0;
                }
            }
        }
        if (step < nmd - 1) {
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    v[j][d] = tfma(hT, (T)f[j][d], v[j][d]);
                    x[j][d] = wrap_coord<T>(tfma(dtT, v[j][d], x[j][d]), Lt[d]);
                }
        }
        // the potential energy is an observable of the last force evaluation
        if (updates)
            chain_collect<T, K, NT>(S, cc, cp, nc, g, Gact, Gpad, nbar, epoch0, step == nmd - 1, cF, PL);
        // colloids (wave 0, in registers): second half kick, RATTLE
        // velocity stage, Verlet-list soundness check (displacement within
        // the interval)
        if (updates && colloid_wave) {
            if (t < nc)
                for (int d = 0; d < 3; ++d) cV[d] = fma(chc, cF[d], cV[d]);
            if (iter) {
                if (t < nc)
                    for (int d = 0; d < 3; ++d) {
                        S.sXc[t][d] = cX[d];
                        S.sVc[t][d] = cV[d];
                    }
                wave_sync();
                uint32_t vflags = 0;
                vflags = rattle_vel_iter(S, cp, dt);
                if (t != 0) vflags = 0;
                if (vflags) atomicOr(&S.sflags, vflags);
                wave_sync();
                if (t < nc)
                    for (int d = 0; d < 3; ++d) cV[d] = S.sVc[t][d];
            } else {
                rattle_vel_lane(BL, cX, cV);
            }
            if (t < nc) {
                double dx = cX[0] - cX0[0], dy = cX[1] - cX0[1], dz = cX[2] - cX0[2];
                if (dot3(dx, dy, dz, dx, dy, dz) >= D.skin_half2)
                    atomicOr(&S.sflags, RMP_FLAG_DISPLACEMENT);
            }
        }
    }
    __syncthreads();
    // write back list entries and bin them for the coming collision
    double s3[3];
    shift_of(D.seed, coll, s3);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!valid[j]) continue;
        const int64_t i = idx[j];
        for (int d = 0; d < 3; ++d) {
            xb[d][i] = x[j][d];
            vb[d][i] = v[j][d];
        }
        stb[i] = st[j];
        uint32_t key = cell_key(D, (double)x[j][0], (double)x[j][1], (double)x[j][2], s3);
        const uint32_t rank = __hip_atomic_fetch_add(G(D.count) + key, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        G(D.keyrank)[i] = ((uint64_t)key << 32) | rank;
    }
    // reaction bookkeeping of this workgroup (combined after the collision)
    __shared__ double sred[NT / 64 + 1];
    eu = block_sum<NT>(eu, sred);
    ef = block_sum<NT>(ef, sred);
    if (t == 0) {
        G(D.epart)[(int64_t)g * 2 + 0] = eu;
        G(D.epart)[(int64_t)g * 2 + 1] = ef;
        if (S.sflags) atomicOr(&rs->flags, S.sflags);
    }
    if (g == 0) {
        if (t < nc) {
            bool fin = true;
            for (int d = 0; d < 3; ++d) {
                rs->X[t][d] = cX[d];
                rs->V[t][d] = cV[d];
                rs->F[t][d] = cF[d];
                fin = fin && isfinite(cF[d]);
            }
            if (!fin) atomicOr(&rs->flags, RMP_FLAG_NONFINITE);
        }
        if (t == 0) {
            rs->U = S.sU;
            rs->md_step = md0 + nmd;
            rs->n_cand_used = ncand;
        }
    }
}

// Work-list position of a chain workgroup.  When every workgroup of the
// launch fits on the device at once it is blockIdx.  Otherwise (TICKET)
// workgroups take their positions in the order they start running, from a
// device counter: the workgroups of one system hold consecutive positions,
// so every system whose positions have all been taken is entirely resident
// and its exchange waits end, even though the launch runs in waves.  The
// last workgroup to finish puts the counters back to zero for the next
// launch.  (The ticket is a separate instantiation because an atomic at
// kernel entry keeps the descriptor loads of the whole kernel off the
// scalar unit.)
template <class T, int K, int NC, int NT>
__device__ __forceinline__ void chain_run(Work w, int item)
{
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int g = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    chain_body<T, K, NC, NT>(w, g, D, chain_const(D, w.budget));
}

template <class T, int K, bool TICKET, int NC, int NT>
__global__ __launch_bounds__(NT) void k_chain(Work w)
{
    // only in the one- and two-colloid variants: with the priority code in
    // the generic variant its 128^3 launches ran 10 % slower even with the
    // flag off
    if constexpr (NC == 1 || NC == 2)
        if (w.flags & WORK_CHAIN_PRIO) __builtin_amdgcn_s_setprio(3);
    if (!TICKET) {
        chain_run<T, K, NC, NT>(w, (int)blockIdx.x);
        return;
    }
    __shared__ int s_item;
    if (threadIdx.x == 0)
        s_item = (int)__hip_atomic_fetch_add(&w.tick[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    chain_run<T, K, NC, NT>(w, s_item);
    if (threadIdx.x == 0) {
        const uint32_t fin = __hip_atomic_fetch_add(&w.tick[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (fin == gridDim.x - 1) {
            __hip_atomic_store(&w.tick[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&w.tick[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------- cell scan

__global__ __launch_bounds__(1024) void k_scan_blocks(Work w)
{
    const int item = blockIdx.x;
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int blk = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active) return;
    __shared__ uint32_t sbuf[16];
    const int64_t c0 = (int64_t)blk * SCAN_BLK;
    uint32_t s = 0;
    for (int k = 0; k < SCAN_BLK / 1024; ++k) {
        int64_t c = c0 + (int64_t)threadIdx.x * (SCAN_BLK / 1024) + k;
        if (c < D.ncell) s += D.count[c];
    }
    uint32_t tot = block_sum_u32<1024>(s, sbuf);
    if (threadIdx.x == 0) D.scanblk[blk] = tot;
}

// `direct`: the launch's grids are small (at most SCAN_DIRECT_BLOCKS blocks
// each), so a block sums the counts of the blocks before it itself and no
// k_scan_blocks pass is launched.
__global__ __launch_bounds__(1024) void k_scan_final(Work w, int direct)
{
    const int item = blockIdx.x;
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int blk = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active) return;
    __shared__ uint32_t sbuf[16];
    uint32_t pre = 0;
    if (direct) {
        // counts of cells [0, blk * SCAN_BLK): 4 loads in flight per thread
        const int64_t m = (int64_t)blk * SCAN_BLK;
        for (int64_t c = threadIdx.x; c < m; c += 4 * 1024) {
            uint32_t q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = c + u * 1024 < m ? D.count[c + u * 1024] : 0u;
            pre += (q[0] + q[1]) + (q[2] + q[3]);
        }
    } else {
        for (int k = threadIdx.x; k < blk; k += 1024) pre += D.scanblk[k];
    }
    pre = block_sum_u32<1024>(pre, sbuf);
    constexpr int PER = SCAN_BLK / 1024;
    const int64_t c0 = (int64_t)blk * SCAN_BLK + (int64_t)threadIdx.x * PER;
    uint32_t cnt[PER];
    uint32_t loc = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int64_t c = c0 + k;
        cnt[k] = c < D.ncell ? D.count[c] : 0u;
        loc += cnt[k];
    }
    uint32_t total;
    uint32_t p = block_exscan_u32<1024>(loc, sbuf, &total) + pre;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int64_t c = c0 + k;
        if (c < D.ncell) {
            D.start[c] = p;
            p += cnt[k];
        }
    }
    if (blk == D.n_scanblk - 1 && threadIdx.x == 0) D.start[D.ncell] = pre + total;
}

// Particle records of the staging array (Rec<T>): packed and unpacked with
// the state byte split into the spare top bits of id and index in FP32.
__device__ __forceinline__ void rec_put(Rec<double>* r, const double (&x)[3], const double (&v)[3],
                                        uint32_t id, uint32_t idx, uint8_t st)
{
    Rec<double> q;
    q.x[0] = x[0]; q.x[1] = x[1]; q.x[2] = x[2];
    q.v[0] = v[0]; q.v[1] = v[1]; q.v[2] = v[2];
    q.id = id; q.idx = idx; q.st = st; q.pad = 0u;
    *r = q;
}
__device__ __forceinline__ void rec_put(Rec<float>* r, const float (&x)[3], const float (&v)[3],
                                        uint32_t id, uint32_t idx, uint8_t st)
{
    Rec<float> q;
    q.x[0] = x[0]; q.x[1] = x[1]; q.x[2] = x[2];
    q.v[0] = v[0]; q.v[1] = v[1]; q.v[2] = v[2];
    q.id_f = id | ((uint32_t)((st >> 1) & 1u) << 31);
    q.idx_s = idx | ((uint32_t)(st & 1u) << 31);
    *r = q;
}
template <class RP>
__device__ __forceinline__ void rec_get(RP r, double (&x)[3], double (&v)[3], uint32_t& id, uint32_t& idx,
                                        uint8_t& st)
{
    x[0] = r->x[0]; x[1] = r->x[1]; x[2] = r->x[2];
    v[0] = r->v[0]; v[1] = r->v[1]; v[2] = r->v[2];
    id = r->id; idx = r->idx; st = (uint8_t)r->st;
}
template <class RP>
__device__ __forceinline__ void rec_get(RP r, float (&x)[3], float (&v)[3], uint32_t& id, uint32_t& idx,
                                        uint8_t& st)
{
    x[0] = r->x[0]; x[1] = r->x[1]; x[2] = r->x[2];
    v[0] = r->v[0]; v[1] = r->v[1]; v[2] = r->v[2];
    const uint32_t id_f = r->id_f, idx_s = r->idx_s;
    id = id_f & 0x7fffffffu;
    idx = idx_s & 0x7fffffffu;
    st = (uint8_t)(((idx_s >> 31) & 1u) | (((id_f >> 31) & 1u) << 1));
}

// single fields of a record (the oversized-cell path reads them one by one)
__device__ __forceinline__ uint32_t rec_idx(const Rec<double>* r) { return r->idx; }
__device__ __forceinline__ uint32_t rec_idx(const Rec<float>* r) { return r->idx_s & 0x7fffffffu; }
__device__ __forceinline__ uint8_t rec_st(const Rec<double>* r) { return (uint8_t)r->st; }
__device__ __forceinline__ uint8_t rec_st(const Rec<float>* r)
{
    return (uint8_t)(((r->idx_s >> 31) & 1u) | (((r->id_f >> 31) & 1u) << 1));
}
__device__ __forceinline__ uint32_t rec_id(const Rec<double>* r) { return r->id; }
__device__ __forceinline__ uint32_t rec_id(const Rec<float>* r) { return r->id_f & 0x7fffffffu; }
template <class T>
__device__ __forceinline__ double rec_v(const Rec<T>* r, int d) { return (double)r->v[d]; }

// Counting-sort scatter: particle i (read in array order, coalesced) goes to
// slot start[key] + rank of the staging array as one whole record, so the
// collision reads each tile of cells as one contiguous run.
template <class T>
__global__ __launch_bounds__(256) void k_scatter(Work w)
{
    const int item = blockIdx.x;
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int chunk = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active) return;
    const int64_t n = D.n;
    const int cur = (int)(D.rs->coll_step & 1);
    const gptr<const T> xs[3] = {G(comp<T>(D.x[cur], n, 0)), G(comp<T>(D.x[cur], n, 1)),
                                 G(comp<T>(D.x[cur], n, 2))};
    const gptr<const T> vs[3] = {G(comp<T>(D.v[cur], n, 0)), G(comp<T>(D.v[cur], n, 1)),
                                 G(comp<T>(D.v[cur], n, 2))};
    const gptr<const uint32_t> ids = G(D.id[cur]);
    const gptr<const uint8_t> sts = G(D.st[cur]);
    const gptr<const uint64_t> keyrank = G(D.keyrank);
    const gptr<const uint32_t> start = G(D.start);
    const int64_t base = (int64_t)chunk * CHUNK;
    // the chunk's four particles per thread: every load before the stores
    constexpr int P = CHUNK / 256;
    constexpr int RW = (int)(sizeof(Rec<T>) / 16);
    int64_t ii[P];
    uint32_t key[P], rank[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
        ii[u] = base + u * 256 + threadIdx.x;
        const uint64_t kr = ii[u] < n ? keyrank[ii[u]] : 0ull;
        key[u] = (uint32_t)(kr >> 32);
        rank[u] = (uint32_t)kr;
    }
    int64_t slot[P];
#pragma unroll
    for (int u = 0; u < P; ++u) slot[u] = ii[u] < n ? (int64_t)start[key[u]] + rank[u] : n;
    T x[P][3], v[P][3];
    uint32_t idv[P];
    uint8_t stv[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const int64_t i = ii[u] < n ? ii[u] : 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) { x[u][d] = xs[d][i]; v[u][d] = vs[d][i]; }
        idv[u] = ids[i];
        stv[u] = sts[i];
    }
    // each record through LDS, then written by RW consecutive lanes (one
    // 16-byte word each), so a record leaves as one contiguous request
    __shared__ Rec<T> s_out[256];
    __shared__ int64_t s_slot[256];
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* s_out4 = reinterpret_cast<const u32x4*>(s_out);
    const gptr<u32x4> stage4 = G(reinterpret_cast<u32x4*>(D.stage));
#pragma unroll
    for (int u = 0; u < P; ++u) {
        if (u) __syncthreads();
        rec_put(&s_out[threadIdx.x], x[u], v[u], idv[u], (uint32_t)ii[u], stv[u]);
        s_slot[threadIdx.x] = (ii[u] < n && slot[u] < n) ? slot[u] : -1;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int k4 = q * 256 + (int)threadIdx.x;
            const int r = k4 / RW, part = k4 - r * RW;
            const int64_t sl = s_slot[r];
            if (sl >= 0) stage4[sl * RW + part] = s_out4[k4];
        }
    }
}

// ------------------------------------------------------------- collision

// Add the Verlet-list flags of the wave's particles to their chunks' counts.
// The particles of one collision group occupy slots [q0, q0 + ns) with
// ns <= CHUNK, so they span the chunks c_lo = q0 / CHUNK and c_lo + 1 at
// most: one atomic per chunk and wave.  All 64 lanes must call it.
__device__ __forceinline__ void count_flag(gptr<uint32_t> chunk_cnt, int64_t o, bool f, int64_t c_lo)
{
    const int64_t ch = o / CHUNK;
    const uint32_t n_lo = (uint32_t)__popcll(__ballot(f && ch == c_lo));
    const uint32_t n_hi = (uint32_t)__popcll(__ballot(f && ch != c_lo));
    if ((threadIdx.x & 63) == 0) {
        if (n_lo) g_add(chunk_cnt + c_lo, n_lo);
        if (n_hi) g_add(chunk_cnt + c_lo + 1, n_hi);
    }
}

// Verlet-list membership (as is_candidate) tested only against the colloids
// of `mask`: the others were found out of reach of every particle of the
// tile, so they cannot change the outcome.
__device__ __forceinline__ bool is_candidate_masked(const RepDesc& D, const ColloidParams* cp, uint32_t mask,
                                                    const double (*Xw)[3], uint8_t st,
                                                    double x0, double x1, double x2,
                                                    double v0, double v1, double v2)
{
    if (D.flow) return false;
    if (st & 2) return true;
    if (mask == 0) return false;
    const double vv = dot3(v0, v1, v2, v0, v1, v2);
    const double reach = sqrt(vv) * D.tau;
    for (uint32_t m = mask; m; m &= m - 1) {
        const int c = __ffs(m) - 1;
        double dx = min_image(x0 - Xw[c][0], D.Ld[0], D.halfL[0]);
        double dy = min_image(x1 - Xw[c][1], D.Ld[1], D.halfL[1]);
        double dz = min_image(x2 - Xw[c][2], D.Ld[2], D.halfL[2]);
        double r2 = dot3(dx, dy, dz, dx, dy, dz);
        double tt = cp->reachR[c] + reach;
        if (r2 < tt * tt) return true;
    }
    return false;
}

constexpr int COLL_TCMAX = 64;       // cells per tile at most

// One cell of the tile holding more particles than a collision group (rare:
// hundreds of particles in one cell).  Its records are contiguous in the
// staging array; the stable order is found by counting ranks of the old
// indices into scratch (the key/rank array is dead after the scatter), then
// the per-cell quantities by one thread in that order, then every particle.
template <class T, int RULE, int NT>
__device__ void collide_big_cell(const RepDesc& D, const ColloidParams* cp, int nc, const double (*s_Xw)[3],
                                 int64_t coll, int64_t cell, uint32_t q0, int nn,
                                 double* s_u, double* s_n, int32_t* s_flip,
                                 double& t_sum, double& t_cells, double& du_sum, double& n_flip)
{
    RepState* rs = D.rs;
    const int t = threadIdx.x;
    const int64_t n = D.n;
    const int cur = (int)(coll & 1), nxt = cur ^ 1;
    T* xn[3] = {comp<T>(D.x[nxt], n, 0), comp<T>(D.x[nxt], n, 1), comp<T>(D.x[nxt], n, 2)};
    T* vn[3] = {comp<T>(D.v[nxt], n, 0), comp<T>(D.v[nxt], n, 1), comp<T>(D.v[nxt], n, 2)};
    uint32_t* idn = D.id[nxt];
    uint8_t* stn = D.st[nxt];
    const Rec<T>* rec = reinterpret_cast<const Rec<T>*>(D.stage) + q0;
    const double ca = D.ca, sa = D.sa, oma = 1.0 - D.ca;
    uint32_t* srt = reinterpret_cast<uint32_t*>(D.keyrank) + q0;   // stable rank -> record
    for (int j = t; j < nn; j += NT) {
        const uint32_t pj = rec_idx(&rec[j]);
        int r = 0;
        for (int q = 0; q < nn; ++q) r += rec_idx(&rec[q]) < pj ? 1 : 0;
        srt[r] = (uint32_t)j;
    }
    __syncthreads();
    if (t == 0) {
        double S0 = 0.0, S1 = 0.0, S2 = 0.0;
        for (int k = 0; k < nn; ++k) {
            const Rec<T>* q = &rec[srt[k] < (uint32_t)nn ? srt[k] : 0u];
            S0 = S0 + rec_v(q, 0);
            S1 = S1 + rec_v(q, 1);
            S2 = S2 + rec_v(q, 2);
        }
        const double u0 = S0 / (double)nn, u1 = S1 / (double)nn, u2 = S2 / (double)nn;
        double tsum = 0.0, G0 = 0.0, G1 = 0.0, G2 = 0.0;
        int nB = 0;
        for (int k = 0; k < nn; ++k) {
            const Rec<T>* q = &rec[srt[k] < (uint32_t)nn ? srt[k] : 0u];
            double w0 = rec_v(q, 0) - u0, w1 = rec_v(q, 1) - u1, w2 = rec_v(q, 2) - u2;
            tsum = tsum + dot3(w0, w1, w2, w0, w1, w2);
            nB += rec_st(q) & 1;
            if constexpr (RULE == 1) {
                uint64_t wv[4]; double z[3];
                philox<true>((uint64_t)coll, rec_id(q), 0, D.seed, TAG_THERMO, wv);
                normals3(wv, z);
                G0 = G0 + (D.vscale * z[0]);
                G1 = G1 + (D.vscale * z[1]);
                G2 = G2 + (D.vscale * z[2]);
            }
        }
        t_sum += (D.mass * tsum) / (double)(nn - 1);
        t_cells += 1.0;
        if (!(isfinite(u0) && isfinite(u1) && isfinite(u2))) atomicOr(&rs->flags, RMP_FLAG_NONFINITE);
        s_u[0] = u0; s_u[1] = u1; s_u[2] = u2;
        if constexpr (RULE == 1) {
            s_n[0] = G0 / (double)nn; s_n[1] = G1 / (double)nn; s_n[2] = G2 / (double)nn;
        }
        int flipk = -1;
        if (D.bulk_on && nB > 0) {
            uint64_t wv[4];
            philox<true>((uint64_t)coll, (uint64_t)cell, 0, D.seed, TAG_BULK, wv);
            double P = D.ptable[nB < RMP_PTABLE ? nB : RMP_PTABLE - 1];
            if (u01(wv[0]) < P) {
                int jb = (int)(u01(wv[1]) * (double)nB);
                if (jb >= nB) jb = nB - 1;
                for (int k = 0; k < nn; ++k)
                    if (rec_st(&rec[srt[k] < (uint32_t)nn ? srt[k] : 0u]) & 1) {
                        if (jb == 0) { flipk = k; break; }
                        jb--;
                    }
            }
        }
        *s_flip = flipk;
    }
    __syncthreads();
    const double u0 = s_u[0], u1 = s_u[1], u2 = s_u[2];
    const int flipk = *s_flip;
    for (int k0 = 0; k0 < nn; k0 += NT) {
        const int k = k0 + t;
        bool cnd = false;
        const int64_t o = (int64_t)q0 + k;
        if (k < nn) {
            T xt[3], vq[3]; uint32_t idq, pq; uint8_t s;
            rec_get(&rec[srt[k] < (uint32_t)nn ? srt[k] : 0u], xt, vq, idq, pq, s);
            const double vv0 = (double)vq[0], vv1 = (double)vq[1], vv2 = (double)vq[2];
            double v3[3];
            if constexpr (RULE == 0) {
                const double nax[3] = {s_n[0], s_n[1], s_n[2]};
                double rw[3];
                rotate(nax, ca, sa, oma, vv0 - u0, vv1 - u1, vv2 - u2, rw);
                v3[0] = u0 + rw[0]; v3[1] = u1 + rw[1]; v3[2] = u2 + rw[2];
            } else {
                uint64_t wv[4]; double z[3];
                philox<true>((uint64_t)coll, idq, 0, D.seed, TAG_THERMO, wv);
                normals3(wv, z);
                v3[0] = u0 + ((D.vscale * z[0]) - s_n[0]);
                v3[1] = u1 + ((D.vscale * z[1]) - s_n[1]);
                v3[2] = u2 + ((D.vscale * z[2]) - s_n[2]);
            }
            if (k == flipk) {
                du_sum += species_dU(D, cp, nc, s_Xw, (double)xt[0], (double)xt[1], (double)xt[2], 1, 0);
                n_flip += 1.0;
                s = 0;
            }
            const T vt[3] = {(T)v3[0], (T)v3[1], (T)v3[2]};
            for (int d = 0; d < 3; ++d) { xn[d][o] = xt[d]; vn[d][o] = vt[d]; }
            idn[o] = idq;
            stn[o] = s;
            cnd = is_candidate(D, cp, nc, s_Xw, s, (double)xt[0], (double)xt[1], (double)xt[2],
                               (double)vt[0], (double)vt[1], (double)vt[2]);
            D.cflag[o] = cnd ? 1 : 0;
        }
        // the wave's slots lie in [q0 + k0, q0 + k0 + NT): at most two chunks
        count_flag(G(D.chunk_cnt), o, cnd, ((int64_t)q0 + k0) / CHUNK);
    }
    __syncthreads();
}

// MPCD collision on one tile of cells of the shifted grid (sort ranks
// [c0, c0 + TC)).  The scatter has put the tile's particles in the
// contiguous slots [start[c0], start[c0 + TC)) of the staging array, cell
// by cell (in scatter order within a cell).  The tile's cells are taken in
// groups whose particles fit the workgroup (NT threads holding PPT particles
// each); usually the whole tile is one group.  Per group:
//   B  each thread reads whole records of the group's slots (coalesced) and
//      looks up each slot's cell (a slot-to-cell map of the tile built at
//      tile start; binary search over the cell starts past its end);
//   C  it ranks its particle by old index among its cell's records (the
//      stable order), writes position and id to the output slot of that
//      rank, velocity and species to LDS at that slot for the per-cell sums;
//   D  one thread per cell: sequential FP64 sums in the stable order,
//      centre-of-mass velocity, temperature term, bulk reaction decision;
//      one lane per colloid: is the colloid within reach of any particle of
//      the tile (the box of the tile's cells, the particles' largest speed)?
//   E  each thread rotates its particles about their cell's axis, applies
//      the reaction, and writes velocity, species and Verlet-list flag.
// The random axes and bulk-reaction uniforms of all cells of the tile, the
// slot-to-cell map and the tile's box are made at tile start (they depend on
// nothing loaded), next to the loads.
// The register file is held to 96 VGPRs (five waves per SIMD) with one
// particle per thread, or two in FP32, and to 128 (four waves) with two in
// FP64; a few bytes of values spill.
template <class T, int RULE, int NT, int PPT>
__global__ __launch_bounds__(NT, (PPT == 1 || sizeof(T) == 4) ? 5 : 4) void k_collide(Work w, int xcd_map)
{
    constexpr int CAP = NT * PPT;
    constexpr int FILLCAP = 2 * CAP;    // leading slots of the tile with their cell in s_cellof
    static_assert(CAP <= CHUNK, "a collision group spans at most two chunks");
    static_assert(NT >= 256, "the tile-start draws use the last two waves");
    int item = blockIdx.x;
    if (xcd_map && (gridDim.x & 7) == 0) {
        // workgroups are dealt to the eight XCDs in turn: give each XCD a
        // contiguous range of tiles so that neighbouring tiles, which gather
        // from the same source lines, share an L2
        const int per = (int)(gridDim.x >> 3);
        item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    }
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int tile = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active || D.rule != RULE) return;
    RepState* rs = D.rs;
    const ColloidParams* cp = D.cp;
    const int nc = cp->nc;
    const int t = threadIdx.x;
    const int lane = t & 63;

    __shared__ uint32_t s_start[COLL_TCMAX + 1];
    __shared__ uint8_t s_cellof[FILLCAP];
    __shared__ uint32_t s_perm[CAP];
    __shared__ T s_v[3][CAP];
    __shared__ double s_g[3][RULE ? CAP : 1];
    __shared__ uint8_t s_st[CAP];
    __shared__ double s_u[COLL_TCMAX][3], s_n[COLL_TCMAX][3];
    __shared__ double s_b[COLL_TCMAX][2];       // bulk-reaction uniforms
    __shared__ double s_z[COLL_TCMAX][3];       // virtual-momentum normal of a plate-layer cell
    __shared__ int32_t s_flip[COLL_TCMAX];
    __shared__ uint8_t s_go[COLL_TCMAX];
    __shared__ double s_Xw[MAXC][3];
    __shared__ double s_box[6];        // the tile's box: lower, upper offsets from s_ref
    __shared__ double s_ref[3];        // lower corner of the tile's first cell (unshifted)
    __shared__ uint64_t s_vmax2;       // max |v|^2 (bit patterns order like the values)
    __shared__ uint32_t s_cmask;
    __shared__ double sred[(NT / 64 + 1) * 4];

    const int64_t coll = rs->coll_step;
    const int nxt = (int)(coll & 1) ^ 1;
    const int64_t n = D.n;
    const int TC = D.tile_cells;
    const int64_t c0 = (int64_t)tile * TC;
    const int64_t c1 = (c0 + TC < D.ncell) ? c0 + TC : D.ncell;
    const int ncl = (int)(c1 - c0);
    // the colloid cull needs a bound on the speed after the collision:
    // the rotation gives one (below), the thermostat's fresh draws do not
    const bool cull = RULE == 0 && nc > 0 && !D.flow;

    // ---- A: cell starts (and the counters zeroed for the next binning);
    //         per-cell random draws; colloid images
    for (int k = t; k <= ncl; k += NT) {
        s_start[k] = G(D.start)[c0 + k];
        if (k < ncl) G(D.count)[c0 + k] = 0;
    }
    if (t >= NT - 128 && t < NT - 64) {
        if constexpr (RULE == 0) {
            for (int lc = t - (NT - 128); lc < ncl; lc += 64) {
                const int64_t cell = D.hbits == KEY_ROW ? c0 + lc : G(D.cell_of)[c0 + lc];
                double nax[3];
                marsaglia_axis<true>(D.seed, (uint64_t)coll, (uint64_t)cell, nax);
                s_n[lc][0] = nax[0]; s_n[lc][1] = nax[1]; s_n[lc][2] = nax[2];
            }
        }
    } else if (t >= NT - 64) {
        if (D.bulk_on)
            for (int lc = t - (NT - 64); lc < ncl; lc += 64) {
                const int64_t cell = D.hbits == KEY_ROW ? c0 + lc : G(D.cell_of)[c0 + lc];
                uint64_t wv[4];
                philox<true>((uint64_t)coll, (uint64_t)cell, 0, D.seed, TAG_BULK, wv);
                s_b[lc][0] = u01(wv[0]);
                s_b[lc][1] = u01(wv[1]);
            }
    } else if (t >= 64 && t < 128) {
        if (D.walls) {
            // plates (flows have no colloids): the virtual-momentum normal of
            // every cell of the first and last layer, used if the cell turns
            // out to be cut and under-filled
            for (int lc = t - 64; lc < ncl; lc += 64) {
                const int64_t cell = D.hbits == KEY_ROW ? c0 + lc : G(D.cell_of)[c0 + lc];
                const int64_t cz = cell / ((int64_t)D.L[0] * D.L[1]);
                if (cz == 0 || cz == D.L[2] - 1) {
                    uint64_t wv[4]; double z[3];
                    philox<true>((uint64_t)coll, (uint64_t)cell, 0, D.seed, TAG_VIRT, wv);
                    normals3(wv, z);
                    s_z[lc][0] = z[0]; s_z[lc][1] = z[1]; s_z[lc][2] = z[2];
                }
            }
        } else if (t < 64 + nc) {
            for (int d = 0; d < 3; ++d) s_Xw[t - 64][d] = colloid_image(G(rs)->X[t - 64][d], D.Ld[d]);
        }
    }
    if (cull && t < 64) {
        // the tile's box for the colloid cull, from its cells: a cell
        // (c0, c1, c2) of the grid shifted by s in [0, 1)^3 holds the points
        // with c + s <= x < c + 1 + s, inside [c, c + 2) whatever the shift;
        // cell offsets from the first cell by minimum image, so a tile
        // across the periodic boundary stays compact
        const uint32_t L0 = (uint32_t)D.L[0], L1 = (uint32_t)D.L[1];
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        int ref[3];
        {
            const uint32_t lin = (uint32_t)(D.hbits == KEY_ROW ? c0 : G(D.cell_of)[c0]);
            ref[0] = (int)(lin % L0);
            ref[1] = (int)((lin / L0) % L1);
            ref[2] = (int)(lin / (L0 * L1));
        }
        if (lane < ncl) {
            const uint32_t lin = (uint32_t)(D.hbits == KEY_ROW ? c0 + lane : G(D.cell_of)[c0 + lane]);
            const int cc[3] = {(int)(lin % L0), (int)((lin / L0) % L1), (int)(lin / (L0 * L1))};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int o = cc[d] - ref[d];
                if (2 * o >= D.L[d]) o -= D.L[d];
                else if (2 * o < -D.L[d]) o += D.L[d];
                lo[d] = hi[d] = o;
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) wave_min_max_i(lo[d], hi[d]);
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                s_ref[d] = (double)ref[d];
                s_box[d] = (double)lo[d];
                s_box[3 + d] = (double)hi[d] + 2.0;
            }
        }
    }
    if (t < 64 && lane < ncl) {
        // tile-local cell of each of the tile's first FILLCAP slots (the
        // cells' slot ranges are contiguous and in order)
        const uint32_t base = G(D.start)[c0], a = G(D.start)[c0 + lane], b = G(D.start)[c0 + lane + 1];
        const uint32_t e = b - base < (uint32_t)FILLCAP ? b - base : (uint32_t)FILLCAP;
        for (uint32_t r = a - base; r < e; ++r) s_cellof[r] = (uint8_t)lane;
    }
    if (t == 64) { s_vmax2 = 0ull; s_cmask = 0u; }
    __syncthreads();

    const gptr<const Rec<T>> stage = G(reinterpret_cast<const Rec<T>*>(D.stage));
    const gptr<T> xn[3] = {G(comp<T>(D.x[nxt], n, 0)), G(comp<T>(D.x[nxt], n, 1)), G(comp<T>(D.x[nxt], n, 2))};
    const gptr<T> vn[3] = {G(comp<T>(D.v[nxt], n, 0)), G(comp<T>(D.v[nxt], n, 1)), G(comp<T>(D.v[nxt], n, 2))};
    const gptr<uint32_t> idn = G(D.id[nxt]);
    const gptr<uint8_t> stn = G(D.st[nxt]);
    const gptr<uint8_t> cflag = G(D.cflag);
    const double ca = D.ca, sa = D.sa, oma = 1.0 - D.ca;

    double t_sum = 0.0, t_cells = 0.0, du_sum = 0.0, n_flip = 0.0;
    uint64_t big = 0;          // tile-local cells left to k_collide_big (uniform)
    int ga = 0;
    while (ga < ncl) {
        int gb;
        if (s_start[ncl] - s_start[ga] <= (uint32_t)CAP) {
            gb = ncl;
        } else {
            // the longest run of cells from ga whose particles fit (at least one cell)
            const int k = ga + 1 + t;
            const bool ok = k <= ncl && s_start[k] - s_start[ga] <= (uint32_t)CAP;
            const int cnt = __syncthreads_count(ok);
            gb = ga + (cnt > 0 ? cnt : 1);
        }
        const uint32_t q0 = s_start[ga], q1 = s_start[gb];
        const int ns = (int)(q1 - q0);
        if (ns > CAP) {
            // one cell beyond a group's capacity: left to k_collide_big
            big |= 1ull << ga;
            ga = gb;
            continue;
        }
        // ---- B: records of the group's slots, cell of each slot
        T xr[PPT][3], vq[PPT][3];
        uint32_t idq[PPT], pj[PPT];
        uint8_t sr[PPT];
        int lcj[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int j = t + u * NT;
            lcj[u] = ga;
            pj[u] = 0u;
            sr[u] = 0;
            if (j < ns) {
                rec_get(&stage[q0 + j], xr[u], vq[u], idq[u], pj[u], sr[u]);
                s_perm[j] = pj[u];
                const uint32_t q = q0 + (uint32_t)j;
                if (q - s_start[0] < (uint32_t)FILLCAP) {
                    lcj[u] = s_cellof[q - s_start[0]];
                } else {
                    int lo = ga, hi = gb - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_start[mid] <= q) lo = mid; else hi = mid - 1;
                    }
                    lcj[u] = lo;
                }
            }
        }
        __syncthreads();
        // ---- C: stable rank; position and id written at the rank's slot
        int slot[PPT];
        double gv2 = 0.0;
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            const int j = t + u * NT;
            slot[u] = -1;
            if (j < ns) {
                const int cb = (int)(s_start[lcj[u]] - q0), ce = (int)(s_start[lcj[u] + 1] - q0);
                const uint32_t p = pj[u];
                int r = 0, q = cb;
                for (; q + 4 <= ce; q += 4)
                    r += (s_perm[q] < p ? 1 : 0) + (s_perm[q + 1] < p ? 1 : 0) + (s_perm[q + 2] < p ? 1 : 0) +
                         (s_perm[q + 3] < p ? 1 : 0);
                for (; q < ce; ++q) r += s_perm[q] < p ? 1 : 0;
                const int sl = cb + r;
                slot[u] = sl;
                const int64_t o = (int64_t)q0 + sl;
                const T (&xr_)[3] = xr[u];
                const T (&vq_)[3] = vq[u];
#pragma unroll
                for (int d = 0; d < 3; ++d) { xn[d][o] = xr_[d]; s_v[d][sl] = vq_[d]; }
                idn[o] = idq[u];
                s_st[sl] = sr[u];
                if constexpr (RULE == 1) {
                    uint64_t wv[4]; double z[3];
                    philox<true>((uint64_t)coll, idq[u], 0, D.seed, TAG_THERMO, wv);
                    normals3(wv, z);
                    s_g[0][sl] = D.vscale * z[0];
                    s_g[1][sl] = D.vscale * z[1];
                    s_g[2][sl] = D.vscale * z[2];
                }
                if (cull) {
                    // the largest speed vmax of the tile's particles, for the
                    // colloid cull: after the rotation a speed is at most
                    // |u| + |v - u| <= 3 vmax
                    const double vv = dot3((double)vq_[0], (double)vq_[1], (double)vq_[2],
                                           (double)vq_[0], (double)vq_[1], (double)vq_[2]);
                    gv2 = vv > gv2 ? vv : gv2;
                    if (!(vv <= 1e300)) gv2 = 1e300;          // inf or NaN: no cull
                }
            }
        }
        if (cull) {
            // wave maximum by DPP (exact), then one LDS atomic per wave
            // (non-negative doubles order like their bit patterns)
            gv2 = wave_max_d(gv2);
            if (lane == 0) atomicMax((unsigned long long*)&s_vmax2, (unsigned long long)__double_as_longlong(gv2));
        }
        __syncthreads();
        // ---- D: per cell (one thread each); colloid cull (second wave)
        for (int cl = ga + t; cl < gb; cl += NT) {
            const int cb = (int)(s_start[cl] - q0), ce = (int)(s_start[cl + 1] - q0);
            const int nn = ce - cb;
            s_flip[cl] = -1;
            // Lamura et al. (2001): a cell of the first or last layer (cut by
            // a plate) with fewer than n0 particles holds n0 - n virtual ones
            // at rest on average; only their summed momentum enters, a normal
            // vector of variance (n0 - n) kT / m per component
            bool virt = false;
            if (D.walls && nn >= 1 && nn < D.wall_n0) {
                const int64_t cell = D.hbits == KEY_ROW ? c0 + cl : G(D.cell_of)[c0 + cl];
                const int64_t cz = cell / ((int64_t)D.L[0] * D.L[1]);
                virt = cz == 0 || cz == D.L[2] - 1;
            }
            const bool go = nn >= 2 || virt;
            s_go[cl] = go ? 1 : 0;
            int nB = 0;
            if (go) {
                double S0 = 0.0, S1 = 0.0, S2 = 0.0;
                for (int q = cb; q < ce; ++q) {
                    S0 = S0 + (double)s_v[0][q];
                    S1 = S1 + (double)s_v[1][q];
                    S2 = S2 + (double)s_v[2][q];
                    nB += s_st[q] & 1;
                }
                double u0, u1, u2;
                if (virt) {
                    const double sd = sqrt((double)(D.wall_n0 - nn)) * D.vscale;
                    const double n0 = (double)D.wall_n0;
                    u0 = (S0 + (sd * s_z[cl][0])) / n0;
                    u1 = (S1 + (sd * s_z[cl][1])) / n0;
                    u2 = (S2 + (sd * s_z[cl][2])) / n0;
                } else {
                    u0 = S0 / (double)nn; u1 = S1 / (double)nn; u2 = S2 / (double)nn;
                    double tsum = 0.0;
                    for (int q = cb; q < ce; ++q) {
                        const double w0 = (double)s_v[0][q] - u0, w1 = (double)s_v[1][q] - u1,
                                     w2 = (double)s_v[2][q] - u2;
                        tsum = tsum + dot3(w0, w1, w2, w0, w1, w2);
                    }
                    t_sum += (D.mass * tsum) / (double)(nn - 1);
                    t_cells += 1.0;
                }
                // a non-finite centre-of-mass velocity would spread through
                // its cell: latched for the caller
                if (!(isfinite(u0) && isfinite(u1) && isfinite(u2))) atomicOr(&rs->flags, RMP_FLAG_NONFINITE);
                s_u[cl][0] = u0; s_u[cl][1] = u1; s_u[cl][2] = u2;
                if constexpr (RULE == 1) {
                    double G0 = 0.0, G1 = 0.0, G2 = 0.0;
                    for (int q = cb; q < ce; ++q) {
                        G0 = G0 + s_g[0][q];
                        G1 = G1 + s_g[1][q];
                        G2 = G2 + s_g[2][q];
                    }
                    s_n[cl][0] = G0 / (double)nn; s_n[cl][1] = G1 / (double)nn; s_n[cl][2] = G2 / (double)nn;
                }
            } else if (nn == 1) {
                nB = s_st[cb] & 1;
            }
            if (D.bulk_on && nB > 0) {
                const double P = G(D.ptable)[nB < RMP_PTABLE ? nB : RMP_PTABLE - 1];
                if (s_b[cl][0] < P) {
                    int jb = (int)(s_b[cl][1] * (double)nB);
                    if (jb >= nB) jb = nB - 1;
                    for (int q = cb; q < ce; ++q)
                        if (s_st[q] & 1) {
                            if (jb == 0) { s_flip[cl] = q; break; }
                            jb--;
                        }
                }
            }
        }
        if (cull && t >= 64 && t < 128) {
            // colloid c can reach a particle of the tile only if its reach
            // sphere, widened by the largest speed times tau, meets the
            // tile's box (minimum image per axis, margin far above rounding)
            bool near = false;
            // c is made opaque here so that the per-thread addresses below
            // are formed inside the group loop: hoisted out of it, they were
            // held across the whole tile and spilled to scratch (FP32 form)
            int c = t - 64;
            asm volatile("" : "+v"(c));
            if (c < nc) {
                const double vmax2 = __longlong_as_double((long long)s_vmax2);
                const double reach = ((3.0 * sqrt(vmax2)) * D.tau + cp->reachR[c]) * (1.0 + 1e-6) + 1e-6;
                double r2 = 0.0;
                bool wide = !(reach < 1e200);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    // box [lo, hi] of offsets from s_ref; the colloid's offset
                    // and its periodic images: the nearest one counts
                    const double lo = s_box[d], hi = s_box[3 + d];
                    if (!(hi - lo < 0.5 * D.Ld[d])) { wide = true; continue; }
                    const double oc = min_image(s_Xw[c][d] - s_ref[d], D.Ld[d], D.halfL[d]);
                    double dd = 1e300;
#pragma unroll
                    for (int img = -1; img <= 1; ++img) {
                        const double ci = oc + (double)img * D.Ld[d];
                        double e = lo - ci > ci - hi ? lo - ci : ci - hi;
                        e = e > 0.0 ? e : 0.0;
                        dd = e < dd ? e : dd;
                    }
                    r2 += dd * dd;
                }
                near = wide || r2 < reach * reach;
            }
            const uint64_t m = __ballot(near);
            if (lane == 0) s_cmask = (uint32_t)m;
        }
        __syncthreads();
        // ---- E: rotate (or thermostat), react, write, Verlet-list flag
        // without the cull every colloid is tested
        const uint32_t cmask = cull ? s_cmask : (nc >= 32 ? 0xffffffffu : ((1u << nc) - 1u));
        const int64_t c_lo = (int64_t)q0 / CHUNK;
        bool fl[PPT];
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
            bool cnd = false;
            fl[u] = false;
            int64_t o = (int64_t)q0;
            if (slot[u] >= 0) {
                const int cl = lcj[u];
                double v3[3] = {(double)s_v[0][slot[u]], (double)s_v[1][slot[u]], (double)s_v[2][slot[u]]};
                if (s_go[cl]) {
                    const double u0 = s_u[cl][0], u1 = s_u[cl][1], u2 = s_u[cl][2];
                    if constexpr (RULE == 0) {
                        const double nax[3] = {s_n[cl][0], s_n[cl][1], s_n[cl][2]};
                        double rw[3];
                        rotate(nax, ca, sa, oma, v3[0] - u0, v3[1] - u1, v3[2] - u2, rw);
                        v3[0] = u0 + rw[0]; v3[1] = u1 + rw[1]; v3[2] = u2 + rw[2];
                    } else {
                        v3[0] = u0 + (s_g[0][slot[u]] - s_n[cl][0]);
                        v3[1] = u1 + (s_g[1][slot[u]] - s_n[cl][1]);
                        v3[2] = u2 + (s_g[2][slot[u]] - s_n[cl][2]);
                    }
                }
                uint8_t s = sr[u];
                o = (int64_t)q0 + slot[u];
                const bool flip = s_flip[cl] == slot[u];
                // the position (written to the output slot in C by this
                // thread) is read back only for a colloid within reach of
                // the tile
                T xo3[3] = {(T)0, (T)0, (T)0};
                if (cmask != 0u)
#pragma unroll
                    for (int d = 0; d < 3; ++d) xo3[d] = xn[d][o];
                if (flip) {
                    fl[u] = true;
                    n_flip += 1.0;
                    s = 0;
                }
                const T vt[3] = {(T)v3[0], (T)v3[1], (T)v3[2]};
#pragma unroll
                for (int d = 0; d < 3; ++d) vn[d][o] = vt[d];
                stn[o] = s;
                cnd = is_candidate_masked(D, cp, cmask, s_Xw, s, (double)xo3[0], (double)xo3[1],
                                          (double)xo3[2], (double)vt[0], (double)vt[1], (double)vt[2]);
                cflag[o] = cnd ? 1 : 0;
            }
            count_flag(G(D.chunk_cnt), o, cnd, c_lo);
        }
        // the potential change of a flipped particle, in the same order per
        // thread, after the writes: inside their loop its colloid loop
        // raised the register peak beyond the budget (spills to scratch)
#pragma unroll
        for (int u = 0; u < PPT; ++u)
            if (fl[u]) {
                const int64_t o = (int64_t)q0 + slot[u];
                du_sum += species_dU(D, cp, nc, s_Xw, (double)xn[0][o], (double)xn[1][o], (double)xn[2][o], 1, 0);
            }
        ga = gb;
        if (ga < ncl) __syncthreads();   // the next group reuses the LDS
    }
    // the tile's sums: the wave trees, then the waves in order (as
    // block_sum_n).  The temperature terms live in wave 0 alone (one thread
    // per cell, at most 64 cells) and the reaction terms only where a flip
    // happened; a wave holding only +0.0 has the tree +0.0, which is not
    // formed (no sum here is ever -0.0)
    {
        constexpr int NW = NT / 64;
        const int wave = t >> 6;
        double red[4] = {0.0, 0.0, 0.0, 0.0};
        if (wave == 0) {
            red[0] = wave_tree_sum(t_sum);
            red[1] = wave_tree_sum(t_cells);
        }
        if (__ballot(n_flip != 0.0) != 0) {
            red[2] = wave_tree_sum(du_sum);
            red[3] = wave_tree_sum(n_flip);
        }
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q) sred[wave * 4 + q] = red[q];
        __syncthreads();
        if (t < 4) {
            double a = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) a = a + sred[w * 4 + t];
            G(D.tpart)[(int64_t)tile * 4 + t] = a;
        }
        if (t == 0) G(D.bigmask)[tile] = big;
    }
}

// The cells that k_collide found beyond a group's capacity (a bit per
// tile-local cell in bigmask[tile]).  Workgroup w looks at tiles
// [64 w, 64 w + 64) of the launch and collides each such cell with all its
// threads (collide_big_cell); the cell's temperature, reaction energy and
// flips are added to its tile's partials after those of the tile's other
// cells, cell by cell, so the sums stay deterministic.
template <class T, int RULE>
__global__ __launch_bounds__(256) void k_collide_big(Work w, int n_items)
{
    constexpr int NT = 256;
    const int t = threadIdx.x;
    __shared__ uint64_t s_mask[64];
    __shared__ double s_u[3], s_n[3];
    __shared__ int32_t s_flip;
    __shared__ double s_Xw[MAXC][3];
    __shared__ double sred[(NT / 64 + 1) * 4];
    const int item0 = blockIdx.x * 64;
    bool any = false;
    if (t < 64) {
        const int item = item0 + t;
        uint64_t m = 0;
        if (item < n_items) {
            const int rep = find_rep(w.prefix, w.nrep, item);
            const RepDesc& D = w.desc[rep];
            if (D.active && D.rule == RULE) m = D.bigmask[item - w.prefix[rep]];
        }
        s_mask[t] = m;
        any = m != 0;
    }
    if (__syncthreads_or(any) == 0) return;
    for (int q = 0; q < 64; ++q) {
        const uint64_t mask = s_mask[q];
        if (mask == 0) continue;
        const int item = item0 + q;
        const int rep = find_rep(w.prefix, w.nrep, item);
        const int tile = item - w.prefix[rep];
        const RepDesc& D = w.desc[rep];
        RepState* rs = D.rs;
        const ColloidParams* cp = D.cp;
        const int nc = cp->nc;
        const int64_t coll = rs->coll_step;
        if (t < nc)
            for (int d = 0; d < 3; ++d) s_Xw[t][d] = colloid_image(rs->X[t][d], D.Ld[d]);
        const int64_t c0 = (int64_t)tile * D.tile_cells;
        double t_sum = 0.0, t_cells = 0.0, du_sum = 0.0, n_flip = 0.0;
        for (uint64_t m = mask; m; m &= m - 1) {
            const int ga = __ffsll((long long)m) - 1;
            const int64_t cell = D.hbits == KEY_ROW ? c0 + ga : D.cell_of[c0 + ga];
            const uint32_t q0 = D.start[c0 + ga];
            const int nn = (int)(D.start[c0 + ga + 1] - q0);
            if (RULE == 0 && t == 0) marsaglia_axis<true>(D.seed, (uint64_t)coll, (uint64_t)cell, s_n);
            __syncthreads();
            collide_big_cell<T, RULE, NT>(D, cp, nc, s_Xw, coll, cell, q0, nn, s_u, s_n, &s_flip,
                                          t_sum, t_cells, du_sum, n_flip);
        }
        double red[4] = {t_sum, t_cells, du_sum, n_flip};
        block_sum_n<NT, 4>(red, sred);
        if (t == 0)
            for (int j = 0; j < 4; ++j) D.tpart[(int64_t)tile * 4 + j] = D.tpart[(int64_t)tile * 4 + j] + red[j];
        __syncthreads();
    }
}

// ---------------------------------------------------------- observables

// part: where the per-chunk partials go (nullptr: the replica's own
// workspace region)
template <class T>
__global__ __launch_bounds__(256) void k_observe(Work w, double* part)
{
    const int item = blockIdx.x;
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int chunk = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active) return;
    __shared__ double sred[8];
    const int cur = (int)(D.rs->coll_step & 1);
    const int64_t n = D.n;
    const int64_t base = (int64_t)chunk * CHUNK;
    double P0 = 0.0, P1 = 0.0, P2 = 0.0, ke = 0.0, nb = 0.0;
    for (int j = threadIdx.x; j < CHUNK; j += 256) {
        int64_t i = base + j;
        if (i >= n) break;
        double v0 = comp<T>(D.v[cur], n, 0)[i], v1 = comp<T>(D.v[cur], n, 1)[i],
               v2 = comp<T>(D.v[cur], n, 2)[i];
        P0 += v0; P1 += v1; P2 += v2;
        ke += dot3(v0, v1, v2, v0, v1, v2);
        nb += (double)(D.st[cur][i] & 1);
    }
    double r[5] = {P0, P1, P2, ke, nb};
    double* out = part ? part : D.obs_part;
    for (int k = 0; k < 5; ++k) {
        double s = block_sum<256>(r[k], sred);
        if (threadIdx.x == 0) out[(int64_t)chunk * 8 + k] = s;
    }
}

// Totals of the k_observe partials: lane k (< 5) adds quantity k over the
// chunks in chunk order, the order of the host-side sum, so both give the
// same totals bit for bit.
__global__ __launch_bounds__(64) void k_observe_total(const double* part, int cnt, double* tot)
{
    const int k = threadIdx.x;
    if (k >= 5) return;
    double s = 0.0;
    for (int c = 0; c < cnt; ++c) s += part[(int64_t)c * 8 + k];
    tot[k] = s;
}

// ------------------------------------------------------------ dimer analysis
// Quantities of the paper's dimer analysis programs ("Applications of
// RMPCDMD"), sampled on the device after a collision: the dimer record
// (centre of mass, its velocity, unit axis from bond_a to bond_b, directed
// velocity) and integer counts of A and B in cylindrical shells around the
// dimer's axis.  The same operations in the same order as the definitions
// (no contraction), so records and counts are exact, independent of launch
// shape.
__device__ __forceinline__ void dimer_record(const ColloidParams* cp, const RepState* rs, int k,
                                             double rec[RMP_SERIES_FIELDS])
{
    const int a = cp->bond_a[k], b = cp->bond_b[k];
    const double ma = cp->mass[a], mb = cp->mass[b];
    double dX[3];
    for (int d = 0; d < 3; ++d) {
        rec[d] = (ma * rs->X[a][d] + mb * rs->X[b][d]) / (ma + mb);
        rec[3 + d] = (ma * rs->V[a][d] + mb * rs->V[b][d]) / (ma + mb);
        dX[d] = rs->X[b][d] - rs->X[a][d];
    }
    const double len = sqrt(dot3(dX[0], dX[1], dX[2], dX[0], dX[1], dX[2]));
    for (int d = 0; d < 3; ++d) rec[6 + d] = dX[d] / len;
    rec[9] = dot3(rec[3], rec[4], rec[5], rec[6], rec[7], rec[8]);
}

// One workgroup per particle chunk (after the collision): chunk 0 also
// stores the series record.  After a collision the arrays are in cell order,
// so a chunk occupies a small region: its bounding box culls, for the whole
// workgroup, every dimer whose cylinder cannot reach it (the cylinder lies
// within a sphere of radius sqrt(zmax^2 + rmax^2) about the centre of mass;
// the bound carries a relative margin far above the rounding of z and rho,
// so no counted particle is ever culled).  Hits are sparse, so they go
// straight to 64-bit device atomics.
template <class T>
__global__ __launch_bounds__(256) void k_analysis(Work w)
{
    constexpr int PPT = CHUNK / 256;
    const int item = blockIdx.x;
    const int rep = find_rep(w.prefix, w.nrep, item);
    const int chunk = item - w.prefix[rep];
    const RepDesc& D = w.desc[rep];
    if (!D.active || D.an == nullptr) return;
    Analysis* A = D.an;
    const RepState* rs = D.rs;
    if (rs->coll_step % A->every != 0) return;
    __shared__ double sR[MAXC][3], sU[MAXC][3];
    __shared__ double sBox[4][6];
    __shared__ int sLive[MAXC];
    const int nb = A->nb;
    const int t = threadIdx.x;
    const int cur = (int)(rs->coll_step & 1);
    const int64_t n = D.n;
    const int64_t base = (int64_t)chunk * CHUNK;
    // every load of the chunk first
    double px[PPT][3];
    int psp[PPT];
    bool pv[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t i = base + t + 256 * q;
        pv[q] = i < n;
        const int64_t ic = pv[q] ? i : base;
        px[q][0] = (double)comp<T>(D.x[cur], n, 0)[ic];
        px[q][1] = (double)comp<T>(D.x[cur], n, 1)[ic];
        px[q][2] = (double)comp<T>(D.x[cur], n, 2)[ic];
        psp[q] = D.st[cur][ic] & 1;
    }
    if (t < nb) {
        double rec[RMP_SERIES_FIELDS];
        dimer_record(D.cp, rs, t, rec);
        for (int d = 0; d < 3; ++d) {
            sR[t][d] = colloid_image(rec[d], D.Ld[d]);
            sU[t][d] = rec[6 + d];
        }
        if (chunk == 0) {
            const int64_t k = A->n_samples;
            if (k < A->cap) {
                double* dst = A->series + (k * nb + t) * RMP_SERIES_FIELDS;
                for (int f = 0; f < RMP_SERIES_FIELDS; ++f) dst[f] = rec[f];
                if (t == 0) A->series_t[k] = rs->md_step;
            }
        }
    }
    // bounding box of the chunk's positions
    double bx[6];
    for (int d = 0; d < 3; ++d) {
        bx[d] = INFINITY;
        bx[3 + d] = -INFINITY;
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q)
        if (pv[q])
            for (int d = 0; d < 3; ++d) {
                bx[d] = fmin(bx[d], px[q][d]);
                bx[3 + d] = fmax(bx[3 + d], px[q][d]);
            }
    for (int m = 1; m < 64; m <<= 1)
        for (int d = 0; d < 3; ++d) {
            bx[d] = fmin(bx[d], __shfl_xor(bx[d], m, 64));
            bx[3 + d] = fmax(bx[3 + d], __shfl_xor(bx[3 + d], m, 64));
        }
    if ((t & 63) == 0)
        for (int k = 0; k < 6; ++k) sBox[t >> 6][k] = bx[k];
    __syncthreads();
    if (chunk == 0 && t == 0) {
        if (A->n_samples < A->cap) A->n_samples += 1;
        else A->n_dropped += 1;
    }
    if (t < nb) {
        bool live = true;
        for (int d = 0; d < 3; ++d) {
            const double lo = fmin(fmin(sBox[0][d], sBox[1][d]), fmin(sBox[2][d], sBox[3][d]));
            const double hi = fmax(fmax(sBox[0][3 + d], sBox[1][3 + d]), fmax(sBox[2][3 + d], sBox[3][3 + d]));
            // periodic distance from the centre's images to [lo, hi]
            double dist = INFINITY;
            for (int k = -1; k <= 1; ++k) {
                const double c = sR[t][d] + (double)k * D.Ld[d];
                dist = fmin(dist, c < lo ? lo - c : (c > hi ? c - hi : 0.0));
            }
            if (dist >= A->cull_r) live = false;
        }
        sLive[t] = live ? 1 : 0;
    }
    __syncthreads();
    const int nz = A->nz, nr = A->nr;
    const double zmax = A->zmax, inv_dz = A->inv_dz, inv_dr = A->inv_dr, skip_r2 = A->skip_r2;
    const double fnz = (double)nz, fnr = (double)nr;
    uint64_t* hist = A->hist;
    for (int b = 0; b < nb; ++b) {
        if (!sLive[b]) continue;
        const double c0 = sR[b][0], c1 = sR[b][1], c2 = sR[b][2];
        const double u0 = sU[b][0], u1 = sU[b][1], u2 = sU[b][2];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            if (!pv[q]) continue;
            const double r0 = min_image(px[q][0] - c0, D.Ld[0], D.halfL[0]);
            const double r1 = min_image(px[q][1] - c1, D.Ld[1], D.halfL[1]);
            const double r2 = min_image(px[q][2] - c2, D.Ld[2], D.halfL[2]);
            const double z = dot3(r0, r1, r2, u0, u1, u2);
            const double zs = (z + zmax) * inv_dz;
            if (!(zs >= 0.0 && zs < fnz)) continue;
            const double p0 = r0 - z * u0, p1 = r1 - z * u1, p2 = r2 - z * u2;
            const double pp = dot3(p0, p1, p2, p0, p1, p2);
            if (!(pp < skip_r2)) continue;
            const double rsc = sqrt(pp) * inv_dr;
            if (!(rsc < fnr)) continue;
            const int iz = (int)zs, ir = (int)rsc;
            atomicAdd((unsigned long long*)&hist[(((int64_t)b * 2 + psp[q]) * nz + iz) * nr + ir], 1ull);
        }
    }
}

// Mean-squared displacement of each dimer's centre of mass over the stored
// series: one thread per (dimer, lag), origins summed in order.
__global__ __launch_bounds__(256) void k_msd(Analysis* A, int32_t max_lag)
{
    const int nb = A->nb;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)nb * (max_lag + 1)) return;
    const int b = (int)(g / (max_lag + 1));
    const int lag = (int)(g % (max_lag + 1));
    const int64_t T = A->n_samples;
    double out = 0.0;
    if (lag < T) {
        double acc = 0.0;
        for (int64_t t0 = 0; t0 + lag < T; ++t0) {
            const double* p = A->series + ((t0 + lag) * nb + b) * RMP_SERIES_FIELDS;
            const double* q = A->series + (t0 * nb + b) * RMP_SERIES_FIELDS;
            const double d0 = p[0] - q[0], d1 = p[1] - q[1], d2 = p[2] - q[2];
            acc += dot3(d0, d1, d2, d0, d1, d2);
        }
        out = acc / (double)(T - lag);
    }
    A->msd[(int64_t)b * A->cap + lag] = out;
}

// ----------------------------------------------------- explicit instances

#define RMP_CHAIN_INST(T, K, NT)                                                 \
    template __global__ void k_chain<T, K, false, 0, NT>(Work);                  \
    template __global__ void k_chain<T, K, false, 1, NT>(Work);                  \
    template __global__ void k_chain<T, K, false, 2, NT>(Work);                  \
    template __global__ void k_chain<T, K, true, 0, NT>(Work);                   \
    template __global__ void k_chain<T, K, true, 1, NT>(Work);                   \
    template __global__ void k_chain<T, K, true, 2, NT>(Work);

#define RMP_INST(T)                                                              \
    template __global__ void k_init<T>(const RepDesc*);                          \
    template __global__ void k_init_sub<T>(const RepDesc*, const double*);       \
    template __global__ void k_list<T>(Work);                                    \
    template __global__ void k_stream_bin<T, 1>(Work, int);                      \
    template __global__ void k_stream_bin<T, 2>(Work, int);                      \
    template __global__ void k_stream_bin<T, 4>(Work, int);                      \
    template __global__ void k_scatter<T>(Work);                                 \
    RMP_CHAIN_INST(T, 1, 256)                                                    \
    RMP_CHAIN_INST(T, 2, 256)                                                    \
    RMP_CHAIN_INST(T, 4, 256)                                                    \
    RMP_CHAIN_INST(T, 1, 512)                                                    \
    RMP_CHAIN_INST(T, 2, 512)                                                    \
    template __global__ void k_collide_big<T, 0>(Work, int);                     \
    template __global__ void k_collide_big<T, 1>(Work, int);                     \
    template __global__ void k_collide<T, 0, 256, 2>(Work, int);                 \
    template __global__ void k_collide<T, 1, 256, 2>(Work, int);                 \
    template __global__ void k_collide<T, 0, 512, 2>(Work, int);                 \
    template __global__ void k_collide<T, 1, 512, 2>(Work, int);                 \
    template __global__ void k_collide<T, 0, 256, 1>(Work, int);                 \
    template __global__ void k_collide<T, 1, 256, 1>(Work, int);                 \
    template __global__ void k_collide<T, 0, 512, 1>(Work, int);                 \
    template __global__ void k_collide<T, 1, 512, 1>(Work, int);                 \
    template __global__ void k_observe<T>(Work, double*);                     \
    template __global__ void k_analysis<T>(Work);

RMP_INST(double)
RMP_INST(float)

}  // namespace rmp
