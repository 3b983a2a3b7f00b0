// Host runtime and C ABI of the rmpmd library (include/rmpmd.h).
//
// A single system is a batch of one replica.  Each replica's arrays are
// carved from a caller-owned workspace; the batch keeps a small control
// block (descriptors and work-list prefixes) in device memory.  One tick
// launches, for all occupied replicas at once:
//
//   [ k_chain  ||  k_stream_bin ]  (fork/join on a side stream)
//   k_scan_blocks, k_scan_final, k_scatter, k_collide, k_chunk_scan,
//   k_cand_write
//
// optionally replayed from a captured hipGraph.
#include "rmp_kernels.hip"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace rmp;

namespace {

constexpr size_t ALIGN = 256;
inline size_t aup(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// number of work items of each kind
struct Sizes {
    int64_t n, ncell;
    int32_t n_chunks, n_tiles_max, n_scanblk, cand_cap, G;
};

constexpr int MIN_TILE_CELLS = 8;
constexpr int MAX_G = MAX_CHAIN_G;
constexpr int K_MAX = 4;

int64_t auto_capacity(const rmp_params* p)
{
    const double vol = (double)p->L[0] * p->L[1] * p->L[2];
    const double rho = vol > 0 ? (double)p->n_solvent / vol : 0.0;
    double cap = 4096.0;
    for (int c = 0; c < p->n_colloids; ++c) {
        double R = 0x1.1f59ac3c7d6c0p+0 * p->sigma[c] + p->skin + 2.5;
        cap += 1.3 * rho * 4.0 / 3.0 * M_PI * R * R * R;
    }
    if (p->n_colloids == 0) cap = 1024.0;
    int64_t c = (int64_t)cap;
    if (c > p->n_solvent) c = p->n_solvent;
    if (c < 1) c = 1;
    return c;
}

bool has_flow(const rmp_params* p)
{
    return p->walls != 0 || p->accel[0] != 0.0 || p->accel[1] != 0.0 || p->accel[2] != 0.0;
}

// bond networks (a colloid in two or more bonds) need the iterative RATTLE
bool iterative_rattle(const rmp_params* p)
{
    if (p->n_bonds <= 0) return false;
    if (p->rattle_iterative) return true;
    int degree[RMP_MAX_COLLOIDS] = {0};
    for (int b = 0; b < p->n_bonds && b < RMP_MAX_BONDS; ++b) {
        const int a0 = p->bond_a[b], a1 = p->bond_b[b];
        if (a0 >= 0 && a0 < RMP_MAX_COLLOIDS && ++degree[a0] > 1) return true;
        if (a1 >= 0 && a1 < RMP_MAX_COLLOIDS && ++degree[a1] > 1) return true;
    }
    return false;
}

rmp_status validate(const rmp_params* p)
{
    if (!p) return RMP_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (p->L[d] < 1 || p->L[d] > 65536) return RMP_EINVAL;
    if (p->precision != 32 && p->precision != 64) return RMP_EINVAL;
    const int64_t ncell = (int64_t)p->L[0] * p->L[1] * p->L[2];
    if (ncell > (int64_t)1 << 31) return RMP_EINVAL;
    if (p->n_solvent < 0 || p->n_solvent >= ((int64_t)1 << 31)) return RMP_EINVAL;
    if (!(p->kT >= 0.0) || !(p->mass > 0.0) || !(p->dt > 0.0) || !(p->skin >= 0.0)) return RMP_EINVAL;
    if (!std::isfinite(p->alpha) || !(p->cat_prob >= 0.0) || !(p->bulk_rate >= 0.0)) return RMP_EINVAL;
    if (p->rule != 0 && p->rule != 1) return RMP_EINVAL;
    if (p->n_colloids < 0 || p->n_colloids > RMP_MAX_COLLOIDS) return RMP_EINVAL;
    if (p->n_bonds < 0 || p->n_bonds > RMP_MAX_BONDS) return RMP_EINVAL;
    if (p->cell_order != 0 && p->cell_order != 1) return RMP_EINVAL;
    if (p->cand_capacity < 0) return RMP_EINVAL;
    if (p->walls != 0 && p->walls != 1) return RMP_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->accel[d])) return RMP_EINVAL;
    if (has_flow(p) && (p->n_colloids != 0 || p->n_bonds != 0)) return RMP_EINVAL;
    if (p->walls && (p->rule != 0 || p->cell_order != 0 || p->accel[2] != 0.0 ||
                     p->wall_density < 1 || p->wall_density > 1024))
        return RMP_EINVAL;
    if ((int64_t)p->L[0] * p->L[1] * (p->L[2] + 1) > (int64_t)1 << 31) return RMP_EINVAL;
    int degree[RMP_MAX_COLLOIDS] = {0};
    for (int c = 0; c < p->n_colloids; ++c) {
        if (!(p->sigma[c] > 0.0) || !(p->colloid_mass[c] > 0.0)) return RMP_EINVAL;
        if (!(p->eps_A[c] >= 0.0) || !(p->eps_B[c] >= 0.0)) return RMP_EINVAL;
        if (p->ctype[c] < 0 || p->ctype[c] > 1) return RMP_EINVAL;
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(p->colloid_x[c][d])) return RMP_EINVAL;
        // minimum image needs the interaction reach within half a box
        double reach = 0x1.1f59ac3c7d6c0p+0 * p->sigma[c] + p->skin;
        for (int d = 0; d < 3; ++d)
            if (2.0 * reach > (double)p->L[d]) return RMP_EINVAL;
    }
    for (int b = 0; b < p->n_bonds; ++b) {
        int a0 = p->bond_a[b], a1 = p->bond_b[b];
        if (a0 < 0 || a1 < 0 || a0 >= p->n_colloids || a1 >= p->n_colloids || a0 == a1) return RMP_EINVAL;
        for (int r = 0; r < b; ++r)
            if ((p->bond_a[r] == a0 && p->bond_b[r] == a1) || (p->bond_a[r] == a1 && p->bond_b[r] == a0))
                return RMP_EINVAL;
        degree[a0]++;
        degree[a1]++;
        if (!(p->bond_d[b] > 0.0) || !std::isfinite(p->bond_d[b])) return RMP_EINVAL;
    }
    if (p->rattle_iterative != 0 && p->rattle_iterative != 1) return RMP_EINVAL;
    if (iterative_rattle(p) && (!(p->rattle_tol > 0.0) || !std::isfinite(p->rattle_tol) ||
                                p->rattle_maxit < 1 || p->rattle_maxit > 100000))
        return RMP_EINVAL;
    return RMP_OK;
}

Sizes sizes_of(const rmp_params* p)
{
    Sizes s;
    s.n = p->n_solvent;
    // with walls the shifted grid needs one layer more across the channel
    s.ncell = (int64_t)p->L[0] * p->L[1] * (p->L[2] + (p->walls ? 1 : 0));
    s.n_chunks = (int32_t)((s.n + CHUNK - 1) / CHUNK);
    if (s.n_chunks < 1) s.n_chunks = 1;
    s.n_tiles_max = (int32_t)((s.ncell + MIN_TILE_CELLS - 1) / MIN_TILE_CELLS);
    s.n_scanblk = (int32_t)((s.ncell + SCAN_BLK - 1) / SCAN_BLK);
    int64_t cap = p->cand_capacity > 0 ? p->cand_capacity : auto_capacity(p);
    if (cap > (int64_t)MAX_G * CHAIN_BLOCK * K_MAX) cap = (int64_t)MAX_G * CHAIN_BLOCK * K_MAX;
    s.cand_cap = (int32_t)cap;
    s.G = (int32_t)((cap + CHAIN_BLOCK - 1) / CHAIN_BLOCK);   // enough for K = 1
    if (s.G > MAX_G) s.G = MAX_G;
    if (s.G < 1) s.G = 1;
    return s;
}

// offsets of every array inside a replica workspace
struct Layout {
    size_t cp, rs, x[2], v[2], id[2], st[2], keyrank, stage, cflag, count, start, scanblk,
        chunk_cnt, chunk_off, cand_idx, order, partials, epart, tpart, bigmask, ptable, obs_part, mean, total;
};

Layout layout_of(const rmp_params* p)
{
    Sizes s = sizes_of(p);
    const size_t tb = p->precision == 32 ? 4 : 8;
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = aup(o + (bytes ? bytes : 1)); return r; };
    L.cp = take(sizeof(ColloidParams));
    L.rs = take(sizeof(RepState));
    for (int b = 0; b < 2; ++b) {
        L.x[b] = take(3 * s.n * tb);
        L.v[b] = take(3 * s.n * tb);
        L.id[b] = take(4 * s.n);
        L.st[b] = take(s.n);
    }
    L.keyrank = take(8 * s.n);
    L.stage = take((tb == 8 ? sizeof(Rec<double>) : sizeof(Rec<float>)) * s.n);
    L.cflag = take(s.n);
    L.count = take(4 * s.ncell);
    L.start = take(4 * (s.ncell + 1));
    L.scanblk = take(4 * (size_t)s.n_scanblk);
    L.chunk_cnt = take(4 * (size_t)s.n_chunks);
    L.chunk_off = take(4 * (size_t)s.n_chunks);
    L.cand_idx = take(4 * (size_t)s.cand_cap);
    L.order = take(2 * 4 * (size_t)s.ncell);
    L.partials = take(2 * ((size_t)s.G * ROWW + BCW) * 8);
    L.epart = take((size_t)s.G * 2 * 8);
    L.tpart = take((size_t)s.n_tiles_max * 4 * 8);
    L.bigmask = take((size_t)s.n_tiles_max * 8);
    L.ptable = take(RMP_PTABLE * 8);
    L.obs_part = take((size_t)s.n_chunks * 8 * 8);
    L.mean = take(4 * 8);
    L.total = o;
    return L;
}

size_t ctl_bytes_for(int32_t nslots)
{
    return aup(sizeof(RepDesc) * (size_t)nslots) + 6 * aup(4 * (size_t)(nslots + 1)) + aup(16);
}

const char* KNAMES[] = {"stream_bin", "chain", "scan_blocks", "scan_final", "scatter",
                        "collide", "chunk_scan", "cand_write", "list", "analysis"};
enum { KN_STREAM, KN_CHAIN, KN_SCANB, KN_SCANF, KN_SCATTER, KN_COLLIDE, KN_CHUNKSCAN,
       KN_CANDW, KN_LIST, KN_ANALYSIS, KN_COUNT };

struct Replica {
    bool used = false;
    rmp_params p{};
    uint64_t seed = 0;
    int32_t n_md = 0;
    char* ws = nullptr;
    Layout lay{};
    Sizes sz{};
    RepDesc desc{};
    bool list_valid = false;
    int32_t list_nmd = -1;
    std::vector<double> ptable;
    std::vector<uint32_t> order;   // host copy of the cell order tables (rank of cell, cell of rank)
    int32_t ptable_nmd = -1;
    int32_t tile_cells = 0;    // per-replica override of the collision tile size
    char* an = nullptr;        // dimer-analysis buffer (caller memory), nullptr when off
    rmp_analysis_params anp{};
};

}  // namespace

struct rmp_batch {
    int32_t nslots = 0;
    int32_t precision = 64;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;
    hipStream_t capture = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    char* ctl = nullptr;
    RepDesc* d_desc = nullptr;
    int32_t* d_prefix[6] = {};
    uint32_t* d_tick = nullptr;     // chain work-list tickets (two counters)
    int32_t chain_resident[2][5] = {}; // chain workgroups the device holds at once, per shape:
                                       // generic variant, one- or two-colloid variant
    int32_t nc_common = -1;         // colloid count shared by every occupied slot, -1 if mixed
    std::vector<Replica> reps;
    std::vector<RepDesc> hdesc;
    std::vector<int32_t> hprefix[6];
    int32_t totals[6] = {};
    bool dirty = true;
    bool have_rule[2] = {false, false};
    bool multi_scan = false;
    int32_t max_scanblk = 0;        // most scan blocks of any occupied slot
    bool any_analysis = false;
    bool any_iterative = false;     // some occupied slot uses the iterative RATTLE
    int64_t n_total = 0;            // solvent particles over the occupied slots
    int32_t device = 0;             // device current at creation (its stream's device)
    rmp_tuning tun{256, 2, 0, 1, 1, 0, 0, 0, 0, 0, 0, 0};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false;
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    size_t ev_used = 0;
    double prof_ms[KN_COUNT] = {};
    int64_t prof_cnt[KN_COUNT] = {};
};

struct rmp_system {
    rmp_batch* b = nullptr;
    rmp_batch storage;
};

// Device scratch of rmp_observables_noalloc: the per-chunk partial sums of
// the observation kernel and their totals.  Each GPU holds its own copy for
// the life of the process.  Host code never uses the array's name as an
// address: the address on a device comes from hipGetSymbolAddress with that
// device current, taken once per device when a batch is created there.
static __device__ __align__(256) unsigned char scratch[RMP_NOALLOC_SCRATCH_BYTES];
constexpr size_t RMP_STATIC_SCRATCH_BYTES = RMP_NOALLOC_SCRATCH_BYTES;

namespace {

enum { PF_CHUNK, PF_TILE, PF_SCAN, PF_CHAIN, PF_REP, PF_IDENT };

thread_local char g_last_error[256] = "";

void note_error(const char* what, hipError_t e)
{
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(x)                                       \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) {                         \
            note_error(#x, e_);                         \
            return RMP_EHIP;                            \
        }                                               \
    } while (0)

// Address of `scratch` on each device (nullptr until taken) and a lock per
// device that keeps the allocation-free calls on one device from
// overlapping.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[MAX_DEVICES] = {};
std::mutex g_scratch_call_mu[MAX_DEVICES];

// With `dev` current: take the address of this device's scratch once.
rmp_status take_scratch_address(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return RMP_EINVAL;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_addr[dev]) return RMP_OK;
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RMP_EHIP;
    g_scratch_addr[dev] = (char*)p;
    return RMP_OK;
}

char* scratch_address(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_addr[dev];
}

rmp_status last_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        note_error(what, e);
        return RMP_EHIP;
    }
    return RMP_OK;
}

constexpr int64_t CHAIN_PRIO_MAX_PARTICLES = (int64_t)1 << 22;

// Shape of the MD-chain workgroups: NT threads with K list entries each.
// Shapes 0, 1, 2: 256 threads with K = 1, 2, 4; shape 3: 512 threads, K = 1.
struct ChainShape {
    int nt, k, q;
};

int chain_groups(const rmp_batch* b, int k, int nt)
{
    int64_t total = 0;
    for (const auto& R : b->reps) {
        if (!R.used) continue;
        int64_t g = (R.sz.cand_cap + (int64_t)nt * k - 1) / ((int64_t)nt * k);
        total += std::max<int64_t>(1, std::min<int64_t>(g, R.sz.G));
    }
    return (int)std::min<int64_t>(total, INT32_MAX);
}

// workgroups per compute unit of each MD-chain shape (per[0]: the generic
// variant, per[1]: the fewer of the one- and two-colloid variants)
template <class T>
hipError_t occupancy_of(int (&per)[2][5])
{
    hipError_t e = hipSuccess;
    int one[5] = {};
#define RMP_OCC(DST, K, NT, NC)                                                                     \
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&(DST), k_chain<T, K, false, NC, NT>, NT, 0);
    RMP_OCC(per[0][0], 1, 256, 0) RMP_OCC(per[0][1], 2, 256, 0) RMP_OCC(per[0][2], 4, 256, 0)
    RMP_OCC(per[0][3], 1, 512, 0) RMP_OCC(per[0][4], 2, 512, 0)
    RMP_OCC(per[1][0], 1, 256, 2) RMP_OCC(per[1][1], 2, 256, 2) RMP_OCC(per[1][2], 4, 256, 2)
    RMP_OCC(per[1][3], 1, 512, 2) RMP_OCC(per[1][4], 2, 512, 2)
    RMP_OCC(one[0], 1, 256, 1) RMP_OCC(one[1], 2, 256, 1) RMP_OCC(one[2], 4, 256, 1)
    RMP_OCC(one[3], 1, 512, 1) RMP_OCC(one[4], 2, 512, 1)
#undef RMP_OCC
    for (int q = 0; q < 5; ++q) per[1][q] = std::min(per[1][q], one[q]);
    return e;
}

// colloid count of the MD-chain variant: the one common to every occupied
// slot when it is 1 or 2 (unrolled variants, with a smaller exchange table
// and so more workgroups per compute unit), else 0 (the generic one, also
// for a mix or an iterative RATTLE)
int chain_nc(const rmp_batch* b)
{
    return !b->any_iterative && (b->nc_common == 1 || b->nc_common == 2) ? b->nc_common : 0;
}

int chain_resident_of(const rmp_batch* b, int q)
{
    return b->tun.chain_resident > 0 ? b->tun.chain_resident : b->chain_resident[chain_nc(b) ? 1 : 0][q];
}

// 256-thread workgroups: the tuned entries per thread, raised until every
// system's list fits its workgroups, then raised to two while the batch's
// chain workgroups exceed what the device holds at once (past that point
// they run in waves through the ticketed work list; measured on 64 dimer
// replicas, two entries per thread in waves 2.10 ms per tick, four
// 2.17 ms, one 3.17 ms).
// 512-thread workgroups with one or two entries per thread are used when
// asked for, or, by default, when a system's list needs more than one entry
// per thread at 256 threads and the 512-thread shape still fits on the
// device (measured at 128^3 with 8 dimers: 512 x 1 1.95 ms, 256 x 4 2.14 ms,
// 256 x 2 2.36 ms per 50-step chain launch).
ChainShape chain_shape_of(const rmp_batch* b)
{
    int k = b->tun.chain_k;
    if (k != 1 && k != 2 && k != 4) k = 1;
    int64_t cap_max = 0;
    for (const auto& R : b->reps)
        if (R.used) cap_max = std::max<int64_t>(cap_max, R.sz.cand_cap);
    while (k < K_MAX && cap_max > (int64_t)MAX_G * 256 * k) k *= 2;
    while (k < 2 && chain_groups(b, k, 256) > chain_resident_of(b, k == 1 ? 0 : (k == 2 ? 1 : 2))) k *= 2;
    const bool want512 = b->tun.chain_block == 512 ||
                         (b->tun.chain_block <= 0 && cap_max > (int64_t)MAX_G * 256);
    if (want512 && cap_max <= (int64_t)MAX_G * 512 && chain_groups(b, 1, 512) <= chain_resident_of(b, 3))
        return ChainShape{512, 1, 3};
    if (want512 && cap_max <= (int64_t)MAX_G * 1024 && chain_groups(b, 2, 512) <= chain_resident_of(b, 4))
        return ChainShape{512, 2, 4};
    return ChainShape{256, k, k == 1 ? 0 : (k == 2 ? 1 : 2)};
}

// Threads and particles per thread of the collision workgroup (a group of
// cells holds at most their product of particles)
int collide_nt(const rmp_batch* b) { return b->tun.collide_block == 512 ? 512 : 256; }
int collide_ppt(const rmp_batch* b) { return b->tun.collide_ppt == 1 ? 1 : 2; }

// Cells per collision tile: the slot's override, else the batch tuning,
// else sized so that the mean tile holds about 0.94 of a group's capacity
// (measured at 128^3, rho 10: 48 cells 1.16 ms, 39 cells 1.29 ms, 32 cells
// 1.49 ms per collision; a tile beyond the capacity takes a second group),
// between MIN_TILE_CELLS and COLL_TCMAX
int tile_cells_of(const rmp_batch* b, int override_cells, int64_t ncell, int64_t n)
{
    int tc = override_cells > 0 ? override_cells : b->tun.collide_cells;
    if (tc <= 0) {
        const double rho = ncell > 0 ? (double)n / (double)ncell : 1.0;
        const double cap = (double)(collide_nt(b) * collide_ppt(b));
        tc = rho > 0.0 ? (int)(0.94 * cap / rho) : COLL_TCMAX;
    }
    if (tc < MIN_TILE_CELLS) tc = MIN_TILE_CELLS;
    if (tc > COLL_TCMAX) tc = COLL_TCMAX;
    return tc;
}

void fill_desc(rmp_batch* b, Replica& r)
{
    RepDesc& D = r.desc;
    const rmp_params* p = &r.p;
    char* w = r.ws;
    const Layout& L = r.lay;
    const Sizes& s = r.sz;
    D = RepDesc{};
    for (int d = 0; d < 3; ++d) {
        D.L[d] = p->L[d];
        D.Ld[d] = (double)p->L[d];
        D.halfL[d] = 0.5 * D.Ld[d];
    }
    D.flow = has_flow(p) ? 1 : 0;
    D.walls = p->walls;
    D.wall_n0 = p->wall_density;
    if (p->walls) D.L[2] = p->L[2] + 1;
    for (int d = 0; d < 3; ++d) D.g[d] = p->accel[d];
    D.active = 1;
    D.n = s.n;
    D.ncell = s.ncell;
    D.n_md = r.n_md;
    D.rule = p->rule;
    D.n_chunks = s.n_chunks;
    D.tile_cells = tile_cells_of(b, r.tile_cells, s.ncell, s.n);
    D.n_tiles = (int32_t)((s.ncell + D.tile_cells - 1) / D.tile_cells);
    D.n_scanblk = s.n_scanblk;
    D.cand_cap = s.cand_cap;
    const ChainShape cs = chain_shape_of(b);
    const int K = cs.k;
    const int64_t per_wg = (int64_t)cs.nt * K;
    int G = (int)((s.cand_cap + per_wg - 1) / per_wg);
    if (G < 1) G = 1;
    if (G > s.G) G = s.G;
    D.G = G;
    D.cand_cap = std::min<int64_t>(s.cand_cap, (int64_t)G * per_wg);
    D.chain_k = K;
    {
        // row-major: rank = cell index (KEY_ROW); compact Hilbert: computed in
        // the kernels for a cubic power-of-two box, else the table
        int bits = 0;
        while ((1 << bits) < p->L[0]) bits++;
        const bool cube2 = p->L[0] == p->L[1] && p->L[1] == p->L[2] && (1 << bits) == p->L[0];
        D.hbits = p->cell_order == 0 ? KEY_ROW : (cube2 ? bits : KEY_TABLE);
    }
    D.dt = p->dt;
    D.h = (0.5 * p->dt) / p->mass;
    D.tau = (double)r.n_md * p->dt;
    D.vscale = std::sqrt(p->kT / p->mass);
    D.mass = p->mass;
    D.ca = std::cos(p->alpha);
    D.sa = std::sin(p->alpha);
    D.cat_prob = p->cat_prob;
    D.skin_half2 = (0.5 * p->skin) * (0.5 * p->skin);
    // the chain's per-interval colloid cull holds while list entries move less
    // than cull_me from their interval-start positions (five thermal speeds
    // over tau, plus room for the colloid forces); past it a wave tests every
    // colloid, so the margin sets speed only, never results
    D.cull_me = 5.0 * std::sqrt(p->kT / p->mass) * (r.n_md * p->dt) + 0.5;
    D.cull_margin = D.cull_me + 0.5 * p->skin;
    D.bulk_on = p->bulk_rate > 0.0 ? 1 : 0;
    D.seed = r.seed;
    for (int q = 0; q < 2; ++q) {
        D.x[q] = w + L.x[q];
        D.v[q] = w + L.v[q];
        D.id[q] = (uint32_t*)(w + L.id[q]);
        D.st[q] = (uint8_t*)(w + L.st[q]);
    }
    D.keyrank = (uint64_t*)(w + L.keyrank);
    D.stage = (void*)(w + L.stage);
    D.cflag = (uint8_t*)(w + L.cflag);
    D.count = (uint32_t*)(w + L.count);
    D.start = (uint32_t*)(w + L.start);
    D.scanblk = (uint32_t*)(w + L.scanblk);
    D.chunk_cnt = (uint32_t*)(w + L.chunk_cnt);
    D.chunk_off = (uint32_t*)(w + L.chunk_off);
    D.cand_idx = (uint32_t*)(w + L.cand_idx);
    D.rank_of = (const uint32_t*)(w + L.order);
    D.cell_of = (const uint32_t*)(w + L.order) + s.ncell;
    D.partials = (double*)(w + L.partials);
    D.epart = (double*)(w + L.epart);
    D.tpart = (double*)(w + L.tpart);
    D.bigmask = (uint64_t*)(w + L.bigmask);
    D.ptable = (double*)(w + L.ptable);
    D.obs_part = (double*)(w + L.obs_part);
    D.cp = (ColloidParams*)(w + L.cp);
    D.rs = (RepState*)(w + L.rs);
    D.an = (Analysis*)r.an;
}

ColloidParams make_cp(const rmp_params* p)
{
    ColloidParams c{};
    c.nc = p->n_colloids;
    c.nbonds = p->n_bonds;
    for (int i = 0; i < RMP_MAX_COLLOIDS; ++i) c.body[i] = i;
    for (int i = 0; i < RMP_MAX_COLLOIDS; ++i) c.bond_of[i] = -1;
    for (int i = 0; i < p->n_colloids; ++i) {
        c.catalytic[i] = p->catalytic[i] ? 1 : 0;
        c.ctype[i] = p->ctype[i];
        c.sigma[i] = p->sigma[i];
        c.sig2[i] = p->sigma[i] * p->sigma[i];
        double rc = 0x1.1f59ac3c7d6c0p+0 * p->sigma[i];
        c.rc2[i] = rc * rc;
        c.reachR[i] = rc + p->skin;
        c.epsA[i] = p->eps_A[i];
        c.epsB[i] = p->eps_B[i];
        c.mass[i] = p->colloid_mass[i];
        c.imass[i] = 1.0 / p->colloid_mass[i];
        c.hc[i] = (0.5 * p->dt) / p->colloid_mass[i];
    }
    for (int a = 0; a < 2; ++a)
        for (int q = 0; q < 2; ++q) c.eps_cc[a][q] = p->eps_cc[a][q];
    for (int b = 0; b < p->n_bonds; ++b) {
        c.bond_a[b] = p->bond_a[b];
        c.bond_b[b] = p->bond_b[b];
        c.bond_d[b] = p->bond_d[b];
        c.bond_of[p->bond_a[b]] = b;
        c.bond_of[p->bond_b[b]] = b;
    }
    c.iterative = iterative_rattle(p) ? 1 : 0;
    c.rattle_maxit = p->rattle_maxit;
    c.rattle_tol = p->rattle_tol;
    if (c.iterative)
        for (int i = 0; i < RMP_MAX_COLLOIDS; ++i) c.bond_of[i] = -1;   // no exact bond stage
    // runs of consecutive bonds touching disjoint colloids (greedy, in order)
    c.n_layers = 0;
    for (int b = 0; b < p->n_bonds;) {
        uint32_t used = 0;
        c.layer_start[c.n_layers++] = b;
        while (b < p->n_bonds) {
            const uint32_t m = (1u << p->bond_a[b]) | (1u << p->bond_b[b]);
            if (used & m) break;
            used |= m;
            ++b;
        }
    }
    c.layer_start[c.n_layers] = p->n_bonds;
    // rigid bodies: merge the two bodies joined by a bond into the smaller
    // label until every bond lies inside one body
    for (bool merged = true; merged;) {
        merged = false;
        for (int b = 0; b < p->n_bonds; ++b) {
            const int la = c.body[p->bond_a[b]], lb = c.body[p->bond_b[b]];
            if (la == lb) continue;
            const int keep = la < lb ? la : lb, drop = la < lb ? lb : la;
            for (int i = 0; i < p->n_colloids; ++i)
                if (c.body[i] == drop) c.body[i] = keep;
            merged = true;
        }
    }
    return c;
}

// Hilbert curve (J. Skilling, "Programming the Hilbert curve", AIP Conf.
// Proc. 707 (2004) 381), from the index to the point: the index's bits are
// dealt to the three axes level by level (first axis most significant), the
// Gray code is undone, then the excess work of the forward transform is
// undone from the lowest level up (invert or exchange low bits with the
// first axis).
void hilbert_point(uint64_t h, int bits, uint32_t X[3])
{
    X[0] = X[1] = X[2] = 0;
    for (int k = 0; k < bits; ++k)
        for (int i = 0; i < 3; ++i) X[i] |= (uint32_t)((h >> (3 * k + 2 - i)) & 1u) << k;
    const uint32_t t = X[2] >> 1;
    X[2] ^= X[1];
    X[1] ^= X[0];
    X[0] ^= t;
    for (uint32_t Q = 2; Q < (1u << bits); Q <<= 1) {
        const uint32_t P = Q - 1;
        for (int i = 2; i >= 0; --i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t e = (X[0] ^ X[i]) & P;
                X[0] ^= e;
                X[i] ^= e;
            }
        }
    }
}

// Cell sort order: the box's cells in the order the Hilbert curve of the
// smallest power-of-two cube containing the box visits them (the paper's
// compact-Hilbert cell ordering).  order[0..ncell) = rank of each cell,
// order[ncell..2 ncell) = cell of each rank.
void make_order(Replica& r)
{
    const int32_t* L = r.p.L;
    const int64_t ncell = r.sz.ncell;
    int bits = 0;
    while ((1 << bits) < std::max(L[0], std::max(L[1], L[2]))) bits++;
    r.order.assign(2 * (size_t)ncell, 0u);
    uint32_t* rank_of = r.order.data();
    uint32_t* cell_of = rank_of + ncell;
    int64_t q = 0;
    const uint64_t end = 1ull << (3 * bits);
    if (r.p.cell_order == 0) {
        for (int64_t c = 0; c < ncell; ++c) { rank_of[c] = (uint32_t)c; cell_of[c] = (uint32_t)c; }
        return;
    }
    for (uint64_t h = 0; h < end && q < ncell; ++h) {
        uint32_t X[3];
        hilbert_point(h, bits, X);
        if ((int32_t)X[0] >= L[0] || (int32_t)X[1] >= L[1] || (int32_t)X[2] >= L[2]) continue;
        const int64_t c = X[0] + (int64_t)L[0] * (X[1] + (int64_t)L[1] * X[2]);
        rank_of[c] = (uint32_t)q;
        cell_of[q] = (uint32_t)c;
        q++;
    }
}

void make_ptable(Replica& r)
{
    if (r.ptable_nmd == r.n_md && !r.ptable.empty()) return;
    r.ptable.assign(RMP_PTABLE, 0.0);
    const double kt = r.p.bulk_rate * ((double)r.n_md * r.p.dt);
    for (int q = 0; q < RMP_PTABLE; ++q) r.ptable[q] = -std::expm1(-(kt * (double)q));
    r.ptable_nmd = r.n_md;
}

// recompute the work-list prefixes and upload descriptors
rmp_status sync_ctl(rmp_batch* b)
{
    if (!b->dirty) return RMP_OK;
    const int S = b->nslots;
    for (int k = 0; k < 6; ++k) b->hprefix[k].assign(S + 1, 0);
    b->have_rule[0] = b->have_rule[1] = false;
    b->multi_scan = false;
    b->max_scanblk = 0;
    b->any_analysis = false;
    b->any_iterative = false;
    b->n_total = 0;
    for (int r = 0; r < S; ++r) {
        Replica& R = b->reps[r];
        int items[6] = {0, 0, 0, 0, 1, 1};
        if (R.used) {
            fill_desc(b, R);
            items[PF_CHUNK] = R.desc.n_chunks;
            items[PF_TILE] = R.desc.n_tiles;
            items[PF_SCAN] = R.desc.n_scanblk;
            items[PF_CHAIN] = R.desc.G;
            b->have_rule[R.p.rule] = true;
            if (R.desc.n_scanblk > 1) b->multi_scan = true;
            b->max_scanblk = std::max(b->max_scanblk, R.desc.n_scanblk);
            if (R.an) b->any_analysis = true;
            if (iterative_rattle(&R.p)) b->any_iterative = true;
            b->n_total += R.p.n_solvent;
            b->hdesc[r] = R.desc;
        } else {
            b->hdesc[r] = RepDesc{};
            b->hdesc[r].active = 0;
        }
        for (int k = 0; k < 6; ++k) b->hprefix[k][r + 1] = b->hprefix[k][r] + items[k];
    }
    for (int k = 0; k < 6; ++k) b->totals[k] = b->hprefix[k][S];
    b->nc_common = -1;
    bool first = true;
    for (int r = 0; r < S; ++r) {
        if (!b->reps[r].used) continue;
        const int nc = b->reps[r].p.n_colloids;
        if (first) b->nc_common = nc;
        else if (b->nc_common != nc) b->nc_common = -1;
        first = false;
    }
    HIPCHK(hipMemcpyAsync(b->d_desc, b->hdesc.data(), sizeof(RepDesc) * S, hipMemcpyHostToDevice, b->stream));
    for (int k = 0; k < 6; ++k)
        HIPCHK(hipMemcpyAsync(b->d_prefix[k], b->hprefix[k].data(), 4 * (S + 1), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->dirty = false;
    b->graph_valid = false;
    return RMP_OK;
}

uint64_t barrier_budget(const rmp_batch* b)
{
    return b->tun.barrier_budget_us > 0 ? (uint64_t)b->tun.barrier_budget_us * 100u : BARRIER_BUDGET_TICKS;
}

Work work(const rmp_batch* b, int kind)
{
    Work w;
    w.desc = b->d_desc;
    w.prefix = b->d_prefix[kind];
    w.tick = b->d_tick;
    w.nrep = b->nslots;
    w.flags = 0;
    w.budget = barrier_budget(b);
    return w;
}

// event-timed launch (profiling mode, no graph)
struct Timer {
    rmp_batch* b;
    int kind;
    hipStream_t s;
    size_t i0;
    Timer(rmp_batch* bb, int k, hipStream_t st) : b(bb), kind(k), s(st), i0(0)
    {
        if (!b->prof) return;
        if (b->ev_used + 2 > b->ev.size()) {
            size_t add = 512;
            for (size_t q = 0; q < add; ++q) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                b->ev.push_back(e);
                b->ev_kind.push_back(-1);
            }
        }
        i0 = b->ev_used;
        b->ev_used += 2;
        b->ev_kind[i0] = kind;
        (void)hipEventRecord(b->ev[i0], s);
    }
    ~Timer()
    {
        if (!b->prof) return;
        (void)hipEventRecord(b->ev[i0 + 1], s);
    }
};

rmp_status flush_profile(rmp_batch* b)
{
    if (!b->prof || b->ev_used == 0) return RMP_OK;
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipStreamSynchronize(b->side));
    for (size_t i = 0; i + 1 < b->ev_used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b->ev[i], b->ev[i + 1]) == hipSuccess) {
            b->prof_ms[b->ev_kind[i]] += ms;
            b->prof_cnt[b->ev_kind[i]] += 1;
        }
    }
    b->ev_used = 0;
    return RMP_OK;
}

template <class T, int K, int NT>
void launch_chain_shape(rmp_batch* b, hipStream_t s, dim3 g, bool ticket, int nc, const Work& w)
{
    const dim3 blk(NT);
    if (ticket && nc == 2) hipLaunchKernelGGL((k_chain<T, K, true, 2, NT>), g, blk, 0, s, w);
    else if (ticket && nc == 1) hipLaunchKernelGGL((k_chain<T, K, true, 1, NT>), g, blk, 0, s, w);
    else if (ticket) hipLaunchKernelGGL((k_chain<T, K, true, 0, NT>), g, blk, 0, s, w);
    else if (nc == 2) hipLaunchKernelGGL((k_chain<T, K, false, 2, NT>), g, blk, 0, s, w);
    else if (nc == 1) hipLaunchKernelGGL((k_chain<T, K, false, 1, NT>), g, blk, 0, s, w);
    else hipLaunchKernelGGL((k_chain<T, K, false, 0, NT>), g, blk, 0, s, w);
}

template <class T>
rmp_status launch_chain(rmp_batch* b, hipStream_t s)
{
    Timer tm(b, KN_CHAIN, s);
    const ChainShape cs = chain_shape_of(b);
    const dim3 g(b->totals[PF_CHAIN]);
    const int nc = chain_nc(b);
    // more workgroups than the device holds at once: ticketed work list
    const bool ticket = b->totals[PF_CHAIN] > b->chain_resident[nc ? 1 : 0][cs.q];
    Work w = work(b, PF_CHAIN);
    // small launches: the chain's dependent steps are the whole critical
    // path, so its waves take issue priority over the streaming kernel that
    // shares the compute units (measured: 32^3 +2 %; at 128^3, where the
    // streaming kernel is long, -1.5 %, hence the size limit)
    if (b->n_total <= CHAIN_PRIO_MAX_PARTICLES) w.flags |= WORK_CHAIN_PRIO;
    switch (cs.q) {
        case 0: launch_chain_shape<T, 1, 256>(b, s, g, ticket, nc, w); break;
        case 1: launch_chain_shape<T, 2, 256>(b, s, g, ticket, nc, w); break;
        case 2: launch_chain_shape<T, 4, 256>(b, s, g, ticket, nc, w); break;
        case 3: launch_chain_shape<T, 1, 512>(b, s, g, ticket, nc, w); break;
        default: launch_chain_shape<T, 2, 512>(b, s, g, ticket, nc, w); break;
    }
    return last_launch("k_chain");
}

template <class T>
rmp_status launch_list(rmp_batch* b)
{
    hipStream_t s = b->stream;
    if (b->totals[PF_CHUNK] == 0) return RMP_OK;
    {
        Timer tm(b, KN_LIST, s);
        hipLaunchKernelGGL((k_list<T>), dim3(b->totals[PF_CHUNK]), dim3(256), 0, s, work(b, PF_CHUNK));
    }
    {
        Timer tm(b, KN_CHUNKSCAN, s);
        hipLaunchKernelGGL(k_chunk_scan, dim3(b->nslots), dim3(1024), 0, s, work(b, PF_IDENT), 0);
    }
    {
        Timer tm(b, KN_CANDW, s);
        hipLaunchKernelGGL(k_cand_write, dim3(b->totals[PF_CHUNK]), dim3(256), 0, s, work(b, PF_CHUNK));
    }
    return last_launch("list build");
}

template <class T, int RULE>
void launch_collide_rule(rmp_batch* b, hipStream_t s)
{
    const dim3 g(b->totals[PF_TILE]);
    const Work w = work(b, PF_TILE);
    const int xcd = b->tun.collide_xcd;
    const int nt = collide_nt(b), ppt = collide_ppt(b);
    if (nt == 512 && ppt == 2) hipLaunchKernelGGL((k_collide<T, RULE, 512, 2>), g, dim3(512), 0, s, w, xcd);
    else if (nt == 512) hipLaunchKernelGGL((k_collide<T, RULE, 512, 1>), g, dim3(512), 0, s, w, xcd);
    else if (ppt == 2) hipLaunchKernelGGL((k_collide<T, RULE, 256, 2>), g, dim3(256), 0, s, w, xcd);
    else hipLaunchKernelGGL((k_collide<T, RULE, 256, 1>), g, dim3(256), 0, s, w, xcd);
}

// every collision launch is followed by the pass over the cells beyond a
// group's capacity (tiles without any such cell cost one mask load each)
template <class T>
void launch_collide(rmp_batch* b, hipStream_t s, int rule)
{
    const int items = b->totals[PF_TILE];
    const dim3 gb((unsigned)((items + 63) / 64));
    if (rule == 0) {
        launch_collide_rule<T, 0>(b, s);
        hipLaunchKernelGGL((k_collide_big<T, 0>), gb, dim3(256), 0, s, work(b, PF_TILE), items);
    } else {
        launch_collide_rule<T, 1>(b, s);
        hipLaunchKernelGGL((k_collide_big<T, 1>), gb, dim3(256), 0, s, work(b, PF_TILE), items);
    }
}

// one interval for every occupied replica
template <class T>
rmp_status launch_interval(rmp_batch* b, hipStream_t s)
{
    const int nch = b->totals[PF_CHUNK];
    if (nch == 0) return RMP_OK;
    // fork: the MD chain runs on the side stream next to the streaming
    // kernel (chain_serial: before it, on the same stream)
    const bool serial = b->tun.chain_serial != 0;
    if (!serial) {
        HIPCHK(hipEventRecord(b->fork, s));
        HIPCHK(hipStreamWaitEvent(b->side, b->fork, 0));
    }
    rmp_status st = launch_chain<T>(b, serial ? s : b->side);
    if (st != RMP_OK) return st;
    {
        Timer tm(b, KN_STREAM, s);
        // stream_block threads holding stream_ppt particles each (1, 2 or 4)
        int bs = b->tun.stream_block;
        if (bs != 64 && bs != 128 && bs != 256) bs = 256;
        const int ppt = b->tun.stream_ppt == 2 || b->tun.stream_ppt == 4 ? b->tun.stream_ppt : 1;
        const int wpc = CHUNK / (bs * ppt);
        const dim3 g(nch * wpc);
        if (ppt == 4) hipLaunchKernelGGL((k_stream_bin<T, 4>), g, dim3(bs), 0, s, work(b, PF_CHUNK), wpc);
        else if (ppt == 2) hipLaunchKernelGGL((k_stream_bin<T, 2>), g, dim3(bs), 0, s, work(b, PF_CHUNK), wpc);
        else hipLaunchKernelGGL((k_stream_bin<T, 1>), g, dim3(bs), 0, s, work(b, PF_CHUNK), wpc);
    }
    if (!serial) {
        HIPCHK(hipEventRecord(b->join, b->side));
        HIPCHK(hipStreamWaitEvent(s, b->join, 0));
    }
    // small grids: each scan block sums the counts before it itself
    const int direct = b->max_scanblk <= SCAN_DIRECT_BLOCKS ? 1 : 0;
    if (b->multi_scan && !direct) {
        Timer tm(b, KN_SCANB, s);
        hipLaunchKernelGGL(k_scan_blocks, dim3(b->totals[PF_SCAN]), dim3(1024), 0, s, work(b, PF_SCAN));
    }
    {
        Timer tm(b, KN_SCANF, s);
        hipLaunchKernelGGL(k_scan_final, dim3(b->totals[PF_SCAN]), dim3(1024), 0, s, work(b, PF_SCAN), direct);
    }
    {
        Timer tm(b, KN_SCATTER, s);
        hipLaunchKernelGGL((k_scatter<T>), dim3(nch), dim3(256), 0, s, work(b, PF_CHUNK));
    }
    {
        Timer tm(b, KN_COLLIDE, s);
        for (int rule = 0; rule < 2; ++rule)
            if (b->have_rule[rule]) launch_collide<T>(b, s, rule);
    }
    {
        Timer tm(b, KN_CHUNKSCAN, s);
        hipLaunchKernelGGL(k_chunk_scan, dim3(b->nslots), dim3(1024), 0, s, work(b, PF_IDENT), 1);
    }
    {
        Timer tm(b, KN_CANDW, s);
        hipLaunchKernelGGL(k_cand_write, dim3(nch), dim3(256), 0, s, work(b, PF_CHUNK));
    }
    if (b->any_analysis) {
        Timer tm(b, KN_ANALYSIS, s);
        hipLaunchKernelGGL((k_analysis<T>), dim3(nch), dim3(256), 0, s, work(b, PF_CHUNK));
    }
    return last_launch("interval");
}

rmp_status run_interval(rmp_batch* b, hipStream_t s)
{
    return b->precision == 32 ? launch_interval<float>(b, s) : launch_interval<double>(b, s);
}

rmp_status capture_graph(rmp_batch* b)
{
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    // capture on the library's private stream (the caller's stream may be
    // the legacy default stream, which cannot be captured); the graph is
    // then launched on the caller's stream
    HIPCHK(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    rmp_status st = run_interval(b, b->capture);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->capture, &g);
    if (e != hipSuccess) note_error("hipStreamEndCapture", e);
    if (st != RMP_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != RMP_OK ? st : RMP_EHIP;
    }
    b->graph = g;
    HIPCHK(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    b->graph_valid = true;
    return RMP_OK;
}

// make every occupied replica's Verlet list valid for its current n_md
rmp_status ensure_lists(rmp_batch* b)
{
    bool need = false;
    for (int r = 0; r < b->nslots; ++r) {
        Replica& R = b->reps[r];
        if (R.used && (!R.list_valid || R.list_nmd != R.n_md)) need = true;
    }
    if (!need) return RMP_OK;
    rmp_status st = b->precision == 32 ? launch_list<float>(b) : launch_list<double>(b);
    if (st != RMP_OK) return st;
    for (int r = 0; r < b->nslots; ++r) {
        Replica& R = b->reps[r];
        if (R.used) { R.list_valid = true; R.list_nmd = R.n_md; }
    }
    return RMP_OK;
}

rmp_status batch_ticks(rmp_batch* b, int32_t n)
{
    if (n < 0) return RMP_EINVAL;
    rmp_status st = sync_ctl(b);
    if (st != RMP_OK) return st;
    st = ensure_lists(b);
    if (st != RMP_OK) return st;
    const bool use_graph = b->tun.use_graph > 0 && !b->prof;
    for (int32_t k = 0; k < n; ++k) {
        if (use_graph) {
            if (!b->graph_valid) {
                st = capture_graph(b);
                if (st != RMP_OK) return st;
            }
            HIPCHK(hipGraphLaunch(b->gexec, b->stream));
        } else {
            st = run_interval(b, b->stream);
            if (st != RMP_OK) return st;
        }
        if (b->prof && b->ev_used > 3000) {
            st = flush_profile(b);
            if (st != RMP_OK) return st;
        }
    }
    return RMP_OK;
}

// initialise one replica's state in its workspace
rmp_status init_replica(rmp_batch* b, int slot)
{
    Replica& R = b->reps[slot];
    hipStream_t s = b->stream;
    HIPCHK(hipMemsetAsync(R.ws, 0, R.lay.total, s));
    ColloidParams cp = make_cp(&R.p);
    RepState rs{};
    rs.list_nmd = -1;
    for (int c = 0; c < R.p.n_colloids; ++c)
        for (int d = 0; d < 3; ++d) rs.X[c][d] = R.p.colloid_x[c][d];
    HIPCHK(hipMemcpyAsync(R.ws + R.lay.cp, &cp, sizeof(cp), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(R.ws + R.lay.rs, &rs, sizeof(rs), hipMemcpyHostToDevice, s));
    make_ptable(R);
    HIPCHK(hipMemcpyAsync(R.ws + R.lay.ptable, R.ptable.data(), RMP_PTABLE * 8, hipMemcpyHostToDevice, s));
    make_order(R);
    HIPCHK(hipMemcpyAsync(R.ws + R.lay.order, R.order.data(), R.order.size() * 4, hipMemcpyHostToDevice, s));
    b->dirty = true;
    rmp_status st = sync_ctl(b);
    if (st != RMP_OK) return st;
    const RepDesc* dD = b->d_desc + slot;
    double* mean = (double*)(R.ws + R.lay.mean);
    const int nch = R.desc.n_chunks;
    if (R.p.precision == 32) {
        hipLaunchKernelGGL((k_init<float>), dim3(nch), dim3(256), 0, s, dD);
        hipLaunchKernelGGL(k_init_mean, dim3(1), dim3(256), 0, s, dD, mean);
        hipLaunchKernelGGL((k_init_sub<float>), dim3(nch), dim3(256), 0, s, dD, (const double*)mean);
    } else {
        hipLaunchKernelGGL((k_init<double>), dim3(nch), dim3(256), 0, s, dD);
        hipLaunchKernelGGL(k_init_mean, dim3(1), dim3(256), 0, s, dD, mean);
        hipLaunchKernelGGL((k_init_sub<double>), dim3(nch), dim3(256), 0, s, dD, (const double*)mean);
    }
    rmp_status le = last_launch("init");
    if (le != RMP_OK) return le;
    R.list_valid = false;
    return RMP_OK;
}

rmp_status admit(rmp_batch* b, int slot, const rmp_params* p, uint64_t seed, int32_t n_md,
                 void* ws, size_t bytes)
{
    rmp_status st = validate(p);
    if (st != RMP_OK) return st;
    if (p->precision != b->precision) return RMP_EINVAL;
    if (n_md < 1) return RMP_EINVAL;
    Layout L = layout_of(p);
    if (!ws || bytes < L.total) return RMP_ENOMEM;
    if (((uintptr_t)ws) % ALIGN) return RMP_EINVAL;
    Replica& R = b->reps[slot];
    R = Replica{};
    R.used = true;
    R.p = *p;
    R.seed = seed;
    R.n_md = n_md;
    R.ws = (char*)ws;
    R.lay = L;
    R.sz = sizes_of(p);
    return init_replica(b, slot);
}

rmp_status batch_init(rmp_batch* b, int32_t nslots, int32_t precision, void* ctl, size_t bytes,
                      void* stream)
{
    if (nslots < 1 || nslots > 4096 || (precision != 32 && precision != 64)) return RMP_EINVAL;
    if (!ctl || bytes < ctl_bytes_for(nslots)) return RMP_ENOMEM;
    if (((uintptr_t)ctl) % ALIGN) return RMP_EINVAL;
    b->nslots = nslots;
    b->precision = precision;
    b->stream = (hipStream_t)stream;
    HIPCHK(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->join, hipEventDisableTiming));
    b->ctl = (char*)ctl;
    size_t o = 0;
    b->d_desc = (RepDesc*)(b->ctl + o);
    o += aup(sizeof(RepDesc) * (size_t)nslots);
    for (int k = 0; k < 6; ++k) {
        b->d_prefix[k] = (int32_t*)(b->ctl + o);
        o += aup(4 * (size_t)(nslots + 1));
    }
    b->d_tick = (uint32_t*)(b->ctl + o);
    o += aup(16);
    HIPCHK(hipMemsetAsync(b->d_tick, 0, 16, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    {
        int dev = 0, ncu = 0;
        HIPCHK(hipGetDevice(&dev));
        b->device = dev;
        rmp_status sst = take_scratch_address(dev);
        if (sst != RMP_OK) return sst;
        HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        // per shape, for the generic and the one- or two-colloid variants
        // (the ticketed instantiations use the same resources)
        int per[2][5] = {};
        if (precision == 64) {
            HIPCHK(occupancy_of<double>(per));
        } else {
            HIPCHK(occupancy_of<float>(per));
        }
        for (int v = 0; v < 2; ++v)
            for (int q = 0; q < 5; ++q) b->chain_resident[v][q] = std::max(1, per[v][q]) * std::max(1, ncu);
    }
    b->reps.assign(nslots, Replica{});
    b->hdesc.assign(nslots, RepDesc{});
    b->dirty = true;
    return RMP_OK;
}

void batch_release(rmp_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto e : b->ev) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    b->gexec = nullptr; b->graph = nullptr; b->fork = b->join = nullptr; b->side = nullptr;
    b->capture = nullptr;
    b->ev.clear();
}

// scr: nullptr for the workspace's partials and a host-side sum; else the
// device's static scratch, which takes the partials and their totals (the
// allocation-free form; the two give identical results)
template <class T>
rmp_status observe(rmp_batch* b, int slot, rmp_obs* o, char* scr = nullptr)
{
    Replica& R = b->reps[slot];
    hipStream_t s = b->stream;
    rmp_status st = sync_ctl(b);
    if (st != RMP_OK) return st;
    // the observation kernel runs over this replica only: a one-replica work
    // list whose prefix is the identity prefix (prefix[0] == 0)
    const int cnt = R.desc.n_chunks;
    const size_t part_bytes = (size_t)cnt * 8 * 8;
    if (scr && part_bytes + 64 > RMP_STATIC_SCRATCH_BYTES) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "rmp_observables_noalloc: %d particle chunks need %zu bytes of static scratch, "
                      "more than its %zu", cnt, part_bytes + 64, (size_t)RMP_STATIC_SCRATCH_BYTES);
        return RMP_ENOMEM;
    }
    Work w;
    w.desc = b->d_desc + slot;
    w.prefix = b->d_prefix[PF_REP];
    w.nrep = 1;
    w.flags = 0;
    w.budget = barrier_budget(b);
    double* part = scr ? (double*)scr : nullptr;
    hipLaunchKernelGGL((k_observe<T>), dim3(cnt), dim3(256), 0, s, w, part);
    st = last_launch("k_observe");
    if (st != RMP_OK) return st;
    double P[3] = {0, 0, 0}, ke = 0, nb = 0;
    RepState rs;
    if (scr) {
        double* tot = (double*)(scr + part_bytes);
        hipLaunchKernelGGL(k_observe_total, dim3(1), dim3(64), 0, s, (const double*)part, cnt, tot);
        st = last_launch("k_observe_total");
        if (st != RMP_OK) return st;
        double t[5];
        HIPCHK(hipMemcpyAsync(t, tot, sizeof(t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&rs, R.ws + R.lay.rs, sizeof(rs), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        P[0] = t[0]; P[1] = t[1]; P[2] = t[2]; ke = t[3]; nb = t[4];
    } else {
        std::vector<double> hpart((size_t)cnt * 8);
        HIPCHK(hipMemcpyAsync(hpart.data(), R.ws + R.lay.obs_part, part_bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&rs, R.ws + R.lay.rs, sizeof(rs), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int k = 0; k < cnt; ++k) {
            for (int d = 0; d < 3; ++d) P[d] += hpart[(size_t)k * 8 + d];
            ke += hpart[(size_t)k * 8 + 3];
            nb += hpart[(size_t)k * 8 + 4];
        }
    }
    if (b->prof) flush_profile(b);
    std::memset(o, 0, sizeof(*o));
    double kec = 0.0;
    for (int d = 0; d < 3; ++d) o->momentum[d] = R.p.mass * P[d];
    for (int c = 0; c < R.p.n_colloids; ++c) {
        double v2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            o->momentum[d] += R.p.colloid_mass[c] * rs.V[c][d];
            v2 += rs.V[c][d] * rs.V[c][d];
            o->colloid_X[c][d] = rs.X[c][d];
            o->colloid_V[c][d] = rs.V[c][d];
        }
        kec += 0.5 * R.p.colloid_mass[c] * v2;
    }
    o->ke_solvent = 0.5 * R.p.mass * ke;
    o->ke_colloid = kec;
    o->potential = rs.U;
    o->temperature = rs.T_cells > 0 ? rs.T_sum / (3.0 * rs.T_cells) : 0.0;
    o->n_cells_T = (int64_t)rs.T_cells;
    o->e_rxn = rs.e_rxn;
    o->n_B = (int64_t)nb;
    o->n_A = R.sz.n - o->n_B;
    o->n_cat_flips = rs.n_cat;
    o->n_bulk_flips = rs.n_bulk;
    o->md_step = rs.md_step;
    o->coll_step = rs.coll_step;
    o->n_candidates = rs.n_cand_used;
    o->flags = rs.flags;
    return rs.flags ? RMP_EDEVICE : RMP_OK;
}

template <class T>
rmp_status get_state_t(rmp_batch* b, int slot, rmp_host_state* dst)
{
    Replica& R = b->reps[slot];
    hipStream_t s = b->stream;
    HIPCHK(hipStreamSynchronize(s));
    RepState rs;
    HIPCHK(hipMemcpy(&rs, R.ws + R.lay.rs, sizeof(rs), hipMemcpyDeviceToHost));
    const int cur = (int)(rs.coll_step & 1);
    const int64_t n = R.sz.n;
    if (dst->x || dst->v) {
        std::vector<T> buf((size_t)3 * n);
        if (dst->x) {
            HIPCHK(hipMemcpy(buf.data(), R.ws + R.lay.x[cur], 3 * n * sizeof(T), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < 3 * n; ++i) dst->x[i] = (double)buf[i];
        }
        if (dst->v) {
            HIPCHK(hipMemcpy(buf.data(), R.ws + R.lay.v[cur], 3 * n * sizeof(T), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < 3 * n; ++i) dst->v[i] = (double)buf[i];
        }
    }
    if (dst->id) HIPCHK(hipMemcpy(dst->id, R.ws + R.lay.id[cur], 4 * n, hipMemcpyDeviceToHost));
    if (dst->state) HIPCHK(hipMemcpy(dst->state, R.ws + R.lay.st[cur], n, hipMemcpyDeviceToHost));
    for (int c = 0; c < R.p.n_colloids; ++c)
        for (int d = 0; d < 3; ++d) {
            if (dst->X) dst->X[3 * c + d] = rs.X[c][d];
            if (dst->V) dst->V[3 * c + d] = rs.V[c][d];
        }
    dst->md_step = rs.md_step;
    dst->coll_step = rs.coll_step;
    return RMP_OK;
}

// A state handed in by the caller (pure host check, before any upload):
// solvent positions inside the box, velocities finite (also once rounded to
// the storage precision), ids a permutation of 0 .. N-1, state bytes with
// only the species and catalysis bits, colloid positions and velocities
// finite, and no solvent particle deep inside a colloid core (r < sigma/2,
// where the WCA potential exceeds 1.6e4 eps: unreachable by a thermal
// state, so the input is corrupt).
rmp_status check_state(const rmp_params* p, const rmp_host_state* src)
{
    if (!p || !src) return RMP_EINVAL;
    if (validate(p) != RMP_OK) return RMP_EINVAL;
    const int64_t n = p->n_solvent;
    if (n > 0 && (!src->x || !src->v || !src->id || !src->state)) return RMP_EINVAL;
    if (p->n_colloids > 0 && (!src->X || !src->V)) return RMP_EINVAL;
    if (src->md_step < 0 || src->coll_step < 0) return RMP_EINVAL;
    for (int d = 0; d < 3; ++d)
        for (int64_t i = 0; i < n; ++i) {
            const double xv = src->x[d * n + i];
            if (!(xv >= 0.0 && xv < (double)p->L[d])) return RMP_EINVAL;
            const double vv = src->v[d * n + i];
            if (!std::isfinite(vv)) return RMP_EINVAL;
            if (p->precision == 32 && !std::isfinite((float)vv)) return RMP_EINVAL;
        }
    std::vector<uint8_t> seen((size_t)n, 0);
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t id = src->id[i];
        if ((int64_t)id >= n || seen[id]) return RMP_EINVAL;
        seen[id] = 1;
        if (src->state[i] > 3) return RMP_EINVAL;
    }
    double Xw[RMP_MAX_COLLOIDS][3];
    for (int c = 0; c < p->n_colloids; ++c)
        for (int d = 0; d < 3; ++d) {
            if (!std::isfinite(src->X[3 * c + d]) || !std::isfinite(src->V[3 * c + d])) return RMP_EINVAL;
            const double L = (double)p->L[d];
            double w = std::fmod(src->X[3 * c + d], L);
            if (w < 0.0) w += L;
            Xw[c][d] = w;
        }
    for (int c = 0; c < p->n_colloids; ++c) {
        const double core2 = 0.25 * p->sigma[c] * p->sigma[c];
        for (int64_t i = 0; i < n; ++i) {
            double r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double L = (double)p->L[d];
                double dd = src->x[d * n + i] - Xw[c][d];
                if (dd > 0.5 * L) dd -= L;
                else if (dd < -0.5 * L) dd += L;
                r2 += dd * dd;
            }
            if (r2 < core2) return RMP_EINVAL;
        }
    }
    return RMP_OK;
}

template <class T>
rmp_status set_state_t(rmp_batch* b, int slot, const rmp_host_state* src)
{
    Replica& R = b->reps[slot];
    rmp_status cst = check_state(&R.p, src);
    if (cst != RMP_OK) return cst;
    hipStream_t s = b->stream;
    HIPCHK(hipStreamSynchronize(s));
    RepState rs;
    HIPCHK(hipMemcpy(&rs, R.ws + R.lay.rs, sizeof(rs), hipMemcpyDeviceToHost));
    const int64_t n = R.sz.n;
    const int cur = (int)(src->coll_step & 1);
    std::vector<T> buf((size_t)3 * n);
    for (int d = 0; d < 3; ++d)
        for (int64_t i = 0; i < n; ++i) {
            T xt = (T)src->x[d * n + i];
            if ((double)xt >= (double)R.p.L[d]) xt = (T)0;
            buf[d * n + i] = xt;
        }
    HIPCHK(hipMemcpy(R.ws + R.lay.x[cur], buf.data(), 3 * n * sizeof(T), hipMemcpyHostToDevice));
    for (int64_t i = 0; i < 3 * n; ++i) buf[i] = (T)src->v[i];
    HIPCHK(hipMemcpy(R.ws + R.lay.v[cur], buf.data(), 3 * n * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(R.ws + R.lay.id[cur], src->id, 4 * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(R.ws + R.lay.st[cur], src->state, n, hipMemcpyHostToDevice));
    for (int c = 0; c < R.p.n_colloids; ++c)
        for (int d = 0; d < 3; ++d) {
            rs.X[c][d] = src->X[3 * c + d];
            rs.V[c][d] = src->V[3 * c + d];
            rs.F[c][d] = 0.0;
        }
    rs.md_step = src->md_step;
    rs.coll_step = src->coll_step;
    HIPCHK(hipMemcpy(R.ws + R.lay.rs, &rs, sizeof(rs), hipMemcpyHostToDevice));
    // the MD chain's exchange words carry epochs derived from the step
    // counters; a state that sets the counters back must not meet words left
    // from the same epochs (epochs start at 1, so zero words never match)
    HIPCHK(hipMemset(R.ws + R.lay.partials, 0, R.lay.epart - R.lay.partials));
    R.list_valid = false;
    return RMP_OK;
}

rmp_status slot_ok(rmp_batch* b, int32_t slot)
{
    if (!b) return RMP_EINVAL;
    if (slot < 0 || slot >= b->nslots) return RMP_EINVAL;
    if (!b->reps[slot].used) return RMP_ESTATE;
    return RMP_OK;
}

}  // namespace

// ===================================================================== ABI

// ------------------------------------------------------------ dimer analysis
namespace {

struct AnLayout {
    size_t hist, series, series_t, msd, total;
};

rmp_status an_validate(const rmp_params* p, const rmp_analysis_params* a)
{
    if (!p || !a) return RMP_EINVAL;
    if (p->n_bonds < 1 || p->n_bonds > RMP_MAX_COLLOIDS) return RMP_EINVAL;
    if (a->every < 1 || a->series_cap < 1 || a->hist_nz < 1 || a->hist_nr < 1) return RMP_EINVAL;
    if ((int64_t)a->hist_nz * a->hist_nr > ((int64_t)1 << 24)) return RMP_EINVAL;
    if (a->series_cap > (1 << 26)) return RMP_EINVAL;
    if (!(a->hist_zmax > 0.0) || !(a->hist_rmax > 0.0) || !std::isfinite(a->hist_zmax) ||
        !std::isfinite(a->hist_rmax))
        return RMP_EINVAL;
    return RMP_OK;
}

AnLayout an_layout(const rmp_params* p, const rmp_analysis_params* a)
{
    const size_t nb = (size_t)p->n_bonds, cap = (size_t)a->series_cap;
    AnLayout L{};
    size_t o = aup(sizeof(Analysis));
    L.hist = o;
    o = aup(o + nb * 2 * (size_t)a->hist_nz * (size_t)a->hist_nr * 8);
    L.series = o;
    o = aup(o + cap * nb * RMP_SERIES_FIELDS * 8);
    L.series_t = o;
    o = aup(o + cap * 8);
    L.msd = o;
    o = aup(o + nb * cap * 8);
    L.total = o;
    return L;
}

rmp_status an_attach(rmp_batch* b, int slot, const rmp_analysis_params* a, void* buf, size_t bytes)
{
    Replica& R = b->reps[slot];
    rmp_status st = an_validate(&R.p, a);
    if (st != RMP_OK) return st;
    const AnLayout L = an_layout(&R.p, a);
    if (!buf || bytes < L.total) return RMP_ENOMEM;
    if (((uintptr_t)buf) % ALIGN) return RMP_EINVAL;
    char* w = (char*)buf;
    Analysis h{};
    h.every = a->every;
    h.cap = a->series_cap;
    h.nz = a->hist_nz;
    h.nr = a->hist_nr;
    h.nb = R.p.n_bonds;
    h.zmax = a->hist_zmax;
    h.rmax = a->hist_rmax;
    h.inv_dz = (double)a->hist_nz / (2.0 * a->hist_zmax);
    h.inv_dr = (double)a->hist_nr / a->hist_rmax;
    // sqrt(rho2) * inv_dr >= nr for every rho2 at or beyond this bound
    const double rs = a->hist_rmax * (1.0 + 1e-6);
    h.skip_r2 = rs * rs;
    // a counted particle has z^2 + rho^2 < zmax^2 + rmax^2 up to rounding
    h.cull_r = std::sqrt(a->hist_zmax * a->hist_zmax + a->hist_rmax * a->hist_rmax) * (1.0 + 1e-6);
    h.hist = (uint64_t*)(w + L.hist);
    h.series = (double*)(w + L.series);
    h.series_t = (int64_t*)(w + L.series_t);
    h.msd = (double*)(w + L.msd);
    // queued intervals may still sample into a previous buffer
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipMemsetAsync(buf, 0, L.total, b->stream));
    HIPCHK(hipMemcpyAsync(buf, &h, sizeof(h), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    R.an = w;
    R.anp = *a;
    b->dirty = true;
    return RMP_OK;
}

rmp_status an_detach(rmp_batch* b, int slot)
{
    HIPCHK(hipStreamSynchronize(b->stream));
    b->reps[slot].an = nullptr;
    b->dirty = true;
    return RMP_OK;
}

rmp_status an_read(rmp_batch* b, int slot, rmp_analysis_out* out)
{
    const Replica& R = b->reps[slot];
    if (!R.an || !out) return RMP_ESTATE;
    HIPCHK(hipStreamSynchronize(b->stream));
    Analysis h{};
    HIPCHK(hipMemcpy(&h, R.an, sizeof(h), hipMemcpyDeviceToHost));
    out->n_samples = h.n_samples;
    out->n_dropped = h.n_dropped;
    const size_t nb = (size_t)h.nb;
    if (out->md_step && h.n_samples > 0)
        HIPCHK(hipMemcpy(out->md_step, h.series_t, (size_t)h.n_samples * 8, hipMemcpyDeviceToHost));
    if (out->series && h.n_samples > 0)
        HIPCHK(hipMemcpy(out->series, h.series, (size_t)h.n_samples * nb * RMP_SERIES_FIELDS * 8,
                         hipMemcpyDeviceToHost));
    if (out->hist)
        HIPCHK(hipMemcpy(out->hist, h.hist, nb * 2 * (size_t)h.nz * (size_t)h.nr * 8,
                         hipMemcpyDeviceToHost));
    return RMP_OK;
}

rmp_status an_msd(rmp_batch* b, int slot, int32_t max_lag, double* msd)
{
    const Replica& R = b->reps[slot];
    if (!R.an) return RMP_ESTATE;
    if (!msd || max_lag < 0 || max_lag >= R.anp.series_cap) return RMP_EINVAL;
    const int nb = R.p.n_bonds;
    const int64_t threads = (int64_t)nb * (max_lag + 1);
    Analysis* A = (Analysis*)R.an;
    hipLaunchKernelGGL(k_msd, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, b->stream, A, max_lag);
    rmp_status le = last_launch("k_msd");
    if (le != RMP_OK) return le;
    const AnLayout L = an_layout(&R.p, &R.anp);
    const double* dmsd = (const double*)(R.an + L.msd);
    for (int k = 0; k < nb; ++k)
        HIPCHK(hipMemcpyAsync(msd + (size_t)k * (max_lag + 1), dmsd + (size_t)k * R.anp.series_cap,
                              (size_t)(max_lag + 1) * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return RMP_OK;
}

}  // namespace

extern "C" {

const char* rmp_last_error(void) { return g_last_error; }

const char* rmp_status_string(rmp_status st)
{
    switch (st) {
    case RMP_OK: return "ok";
    case RMP_EINVAL: return "invalid argument";
    case RMP_ENOMEM: return "workspace too small";
    case RMP_EHIP: return "HIP runtime error";
    case RMP_EDEVICE: return "device flag set";
    case RMP_ESTATE: return "invalid state for this call";
    }
    return "unknown status";
}

size_t rmp_workspace_bytes(const rmp_params* p, rmp_status* st)
{
    rmp_status s = validate(p);
    if (st) *st = s;
    if (s != RMP_OK) return 0;
    return aup(layout_of(p).total) + ctl_bytes_for(1);
}

rmp_status rmp_init_system(const rmp_params* p, uint64_t seed, void* d_workspace,
                           size_t workspace_bytes, void* stream, rmp_system** out)
{
    if (!out) return RMP_EINVAL;
    *out = nullptr;
    rmp_status st = validate(p);
    if (st != RMP_OK) return st;
    const size_t rep_bytes = aup(layout_of(p).total);
    if (!d_workspace || workspace_bytes < rep_bytes + ctl_bytes_for(1)) return RMP_ENOMEM;
    if (((uintptr_t)d_workspace) % ALIGN) return RMP_EINVAL;
    rmp_system* s = new (std::nothrow) rmp_system();
    if (!s) return RMP_ENOMEM;
    s->b = &s->storage;
    st = batch_init(s->b, 1, p->precision, (char*)d_workspace + rep_bytes, ctl_bytes_for(1), stream);
    if (st == RMP_OK) st = admit(s->b, 0, p, seed, 1, d_workspace, rep_bytes);
    if (st != RMP_OK) {
        batch_release(s->b);
        delete s;
        return st;
    }
    *out = s;
    return RMP_OK;
}

rmp_status rmp_step(rmp_system* s, int32_t n_md, int32_t n_collide)
{
    if (!s || n_md < 1 || n_collide < 0) return RMP_EINVAL;
    Replica& R = s->b->reps[0];
    if (R.n_md != n_md) {
        R.n_md = n_md;
        make_ptable(R);
        HIPCHK(hipMemcpyAsync(R.ws + R.lay.ptable, R.ptable.data(), RMP_PTABLE * 8,
                              hipMemcpyHostToDevice, s->b->stream));
        HIPCHK(hipStreamSynchronize(s->b->stream));
        s->b->dirty = true;
    }
    return batch_ticks(s->b, n_collide);
}

rmp_status rmp_observables(rmp_system* s, rmp_obs* out)
{
    if (!s || !out) return RMP_EINVAL;
    return s->b->precision == 32 ? observe<float>(s->b, 0, out) : observe<double>(s->b, 0, out);
}

rmp_status rmp_observables_noalloc(rmp_system* s, rmp_obs* out)
{
    g_last_error[0] = 0;
    if (!s || !out) return RMP_EINVAL;
    rmp_batch* b = s->b;
    char* scr = scratch_address(b->device);
    if (!scr) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "rmp_observables_noalloc: no scratch address for device %d", b->device);
        return RMP_ESTATE;
    }
    std::lock_guard<std::mutex> g(g_scratch_call_mu[b->device]);
    return b->precision == 32 ? observe<float>(b, 0, out, scr) : observe<double>(b, 0, out, scr);
}

rmp_status rmp_get_state(rmp_system* s, rmp_host_state* dst)
{
    if (!s || !dst) return RMP_EINVAL;
    return s->b->precision == 32 ? get_state_t<float>(s->b, 0, dst) : get_state_t<double>(s->b, 0, dst);
}

rmp_status rmp_check_state(const rmp_params* p, const rmp_host_state* src)
{
    return check_state(p, src);
}

rmp_status rmp_set_state(rmp_system* s, const rmp_host_state* src)
{
    if (!s || !src) return RMP_EINVAL;
    return s->b->precision == 32 ? set_state_t<float>(s->b, 0, src) : set_state_t<double>(s->b, 0, src);
}

rmp_status rmp_destroy(rmp_system* s)
{
    if (!s) return RMP_EINVAL;
    if (s->b->stream) (void)hipStreamSynchronize(s->b->stream);
    batch_release(s->b);
    delete s;
    return RMP_OK;
}

rmp_status rmp_set_tuning(rmp_system* s, const rmp_tuning* t)
{
    if (!s) return RMP_EINVAL;
    return rmp_batch_set_tuning(s->b, t);
}

rmp_status rmp_get_tuning(rmp_system* s, rmp_tuning* t)
{
    if (!s || !t) return RMP_EINVAL;
    *t = s->b->tun;
    return RMP_OK;
}

rmp_status rmp_profile(rmp_system* s, int32_t enable)
{
    if (!s) return RMP_EINVAL;
    rmp_batch* b = s->b;
    flush_profile(b);
    b->prof = enable != 0;
    for (int k = 0; k < KN_COUNT; ++k) { b->prof_ms[k] = 0.0; b->prof_cnt[k] = 0; }
    return RMP_OK;
}

int32_t rmp_profile_read(rmp_system* s, const char** names, double* ms_total, int64_t* count, int32_t cap)
{
    if (!s) return 0;
    flush_profile(s->b);
    int32_t m = 0;
    for (int k = 0; k < KN_COUNT && m < cap; ++k, ++m) {
        if (names) names[m] = KNAMES[k];
        if (ms_total) ms_total[m] = s->b->prof_ms[k];
        if (count) count[m] = s->b->prof_cnt[k];
    }
    return m;
}

size_t rmp_batch_ctl_bytes(int32_t n_slots)
{
    if (n_slots < 1) return 0;
    return ctl_bytes_for(n_slots);
}

rmp_status rmp_batch_create(int32_t n_slots, int32_t precision, void* d_ctl, size_t ctl_bytes,
                            void* stream, rmp_batch** out)
{
    if (!out) return RMP_EINVAL;
    *out = nullptr;
    rmp_batch* b = new (std::nothrow) rmp_batch();
    if (!b) return RMP_ENOMEM;
    rmp_status st = batch_init(b, n_slots, precision, d_ctl, ctl_bytes, stream);
    if (st != RMP_OK) {
        batch_release(b);
        delete b;
        return st;
    }
    *out = b;
    return RMP_OK;
}

rmp_status rmp_batch_set_slot(rmp_batch* b, int32_t slot, const rmp_params* p, uint64_t seed,
                              int32_t n_md, void* d_workspace, size_t workspace_bytes)
{
    if (!b || slot < 0 || slot >= b->nslots) return RMP_EINVAL;
    if (b->reps[slot].used) return RMP_ESTATE;
    rmp_status st = admit(b, slot, p, seed, n_md, d_workspace, workspace_bytes);
    if (st != RMP_OK) b->reps[slot] = Replica{};
    b->dirty = true;
    return st;
}

rmp_status rmp_batch_clear_slot(rmp_batch* b, int32_t slot)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    HIPCHK(hipStreamSynchronize(b->stream));
    b->reps[slot] = Replica{};
    b->dirty = true;
    return RMP_OK;
}

rmp_status rmp_batch_step(rmp_batch* b, int32_t n_ticks)
{
    if (!b) return RMP_EINVAL;
    return batch_ticks(b, n_ticks);
}

rmp_status rmp_batch_slot_observables(rmp_batch* b, int32_t slot, rmp_obs* out)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    if (!out) return RMP_EINVAL;
    return b->precision == 32 ? observe<float>(b, slot, out) : observe<double>(b, slot, out);
}

rmp_status rmp_batch_get_state(rmp_batch* b, int32_t slot, rmp_host_state* dst)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    if (!dst) return RMP_EINVAL;
    return b->precision == 32 ? get_state_t<float>(b, slot, dst) : get_state_t<double>(b, slot, dst);
}

rmp_status rmp_batch_set_state(rmp_batch* b, int32_t slot, const rmp_host_state* src)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    if (!src) return RMP_EINVAL;
    return b->precision == 32 ? set_state_t<float>(b, slot, src) : set_state_t<double>(b, slot, src);
}

rmp_status rmp_batch_set_tuning(rmp_batch* b, const rmp_tuning* t)
{
    if (!b || !t) return RMP_EINVAL;
    rmp_tuning n = b->tun;
    if (t->stream_block > 0) n.stream_block = t->stream_block;
    if (t->stream_ppt > 0) n.stream_ppt = t->stream_ppt;
    if (t->collide_cells > 0) n.collide_cells = t->collide_cells;
    if (t->chain_k > 0) n.chain_k = t->chain_k;
    if (t->use_graph >= 0) n.use_graph = t->use_graph;
    if (t->chain_resident >= 0) n.chain_resident = t->chain_resident;
    if (t->chain_block >= 0) n.chain_block = t->chain_block;
    if (t->barrier_budget_us >= 0) n.barrier_budget_us = t->barrier_budget_us;
    if (t->collide_block >= 0) n.collide_block = t->collide_block;
    if (t->collide_ppt >= 0) n.collide_ppt = t->collide_ppt;
    if (t->collide_xcd >= 0) n.collide_xcd = t->collide_xcd;
    if (t->chain_serial >= 0) n.chain_serial = t->chain_serial;
    if (n.chain_serial != 0 && n.chain_serial != 1) return RMP_EINVAL;
    if (n.collide_block != 0 && n.collide_block != 256 && n.collide_block != 512) return RMP_EINVAL;
    if (n.collide_ppt < 0 || n.collide_ppt > 2) return RMP_EINVAL;
    if (n.collide_xcd != 0 && n.collide_xcd != 1) return RMP_EINVAL;
    if (n.collide_cells > COLL_TCMAX) return RMP_EINVAL;
    if (n.chain_block != 0 && n.chain_block != 256 && n.chain_block != 512) return RMP_EINVAL;
    if (n.barrier_budget_us > BARRIER_BUDGET_MAX_US) return RMP_EINVAL;
    if (n.chain_k != 1 && n.chain_k != 2 && n.chain_k != 4) return RMP_EINVAL;
    if (n.stream_block != 64 && n.stream_block != 128 && n.stream_block != 256) return RMP_EINVAL;
    b->tun = n;
    b->dirty = true;
    b->graph_valid = false;
    return RMP_OK;
}

rmp_status rmp_batch_set_slot_tuning(rmp_batch* b, int32_t slot, const rmp_tuning* t)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    if (!t) return RMP_EINVAL;
    b->reps[slot].tile_cells = t->collide_cells > 0 ? t->collide_cells : 0;
    b->dirty = true;
    b->graph_valid = false;
    return RMP_OK;
}

rmp_status rmp_batch_destroy(rmp_batch* b)
{
    if (!b) return RMP_EINVAL;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_release(b);
    delete b;
    return RMP_OK;
}

size_t rmp_analysis_bytes(const rmp_params* p, const rmp_analysis_params* a, rmp_status* st)
{
    rmp_status v = validate(p);
    if (v == RMP_OK) v = an_validate(p, a);
    if (st) *st = v;
    if (v != RMP_OK) return 0;
    return an_layout(p, a).total;
}

rmp_status rmp_analysis_attach(rmp_system* s, const rmp_analysis_params* a, void* d_buf, size_t bytes)
{
    if (!s) return RMP_EINVAL;
    return an_attach(s->b, 0, a, d_buf, bytes);
}

rmp_status rmp_analysis_detach(rmp_system* s)
{
    if (!s) return RMP_EINVAL;
    return an_detach(s->b, 0);
}

rmp_status rmp_analysis_read(rmp_system* s, rmp_analysis_out* out)
{
    if (!s || !out) return RMP_EINVAL;
    return an_read(s->b, 0, out);
}

rmp_status rmp_analysis_msd(rmp_system* s, int32_t max_lag, double* msd)
{
    if (!s) return RMP_EINVAL;
    return an_msd(s->b, 0, max_lag, msd);
}

rmp_status rmp_batch_analysis_attach(rmp_batch* b, int32_t slot, const rmp_analysis_params* a,
                                     void* d_buf, size_t bytes)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    return an_attach(b, slot, a, d_buf, bytes);
}

rmp_status rmp_batch_analysis_detach(rmp_batch* b, int32_t slot)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    return an_detach(b, slot);
}

rmp_status rmp_batch_analysis_read(rmp_batch* b, int32_t slot, rmp_analysis_out* out)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    if (!out) return RMP_EINVAL;
    return an_read(b, slot, out);
}

rmp_status rmp_batch_analysis_msd(rmp_batch* b, int32_t slot, int32_t max_lag, double* msd)
{
    rmp_status st = slot_ok(b, slot);
    if (st != RMP_OK) return st;
    return an_msd(b, slot, max_lag, msd);
}

}  // extern "C"
