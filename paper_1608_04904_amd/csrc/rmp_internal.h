// Internal layout shared by the host runtime and the gfx950 kernels of the
// rmpmd library.  Not part of the public C ABI (include/rmpmd.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rmpmd.h"

namespace rmp {

constexpr int MAXC = RMP_MAX_COLLOIDS;
constexpr int CHUNK = 1024;          // particles per chunk (list compaction, init, observables)
constexpr int SCAN_BLK = 4096;       // cells per block of the multi-block cell scan
constexpr int SCAN_DIRECT_BLOCKS = 8; // up to this many blocks, no separate block-sum pass
constexpr int CHAIN_BLOCK = 256;     // threads per Verlet-list workgroup
constexpr int NVAL_MAX = 3 * MAXC + 1;  // reduced values per MD step: F per colloid + U
constexpr int MAX_CHAIN_G = 256;      // MD-chain workgroups per system at most
constexpr int ROWW = 2 * NVAL_MAX + 2;    // MD-chain exchange: words per workgroup
constexpr int BCW = 6 * MAXC + 2;         // MD-chain broadcast of the colloid positions: words
constexpr int XTAB_V = 49, XTAB_R = 128;   // MD-chain master: values and rows per table chunk
constexpr uint64_t BARRIER_BUDGET_TICKS = 25000000;  // 0.25 s of the 100 MHz wall clock (default)
constexpr int32_t BARRIER_BUDGET_MAX_US = 10000000;  // largest budget a caller may set (10 s)
constexpr int32_t KEY_TABLE = -1;                    // cell sort rank from rank_of[]
constexpr int32_t KEY_ROW = -2;                      // row-major: rank = cell index

// Philox stream tags (key word 1); key word 0 is the replica seed.
enum : uint64_t {
    TAG_SHIFT = 1, TAG_ROT = 2, TAG_BULK = 3, TAG_CAT = 4, TAG_THERMO = 5,
    TAG_INIT_POS = 6, TAG_INIT_VEL = 7, TAG_VIRT = 8
};

// Per-replica colloid parameters with host-derived constants.
struct ColloidParams {
    int32_t nc, nbonds;
    int32_t catalytic[MAXC], ctype[MAXC];
    int32_t body[MAXC];                                  // rigid body: smallest colloid of its bonded group
    int32_t bond_of[MAXC];                               // the single bond of a colloid (exact RATTLE), -1 if none
    int32_t bond_a[RMP_MAX_BONDS], bond_b[RMP_MAX_BONDS];
    double bond_d[RMP_MAX_BONDS];
    int32_t iterative, rattle_maxit;                     // iterative RATTLE for bond networks
    double rattle_tol;
    // the bond order cut into runs of consecutive bonds with no colloid in
    // common: within a run the sweep's corrections commute exactly
    int32_t n_layers;
    int32_t layer_start[RMP_MAX_BONDS + 1];
    double sigma[MAXC], sig2[MAXC], rc2[MAXC], reachR[MAXC];
    double epsA[MAXC], epsB[MAXC];
    double mass[MAXC], imass[MAXC], hc[MAXC];
    double eps_cc[2][2];
};

// Per-replica mutable state, device resident.
struct RepState {
    int64_t md_step, coll_step;
    int64_t n_cand;            // Verlet-list length for the coming interval
    int64_t n_cand_used;       // ... of the last interval run
    int64_t n_cat, n_bulk;
    int64_t list_nmd;          // n_md the current Verlet list was built for (-1: none)
    uint32_t flags;
    uint32_t bar;              // inter-workgroup barrier counter of the MD chain
    double U, e_rxn;
    double T_sum, T_cells;     // temperature estimator of the last collision
    double X[MAXC][3], V[MAXC][3], F[MAXC][3];
};

// Dimer-analysis state of one replica, at the start of the caller's
// analysis buffer (the arrays follow it in the same buffer).
struct Analysis {
    int64_t n_samples, n_dropped;
    int32_t every, cap, nz, nr, nb, pad;
    double zmax, rmax, inv_dz, inv_dr;
    double skip_r2;            // rho^2 beyond which rho certainly falls past the last shell
    double cull_r;             // distance beyond which a point is certainly outside the cylinder
    uint64_t* hist;            // [nb][2][nz][nr]
    double* series;            // [cap][nb][RMP_SERIES_FIELDS]
    int64_t* series_t;         // [cap] MD step of each stored sample
    double* msd;               // [nb][cap]
};

// A particle's record in the staging array that the scatter fills in cell
// order for the collision: one aligned 64-byte record in FP64 (32 bytes in
// FP32), so that the scatter writes and the collision reads whole sectors.
// FP64: x[3], v[3], id, old index, state byte.  FP32: x[3], v[3], then id and
// old index (both < 2^31) with the state's catalysis bit in bit 31 of the id
// word and its species bit in bit 31 of the index word.
template <class T> struct Rec;
template <> struct alignas(64) Rec<double> {
    double x[3], v[3];
    uint32_t id, idx;
    uint32_t st, pad;
};
template <> struct alignas(32) Rec<float> {
    float x[3], v[3];
    uint32_t id_f, idx_s;
};
static_assert(sizeof(Rec<double>) == 64 && sizeof(Rec<float>) == 32, "record sizes");

// Per-replica descriptor, written by the host.
struct RepDesc {
    int32_t L[3];              // cell grid (with walls L[2] is one layer more than the box)
    int32_t active;
    int64_t n, ncell;
    int32_t n_md, rule;
    int32_t n_chunks, n_tiles, n_scanblk, tile_cells;
    int32_t cand_cap, G;       // Verlet-list capacity, MD-chain workgroups
    int32_t chain_k;
    int32_t hbits;             // cell sort rank: >= 0 Hilbert index with hbits bits, KEY_TABLE, KEY_ROW
    double Ld[3], halfL[3];
    double dt, h, tau, vscale, mass, ca, sa, cat_prob, skin_half2;
    double cull_me, cull_margin; // MD chain cull: entry displacement allowed per interval; + skin/2
    int32_t bulk_on, pad1;
    int32_t flow;              // constant acceleration and/or walls: every particle streams
    int32_t walls;             // plates at z = 0 and z = Ld[2]
    int32_t wall_n0;           // particles of a full cell (virtual fill of cut cells)
    int32_t pad2;
    double g[3];               // constant acceleration
    uint64_t seed;
    void* x[2];                // [3][n] storage-type arrays, double-buffered
    void* v[2];
    uint32_t* id[2];
    uint8_t* st[2];
    uint64_t* keyrank;         // (key << 32) | rank
    void* stage;               // [n] particle records in cell order (Rec<T>), written by the scatter
    uint32_t* count;           // [ncell]
    uint32_t* start;           // [ncell + 1]
    uint32_t* scanblk;         // [n_scanblk]
    uint8_t* cflag;            // [n] Verlet-list membership for the coming interval
    uint32_t* chunk_cnt;       // [n_chunks]
    uint32_t* chunk_off;       // [n_chunks]
    uint32_t* cand_idx;        // [cand_cap]
    const uint32_t* rank_of;   // [ncell] sort rank of a cell (Hilbert order)
    const uint32_t* cell_of;   // [ncell] cell of a sort rank
    double* partials;          // [2][G * ROWW + BCW] 64-bit exchange words of the MD chain
    double* epart;             // [G][2] reaction energy / flips of the interval
    double* tpart;             // [n_tiles][4] collision partials: temperature sum, cells, reaction energy, flips
    uint64_t* bigmask;         // [n_tiles] cells of a tile beyond a collision group's capacity
    double* ptable;            // [RMP_PTABLE]
    double* obs_part;          // [n_chunks][8]
    ColloidParams* cp;
    RepState* rs;
    Analysis* an;              // dimer analysis, nullptr when off
};

constexpr int32_t WORK_CHAIN_PRIO = 1;

// Work lists: items of one kind (particle chunks, cell tiles, scan blocks,
// chain workgroups) concatenated over replicas.  prefix[r] is the first item
// of replica r, prefix[nrep] the total.
struct Work {
    const RepDesc* desc;
    const int32_t* prefix;
    uint32_t* tick;   // [0] next ticket, [1] finished workgroups; zero between launches
    int32_t nrep;
    int32_t flags;    // WORK_CHAIN_PRIO: the MD chain raises its waves' issue priority
    uint64_t budget;  // MD chain: longest wait for the other workgroups, 100 MHz ticks
};

}  // namespace rmp
