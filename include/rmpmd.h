/*
 * rmpmd -- MI355X (gfx950) library for the solvent hot path of hybrid
 * Reactive Multiparticle Collision Dynamics + Molecular Dynamics
 * (RMPCDMD, de Buyl, Huang, Deprez, arXiv:1608.04904).
 *
 * One interval of the method = n_md velocity-Verlet MD steps of solvent and
 * colloids ("Algorithms": velocity-Verlet; WCA colloid-solvent and
 * colloid-colloid forces via Verlet and cell lists; exact RATTLE for the
 * dimer; catalytic A->B conversion), followed by one MPCD collision on a
 * randomly shifted grid ("Algorithms": original MPCD rule, grid shifting,
 * Anderson thermostat; Overview: RMPCD bulk reactions) with the stable cell
 * sort it shares with the cell lists.
 *
 * Conventions for every entry point:
 *   - Device memory is owned by the caller: the library carves its arrays out
 *     of a workspace the caller allocates (size from *_workspace_bytes) and
 *     never frees it.  Host buffers are owned by the caller.  Handles are
 *     owned by the library and released by the matching destroy call.
 *   - `stream` is a hipStream_t passed as void*; all device work of a handle
 *     is ordered on that stream.  Calls are asynchronous unless stated.
 *   - Every call returns an rmp_status and never aborts or throws.  Device
 *     side faults (list overflow, unsound Verlet list, barrier time-out,
 *     non-finite force) are latched in a per-replica flag word and reported
 *     by the next observables call as RMP_EDEVICE with `flags` filled in.
 *   - Units are the paper's reduced units: cell size a = 1, energies in kT,
 *     lengths in a, masses in the solvent mass.
 *   - Arrays exchanged with the host are structure-of-arrays: x[3*N] holds
 *     all x components, then all y, then all z.
 */
#ifndef RMPMD_H
#define RMPMD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RMP_MAX_COLLOIDS 32
#define RMP_MAX_BONDS 96
#define RMP_PTABLE 1024

typedef enum rmp_status {
    RMP_OK = 0,
    RMP_EINVAL = -1,   /* invalid argument or parameter set               */
    RMP_ENOMEM = -2,   /* workspace smaller than *_workspace_bytes        */
    RMP_EHIP = -3,     /* a HIP runtime call failed                       */
    RMP_EDEVICE = -4,  /* a device-side flag is set (see rmp_observables) */
    RMP_ESTATE = -5    /* call not valid in the handle's current state    */
} rmp_status;

/* device flag bits (rmp_observables.flags) */
#define RMP_FLAG_DISPLACEMENT  1u  /* colloid moved >= skin/2 in one interval     */
#define RMP_FLAG_RATTLE        2u  /* RATTLE quadratic had no real root           */
#define RMP_FLAG_NONFINITE     4u  /* non-finite colloid force, or non-finite
                                      centre-of-mass velocity of a solvent cell */
#define RMP_FLAG_INIT          8u  /* init rejection sampling hit its cap         */
#define RMP_FLAG_LIST_OVERFLOW 16u /* Verlet list longer than its capacity        */
#define RMP_FLAG_BARRIER       32u /* inter-workgroup barrier timed out           */

/*
 * System parameters.  Names follow the paper's configuration file
 * (appendix "Example configuration file": T -> kT, L, tau = n_md * dt,
 * probability -> cat_prob, bulk_rate, sigma_*, epsilon_*, d -> bond_d).
 * Colloid-solvent interaction: WCA with (sigma[c], eps_A[c] or eps_B[c] by
 * solvent species).  Colloid-colloid: WCA with sigma_a + sigma_b and
 * eps_cc[ctype[a]][ctype[b]], bonded pairs excluded.
 */
typedef struct rmp_params {
    int32_t L[3];              /* box edge in cells, each >= 1                     */
    int32_t precision;         /* 64: FP64 state; 32: FP32 state, FP64 cell sums   */
    int64_t n_solvent;         /* N >= 0, N < 2^31                                 */
    double  kT;                /* temperature for init and the thermostat          */
    double  mass;              /* solvent particle mass m > 0                      */
    double  dt;                /* MD time step > 0                                 */
    double  alpha;             /* rotation angle in radians                        */
    double  skin;              /* Verlet-list skin >= 0                            */
    double  cat_prob;          /* probability of A->B on leaving a catalytic sphere */
    double  bulk_rate;         /* bulk B->A rate k; 0 switches it off              */
    int32_t rule;              /* 0: rotation (SRD) rule; 1: Anderson thermostat   */
    int32_t n_colloids;        /* 0 .. RMP_MAX_COLLOIDS                            */
    int32_t n_bonds;           /* rigid bonds (each colloid in at most one)        */
    int32_t cand_capacity;     /* Verlet-list capacity; 0 = automatic              */
    double  colloid_x[RMP_MAX_COLLOIDS][3];   /* initial positions (unwrapped)     */
    double  colloid_mass[RMP_MAX_COLLOIDS];
    double  sigma[RMP_MAX_COLLOIDS];
    double  eps_A[RMP_MAX_COLLOIDS];
    double  eps_B[RMP_MAX_COLLOIDS];
    int32_t catalytic[RMP_MAX_COLLOIDS];      /* 1: converts A to B                */
    int32_t ctype[RMP_MAX_COLLOIDS];          /* 0 or 1, index into eps_cc         */
    double  eps_cc[2][2];
    int32_t bond_a[RMP_MAX_BONDS];            /* rigid bonds: colloids bond_a[k] and */
    int32_t bond_b[RMP_MAX_BONDS];            /* bond_b[k] at distance bond_d[k]      */
    double  bond_d[RMP_MAX_BONDS];
    int32_t cell_order;        /* order of cells in the sorted particle arrays:
                                  0 row-major (x fastest); 1 compact Hilbert (the
                                  box's cells along the Hilbert curve of the
                                  enclosing power-of-two cube, "Implementation
                                  and architecture": cell sorting)              */
    int32_t pad_order;
    /* Flows ("Algorithms": flows from a constant acceleration of the solvent;
     * stick walls by the bounce-back rule with virtual particles in the
     * collision, Lamura et al. 2001).  Only for systems without colloids
     * (n_colloids = 0); then there is no Verlet list. */
    int32_t walls;             /* 1: plates at z = 0 and z = L[2]; the drift of a
                                  particle that crosses one is cut at the
                                  crossing, its velocity reversed and the rest
                                  of the step travelled back.  The shifted grid
                                  then has L[2] + 1 layers; cells of the first
                                  and last layer holding fewer than
                                  wall_density particles get the summed
                                  momentum of the missing ones, drawn from
                                  Maxwell-Boltzmann at rest, in their mean
                                  velocity.  Needs rule 0, cell_order 0 and
                                  accel[2] = 0.                                  */
    int32_t wall_density;      /* particles of a full cell, 1 .. 1024 (walls)  */
    double  accel[3];          /* constant acceleration of every solvent
                                  particle, applied as velocity-Verlet half
                                  kicks around each drift (0: none)             */
    /* Rigid bodies ("Algorithms": RATTLE, exact for the dimer, iterative for
     * the Janus particle).  Bonded colloids form rigid bodies whose colloids
     * do not interact with each other.  A colloid in one bond at most is
     * constrained by the exact RATTLE; a bond network (a colloid in two or
     * more bonds) by the iterative RATTLE (Andersen 1983): sweeps over the
     * bonds in order, correcting a bond whose squared length misses d^2 by
     * more than 2 rattle_tol d^2 (velocity stage: |r.v| > rattle_tol d^2 / dt),
     * until a sweep changes nothing; after rattle_maxit sweeps the RATTLE
     * flag is raised. */
    double  rattle_tol;        /* > 0 when iterative                            */
    int32_t rattle_maxit;      /* 1 .. 100000 when iterative                    */
    int32_t rattle_iterative;  /* 1: iterative also for single bonds            */
} rmp_params;

/* FP64 observables.  `potential` is the colloid-solvent plus colloid-colloid
 * WCA energy at the last force evaluation; `temperature` is the cell-frame
 * estimator ("Algorithms", temperature equation) of the last collision,
 * averaged over the n_cells_T cells holding two or more particles. */
typedef struct rmp_obs {
    double   momentum[3];
    double   ke_solvent, ke_colloid, potential, temperature, e_rxn;
    int64_t  n_A, n_B, n_cat_flips, n_bulk_flips;
    int64_t  md_step, coll_step, n_candidates, n_cells_T;
    uint32_t flags;
    int32_t  pad;
    double   colloid_X[RMP_MAX_COLLOIDS][3];
    double   colloid_V[RMP_MAX_COLLOIDS][3];
} rmp_obs;

/* Host-side state exchange, caller-owned buffers.  x, v: 3*N doubles (SoA;
 * FP32 systems convert exactly on get and round on set); id: N; state: N
 * bytes (bit 0 species B, bit 1 catalytic flag); X, V: 3*n_colloids
 * doubles, row per colloid.  Any pointer may be NULL on get to skip it. */
typedef struct rmp_host_state {
    double*   x;
    double*   v;
    uint32_t* id;
    uint8_t*  state;
    double*   X;
    double*   V;
    int64_t   md_step;
    int64_t   coll_step;
} rmp_host_state;

typedef struct rmp_system rmp_system;
typedef struct rmp_batch rmp_batch;

const char* rmp_status_string(rmp_status st);
/* Text of the last HIP failure seen by the calling thread (RMP_EHIP). */
const char* rmp_last_error(void);

/* ---------------------------------------------------------------- single */

/* Device bytes needed by one system with these parameters; 0 and *st set on
 * invalid parameters.  Pure host function, used for HBM admission. */
size_t rmp_workspace_bytes(const rmp_params* p, rmp_status* st);

/* Validate p, carve d_workspace, and initialise the solvent on `stream`:
 * positions uniform in the box, rejected inside colloid cores (r < sigma),
 * velocities Maxwellian at kT with the mean removed, all species A, colloids
 * at rest at colloid_x (Overview: N solvent particles with mass, position and
 * velocity in a cuboid domain).  Randomness: Philox4x64-10 keyed by seed. */
rmp_status rmp_init_system(const rmp_params* p, uint64_t seed, void* d_workspace,
                           size_t workspace_bytes, void* stream, rmp_system** out);

/* Advance n_collide intervals of (n_md MD steps, one collision); tau =
 * n_md * dt.  Asynchronous.  n_md >= 1, n_collide >= 0. */
rmp_status rmp_step(rmp_system* s, int32_t n_md, int32_t n_collide);

/* FP64 reductions of the current state; synchronises the stream.  Returns
 * RMP_EDEVICE (with out filled) if a device flag is set. */
rmp_status rmp_observables(rmp_system* s, rmp_obs* out);

/* For callers that cannot allocate device memory (code under graph capture
 * elsewhere in the process, serving loops, harnesses that forbid
 * hipMalloc): the same results as rmp_observables, bit for bit, with its
 * per-chunk partial sums and their totals kept in a static device array of
 * RMP_NOALLOC_SCRATCH_BYTES per GPU instead of the workspace.  The array
 * holds 64 bytes per 1024 solvent particles plus 64, so systems up to
 * 33,553,408 particles; a larger system gets RMP_ENOMEM and a message in
 * rmp_last_error().  No device or host allocation in the call; it
 * synchronises the system's stream.  All calls on one GPU share that GPU's
 * array and keep no result in it between calls; the library serialises
 * calls from different host threads on one device with a lock, and work on
 * other streams that reads the array while a call runs would race.  The
 * array's address is taken per device when a system is created there
 * (rmp_init_system); RMP_ESTATE if none was. */
#define RMP_NOALLOC_SCRATCH_BYTES (2u << 20)
rmp_status rmp_observables_noalloc(rmp_system* s, rmp_obs* out);

/* Copy the state to / from caller-owned host buffers (synchronous).  After
 * set_state the next interval rebuilds the Verlet list and forces.
 * set_state first applies rmp_check_state and uploads nothing on
 * RMP_EINVAL. */
rmp_status rmp_get_state(rmp_system* s, rmp_host_state* dst);
rmp_status rmp_set_state(rmp_system* s, const rmp_host_state* src);

/* Pure host check of a state for parameters p (no device needed): RMP_OK, or
 * RMP_EINVAL when a solvent position lies outside [0, L), a velocity is not
 * finite (for precision 32 also after rounding to float), the ids are not a
 * permutation of 0 .. n_solvent-1, a state byte has bits other than the
 * species (bit 0) and catalysis flag (bit 1), a colloid position or velocity
 * is not finite, a solvent particle lies within sigma/2 of a colloid centre
 * (minimum image; the WCA potential there exceeds 1.6e4 eps, which no
 * thermal state reaches), or a required pointer is NULL. */
rmp_status rmp_check_state(const rmp_params* p, const rmp_host_state* src);

/* Release the handle; the workspace is not freed. */
rmp_status rmp_destroy(rmp_system* s);

/* Per-kernel launch parameters (autotuning).  A negative field keeps its
 * current value; so does 0, except for use_graph, chain_resident,
 * chain_block, collide_block, collide_ppt, collide_xcd and chain_serial,
 * where 0 is a value (collide_cells is 0 until set).  Applies to the next rmp_step /
 * rmp_batch_step. */
typedef struct rmp_tuning {
    int32_t stream_block;      /* threads per workgroup, particle kernels       */
    int32_t stream_ppt;        /* particles per thread in the streaming kernel
                                  (1, 2 or 4; default 2)                        */
    int32_t collide_cells;     /* cells per collision tile, 8 .. 64 (0: sized
                                  from the density so that a tile fills about
                                  0.94 of a collision group, the default)      */
    int32_t chain_k;           /* Verlet-list entries per thread (1, 2 or 4)    */
    int32_t use_graph;         /* 1: replay a captured hipGraph per interval    */
    int32_t chain_resident;    /* chain workgroups taken to fit on the device at
                                  once when raising chain_k (0: the device's
                                  own occupancy figure)                         */
    int32_t chain_block;       /* MD-chain workgroup size: 256, 512 (one or two
                                  list entries per thread), or 0: 512 when a
                                  list needs more than one entry per thread at
                                  256 threads                                   */
    int32_t barrier_budget_us; /* longest wait of an MD-chain workgroup for the
                                  other workgroups' values, in microseconds
                                  (0: the default, 250000; at most 10000000);
                                  beyond it the workgroup gives up, raises
                                  RMP_FLAG_BARRIER and waits no more in that
                                  launch, so the launch always ends          */
    int32_t collide_block;     /* collision workgroup size: 256 or 512 threads
                                  (0: 256)                                      */
    int32_t collide_ppt;       /* particles each collision thread holds: 1 or 2
                                  (0: 2); a group of cells holds at most
                                  collide_block * collide_ppt particles         */
    int32_t collide_xcd;       /* 1: tiles dealt to the eight XCDs in
                                  contiguous ranges (0: in launch order)        */
    int32_t chain_serial;      /* 1: the MD chain runs before the streaming
                                  kernel on the same stream (0: next to it on a
                                  side stream)                                  */
} rmp_tuning;
rmp_status rmp_set_tuning(rmp_system* s, const rmp_tuning* t);
rmp_status rmp_get_tuning(rmp_system* s, rmp_tuning* t);

/* Average device time per launch of each hot kernel over the calls since
 * the last reset, measured with HIP events on the handle's stream (enabled
 * by rmp_profile(s, 1)).  names/ms/count hold up to cap entries. */
rmp_status rmp_profile(rmp_system* s, int32_t enable);
int32_t    rmp_profile_read(rmp_system* s, const char** names, double* ms_total,
                            int64_t* count, int32_t cap);

/* ----------------------------------------------------------------- batch */
/* A batch advances many independent replicas together (uneven box sizes,
 * per-replica seeds and n_md), one interval per replica per tick.  All
 * replicas of a batch share the precision.  Each replica's state lives in a
 * caller-provided workspace of rmp_workspace_bytes(params).  Slots can be
 * filled and emptied between ticks (continuous batching). */
size_t     rmp_batch_ctl_bytes(int32_t n_slots);
rmp_status rmp_batch_create(int32_t n_slots, int32_t precision, void* d_ctl,
                            size_t ctl_bytes, void* stream, rmp_batch** out);
/* Admit a replica into an empty slot: validates, carves d_workspace and
 * initialises the state (as rmp_init_system); it takes part from the next
 * tick with its own n_md. */
rmp_status rmp_batch_set_slot(rmp_batch* b, int32_t slot, const rmp_params* p,
                              uint64_t seed, int32_t n_md, void* d_workspace,
                              size_t workspace_bytes);
/* Retire a slot; its workspace may then be reused by the caller. */
rmp_status rmp_batch_clear_slot(rmp_batch* b, int32_t slot);
/* n_ticks ticks: every occupied slot advances one interval per tick. */
rmp_status rmp_batch_step(rmp_batch* b, int32_t n_ticks);
rmp_status rmp_batch_slot_observables(rmp_batch* b, int32_t slot, rmp_obs* out);
rmp_status rmp_batch_get_state(rmp_batch* b, int32_t slot, rmp_host_state* dst);
rmp_status rmp_batch_set_state(rmp_batch* b, int32_t slot, const rmp_host_state* src);
rmp_status rmp_batch_set_tuning(rmp_batch* b, const rmp_tuning* t);
/* Per-replica override of the collision tile size (t->collide_cells; the
 * other fields are batch-wide and ignored here); <= 0 restores the batch
 * value.  Used to apply a per-box-class autotuned tile size. */
rmp_status rmp_batch_set_slot_tuning(rmp_batch* b, int32_t slot, const rmp_tuning* t);
rmp_status rmp_batch_destroy(rmp_batch* b);

/* ------------------------------------------------------- dimer analysis */
/* On-device analysis of dimer motors, the quantities the paper's analysis
 * programs report ("Applications of RMPCDMD": laboratory-frame and directed
 * velocity of the dimer, mean-squared displacement of its centre of mass,
 * cylindrical shell histogram of the product concentration), accumulated
 * during the run instead of storing solvent data (pre-averaging, "Overview").
 *
 * Every bond (a, b) of the system is one dimer.  A sample is taken at the
 * end of every interval whose collision count (coll_step) is a multiple of
 * `every`, from the state after the collision:
 *   - series record of each dimer (RMP_SERIES_FIELDS doubles): centre of
 *     mass R = (m_a X_a + m_b X_b) / (m_a + m_b) (unwrapped), its velocity V,
 *     unit axis u = (X_b - X_a) / |X_b - X_a|, directed velocity V.u;
 *     stored while fewer than series_cap samples are held, later samples
 *     are counted in n_dropped;
 *   - histogram: for every solvent particle, r = minimum image of its
 *     position minus the image of R in the box, z = r.u, rho = |r - z u|;
 *     counted per species (A, B) in bin iz = floor((z + zmax) nz / (2 zmax)),
 *     ir = floor(rho nr / rmax) when 0 <= iz < nz and ir < nr (integer
 *     counts, added at every sample, including dropped ones).
 * Memory: the caller provides device memory of rmp_analysis_bytes(), 256-byte
 * aligned, and keeps it until detach; attach clears it.  Counts and records
 * do not depend on the launch configuration. */
#define RMP_SERIES_FIELDS 10   /* R[3], V[3], u[3], V.u */

typedef struct rmp_analysis_params {
    int32_t every;             /* sample after collisions that are multiples of this (>= 1) */
    int32_t series_cap;        /* samples of the series kept (>= 1)              */
    int32_t hist_nz, hist_nr;  /* bins along the axis and across it (>= 1)       */
    double  hist_zmax;         /* axial range [-zmax, zmax) (> 0)                */
    double  hist_rmax;         /* radial range [0, rmax) (> 0)                   */
} rmp_analysis_params;

typedef struct rmp_analysis_out {
    int64_t   n_samples;       /* samples stored in the series (<= series_cap)   */
    int64_t   n_dropped;       /* samples taken after the series was full        */
    int64_t*  md_step;         /* host [series_cap]: MD step of each sample, or NULL */
    double*   series;          /* host [series_cap][n_bonds][RMP_SERIES_FIELDS], or NULL */
    uint64_t* hist;            /* host [n_bonds][2][hist_nz][hist_nr], or NULL   */
} rmp_analysis_out;

/* Device bytes for the analysis of a system with parameters p; 0 and *st
 * set on invalid arguments (no bonds, non-positive sizes or ranges). */
size_t     rmp_analysis_bytes(const rmp_params* p, const rmp_analysis_params* a, rmp_status* st);
/* Start (or restart, clearing the counts) the analysis of a system. */
rmp_status rmp_analysis_attach(rmp_system* s, const rmp_analysis_params* a, void* d_buf,
                               size_t bytes);
/* Stop sampling; waits for queued work, after which d_buf may be freed. */
rmp_status rmp_analysis_detach(rmp_system* s);
/* Copy the counts, series and histogram to host memory (synchronous). */
rmp_status rmp_analysis_read(rmp_system* s, rmp_analysis_out* out);
/* Mean-squared displacement of each dimer's centre of mass over the stored
 * series, computed on the device: msd[k][lag] = average over the origins t
 * of |R(t + lag) - R(t)|^2 (summed in order of t), lag = 0 .. max_lag
 * (< series_cap; 0 where lag >= n_samples).  msd is host memory of
 * n_bonds * (max_lag + 1) doubles; synchronous. */
rmp_status rmp_analysis_msd(rmp_system* s, int32_t max_lag, double* msd);
/* The same for one slot of a batch. */
rmp_status rmp_batch_analysis_attach(rmp_batch* b, int32_t slot, const rmp_analysis_params* a,
                                     void* d_buf, size_t bytes);
rmp_status rmp_batch_analysis_detach(rmp_batch* b, int32_t slot);
rmp_status rmp_batch_analysis_read(rmp_batch* b, int32_t slot, rmp_analysis_out* out);
rmp_status rmp_batch_analysis_msd(rmp_batch* b, int32_t slot, int32_t max_lag, double* msd);

#ifdef __cplusplus
}
#endif
#endif /* RMPMD_H */
