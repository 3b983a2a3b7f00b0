/*
 * FP64 CPU oracle for the MPCD+MD solvent path (test infrastructure only).
 *
 * This library is the plain, slow reference against which the HIP path is
 * checked.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg load it; the product library never links or calls it, and the
 * two share no source.
 *
 * Method (paper: "Algorithms" section and the Overview):
 *   - solvent streaming / velocity-Verlet for solvent and colloids,
 *   - purely repulsive cut-off 12-6 Lennard-Jones (WCA) colloid-solvent and
 *     colloid-colloid forces (the equation in "Algorithms"), computed over a
 *     Verlet list built from the solvent positions,
 *   - the MPCD collision on a randomly shifted cell grid (rotation rule) and
 *     the Anderson-thermostat variant,
 *   - exact RATTLE for the rigid dimer bond,
 *   - catalytic A->B conversion at the catalytic sphere and RMPCD bulk B->A
 *     reactions per cell,
 *   - the cell-frame temperature estimator (equation in "Algorithms").
 * Randomness: Philox4x64-10 keyed by (seed, stream tag), counter
 * (step, cell-or-id, sub, 0).  The paper uses Threefry-2x64 from the same
 * counter-based family; see the readings listed in the design notes.
 */
#ifndef RMP_ORACLE_H
#define RMP_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXC 32          /* max colloids per system */
#define ORC_MAXB 96          /* max rigid bonds per system */
#define ORC_PTABLE 1024      /* bulk-reaction probability table length */

typedef struct orc_params {
    int32_t L[3];            /* box edge in cells (cell size a = 1)            */
    int32_t rule;            /* 0 = rotation (SRD), 1 = Anderson thermostat     */
    int64_t n_solvent;       /* N                                               */
    double  kT;              /* temperature (init and thermostat)               */
    double  mass;            /* solvent mass m                                  */
    double  dt;              /* MD time step                                    */
    double  alpha;           /* rotation angle (radians)                        */
    double  skin;            /* Verlet-list skin                                */
    double  cat_prob;        /* catalytic conversion probability                */
    double  bulk_rate;       /* bulk B->A rate k (0 = off)                      */
    int32_t n_colloids;
    int32_t n_bonds;
    double  cx[ORC_MAXC][3]; /* initial colloid positions                       */
    double  cmass[ORC_MAXC];
    double  sigma[ORC_MAXC];
    double  epsA[ORC_MAXC];  /* colloid-solvent epsilon for species A           */
    double  epsB[ORC_MAXC];  /* ... for species B                               */
    int32_t catalytic[ORC_MAXC];
    int32_t ctype[ORC_MAXC]; /* 0 or 1: row/column of eps_cc                     */
    double  eps_cc[2][2];    /* colloid-colloid epsilon by type                 */
    int32_t bond_a[ORC_MAXB];
    int32_t bond_b[ORC_MAXB];
    double  bond_d[ORC_MAXB];
    int32_t cell_order;      /* 0 row-major cell order, 1 compact Hilbert       */
    int32_t pad;
    /* flows ("Algorithms": constant acceleration; stick walls by bounce-back
     * and virtual particles).  Only for systems without colloids.          */
    int32_t walls;           /* 1: plates at z = 0 and z = L_z              */
    int32_t wall_density;    /* particles of a full cell (virtual fill)    */
    double  accel[3];        /* constant acceleration of every solvent particle */
    /* rigid bodies of several bonded colloids ("Algorithms": RATTLE in its
     * iterative form for the Janus particle, exact for the dimer)         */
    double  rattle_tol;      /* relative tolerance of the iterative RATTLE  */
    int32_t rattle_maxit;    /* sweeps over the bonds at most               */
    int32_t rattle_iterative;/* 1: iterative RATTLE also for single bonds   */
} orc_params;

typedef struct orc_obs {
    double  momentum[3];
    double  ke_solvent, ke_colloid, potential, temperature, e_rxn;
    int64_t n_A, n_B, n_cat_flips, n_bulk_flips;
    int64_t md_step, coll_step, n_candidates, n_cells_T;
    int32_t flags;
    int32_t pad;
} orc_obs;

/* error / warning flags, latched */
#define ORC_F_DISPLACEMENT 1u   /* a colloid moved >= skin/2 within one interval */
#define ORC_F_RATTLE       2u   /* RATTLE quadratic had no real root             */
#define ORC_F_NONFINITE    4u   /* non-finite colloid force or cell velocity     */
#define ORC_F_INIT         8u   /* init rejection sampling hit its cap           */

typedef struct orc_system orc_system;

void        orc_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void        orc_wca(double r2, double sigma, double eps, double* coef, double* pot);
double      orc_tree_sum(const double* a, int64_t n);

orc_system* orc_create(const orc_params* p, uint64_t seed);
void        orc_destroy(orc_system* s);
int         orc_init(orc_system* s);
int         orc_set_state(orc_system* s, const double* x, const double* v,
                          const uint32_t* id, const uint8_t* st,
                          const double* X, const double* V,
                          int64_t md_step, int64_t coll_step);
int         orc_get_state(const orc_system* s, double* x, double* v, uint32_t* id,
                          uint8_t* st, double* X, double* V, double* F,
                          int64_t* md_step, int64_t* coll_step);
/* n_collide intervals of (Verlet-list build, n_md MD steps, collision). */
int         orc_run(orc_system* s, int32_t n_md, int32_t n_collide);
/* one interval with the collision optional (MD-only tests) */
int         orc_interval(orc_system* s, int32_t n_md, int32_t do_collide);
int         orc_collide(orc_system* s, int32_t n_md);
void        orc_observables(const orc_system* s, orc_obs* o);

/* inspection for tests */
int64_t     orc_candidates(const orc_system* s, int64_t* idx, int64_t cap);
void        orc_forces(const orc_system* s, double* f);            /* 3N SoA, last eval */
int         orc_build_list(orc_system* s, int32_t n_md);            /* list + forces */
void        orc_forces_allpairs(orc_system* s, double* f, double* F);/* 3N, 3*nc */
void        orc_cell_keys(const orc_system* s, const double shift[3], uint32_t* keys);
void        orc_shift(const orc_system* s, int64_t coll_step, double shift[3]);
int64_t     orc_last_cells(const orc_system* s, uint32_t* start, int64_t cap); /* by sort rank */
int64_t     orc_cell_ranks(const orc_system* s, uint32_t* rank_of, int64_t cap);
uint64_t    orc_hilbert(uint32_t x, uint32_t y, uint32_t z, int bits);
void        orc_marsaglia(uint64_t seed, int64_t coll_step, int64_t cell, double n[3]);
void        orc_rotate(const double n[3], double ca, double sa, const double w[3], double out[3]);
void        orc_ptable(double bulk_rate, double tau, double* table);

/* dimer analysis of bond k: rec = R_com[3], V_com[3], axis u[3], V_com.u */
int         orc_dimer_sample(const orc_system* s, int32_t k, double rec[10]);
/* adds the current species counts per (z, rho) bin to hist[2][nz][nr] */
int         orc_cyl_hist(const orc_system* s, int32_t k, int32_t nz, int32_t nr,
                         double zmax, double rmax, uint64_t* hist);
void        orc_msd(const double* R, int64_t T, int32_t max_lag, double* msd);

#ifdef __cplusplus
}
#endif
#endif
