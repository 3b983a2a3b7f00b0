/*
 * FP64 CPU oracle for the MPCD+MD solvent path.  TEST INFRASTRUCTURE ONLY:
 * loaded by the tests, the smoke check and the benchmark's CPU-baseline leg;
 * the product library does not use it.
 *
 * Every function states the passage of the paper (section / equation) it
 * follows.  Where the paper is silent the reading used is stated inline; the
 * full list of readings is kept with the design notes.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.  Contraction is
 * off so that every multiply and add rounds separately; where the method uses
 * a fused multiply-add it is written as fma().
 *
 * Parity status: every function here is pinned by a CPU test (numpy Philox,
 * brute-force forces, stable argsort, conservation laws, closed forms of
 * MPCD transport, analytic special cases); the dimer's propulsion speed is
 * not (parity unpinned: no reference values are available).
 */
#include "rmp_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11), the counter-based RNG family the     */
/* paper's "Algorithms" section names.                                        */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { TAG_SHIFT = 1, TAG_ROT = 2, TAG_BULK = 3, TAG_CAT = 4, TAG_THERMO = 5,
       TAG_INIT_POS = 6, TAG_INIT_VEL = 7, TAG_VIRT = 8 };

static void draw(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t c,
                 uint64_t w[4])
{
    uint64_t ctr[4] = { a, b, c, 0 };
    uint64_t key[2] = { seed, tag };
    orc_philox(ctr, key, w);
}

/* uniform in [0,1) from the top 53 bits */
static double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
/* uniform in (0,1] (for logarithms) */
static double u01o(uint64_t w) { return ((double)(w >> 11) + 1.0) * 0x1.0p-53; }

/* Box-Muller: three standard normals from one Philox block. */
static void normals3(const uint64_t w[4], double z[3])
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

/* ------------------------------------------------------------------------ */
/* WCA potential ("Algorithms", the cut-off 12-6 Lennard-Jones equation):    */
/*   V(r) = 4 eps ((s/r)^12 - (s/r)^6 + 1/4) for r < 2^(1/6) s, else 0.     */
/* Returns coef = -(dV/dr)/r so that the force on the solvent particle is    */
/* coef * (x_solvent - X_colloid), and the potential.                        */
/* ------------------------------------------------------------------------ */
static const double TWO_1_6 = 0x1.1f59ac3c7d6c0p+0;   /* 2^(1/6) */

void orc_wca(double r2, double sigma, double eps, double* coef, double* pot)
{
    double sig2 = sigma * sigma;
    double ir2 = 1.0 / r2;
    double s2 = sig2 * ir2;
    double s6 = (s2 * s2) * s2;
    *coef = (((24.0 * eps) * ir2) * s6) * ((2.0 * s6) - 1.0);
    *pot = (4.0 * eps) * (((s6 * s6) - s6) + 0.25);
}

/* Fixed binary-tree sum over list positions, padded with zeros to a power   */
/* of two: node(l, j) = node(l-1, 2j) + node(l-1, 2j+1).  The reduction order */
/* of the colloid forces is not given in the paper; this definition makes    */
/* the result independent of how the work is split.                          */
static double tree_rec(const double* a, int64_t n, int64_t lo, int64_t size)
{
    if (lo >= n) return 0.0;
    if (size == 1) return a[lo];
    int64_t h = size >> 1;
    return tree_rec(a, n, lo, h) + tree_rec(a, n, lo + h, h);
}

double orc_tree_sum(const double* a, int64_t n)
{
    if (n <= 0) return 0.0;
    int64_t p = 1;
    while (p < n) p <<= 1;
    return tree_rec(a, n, 0, p);
}

/* ------------------------------------------------------------------------ */
struct orc_system {
    orc_params p;
    uint64_t seed;
    int64_t n;
    double Ld[3], halfL[3];
    double *x[3], *v[3], *f[3];
    uint32_t* id;
    uint8_t* st;
    /* colloids */
    int nc;
    int body[ORC_MAXC];       /* rigid body of a colloid: smallest colloid of its bonded group */
    int iterative;            /* some colloid has two or more bonds: iterative RATTLE */
    double X[ORC_MAXC][3], V[ORC_MAXC][3], F[ORC_MAXC][3], X0[ORC_MAXC][3];
    double hc[ORC_MAXC];      /* 0.5*dt/M */
    double imass[ORC_MAXC];   /* 1/M */
    double rc2[ORC_MAXC], sig2[ORC_MAXC], reachR[ORC_MAXC];
    double h;                 /* 0.5*dt/m */
    double ca, sa, oma;       /* cos, sin, 1-cos of alpha */
    /* Verlet list */
    int64_t ncand, cap;
    int64_t* idx;
    double* contrib;          /* [nc][3][cap] */
    double* upart;            /* [cap] */
    uint8_t* inside;          /* [cap] inside a catalytic colloid's range */
    /* scratch for the sort */
    uint32_t* keys;
    uint32_t* start;          /* [ncell+1] of the last collision, by sort rank */
    uint32_t* rank_of;        /* [ncell] sort rank of a cell (Hilbert order)  */
    uint32_t* cell_of;        /* [ncell] cell of a sort rank                  */
    int64_t ncell;
    double *tx[3], *tv[3];
    uint32_t* tid;
    uint8_t* tst;
    /* counters and observables */
    int64_t md_step, coll_step;
    double potential, e_rxn, temperature;
    int64_t n_cat, n_bulk, n_cells_T;
    uint32_t flags;
    double ptable[ORC_PTABLE];
    int32_t ptable_nmd;
};

static double wrap1(double x, double L)
{
    if (x >= L) x -= L;
    else if (x < 0.0) { x += L; if (x >= L) x -= L; }
    return x;
}

static double mimg(double d, double L, double halfL)
{
    if (d > halfL) d -= L;
    else if (d < -halfL) d += L;
    return d;
}

/* colloid positions are kept unwrapped; forces use the image in [0,L) */
static double wrapX(double X, double L)
{
    double k = floor(X / L);
    double w = X - k * L;
    if (w >= L) w -= L;
    else if (w < 0.0) { w += L; if (w >= L) w -= L; }
    return w;
}

static int has_flow(const orc_params* p)
{
    return p->walls != 0 || p->accel[0] != 0.0 || p->accel[1] != 0.0 || p->accel[2] != 0.0;
}

static void *xalloc(size_t n) { void* q = calloc(n ? n : 1, 1); return q; }

/* Position of the point (x, y, z) along the Hilbert curve through the
 * 2^bits cube (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc.
 * 707 (2004) 381): the coordinates are turned into the curve's "transpose"
 * form by undoing the excess work (for each level Q from the top: invert the
 * low bits of the first coordinate where a coordinate's Q bit is set, else
 * exchange the low bits of the first coordinate and that one), then Gray
 * encoding; the index takes one bit from each coordinate per level, first
 * coordinate most significant. */
uint64_t orc_hilbert(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint32_t X[3] = { x, y, z };
    if (bits <= 0) return 0;
    const uint32_t top = 1u << (bits - 1);
    for (uint32_t Q = top; Q > 1; Q >>= 1) {
        const uint32_t low = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= low;
            } else {
                uint32_t t = (X[0] ^ X[i]) & low;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t g = 0;
    for (uint32_t Q = top; Q > 1; Q >>= 1)
        if (X[2] & Q) g ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= g;
    uint64_t h = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
    return h;
}

/* Sort order of the cells when the compact-Hilbert ordering of the paper's
 * cell sort is selected, read as: cells of the box ranked by their position
 * along the Hilbert curve of the smallest power-of-two cube that contains the
 * box.  The default order is row-major (rank = cell index). */
static int cmp_u64_pair(const void* a, const void* b)
{
    const uint64_t* p = (const uint64_t*)a;
    const uint64_t* q = (const uint64_t*)b;
    return p[0] < q[0] ? -1 : (p[0] > q[0] ? 1 : 0);
}

static void hilbert_order(const int32_t L[3], uint32_t* rank_of, uint32_t* cell_of)
{
    int bits = 0;
    int32_t m = L[0] > L[1] ? L[0] : L[1];
    if (L[2] > m) m = L[2];
    while ((1 << bits) < m) bits++;
    const int64_t ncell = (int64_t)L[0] * L[1] * L[2];
    uint64_t* pairs = (uint64_t*)xalloc(sizeof(uint64_t) * 2 * ncell);
    for (int64_t c = 0; c < ncell; ++c) {
        const uint32_t x = (uint32_t)(c % L[0]);
        const uint32_t y = (uint32_t)((c / L[0]) % L[1]);
        const uint32_t z = (uint32_t)(c / ((int64_t)L[0] * L[1]));
        pairs[2 * c] = orc_hilbert(x, y, z, bits);
        pairs[2 * c + 1] = (uint64_t)c;
    }
    qsort(pairs, (size_t)ncell, 2 * sizeof(uint64_t), cmp_u64_pair);
    for (int64_t r = 0; r < ncell; ++r) {
        cell_of[r] = (uint32_t)pairs[2 * r + 1];
        rank_of[pairs[2 * r + 1]] = (uint32_t)r;
    }
    free(pairs);
}

orc_system* orc_create(const orc_params* p, uint64_t seed)
{
    if (p->L[0] < 1 || p->L[1] < 1 || p->L[2] < 1 || p->n_solvent < 0 ||
        (p->cell_order != 0 && p->cell_order != 1) ||
        p->n_colloids < 0 || p->n_colloids > ORC_MAXC || p->dt <= 0.0 || p->mass <= 0.0)
        return NULL;
    /* flows: no colloids; walls with the rotation rule, row-major cells, a
     * fill density and no acceleration across the plates */
    if (p->walls != 0 && p->walls != 1) return NULL;
    if (has_flow(p) && (p->n_colloids != 0 || p->n_bonds != 0)) return NULL;
    if (p->walls && (p->rule != 0 || p->cell_order != 0 || p->accel[2] != 0.0 ||
                     p->wall_density < 1 || p->wall_density > 1024))
        return NULL;
    if (p->n_bonds < 0 || p->n_bonds > ORC_MAXB) return NULL;
    int degree[ORC_MAXC] = { 0 };
    for (int q = 0; q < p->n_bonds; ++q) {
        const int a = p->bond_a[q], b = p->bond_b[q];
        if (a < 0 || b < 0 || a >= p->n_colloids || b >= p->n_colloids || a == b || !(p->bond_d[q] > 0.0))
            return NULL;
        for (int r = 0; r < q; ++r)
            if ((p->bond_a[r] == a && p->bond_b[r] == b) || (p->bond_a[r] == b && p->bond_b[r] == a))
                return NULL;
        degree[a]++;
        degree[b]++;
    }
    int iterative = p->rattle_iterative != 0 && p->n_bonds > 0;
    for (int c = 0; c < p->n_colloids; ++c) if (degree[c] > 1) iterative = 1;
    if (iterative && (!(p->rattle_tol > 0.0) || p->rattle_maxit < 1 || p->rattle_maxit > 100000)) return NULL;
    orc_system* s = (orc_system*)xalloc(sizeof(orc_system));
    s->p = *p;
    s->seed = seed;
    s->n = p->n_solvent;
    for (int d = 0; d < 3; ++d) {
        s->Ld[d] = (double)p->L[d];
        s->halfL[d] = 0.5 * s->Ld[d];
        s->x[d] = (double*)xalloc(sizeof(double) * s->n);
        s->v[d] = (double*)xalloc(sizeof(double) * s->n);
        s->f[d] = (double*)xalloc(sizeof(double) * s->n);
        s->tx[d] = (double*)xalloc(sizeof(double) * s->n);
        s->tv[d] = (double*)xalloc(sizeof(double) * s->n);
    }
    s->id = (uint32_t*)xalloc(sizeof(uint32_t) * s->n);
    s->st = (uint8_t*)xalloc(s->n);
    s->tid = (uint32_t*)xalloc(sizeof(uint32_t) * s->n);
    s->tst = (uint8_t*)xalloc(s->n);
    s->keys = (uint32_t*)xalloc(sizeof(uint32_t) * s->n);
    /* with walls the shifted grid needs L_z + 1 layers of cells across the channel */
    s->ncell = (int64_t)p->L[0] * p->L[1] * (p->L[2] + (p->walls ? 1 : 0));
    s->start = (uint32_t*)xalloc(sizeof(uint32_t) * (s->ncell + 1));
    s->rank_of = (uint32_t*)xalloc(sizeof(uint32_t) * s->ncell);
    s->cell_of = (uint32_t*)xalloc(sizeof(uint32_t) * s->ncell);
    if (p->cell_order == 1) {
        hilbert_order(p->L, s->rank_of, s->cell_of);
    } else {
        for (int64_t c = 0; c < s->ncell; ++c) { s->rank_of[c] = (uint32_t)c; s->cell_of[c] = (uint32_t)c; }
    }
    s->nc = p->n_colloids;
    s->iterative = iterative;
    /* rigid bodies: connected groups of the bond graph, each named by its
     * smallest colloid (relabel until no bond joins two labels) */
    for (int c = 0; c < s->nc; ++c) s->body[c] = c;
    for (int changed = 1; changed;) {
        changed = 0;
        for (int q = 0; q < p->n_bonds; ++q) {
            const int a = p->bond_a[q], b = p->bond_b[q];
            const int m = s->body[a] < s->body[b] ? s->body[a] : s->body[b];
            if (s->body[a] != m || s->body[b] != m) {
                const int oa = s->body[a], ob = s->body[b];
                for (int c = 0; c < s->nc; ++c)
                    if (s->body[c] == oa || s->body[c] == ob) s->body[c] = m;
                changed = 1;
            }
        }
    }
    s->h = (0.5 * p->dt) / p->mass;
    s->ca = cos(p->alpha);
    s->sa = sin(p->alpha);
    s->oma = 1.0 - s->ca;
    for (int c = 0; c < s->nc; ++c) {
        for (int d = 0; d < 3; ++d) { s->X[c][d] = p->cx[c][d]; s->V[c][d] = 0.0; s->F[c][d] = 0.0; }
        s->hc[c] = (0.5 * p->dt) / p->cmass[c];
        s->imass[c] = 1.0 / p->cmass[c];
        double rc = TWO_1_6 * p->sigma[c];
        s->rc2[c] = rc * rc;
        s->sig2[c] = p->sigma[c] * p->sigma[c];
        s->reachR[c] = rc + p->skin;
    }
    s->cap = 0;
    s->ptable_nmd = -1;
    return s;
}

void orc_destroy(orc_system* s)
{
    if (!s) return;
    for (int d = 0; d < 3; ++d) { free(s->x[d]); free(s->v[d]); free(s->f[d]); free(s->tx[d]); free(s->tv[d]); }
    free(s->id); free(s->st); free(s->tid); free(s->tst); free(s->keys); free(s->start);
    free(s->rank_of); free(s->cell_of);
    free(s->idx); free(s->contrib); free(s->upart); free(s->inside);
    free(s);
}

/* Initial state (overview: N solvent particles with mass, position and
 * velocity in a cuboid domain; velocities Maxwellian at kT, mean removed).
 * Positions are uniform and rejected inside colloid cores (r < sigma). */
int orc_init(orc_system* s)
{
    const orc_params* p = &s->p;
    double Xw[ORC_MAXC][3];
    for (int c = 0; c < s->nc; ++c)
        for (int d = 0; d < 3; ++d) Xw[c][d] = wrapX(s->X[c][d], s->Ld[d]);
    uint32_t bad = 0;
    #pragma omp parallel for schedule(static) reduction(|:bad)
    for (int64_t i = 0; i < s->n; ++i) {
        double xi[3];
        int ok = 0;
        for (uint64_t att = 0; att < 4096 && !ok; ++att) {
            uint64_t w[4];
            draw(s->seed, TAG_INIT_POS, att, (uint64_t)i, 0, w);
            for (int d = 0; d < 3; ++d) {
                xi[d] = u01(w[d]) * s->Ld[d];
            }
            ok = 1;
            for (int c = 0; c < s->nc && ok; ++c) {
                double dx = mimg(xi[0] - Xw[c][0], s->Ld[0], s->halfL[0]);
                double dy = mimg(xi[1] - Xw[c][1], s->Ld[1], s->halfL[1]);
                double dz = mimg(xi[2] - Xw[c][2], s->Ld[2], s->halfL[2]);
                double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
                if (r2 < s->sig2[c]) ok = 0;
            }
        }
        if (!ok) bad |= ORC_F_INIT;
        for (int d = 0; d < 3; ++d) s->x[d][i] = xi[d];
        uint64_t w[4];
        double z[3];
        draw(s->seed, TAG_INIT_VEL, 0, (uint64_t)i, 0, w);
        normals3(w, z);
        double sc = sqrt(p->kT / p->mass);
        for (int d = 0; d < 3; ++d) s->v[d][i] = sc * z[d];
        s->id[i] = (uint32_t)i;
        s->st[i] = 0;
    }
    s->flags |= bad;
    if (s->n > 0) {
        for (int d = 0; d < 3; ++d) {
            double m = 0.0;
            for (int64_t i = 0; i < s->n; ++i) m += s->v[d][i];
            m = m / (double)s->n;
            for (int64_t i = 0; i < s->n; ++i) s->v[d][i] = s->v[d][i] - m;
        }
    }
    s->md_step = 0;
    s->coll_step = 0;
    return 0;
}

int orc_set_state(orc_system* s, const double* x, const double* v, const uint32_t* id,
                  const uint8_t* st, const double* X, const double* V,
                  int64_t md_step, int64_t coll_step)
{
    for (int d = 0; d < 3; ++d) {
        memcpy(s->x[d], x + d * s->n, sizeof(double) * s->n);
        memcpy(s->v[d], v + d * s->n, sizeof(double) * s->n);
        memset(s->f[d], 0, sizeof(double) * s->n);
    }
    memcpy(s->id, id, sizeof(uint32_t) * s->n);
    memcpy(s->st, st, s->n);
    for (int c = 0; c < s->nc; ++c)
        for (int d = 0; d < 3; ++d) { s->X[c][d] = X[3 * c + d]; s->V[c][d] = V[3 * c + d]; s->F[c][d] = 0.0; }
    s->md_step = md_step;
    s->coll_step = coll_step;
    s->ncand = 0;
    return 0;
}

int orc_get_state(const orc_system* s, double* x, double* v, uint32_t* id, uint8_t* st,
                  double* X, double* V, double* F, int64_t* md_step, int64_t* coll_step)
{
    for (int d = 0; d < 3; ++d) {
        if (x) memcpy(x + d * s->n, s->x[d], sizeof(double) * s->n);
        if (v) memcpy(v + d * s->n, s->v[d], sizeof(double) * s->n);
    }
    if (id) memcpy(id, s->id, sizeof(uint32_t) * s->n);
    if (st) memcpy(st, s->st, s->n);
    for (int c = 0; c < s->nc; ++c)
        for (int d = 0; d < 3; ++d) {
            if (X) X[3 * c + d] = s->X[c][d];
            if (V) V[3 * c + d] = s->V[c][d];
            if (F) F[3 * c + d] = s->F[c][d];
        }
    if (md_step) *md_step = s->md_step;
    if (coll_step) *coll_step = s->coll_step;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Verlet list ("Algorithms": Verlet and cell lists for the colloid-solvent  */
/* forces).  A particle enters the list for the coming interval of n_md MD   */
/* steps if it is flagged (catalysis memory) or if, for some colloid c,      */
/*    r_ic < r_cut,c + skin + |v_i| tau        (tau = n_md dt),              */
/* evaluated as r2 < t*t with t = (r_cut,c + skin) + sqrt(v.v)*tau.  A      */
/* particle outside the list moves ballistically for the whole interval and  */
/* cannot reach any cut-off sphere unless a colloid moves by more than the   */
/* skin; colloid displacement >= skin/2 sets ORC_F_DISPLACEMENT.            */
/* The list keeps array order.                                               */
/* ------------------------------------------------------------------------ */
static void ensure_cap(orc_system* s, int64_t need)
{
    if (need <= s->cap) return;
    int64_t cap = need + need / 4 + 64;
    free(s->idx); free(s->contrib); free(s->upart); free(s->inside);
    s->idx = (int64_t*)xalloc(sizeof(int64_t) * cap);
    s->contrib = (double*)xalloc(sizeof(double) * cap * 3 * (s->nc ? s->nc : 1));
    s->upart = (double*)xalloc(sizeof(double) * cap);
    s->inside = (uint8_t*)xalloc(cap);
    s->cap = cap;
}

static int is_candidate(const orc_system* s, int64_t i, const double Xw[][3], double tau)
{
    if (s->st[i] & 2) return 1;
    double vx = s->v[0][i], vy = s->v[1][i], vz = s->v[2][i];
    double v2 = ((vx * vx) + (vy * vy)) + (vz * vz);
    double reach = sqrt(v2) * tau;
    for (int c = 0; c < s->nc; ++c) {
        double dx = mimg(s->x[0][i] - Xw[c][0], s->Ld[0], s->halfL[0]);
        double dy = mimg(s->x[1][i] - Xw[c][1], s->Ld[1], s->halfL[1]);
        double dz = mimg(s->x[2][i] - Xw[c][2], s->Ld[2], s->halfL[2]);
        double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
        double t = s->reachR[c] + reach;
        if (r2 < t * t) return 1;
    }
    return 0;
}

static void wrapped_colloids(const orc_system* s, double Xw[][3])
{
    for (int c = 0; c < s->nc; ++c)
        for (int d = 0; d < 3; ++d) Xw[c][d] = wrapX(s->X[c][d], s->Ld[d]);
}

/* Forces over the Verlet list (WCA equation), colloid forces by Newton's
 * third law summed with the fixed tree, colloid-colloid WCA with
 * sigma_ij = sigma_i + sigma_j and eps from the type table, bonded pairs
 * excluded (their distance is held by RATTLE). */
static void compute_forces(orc_system* s)
{
    const int nc = s->nc;
    double Xw[ORC_MAXC][3];
    wrapped_colloids(s, Xw);
    const int64_t nl = s->ncand;
    double* cb = s->contrib;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nl; ++k) {
        int64_t i = s->idx[k];
        int sp = s->st[i] & 1;
        double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0;
        int in = 0;
        for (int c = 0; c < nc; ++c) {
            double dx = mimg(s->x[0][i] - Xw[c][0], s->Ld[0], s->halfL[0]);
            double dy = mimg(s->x[1][i] - Xw[c][1], s->Ld[1], s->halfL[1]);
            double dz = mimg(s->x[2][i] - Xw[c][2], s->Ld[2], s->halfL[2]);
            double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
            double gx = 0.0, gy = 0.0, gz = 0.0;
            if (r2 < s->rc2[c]) {
                double eps = sp ? s->p.epsB[c] : s->p.epsA[c];
                double coef, pot;
                orc_wca(r2, s->p.sigma[c], eps, &coef, &pot);
                gx = coef * dx; gy = coef * dy; gz = coef * dz;
                fx = fx + gx; fy = fy + gy; fz = fz + gz;
                u = u + pot;
                if (s->p.catalytic[c]) in = 1;
            }
            cb[((size_t)c * 3 + 0) * s->cap + k] = gx;
            cb[((size_t)c * 3 + 1) * s->cap + k] = gy;
            cb[((size_t)c * 3 + 2) * s->cap + k] = gz;
        }
        s->f[0][i] = fx; s->f[1][i] = fy; s->f[2][i] = fz;
        s->upart[k] = u;
        s->inside[k] = (uint8_t)in;
    }
    for (int c = 0; c < nc; ++c)
        for (int d = 0; d < 3; ++d)
            s->F[c][d] = -orc_tree_sum(cb + ((size_t)c * 3 + d) * s->cap, nl);
    double ucc = 0.0;
    for (int a = 0; a < nc; ++a) {
        for (int b = a + 1; b < nc; ++b) {
            /* colloids of one rigid body do not interact */
            if (s->body[a] == s->body[b]) continue;
            double dx = mimg(Xw[a][0] - Xw[b][0], s->Ld[0], s->halfL[0]);
            double dy = mimg(Xw[a][1] - Xw[b][1], s->Ld[1], s->halfL[1]);
            double dz = mimg(Xw[a][2] - Xw[b][2], s->Ld[2], s->halfL[2]);
            double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
            double sab = s->p.sigma[a] + s->p.sigma[b];
            double rc = TWO_1_6 * sab;
            if (r2 < rc * rc) {
                double coef, pot;
                orc_wca(r2, sab, s->p.eps_cc[s->p.ctype[a]][s->p.ctype[b]], &coef, &pot);
                double g[3] = { coef * dx, coef * dy, coef * dz };
                for (int d = 0; d < 3; ++d) { s->F[a][d] = s->F[a][d] + g[d]; s->F[b][d] = s->F[b][d] - g[d]; }
                ucc = ucc + pot;
            }
        }
    }
    s->potential = orc_tree_sum(s->upart, nl) + ucc;
    for (int c = 0; c < nc; ++c)
        for (int d = 0; d < 3; ++d)
            if (!isfinite(s->F[c][d])) s->flags |= ORC_F_NONFINITE;
}

int orc_build_list(orc_system* s, int32_t n_md)
{
    if (has_flow(&s->p)) {
        /* flows have no colloids: every particle streams, no list */
        s->ncand = 0;
        return 0;
    }
    double Xw[ORC_MAXC][3];
    wrapped_colloids(s, Xw);
    double tau = (double)n_md * s->p.dt;
    int64_t cnt = 0;
    for (int64_t i = 0; i < s->n; ++i) cnt += is_candidate(s, i, (const double (*)[3])Xw, tau);
    ensure_cap(s, cnt);
    int64_t k = 0;
    for (int64_t i = 0; i < s->n; ++i) {
        s->f[0][i] = 0.0; s->f[1][i] = 0.0; s->f[2][i] = 0.0;
        if (is_candidate(s, i, (const double (*)[3])Xw, tau)) s->idx[k++] = i;
    }
    s->ncand = cnt;
    for (int c = 0; c < s->nc; ++c)
        for (int d = 0; d < 3; ++d) s->X0[c][d] = s->X[c][d];
    compute_forces(s);
    return 0;
}

/* Exact RATTLE for one bond ("Algorithms": RATTLE, exact for the dimer).
 * Position stage: the constraint displacement is along the bond vector at
 * the start of the step, r0; with s = X_a - X_b after the free drift and
 * mu = 1/M_a + 1/M_b, |s - g mu r0| = d gives the quadratic
 *   (mu^2 r0.r0) g^2 - 2 (mu s.r0) g + (s.s - d^2) = 0,
 * solved for the small root g = C / (Bh + sqrt(Bh^2 - A C)). */
static void rattle_pos(orc_system* s, double Xold[][3])
{
    const double dt = s->p.dt;
    for (int q = 0; q < s->p.n_bonds; ++q) {
        int a = s->p.bond_a[q], b = s->p.bond_b[q];
        double dd = s->p.bond_d[q];
        double r0[3], sv[3];
        for (int d = 0; d < 3; ++d) { r0[d] = Xold[a][d] - Xold[b][d]; sv[d] = s->X[a][d] - s->X[b][d]; }
        double mu = s->imass[a] + s->imass[b];
        double r0r0 = ((r0[0] * r0[0]) + (r0[1] * r0[1])) + (r0[2] * r0[2]);
        double sr0 = ((sv[0] * r0[0]) + (sv[1] * r0[1])) + (sv[2] * r0[2]);
        double ss = ((sv[0] * sv[0]) + (sv[1] * sv[1])) + (sv[2] * sv[2]);
        double A = (mu * mu) * r0r0;
        double Bh = mu * sr0;
        double C = ss - (dd * dd);
        double disc = (Bh * Bh) - (A * C);
        if (disc < 0.0) { s->flags |= ORC_F_RATTLE; disc = 0.0; }
        double g = C / (Bh + sqrt(disc));
        double ga = g * s->imass[a], gb = g * s->imass[b];
        double gad = ga / dt, gbd = gb / dt;
        for (int d = 0; d < 3; ++d) {
            s->X[a][d] = s->X[a][d] - (ga * r0[d]);
            s->X[b][d] = s->X[b][d] + (gb * r0[d]);
            s->V[a][d] = s->V[a][d] - (gad * r0[d]);
            s->V[b][d] = s->V[b][d] + (gbd * r0[d]);
        }
    }
}

/* Iterative RATTLE (Andersen 1983), position stage, for bond networks (a
 * colloid in two or more bonds, as in a composite Janus particle): sweeps
 * over the bonds in their order; a bond whose squared length s.s misses
 * d^2 by more than 2 tol d^2 is corrected along its direction before the
 * drift, r0: both colloids move by g r0 / m (g = (d^2 - s.s) / (2 mu s.r0),
 * mu = 1/m_a + 1/m_b) and their velocities by the same displacement over dt.
 * Sweeps repeat until one changes nothing; after rattle_maxit sweeps the
 * RATTLE flag is raised. */
static void rattle_pos_iter(orc_system* s, double Xold[][3])
{
    const double dt = s->p.dt, tol = s->p.rattle_tol;
    int sweep = 0, moved = 1;
    for (; sweep < s->p.rattle_maxit && moved; ++sweep) {
        moved = 0;
        for (int q = 0; q < s->p.n_bonds; ++q) {
            const int a = s->p.bond_a[q], b = s->p.bond_b[q];
            const double dd2 = s->p.bond_d[q] * s->p.bond_d[q];
            double sv[3], r0[3];
            for (int d = 0; d < 3; ++d) { sv[d] = s->X[a][d] - s->X[b][d]; r0[d] = Xold[a][d] - Xold[b][d]; }
            const double ss = ((sv[0] * sv[0]) + (sv[1] * sv[1])) + (sv[2] * sv[2]);
            const double diff = dd2 - ss;
            if (fabs(diff) > (2.0 * tol) * dd2) {
                const double mu = s->imass[a] + s->imass[b];
                const double sr0 = ((sv[0] * r0[0]) + (sv[1] * r0[1])) + (sv[2] * r0[2]);
                const double g = diff / ((2.0 * mu) * sr0);
                const double ga = g * s->imass[a], gb = g * s->imass[b];
                const double gad = ga / dt, gbd = gb / dt;
                for (int d = 0; d < 3; ++d) {
                    s->X[a][d] = s->X[a][d] + (ga * r0[d]);
                    s->X[b][d] = s->X[b][d] - (gb * r0[d]);
                    s->V[a][d] = s->V[a][d] + (gad * r0[d]);
                    s->V[b][d] = s->V[b][d] - (gbd * r0[d]);
                }
                moved = 1;
            }
        }
    }
    if (moved) s->flags |= ORC_F_RATTLE;
}

/* Iterative RATTLE, velocity stage: sweeps removing the relative velocity
 * along each bond, k = (r.v) / (mu d^2), while |r.v| exceeds tol d^2 / dt. */
static void rattle_vel_iter(orc_system* s)
{
    const double tol = s->p.rattle_tol, dt = s->p.dt;
    int sweep = 0, moved = 1;
    for (; sweep < s->p.rattle_maxit && moved; ++sweep) {
        moved = 0;
        for (int q = 0; q < s->p.n_bonds; ++q) {
            const int a = s->p.bond_a[q], b = s->p.bond_b[q];
            const double dd2 = s->p.bond_d[q] * s->p.bond_d[q];
            double r[3], vr[3];
            for (int d = 0; d < 3; ++d) { r[d] = s->X[a][d] - s->X[b][d]; vr[d] = s->V[a][d] - s->V[b][d]; }
            const double rv = ((r[0] * vr[0]) + (r[1] * vr[1])) + (r[2] * vr[2]);
            if (fabs(rv) > (tol * dd2) / dt) {
                const double mu = s->imass[a] + s->imass[b];
                const double k = rv / (mu * dd2);
                const double ka = k * s->imass[a], kb = k * s->imass[b];
                for (int d = 0; d < 3; ++d) {
                    s->V[a][d] = s->V[a][d] - (ka * r[d]);
                    s->V[b][d] = s->V[b][d] + (kb * r[d]);
                }
                moved = 1;
            }
        }
    }
    if (moved) s->flags |= ORC_F_RATTLE;
}

/* Velocity stage: remove the relative velocity along the bond. */
static void rattle_vel(orc_system* s)
{
    for (int q = 0; q < s->p.n_bonds; ++q) {
        int a = s->p.bond_a[q], b = s->p.bond_b[q];
        double r[3], vr[3];
        for (int d = 0; d < 3; ++d) { r[d] = s->X[a][d] - s->X[b][d]; vr[d] = s->V[a][d] - s->V[b][d]; }
        double mu = s->imass[a] + s->imass[b];
        double rr = ((r[0] * r[0]) + (r[1] * r[1])) + (r[2] * r[2]);
        double vrr = ((vr[0] * r[0]) + (vr[1] * r[1])) + (vr[2] * r[2]);
        double k = vrr / (mu * rr);
        double ka = k * s->imass[a], kb = k * s->imass[b];
        for (int d = 0; d < 3; ++d) {
            s->V[a][d] = s->V[a][d] - (ka * r[d]);
            s->V[b][d] = s->V[b][d] + (kb * r[d]);
        }
    }
}

/* potential-energy change of particle i when its species changes from
 * `from` to `to` (reaction energy bookkeeping; not part of the dynamics). */
static double species_dU(const orc_system* s, int64_t i, int from, int to)
{
    double Xw[ORC_MAXC][3];
    wrapped_colloids(s, Xw);
    double du = 0.0;
    for (int c = 0; c < s->nc; ++c) {
        double dx = mimg(s->x[0][i] - Xw[c][0], s->Ld[0], s->halfL[0]);
        double dy = mimg(s->x[1][i] - Xw[c][1], s->Ld[1], s->halfL[1]);
        double dz = mimg(s->x[2][i] - Xw[c][2], s->Ld[2], s->halfL[2]);
        double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
        if (r2 < s->rc2[c]) {
            double cf, p0, p1;
            orc_wca(r2, s->p.sigma[c], from ? s->p.epsB[c] : s->p.epsA[c], &cf, &p0);
            orc_wca(r2, s->p.sigma[c], to ? s->p.epsB[c] : s->p.epsA[c], &cf, &p1);
            du += p1 - p0;
        }
    }
    return du;
}

/* One streaming step of a solvent particle under the constant acceleration g
 * ("Algorithms": flows from a constant acceleration on the solvent), as a
 * velocity-Verlet step with the force m g: half kick, drift, half kick.
 * With walls (plates at z = 0 and z = L_z, stick boundary by the bounce-back
 * rule) a drift that leaves the channel is cut at the crossing time t*: the
 * particle moves to the wall, its velocity is reversed, and it travels the
 * rest of the step, dt - t*, with the reversed velocity. */
static void flow_step(const orc_system* s, double x[3], double v[3])
{
    const double dt = s->p.dt, hdt = 0.5 * dt;
    double y[3];
    for (int d = 0; d < 3; ++d) {
        v[d] = fma(hdt, s->p.accel[d], v[d]);
        y[d] = fma(dt, v[d], x[d]);
    }
    if (s->p.walls) {
        const double Lz = s->Ld[2];
        if (y[2] < 0.0 || y[2] >= Lz) {
            const double wz = y[2] < 0.0 ? 0.0 : Lz;
            const double ts = (wz - x[2]) / v[2];
            const double rem = dt - ts;
            for (int d = 0; d < 3; ++d) {
                const double xc = fma(ts, v[d], x[d]);
                v[d] = -v[d];
                y[d] = fma(rem, v[d], xc);
            }
            /* rounding can leave the reflected point on a plate */
            if (y[2] >= Lz) y[2] = nextafter(Lz, 0.0);
            if (y[2] < 0.0) y[2] = 0.0;
        }
        x[0] = wrap1(y[0], s->Ld[0]);
        x[1] = wrap1(y[1], s->Ld[1]);
        x[2] = y[2];
    } else {
        for (int d = 0; d < 3; ++d) x[d] = wrap1(y[d], s->Ld[d]);
    }
    for (int d = 0; d < 3; ++d) v[d] = fma(hdt, s->p.accel[d], v[d]);
}

/* One velocity-Verlet step ("Algorithms": velocity-Verlet for solvent and
 * colloids; Overview: Newton's equations solved with velocity-Verlet), in
 * kick-drift-kick form with fused multiply-adds, followed by the catalytic
 * conversion (A becomes B with probability p when it leaves the catalytic
 * sphere's interaction range; "Applications" and the configuration's
 * `probability`). */
static void md_step(orc_system* s)
{
    const double dt = s->p.dt;
    const int nc = s->nc;
    if (has_flow(&s->p)) {
        /* no colloids: every particle streams under the acceleration */
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < s->n; ++i) {
            double x[3], v[3];
            for (int d = 0; d < 3; ++d) { x[d] = s->x[d][i]; v[d] = s->v[d][i]; }
            flow_step(s, x, v);
            for (int d = 0; d < 3; ++d) { s->x[d][i] = x[d]; s->v[d][i] = v[d]; }
        }
        s->md_step++;
        return;
    }
    double Xold[ORC_MAXC][3];
    for (int c = 0; c < nc; ++c)
        for (int d = 0; d < 3; ++d) {
            s->V[c][d] = fma(s->hc[c], s->F[c][d], s->V[c][d]);
            Xold[c][d] = s->X[c][d];
            s->X[c][d] = fma(dt, s->V[c][d], s->X[c][d]);
        }
    if (s->iterative) rattle_pos_iter(s, Xold);
    else rattle_pos(s, Xold);
    const int64_t nl = s->ncand;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nl; ++k) {
        int64_t i = s->idx[k];
        for (int d = 0; d < 3; ++d) s->v[d][i] = fma(s->h, s->f[d][i], s->v[d][i]);
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->n; ++i)
        for (int d = 0; d < 3; ++d)
            s->x[d][i] = wrap1(fma(dt, s->v[d][i], s->x[d][i]), s->Ld[d]);
    compute_forces(s);
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nl; ++k) {
        int64_t i = s->idx[k];
        for (int d = 0; d < 3; ++d) s->v[d][i] = fma(s->h, s->f[d][i], s->v[d][i]);
    }
    for (int c = 0; c < nc; ++c)
        for (int d = 0; d < 3; ++d) s->V[c][d] = fma(s->hc[c], s->F[c][d], s->V[c][d]);
    if (s->iterative) rattle_vel_iter(s);
    else rattle_vel(s);
    /* catalysis, in list order */
    for (int64_t k = 0; k < nl; ++k) {
        int64_t i = s->idx[k];
        uint8_t st = s->st[i];
        if (st & 1) continue;                 /* only A converts */
        if (s->inside[k]) { s->st[i] = (uint8_t)(st | 2); continue; }
        if (st & 2) {
            int flip = 1;
            if (s->p.cat_prob < 1.0) {
                uint64_t w[4];
                draw(s->seed, TAG_CAT, (uint64_t)s->md_step, s->id[i], 0, w);
                flip = u01(w[0]) < s->p.cat_prob;
            }
            if (flip) {
                s->st[i] = 1;
                s->n_cat++;
                s->e_rxn += species_dU(s, i, 0, 1);
            } else {
                s->st[i] = 0;
            }
        }
    }
    /* list soundness: colloid displacement since the list was built */
    double lim = 0.5 * s->p.skin;
    for (int c = 0; c < nc; ++c) {
        double dx = s->X[c][0] - s->X0[c][0], dy = s->X[c][1] - s->X0[c][1], dz = s->X[c][2] - s->X0[c][2];
        if (((dx * dx) + (dy * dy)) + (dz * dz) >= lim * lim) s->flags |= ORC_F_DISPLACEMENT;
    }
    s->md_step++;
}

/* ------------------------------------------------------------------------ */
/* MPCD collision ("Algorithms": original MPCD collision rule with random    */
/* grid shifting; the Anderson thermostat variant; RMPCD bulk reaction).     */
/* ------------------------------------------------------------------------ */
void orc_shift(const orc_system* s, int64_t coll_step, double shift[3])
{
    uint64_t w[4];
    draw(s->seed, TAG_SHIFT, (uint64_t)coll_step, 0, 0, w);
    for (int d = 0; d < 3; ++d) shift[d] = u01(w[d]);
}

/* cell of the shifted position: c_d = floor(x_d - s_d) wrapped to [0, L_d);
 * key = c_x + L_x (c_y + L_y c_z).  With walls the z layers are not periodic:
 * c_z = floor(z - s_z) + 1 in [0, L_z], layer j covering [j - 1 + s_z, j + s_z),
 * so the first and last layers are cut by the plates. */
void orc_cell_keys(const orc_system* s, const double shift[3], uint32_t* keys)
{
    const int32_t* L = s->p.L;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->n; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) {
            int64_t q = (int64_t)floor(s->x[d][i] - shift[d]);
            if (d == 2 && s->p.walls) {
                c[d] = q + 1;
                continue;
            }
            if (q < 0) q += L[d];
            if (q >= L[d]) q -= L[d];
            c[d] = q;
        }
        keys[i] = (uint32_t)(c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * c[2]));
    }
}

/* Marsaglia (1972) point on the unit sphere: (a, b) uniform in the square,
 * accepted if s = a^2 + b^2 < 1; n = (2a sqrt(1-s), 2b sqrt(1-s), 1 - 2s).
 * Two tries per Philox block, `sub` counts blocks, 64 blocks at most. */
void orc_marsaglia(uint64_t seed, int64_t coll_step, int64_t cell, double n[3])
{
    for (uint64_t sub = 0; sub < 64; ++sub) {
        uint64_t w[4];
        draw(seed, TAG_ROT, (uint64_t)coll_step, (uint64_t)cell, sub, w);
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

/* Rotation of w by the angle alpha about the unit axis n (Rodrigues):
 *   R w = cos(a) w + sin(a) (n x w) + (1 - cos(a)) (n.w) n. */
void orc_rotate(const double n[3], double ca, double sa, const double w[3], double out[3])
{
    double oma = 1.0 - ca;
    double nw = ((n[0] * w[0]) + (n[1] * w[1])) + (n[2] * w[2]);
    double cx = (n[1] * w[2]) - (n[2] * w[1]);
    double cy = (n[2] * w[0]) - (n[0] * w[2]);
    double cz = (n[0] * w[1]) - (n[1] * w[0]);
    double k = oma * nw;
    out[0] = ((ca * w[0]) + (sa * cx)) + (k * n[0]);
    out[1] = ((ca * w[1]) + (sa * cy)) + (k * n[1]);
    out[2] = ((ca * w[2]) + (sa * cz)) + (k * n[2]);
}

/* probability of one bulk B->A event in a cell with nB B-particles during
 * tau: P = 1 - exp(-k nB tau), tabulated (host libm) for nB < ORC_PTABLE. */
void orc_ptable(double bulk_rate, double tau, double* table)
{
    double kt = bulk_rate * tau;
    for (int q = 0; q < ORC_PTABLE; ++q) table[q] = -expm1(-(kt * (double)q));
}

static void collide(orc_system* s, int32_t n_md)
{
    const int64_t n = s->n;
    const int64_t ncell = s->ncell;
    double shift[3];
    orc_shift(s, s->coll_step, shift);
    orc_cell_keys(s, shift, s->keys);
    /* stable counting sort by the cell's rank in the Hilbert order
     * (cell_system / particle_system sorting with the compact-Hilbert key) */
    uint32_t* cnt = (uint32_t*)xalloc(sizeof(uint32_t) * (ncell + 1));
    for (int64_t i = 0; i < n; ++i) cnt[s->rank_of[s->keys[i]]]++;
    s->start[0] = 0;
    for (int64_t r = 0; r < ncell; ++r) s->start[r + 1] = s->start[r] + cnt[r];
    for (int64_t r = 0; r < ncell; ++r) cnt[r] = s->start[r];
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = cnt[s->rank_of[s->keys[i]]]++;
        for (int d = 0; d < 3; ++d) { s->tx[d][j] = s->x[d][i]; s->tv[d][j] = s->v[d][i]; }
        s->tid[j] = s->id[i];
        s->tst[j] = s->st[i];
    }
    free(cnt);
    for (int d = 0; d < 3; ++d) {
        double* t = s->x[d]; s->x[d] = s->tx[d]; s->tx[d] = t;
        t = s->v[d]; s->v[d] = s->tv[d]; s->tv[d] = t;
    }
    { uint32_t* t = s->tid; s->tid = s->id; s->id = t; }
    { uint8_t* t = s->tst; s->tst = s->st; s->st = t; }

    if (s->ptable_nmd != n_md) {
        orc_ptable(s->p.bulk_rate, (double)n_md * s->p.dt, s->ptable);
        s->ptable_nmd = n_md;
    }
    double* tterm = (double*)xalloc(sizeof(double) * (ncell ? ncell : 1));
    double* erx = (double*)xalloc(sizeof(double) * (ncell ? ncell : 1));
    uint8_t* flipped = (uint8_t*)xalloc(ncell ? ncell : 1);
    const double sc = sqrt(s->p.kT / s->p.mass);
    const int64_t layer = (int64_t)s->p.L[0] * s->p.L[1];
    const int64_t top = s->p.L[2];
    uint8_t* virt = (uint8_t*)xalloc(ncell ? ncell : 1);
    /* cells in sort order: rank r holds the particles of cell c = cell_of[r];
     * per-cell random streams are keyed by the cell c */
    uint32_t nonfinite = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(|:nonfinite)
    for (int64_t r = 0; r < ncell; ++r) {
        const int64_t c = s->cell_of[r];
        int64_t b = s->start[r], e = s->start[r + 1];
        int64_t nn = e - b;
        tterm[c] = 0.0;
        /* Lamura et al. (2001): a cell cut by a wall with fewer particles
         * than a full cell (n0) is filled with n0 - n virtual particles at
         * rest on average with Maxwell-Boltzmann velocities; they enter the
         * cell's mean velocity only, through their summed momentum, a
         * normal vector of variance (n0 - n) kT / m per component. */
        const int64_t cz = c / layer;
        const int64_t n0 = s->p.wall_density;
        virt[c] = (uint8_t)(s->p.walls && (cz == 0 || cz == top) && nn >= 1 && nn < n0);
        if (nn >= 2 || virt[c]) {
            double S[3] = { 0.0, 0.0, 0.0 };
            for (int64_t j = b; j < e; ++j)
                for (int d = 0; d < 3; ++d) S[d] = S[d] + s->v[d][j];
            double u[3];
            if (virt[c]) {
                uint64_t w[4]; double z[3];
                draw(s->seed, TAG_VIRT, (uint64_t)s->coll_step, (uint64_t)c, 0, w);
                normals3(w, z);
                const double sd = sqrt((double)(n0 - nn)) * sc;
                for (int d = 0; d < 3; ++d) u[d] = (S[d] + (sd * z[d])) / (double)n0;
            } else {
                for (int d = 0; d < 3; ++d) u[d] = S[d] / (double)nn;
                double tsum = 0.0;
                for (int64_t j = b; j < e; ++j) {
                    double w0 = s->v[0][j] - u[0], w1 = s->v[1][j] - u[1], w2 = s->v[2][j] - u[2];
                    tsum = tsum + (((w0 * w0) + (w1 * w1)) + (w2 * w2));
                }
                tterm[c] = (s->p.mass * tsum) / (double)(nn - 1);
            }
            /* a non-finite cell velocity would spread through the cell */
            if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]))) nonfinite |= ORC_F_NONFINITE;
            if (s->p.rule == 0) {
                double nv[3];
                orc_marsaglia(s->seed, s->coll_step, c, nv);
                for (int64_t j = b; j < e; ++j) {
                    double w[3] = { s->v[0][j] - u[0], s->v[1][j] - u[1], s->v[2][j] - u[2] };
                    double rw[3];
                    orc_rotate(nv, s->ca, s->sa, w, rw);
                    for (int d = 0; d < 3; ++d) s->v[d][j] = u[d] + rw[d];
                }
            } else {
                /* Anderson thermostat: v_i = u + (g_i - <g>), g_i ~ N(0, kT/m) */
                double G[3] = { 0.0, 0.0, 0.0 };
                for (int64_t j = b; j < e; ++j) {
                    uint64_t w[4]; double z[3];
                    draw(s->seed, TAG_THERMO, (uint64_t)s->coll_step, s->id[j], 0, w);
                    normals3(w, z);
                    for (int d = 0; d < 3; ++d) G[d] = G[d] + (sc * z[d]);
                }
                double gm[3];
                for (int d = 0; d < 3; ++d) gm[d] = G[d] / (double)nn;
                for (int64_t j = b; j < e; ++j) {
                    uint64_t w[4]; double z[3];
                    draw(s->seed, TAG_THERMO, (uint64_t)s->coll_step, s->id[j], 0, w);
                    normals3(w, z);
                    for (int d = 0; d < 3; ++d) s->v[d][j] = u[d] + ((sc * z[d]) - gm[d]);
                }
            }
        }
        /* bulk reaction B -> A (RMPCD): at most one event per cell */
        flipped[c] = 0;
        erx[c] = 0.0;
        if (s->p.bulk_rate > 0.0 && nn > 0) {
            int64_t nB = 0;
            for (int64_t j = b; j < e; ++j) nB += (s->st[j] & 1);
            if (nB > 0) {
                uint64_t w[4];
                draw(s->seed, TAG_BULK, (uint64_t)s->coll_step, (uint64_t)c, 0, w);
                double P = s->ptable[nB < ORC_PTABLE ? nB : ORC_PTABLE - 1];
                if (u01(w[0]) < P) {
                    int64_t jb = (int64_t)(u01(w[1]) * (double)nB);
                    if (jb >= nB) jb = nB - 1;
                    for (int64_t j = b; j < e; ++j) {
                        if (s->st[j] & 1) {
                            if (jb == 0) {
                                s->st[j] = 0;
                                flipped[c] = 1;
                                erx[c] = species_dU(s, j, 1, 0);
                                break;
                            }
                            jb--;
                        }
                    }
                }
            }
        }
    }
    s->flags |= nonfinite;
    double T = 0.0;
    int64_t ncT = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        const int64_t r = s->rank_of[c];
        int64_t nn = (int64_t)s->start[r + 1] - s->start[r];
        if (nn >= 2 && !virt[c]) { T = T + tterm[c]; ncT++; }
        if (flipped[c]) { s->n_bulk++; s->e_rxn += erx[c]; }
    }
    s->temperature = ncT ? T / (3.0 * (double)ncT) : 0.0;
    s->n_cells_T = ncT;
    free(tterm); free(erx); free(flipped); free(virt);
    s->coll_step++;
}

int orc_interval(orc_system* s, int32_t n_md, int32_t do_collide)
{
    if (n_md < 1) return -1;
    orc_build_list(s, n_md);
    for (int32_t k = 0; k < n_md; ++k) md_step(s);
    if (do_collide) collide(s, n_md);
    return 0;
}

/* the collision alone (tau = n_md dt sets the bulk-reaction probability) */
int orc_collide(orc_system* s, int32_t n_md)
{
    if (n_md < 1) return -1;
    collide(s, n_md);
    return 0;
}

int orc_run(orc_system* s, int32_t n_md, int32_t n_collide)
{
    if (n_md < 1 || n_collide < 0) return -1;
    for (int32_t q = 0; q < n_collide; ++q) orc_interval(s, n_md, 1);
    return 0;
}

void orc_observables(const orc_system* s, orc_obs* o)
{
    memset(o, 0, sizeof(*o));
    double P[3] = { 0, 0, 0 }, ke = 0.0;
    int64_t nB = 0;
    for (int64_t i = 0; i < s->n; ++i) {
        double v2 = 0.0;
        for (int d = 0; d < 3; ++d) { P[d] += s->p.mass * s->v[d][i]; v2 += s->v[d][i] * s->v[d][i]; }
        ke += v2;
        nB += s->st[i] & 1;
    }
    double kec = 0.0;
    for (int c = 0; c < s->nc; ++c) {
        double v2 = 0.0;
        for (int d = 0; d < 3; ++d) { P[d] += s->p.cmass[c] * s->V[c][d]; v2 += s->V[c][d] * s->V[c][d]; }
        kec += 0.5 * s->p.cmass[c] * v2;
    }
    for (int d = 0; d < 3; ++d) o->momentum[d] = P[d];
    o->ke_solvent = 0.5 * s->p.mass * ke;
    o->ke_colloid = kec;
    o->potential = s->potential;
    o->temperature = s->temperature;
    o->e_rxn = s->e_rxn;
    o->n_B = nB;
    o->n_A = s->n - nB;
    o->n_cat_flips = s->n_cat;
    o->n_bulk_flips = s->n_bulk;
    o->md_step = s->md_step;
    o->coll_step = s->coll_step;
    o->n_candidates = s->ncand;
    o->n_cells_T = s->n_cells_T;
    o->flags = (int32_t)s->flags;
}

int64_t orc_candidates(const orc_system* s, int64_t* idx, int64_t cap)
{
    int64_t m = s->ncand < cap ? s->ncand : cap;
    if (idx) memcpy(idx, s->idx, sizeof(int64_t) * m);
    return s->ncand;
}

void orc_forces(const orc_system* s, double* f)
{
    for (int d = 0; d < 3; ++d) memcpy(f + d * s->n, s->f[d], sizeof(double) * s->n);
}

/* all-pairs forces on every solvent particle (no list), for list soundness */
void orc_forces_allpairs(orc_system* s, double* f, double* F)
{
    double Xw[ORC_MAXC][3];
    wrapped_colloids(s, Xw);
    for (int c = 0; c < s->nc; ++c) for (int d = 0; d < 3; ++d) F[3 * c + d] = 0.0;
    for (int64_t i = 0; i < s->n; ++i) {
        int sp = s->st[i] & 1;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int c = 0; c < s->nc; ++c) {
            double dx = mimg(s->x[0][i] - Xw[c][0], s->Ld[0], s->halfL[0]);
            double dy = mimg(s->x[1][i] - Xw[c][1], s->Ld[1], s->halfL[1]);
            double dz = mimg(s->x[2][i] - Xw[c][2], s->Ld[2], s->halfL[2]);
            double r2 = ((dx * dx) + (dy * dy)) + (dz * dz);
            if (r2 < s->rc2[c]) {
                double coef, pot;
                orc_wca(r2, s->p.sigma[c], sp ? s->p.epsB[c] : s->p.epsA[c], &coef, &pot);
                fx = fx + coef * dx; fy = fy + coef * dy; fz = fz + coef * dz;
                F[3 * c + 0] -= coef * dx; F[3 * c + 1] -= coef * dy; F[3 * c + 2] -= coef * dz;
            }
        }
        f[i] = fx; f[s->n + i] = fy; f[2 * s->n + i] = fz;
    }
}

int64_t orc_cell_ranks(const orc_system* s, uint32_t* rank_of, int64_t cap)
{
    int64_t m = s->ncell < cap ? s->ncell : cap;
    if (rank_of) memcpy(rank_of, s->rank_of, sizeof(uint32_t) * m);
    return s->ncell;
}

int64_t orc_last_cells(const orc_system* s, uint32_t* start, int64_t cap)
{
    int64_t m = s->ncell + 1 < cap ? s->ncell + 1 : cap;
    if (start) memcpy(start, s->start, sizeof(uint32_t) * m);
    return s->ncell + 1;
}

/* ------------------------------------------------------------------------
 * Dimer analysis ("Applications of RMPCDMD": the dimer's directed velocity,
 * the mean-squared displacement of its centre of mass and the cylindrical
 * shell histogram of the product concentration).  The paper names these
 * quantities without formulas; the definitions written out here are the
 * readings stated in the design notes:
 *   centre of mass R = (m_a X_a + m_b X_b) / (m_a + m_b) of bond (a, b),
 *   velocity V likewise, axis u = (X_b - X_a) / |X_b - X_a|, directed
 *   velocity V.u;  relative position r of a solvent particle = minimum image
 *   of x minus the image of R in the box; z = r.u, rho = |r - z u|;
 *   bins iz = floor((z + zmax) * nz / (2 zmax)), ir = floor(rho * nr / rmax),
 *   counted when 0 <= iz < nz and ir < nr, separately for A and B.
 */
static double dot3o(const double a[3], const double b[3])
{
    return ((a[0] * b[0]) + (a[1] * b[1])) + (a[2] * b[2]);
}

int orc_dimer_sample(const orc_system* s, int32_t k, double rec[10])
{
    if (k < 0 || k >= s->p.n_bonds) return -1;
    const int a = s->p.bond_a[k], b = s->p.bond_b[k];
    const double ma = s->p.cmass[a], mb = s->p.cmass[b];
    double dX[3];
    for (int d = 0; d < 3; ++d) {
        rec[d] = (ma * s->X[a][d] + mb * s->X[b][d]) / (ma + mb);
        rec[3 + d] = (ma * s->V[a][d] + mb * s->V[b][d]) / (ma + mb);
        dX[d] = s->X[b][d] - s->X[a][d];
    }
    const double len = sqrt(dot3o(dX, dX));
    for (int d = 0; d < 3; ++d) rec[6 + d] = dX[d] / len;
    rec[9] = dot3o(&rec[3], &rec[6]);
    return 0;
}

int orc_cyl_hist(const orc_system* s, int32_t k, int32_t nz, int32_t nr, double zmax, double rmax,
                 uint64_t* hist)
{
    if (k < 0 || k >= s->p.n_bonds || nz < 1 || nr < 1 || !(zmax > 0.0) || !(rmax > 0.0)) return -1;
    double rec[10];
    orc_dimer_sample(s, k, rec);
    const double* u = &rec[6];
    double Rw[3];
    for (int d = 0; d < 3; ++d) Rw[d] = wrapX(rec[d], s->Ld[d]);
    const double inv_dz = (double)nz / (2.0 * zmax), inv_dr = (double)nr / rmax;
    for (int64_t i = 0; i < s->n; ++i) {
        double r[3], p[3];
        for (int d = 0; d < 3; ++d) r[d] = mimg(s->x[d][i] - Rw[d], s->Ld[d], s->halfL[d]);
        const double z = dot3o(r, u);
        for (int d = 0; d < 3; ++d) p[d] = r[d] - z * u[d];
        const double rho = sqrt(dot3o(p, p));
        const double zs = (z + zmax) * inv_dz, rs = rho * inv_dr;
        if (!(zs >= 0.0 && zs < (double)nz && rs < (double)nr)) continue;
        const int64_t iz = (int64_t)floor(zs), ir = (int64_t)floor(rs);
        hist[((int64_t)(s->st[i] & 1) * nz + iz) * nr + ir] += 1;
    }
    return 0;
}

/* msd[lag] = average over the origins t = 0 .. T-1-lag of |R(t+lag) - R(t)|^2,
 * summed in order of t; R is [T][3]. */
void orc_msd(const double* R, int64_t T, int32_t max_lag, double* msd)
{
    for (int32_t lag = 0; lag <= max_lag; ++lag) {
        if (lag >= T) { msd[lag] = 0.0; continue; }
        double acc = 0.0;
        for (int64_t t = 0; t + lag < T; ++t) {
            double d[3];
            for (int c = 0; c < 3; ++c) d[c] = R[(t + lag) * 3 + c] - R[t * 3 + c];
            acc += dot3o(d, d);
        }
        msd[lag] = acc / (double)(T - lag);
    }
}
