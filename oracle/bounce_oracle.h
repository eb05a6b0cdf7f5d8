/*
 * bounce_oracle.h -- plain FP64 CPU oracle of the BOUNCE velocity-jump process.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the reference the GPU path is
 * checked against; it is called by the test-suite, by the entry module's smoke
 * check and by the benchmark's CPU-baseline leg, and by nothing else.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Everything is written for clarity, not speed: brute-force pair searches,
 * double precision throughout, one obvious loop per formula.  Each function
 * names the passage of Monmarche, Weisman, Lagardere & Piquemal,
 * "Velocity jump processes: an alternative to multi-timestep methods for faster
 * and accurate molecular dynamics simulations" (arXiv:2002.07109) it follows.
 *
 * Units: Angstrom, fs, amu, kcal/mol, e.  "Gradient" means nabla E (the paper's
 * F_i are gradients, so the force is minus what is returned here).
 */
#ifndef BOUNCE_ORACLE_H
#define BOUNCE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXT 8
#define ORC_MAX_PME_ORDER 8

/* physical constants (proposed readings: the paper does not state units) */
#define ORC_KE 332.0637          /* Coulomb constant, kcal A / (mol e^2) */
#define ORC_KB 0.0019872041      /* Boltzmann constant, kcal / (mol K)   */
#define ORC_ACC 4.184e-4         /* (kcal/mol/A)/amu -> A/fs^2            */

enum { ORC_BOUNCE = 0, ORC_BAOAB = 1 };
enum { ORC_COUL_BARE = 0, ORC_COUL_EWALD = 1 };
/* random-stream phases (counter word 1 = phase << 32 | atom) */
enum { ORC_PH_JA = 0, ORC_PH_O = 1, ORC_PH_JB = 2 };
/* gradient components */
enum { ORC_G_BONDED = 1, ORC_G_SHORT = 2, ORC_G_LONG = 4, ORC_G_FULL = 8, ORC_G_RECIP = 16 };
/* rate bounds of the jump mechanisms (Sec. III.D thinning; Sec. V: the bound may
   depend on the types of both atoms).  ATOM: every partner of an atom of type a
   gets the bound L_a = max_b L_ab, one Poisson count over all candidates.
   PAIR: partner j of type b gets the bound L_ab; the per-pair Poisson clocks
   are superposed (Sec. II.B), so the count has mean beta |v| dt/2 sum_j L_ab
   and each proposal picks j with probability proportional to its bound. */
enum { ORC_RATE_ATOM = 0, ORC_RATE_PAIR = 1 };
/* bounds are used as integer multiples of a unit per atom type: L_ab is
   rounded up to Lq_ab / 2^20 of L_a (less a slack of 1e-4 of a unit), which
   keeps it a bound and makes the weighted partner draw exact integer
   arithmetic */
#define ORC_WEIGHT_BITS 20
#define ORC_WEIGHT_SLACK 1e-4
/* status codes (same meaning as the GPU library's) */
enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_SKIN = -4, ORC_E_BOUND = -5,
       ORC_E_POISSON_CAP = -6, ORC_E_NONFINITE = -7, ORC_E_GRID = -9 };

typedef struct {
    int32_t integrator;        /* ORC_BOUNCE (B J A O A J B) or ORC_BAOAB           */
    int32_t coulomb;           /* ORC_COUL_BARE (1/r) or ORC_COUL_EWALD (erfc(a r)/r) */
    int32_t periodic;          /* 1: orthorhombic box, minimum image                */
    int32_t n_types;
    int32_t rebuild_interval;  /* lists rebuilt at q_n when n % K == 0              */
    int32_t max_proposals;     /* Poisson cap per atom per half step                */
    double dt, gamma, temperature;          /* fs, 1/fs, K                          */
    double r_on, r_off, r_cut, skin;        /* r', r'', cutoff, Verlet skin (A)     */
    double ewald_alpha;                     /* 1/A                                  */
    double bound_scale;                     /* rate bound used = bound_scale * L    */
    double box[3];
    double cell_size;                       /* canonical-order cell grid            */
    double grid_origin[3];                  /* droplet grid                         */
    int32_t grid_dims[3];
    int32_t rate_mode;                      /* ORC_RATE_ATOM or ORC_RATE_PAIR       */
    uint64_t seed, replica;                 /* Philox key                           */
    double charge[ORC_MAXT], eps[ORC_MAXT], sigma[ORC_MAXT];
    /* reciprocal-space Ewald (Sec. V: SPME) for periodic boxes: grid points
       per edge (pme_grid[0] = 0: no reciprocal part), B-spline order, and the
       schedule: respa_m = 0 adds the reciprocal force to F_0 every step (the
       basic algorithm), respa_m >= 1 applies it as half kicks of m dt around
       every m steps (the RESPA outer step).  respa_outer = ORC_OUTER_NONBONDED
       (with respa_m >= 1) also moves the short-range pair force out of F_0
       onto the outer step (Sec. V: F_out = short direct + short VdW + recip;
       bonded terms stay inner), with or without the mesh */
    int32_t pme_grid[3];
    int32_t pme_order;
    int32_t respa_m;
    int32_t respa_outer;
    /* jump_split = 1: the long-range part of every pair is carried by two jump
       mechanisms of its own (Sec. V treats the Coulomb and the van der Waals
       long-range forces as jumps, and Sec. VI reports the VdW jumps apart):
       Coulomb (mechanism 0) with the switch on [r_on, r_off], Lennard-Jones
       (mechanism 1) with its own switch on [r_on_lj, r_off_lj]; each has its own
       bound per pair of types, L_C(a,b) and L_V(a,b), and the per-(mechanism,
       partner type) clocks are superposed as with ORC_RATE_PAIR */
    int32_t jump_split;
    double r_on_lj, r_off_lj;
} orc_params;

enum { ORC_OUTER_RECIP = 0, ORC_OUTER_NONBONDED = 1 };

typedef struct {
    int32_t n_atoms;
    int32_t n_bonds, n_angles, n_excl;
    const int32_t *type;       /* [n]       */
    const double *mass;        /* [n]       */
    const int32_t *bonds;      /* [nb][2]   */
    const double *bond_k, *bond_r0;
    const int32_t *angles;     /* [na][3], vertex in the middle */
    const double *angle_k, *angle_t0;
    const int32_t *excl;       /* [ne][2] excluded nonbonded pairs */
} orc_topology;

typedef struct {
    int64_t proposals, accepted, bound_violations, rebuilds, pair_evals, steps;
    double list_seconds;       /* wall time spent building lists (timing only) */
} orc_counters;

/* one jump proposal; margin = U |v_i| L - v_i.F (accepted iff margin < 0) and
   scale = |v_i| |F| (how far rounding of F can move v_i.F) let a test tell a
   near-tie of the accept test from a real disagreement */
typedef struct {
    int64_t step;
    int32_t phase, atom, k, partner, accepted;
    int32_t mech;      /* jump mechanism: 0 (Coulomb, or the combined one), 1 (Lennard-Jones) */
    double margin, scale;
} orc_event;

/* Philox4x64-10 block (Salmon et al., SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double orc_u01(uint64_t w);
uint64_t orc_umulh(uint64_t a, uint64_t b);

/* pair potential u, shifted-force W_sf and switch chi */
void orc_pair_u(const orc_params *p, int a, int b, double r, double *u, double *du);
void orc_pair_wsf(const orc_params *p, int a, int b, double r, double *w, double *dw);
double orc_chi(const orc_params *p, double r);
/* the Coulomb and Lennard-Jones parts of W'_sf (their sum is orc_pair_wsf's dw) */
void orc_pair_dw_parts(const orc_params *p, int a, int b, double r, double *dwc, double *dwv);
/* switch of mechanism m (0: Coulomb or combined, 1: Lennard-Jones with jump_split) */
double orc_chi_mech(const orc_params *p, int m, double r);
/* number of jump mechanisms per pair: 2 with jump_split, else 1 */
int orc_n_mech(const orc_params *p);
/* L[m][a][b] >= sup |chi_m W'_m| per mechanism and type pair (n_mech x n_types x
   n_types; the combined mechanism: chi W'_sf) and L_a = max over m, b */
void orc_rate_bounds(const orc_params *p, double *L_ab, double *L_a);
/* integer bound weights Lq[a][m n_types + b] = ceil(2^20 L[m][a][b] / L_a - 1e-4)
   (n_types x n_mech n_types) and the unit of each row, bound_scale L_a 2^-20:
   the bound of a partner of type b under mechanism m is Lq * unit_a
   (ORC_RATE_ATOM without jump_split: Lq = 2^20 for every b) */
void orc_rate_weights(const orc_params *p, uint32_t *Lq, double *unit);
/* reflection of v on F (scalar mass) */
void orc_reflect(const double v[3], const double F[3], double out[3]);

/* canonical atom order: ascending (cell, atom id); returns ORC_E_GRID if an atom
   is outside a droplet grid.  order[k] = atom at sorted position k. */
int orc_sort_order(const orc_params *p, int32_t n, const double *q, int32_t *order, int64_t *cell);
/* per-atom lists: j != i, not excluded, rmin <= |d| < rmax (no lower bound if
   rmin <= 0), rows in canonical order.  Returns total entries or -1 if > cap. */
int64_t orc_build_list(const orc_params *p, const orc_topology *t, const double *q,
                       double rmin, double rmax, const int32_t *order,
                       int64_t *row_ptr, int32_t *col, int64_t cap);
/* one row of the same list, for sampled checks at large N */
int32_t orc_list_row(const orc_params *p, const orc_topology *t, const double *q,
                     double rmin, double rmax, const int32_t *order, int32_t i,
                     int32_t *col, int32_t cap);

/* gradient components (sum of the ORC_G_* bits in which), brute force */
void orc_gradient(const orc_params *p, const orc_topology *t, const double *q, int which, double *g);
void orc_gradient_atom(const orc_params *p, const orc_topology *t, const double *q, int which,
                       int32_t i, double g[3]);
/* E_bond, E_angle, E_coul, E_lj, E_pair, E_kin, T_kin */
void orc_energies(const orc_params *p, const orc_topology *t, const double *q, const double *v,
                  double out[7]);

/* one J half-step (velocities only) over all atoms at fixed q with given
   candidate lists; step/phase select the random stream. */
int orc_jump_halfstep(const orc_params *p, const orc_topology *t, const double *q, double *v,
                      const int64_t *row_ptr, const int32_t *col, int64_t step, int32_t phase,
                      orc_event *ev, int64_t ev_cap, int64_t *n_ev, orc_counters *cnt);

/* nsteps of BOUNCE or BAOAB from (q,v) at step0, lists built at the first step
   and whenever n % K == 0.  q, v updated in place. */
int orc_run(const orc_params *p, const orc_topology *t, double *q, double *v, int64_t step0,
            int32_t nsteps, orc_event *ev, int64_t ev_cap, int64_t *n_ev, orc_counters *cnt);

/* ordered non-excluded pairs (i != j) with r < r_max per type pair and bin:
   counts[(t_i * n_types + t_j) * nbins + k], (k dr)^2 <= r^2 < ((k+1) dr)^2,
   dr = r_max / nbins */
void orc_rdf_counts(const orc_params *p, const orc_topology *t, const double *q, double r_max,
                    int32_t nbins, int64_t *counts);

/* Reciprocal-space Ewald by smooth particle-mesh Ewald (Sec. V; Essmann et al.,
   J. Chem. Phys. 103, 8577 (1995)): energy parts e[0] = E_rec (mesh),
   e[1] = E_self = -k_e alpha/sqrt(pi) sum q^2, e[2] = E_excl = -k_e sum over
   excluded pairs q_i q_j erf(alpha r)/r, and the gradient of E_rec + E_excl
   (NULL = skip).  Charges are the per-type charges. */
void orc_pme(const orc_params *p, const orc_topology *t, const double *q, double *grad, double e[3]);
/* the same reciprocal energy and gradient by the plain Ewald sum over
   reciprocal vectors with |k_a| <= kmax per axis (E_rec only; for checks) */
double orc_ewald_recip(const orc_params *p, const orc_topology *t, const double *q, int32_t kmax,
                       double *grad);

/* direct-space energy sum_{i<j, not excluded, r<rc} W_sf and its gradients with
   respect to positions and per-type charge, epsilon, sigma (NULL = skip). */
double orc_direct_energy(const orc_params *p, const orc_topology *t, const double *q,
                         double *grad_q, double *grad_charge, double *grad_eps, double *grad_sigma);

#ifdef __cplusplus
}
#endif
#endif
