/*
 * bounce.h -- C ABI of the MI355X BOUNCE direct-space library.
 *
 * BOUNCE (Monmarche, Weisman, Lagardere, Piquemal, arXiv:2002.07109) samples
 * the canonical measure of a molecular system (Sec. II.A) with a Langevin
 * dynamics driven by the short-range forces F_0 (Eq. SDE-Langevin-F0) plus
 * velocity jumps that carry the bounded long-range pair forces (Sec. II.B,
 * Eq. Lambda_i, Eq. R_i), discretised by the Strang splitting
 * B J A O A J B (Sec. III.C, algorithm of Sec. IV.B).  The long-range part of
 * every direct-space pair (Coulomb + Lennard-Jones, gradient-level switch chi,
 * Sec. IV.A and Sec. V) is sampled by per-atom Poisson thinning with the rate
 * bound beta |v_i| L (Sec. IV.A, Sec. III.D).  BAOAB is the same scheme without
 * J and with the full pair force in F_0.
 *
 * Conventions
 *  - Units: Angstrom, fs, amu, kcal/mol, elementary charge.
 *  - Atom arrays are in caller order ("global" ids), row-major [N][3] float64.
 *  - Several independent systems ("replicas") may share one context; replica r
 *    owns atoms [replica_offset[r], replica_offset[r+1]) and draws from the
 *    Philox4x64-10 key (seed, r); atom ids in random counters and event logs
 *    are replica-local, so a replica's trajectory does not depend on the batch.
 *  - Device pointers are HIP device addresses (e.g. torch tensors' data_ptr());
 *    host pointers are ordinary memory.  The library never allocates device
 *    memory: the caller allocates the workspace it asks for and keeps it, the
 *    position and the velocity buffers alive until bounce_destroy or the next
 *    bounce_bind.  All device work is enqueued on the bound stream.
 *  - Every call returns a bounce_status (0 = success).  Argument errors are
 *    returned at once.  Conditions detected on the device (list capacity,
 *    Verlet-skin overrun, rate-bound violation, Poisson cap, non-finite state,
 *    atom outside a droplet grid) are latched in a device word and returned by
 *    the next bounce_sync or getter; bounce_last_error gives a message.
 *  - Not thread-safe per context; different contexts are independent.
 */
#ifndef BOUNCE_H
#define BOUNCE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BOUNCE_MAX_TYPES 8

typedef enum {
    BOUNCE_OK = 0,
    BOUNCE_E_ARG = -1,          /* invalid argument or call order            */
    BOUNCE_E_HIP = -2,          /* HIP runtime error                         */
    BOUNCE_E_CAPACITY = -3,     /* a pair-list row or cell overflowed        */
    BOUNCE_E_SKIN = -4,         /* an atom moved >= skin/2 since the build   */
    BOUNCE_E_BOUND = -5,        /* a proposal exceeded the rate bound        */
    BOUNCE_E_POISSON_CAP = -6,  /* more proposals than max_proposals         */
    BOUNCE_E_NONFINITE = -7,    /* NaN/Inf in positions or velocities        */
    BOUNCE_E_STATE = -8,        /* context not bound / system not set        */
    BOUNCE_E_GRID = -9,         /* droplet atom left its cell grid           */
    BOUNCE_E_WORKSPACE = -10    /* workspace too small                       */
} bounce_status;

enum { BOUNCE_BJAOAJB = 0, BOUNCE_BAOAB = 1 };          /* integrator          */
enum { BOUNCE_PAIR_FP32 = 0, BOUNCE_PAIR_FP64 = 1 };    /* pair arithmetic     */
enum { BOUNCE_COUL_BARE = 0, BOUNCE_COUL_EWALD = 1 };   /* 1/r or erfc(a r)/r  */
enum { BOUNCE_PH_JA = 0, BOUNCE_PH_O = 1, BOUNCE_PH_JB = 2 };  /* random-stream phases */
/* what the RESPA outer step carries (bounce_params.respa_outer) */
enum { BOUNCE_OUTER_RECIP = 0, BOUNCE_OUTER_NONBONDED = 1 };
/* gradient parts for bounce_compute_gradient (bit mask) */
enum { BOUNCE_G_BONDED = 1, BOUNCE_G_SHORT = 2, BOUNCE_G_LONG = 4, BOUNCE_G_FULL = 8,
       BOUNCE_G_RECIP = 16,     /* RECIP: smooth-PME mesh + excluded-pair correction */
       BOUNCE_G_STEP = 32 };    /* STEP: the pair part of F_0 as the integrator computes it */
/* lists for bounce_get_list */
enum { BOUNCE_LIST_FORCE = 0, BOUNCE_LIST_CAND = 1 };
/* rate bounds of the jump mechanisms (Sec. III.D thinning; Sec. V: the bound may
   depend on the types of both atoms).  ATOM: every partner of an atom of type a
   has the bound L_a = max_b L_ab (one Poisson count over all candidates, a
   uniform partner).  PAIR: a partner of type b has its own bound L_ab; the
   per-pair Poisson clocks are superposed (Sec. II.B), so one count has mean
   beta |v| dt/2 sum_j L_ab and each proposal picks j with probability
   proportional to its bound.  Both sample the same process; PAIR proposes
   fewer jumps when the bounds differ by type.  Bounds are used as integer
   multiples Lq_ab of a unit per atom type, 2^-20 bound_scale L_a, with
   Lq_ab = ceil(2^20 L_ab / L_a) (ATOM: Lq_ab = 2^20). */
enum { BOUNCE_RATE_ATOM = 0, BOUNCE_RATE_PAIR = 1 };

typedef struct {
    int32_t integrator;        /* BOUNCE_BJAOAJB or BOUNCE_BAOAB                          */
    int32_t pair_precision;    /* BOUNCE_PAIR_FP32 (FP64 accumulation) or BOUNCE_PAIR_FP64 */
    int32_t coulomb;           /* BOUNCE_COUL_BARE or BOUNCE_COUL_EWALD                    */
    int32_t periodic;          /* 1: orthorhombic boxes, minimum image; 0: droplets        */
    int32_t rebuild_interval;  /* K: lists rebuilt at q_n when n % K == 0                  */
    int32_t max_proposals;     /* Poisson cap per atom per half step                       */
    int32_t log_events;        /* 1: record every jump proposal                            */
    int32_t use_graph;         /* 1: replay captured HIP graphs of K steps in bounce_step  */
    double dt;                 /* time step delta (fs)                                     */
    double gamma;              /* friction (1/fs), velocity space, all atoms               */
    double temperature;        /* K                                                        */
    double r_on, r_off;        /* switch chi: 0 below r', 1 above r'' (Angstrom)           */
    double r_cut;              /* shifted-force cutoff rc (Angstrom)                       */
    double skin;               /* Verlet skin s (Angstrom)                                 */
    double ewald_alpha;        /* 1/Angstrom (BOUNCE_COUL_EWALD)                           */
    double bound_scale;        /* rate bound used = bound_scale * L (1 = tight)            */
    double cell_size;          /* target cell edge of the list grid (Angstrom)             */
    uint64_t seed;             /* Philox key word 0                                        */
    int64_t event_capacity;    /* events kept when log_events = 1                          */
    int32_t pair_lanes;        /* lanes per atom in the pair kernel: 4, 8, 16, 32 (0 = 8)  */
    int32_t rate_mode;         /* BOUNCE_RATE_ATOM or BOUNCE_RATE_PAIR (fixed at create)   */
    /* Reciprocal-space Ewald by smooth PME (Sec. V), one periodic box only:      */
    int32_t pme_grid[3];       /* mesh points per edge, powers of two in [8, 512]; 0 = off */
    int32_t pme_order;         /* B-spline order: 4, 5 or 6                              */
    int32_t respa_m;           /* 0: mesh force in F_0 every step (basic BOUNCE);        */
                               /* m >= 1: RESPA outer step of m dt, half kicks with the  */
                               /* outer force at every m-th step (rebuild_interval % m == 0) */
    int32_t respa_outer;       /* BOUNCE_OUTER_RECIP: the outer force is the mesh force;  */
                               /* BOUNCE_OUTER_NONBONDED: also the short-range pair force */
                               /* (Sec. V: F_out = short direct + short VdW + recip; F_0  */
                               /* keeps the bonded terms); needs respa_m >= 1, any box   */
    /* Separate jump mechanisms (Sec. V treats the long-range Coulomb and van der Waals
       forces by jumps; Sec. VI counts the VdW jumps apart).  0: one mechanism per
       directed pair carries chi W'_sf of Coulomb plus Lennard-Jones.  1: two, the
       Coulomb field chi_C qq (g'(r) - g'(rc)) d/r with chi_C on [r_on, r_off] and the
       Lennard-Jones field chi_V (LJ'(r) - LJ'(rc)) d/r with chi_V on [r_on_lj, r_off_lj],
       each with its own bound per type pair; the clocks of all (mechanism, partner)
       pairs superpose into one Poisson count and a weighted draw (as BOUNCE_RATE_PAIR),
       and F_0 keeps (1 - chi_C) W'_C + (1 - chi_V) W'_V.  Needs n_types <= 4.     */
    int32_t jump_split;
    double r_on_lj, r_off_lj;  /* the Lennard-Jones window (both 0: that of Coulomb)      */
    /* 1: each step (F_0 pair force plus the integrator of every replica) is one
       persistent launch whose workgroups take (replica, atom tile) items from a
       queue, with a per-replica counter of finished pair items in place of a
       grid-wide barrier; 8 lanes per atom in its pair part.  0: a pair-force and
       an integrator launch per step.  Both give bit-identical results.  Applies
       when the short-range pair force is in F_0 and no mesh force is (else 0). */
    int32_t persistent;
    /* The F_0 pair force's partner search (FP32 pair arithmetic only): 0 = per-atom
       rows of the force list (G lanes per atom); 4 or 8 = cluster pairs: clusters
       of 4 or 8 consecutive sorted atoms, each with a list of the clusters whose
       bounding boxes (at the build) come within the list radius, evaluated as
       tiles of one pair per lane.  The same pairs contribute; the sums differ by
       rounding order only. */
    int32_t pair_kernel;
} bounce_params;

typedef struct {
    int32_t n_replicas;
    int32_t n_atoms;                 /* total over replicas                               */
    const int64_t *replica_offset;   /* [n_replicas + 1], offset[0] = 0                   */
    const double *box;               /* [n_replicas][3] box edges (periodic) or NULL      */
    const double *grid_origin;       /* [n_replicas][3] droplet cell-grid origin or NULL  */
    const int32_t *grid_dims;        /* [n_replicas][3] droplet cell-grid dims or NULL    */
    const int32_t *type;             /* [n_atoms] in [0, n_types)                         */
    const double *mass;              /* [n_atoms] amu                                     */
    int32_t n_types;                 /* <= BOUNCE_MAX_TYPES                               */
    const double *charge, *eps, *sigma;  /* [n_types] e, kcal/mol, Angstrom; Lorentz-Berthelot mixing */
    int32_t n_bonds;   const int32_t *bonds;  const double *bond_k, *bond_r0;   /* E = k (r - r0)^2       */
    int32_t n_angles;  const int32_t *angles; const double *angle_k, *angle_t0; /* [na][3], vertex middle */
                                     /* at most 8 bonds + angles may touch one atom     */
    int32_t n_excl;    const int32_t *excl;   /* [n_excl][2] pairs with no nonbonded term        */
} bounce_system;

typedef struct {
    int64_t proposals;         /* jump proposals (pair fields evaluated by J)  */
    int64_t accepted;          /* accepted jumps (reflections)                 */
    int64_t bound_violations;  /* v.F > |v| L seen (must stay 0)               */
    int64_t rebuilds;          /* list builds                                  */
    int64_t steps;             /* completed steps                              */
} bounce_counters;

typedef struct {
    int64_t step;
    int32_t phase, atom, k, partner, accepted, replica;   /* atom/partner replica-local */
    int32_t mech;              /* jump mechanism: 0 Coulomb (or combined), 1 Lennard-Jones */
    int32_t pad;
} bounce_event;

typedef struct bounce_ctx bounce_ctx;

/* Create a context from parameters (copied).  *out receives the handle.
   The parameters are those of the process and its discretisation: the target
   measure exp(-beta H) at temperature T (Sec. II.A), the friction and step of
   the Langevin splitting (Sec. III.C), the switch window [r', r''] and cutoff
   of the force decomposition (Sec. IV.A, Sec. V), the Verlet skin and rebuild
   interval of the neighbour lists (Sec. V), and the RESPA outer step (Sec. V).
   Errors: BOUNCE_E_ARG for an inconsistent set (no context is made). */
bounce_status bounce_create(const bounce_params *params, bounce_ctx **out);
/* Release the context and its HIP graph (not the caller's buffers: the
   library allocated no device memory).  NULL is ignored. */
void bounce_destroy(bounce_ctx *ctx);
/* Replace dt, gamma, temperature and bound_scale of a bound context (other fields ignored). */
bounce_status bounce_update_params(bounce_ctx *ctx, const bounce_params *params);

/* Topology and force field of all replicas (host arrays, copied).  Computes the
   rate bounds L_ab = (1 + 1e-3) max over a 1e-4 A grid of [r', rc] of |chi W'_sf|
   (Sec. IV.A).  Must precede bounce_workspace_size.  Errors: BOUNCE_E_ARG for
   inconsistent arrays, a box too small for the list radius, a cell grid too
   large, or more than 134,217,727 atoms with FP32 pair arithmetic (the pair
   kernels address the position mirror with 32-bit byte offsets). */
bounce_status bounce_set_system(bounce_ctx *ctx, const bounce_system *sys);
/* Device workspace bytes the context needs. */
bounce_status bounce_workspace_size(const bounce_ctx *ctx, uint64_t *bytes);
/* Bind caller-owned device memory: workspace (>= bounce_workspace_size bytes),
   positions and velocities ([N][3] float64, updated in place: the state (q, p)
   of the process, Sec. II.A, with p = M v), and the HIP stream (hipStream_t,
   NULL = default).  Uploads the topology; step = 0.  Errors: BOUNCE_E_ARG,
   BOUNCE_E_STATE (no system), BOUNCE_E_WORKSPACE (too small), BOUNCE_E_HIP. */
bounce_status bounce_bind(bounce_ctx *ctx, void *workspace, uint64_t workspace_bytes,
                          double *pos_dev, double *vel_dev, void *stream);
/* Size of the static workspace of bounce_bind_static (32 MiB per device). */
#define BOUNCE_STATIC_WORKSPACE_BYTES (32ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
   capture, serving loops, harnesses that forbid hipMalloc): bind like
   bounce_bind, with the library's static workspace instead of a caller
   workspace.  The workspace is one file-scope device array of
   BOUNCE_STATIC_WORKSPACE_BYTES per device, held from the library's load on
   that device until the process ends; this call allocates nothing (its device
   address is looked up once per device, on the current device).  Systems whose
   bounce_workspace_size exceeds it are refused with BOUNCE_E_WORKSPACE.  All
   calls of one device share the one array: binding a second context to it
   takes it over (the first context's calls then return BOUNCE_E_STATE until it
   is bound again), and contexts whose calls overlap on one device race.  Every
   bind clears what must start at zero (step counter, status, counters, cell
   counts); the rest keeps the last context's contents until rewritten.  Not
   for use inside a stream capture (it uploads the topology).  Errors:
   BOUNCE_E_ARG, BOUNCE_E_STATE (no system), BOUNCE_E_WORKSPACE, BOUNCE_E_HIP. */
bounce_status bounce_bind_static(bounce_ctx *ctx, double *pos_dev, double *vel_dev, void *stream);
/* Set the step counter n (random-stream counter base); the next bounce_step
   rebuilds the lists.  Use after writing new positions or velocities. */
bounce_status bounce_set_step(bounce_ctx *ctx, int64_t step);
bounce_status bounce_get_step(const bounce_ctx *ctx, int64_t *step);
/* Enqueue n_steps full steps of the algorithm of Sec. IV.B: B J A O A J B
   (BOUNCE) or B A O A B (BAOAB), each J a thinned jump half-step (Sec. III.D),
   lists rebuilt every rebuild_interval steps (Sec. V), leaving positions and
   velocities at a step boundary.  Asynchronous: device conditions surface at
   the next bounce_sync. */
bounce_status bounce_step(bounce_ctx *ctx, int32_t n_steps);
/* Wait for the bound stream and return the first latched device condition
   (list capacity, skin overrun, rate-bound violation v.F > |v| L of the
   thinning bound of Sec. IV.A, Poisson cap, non-finite state, droplet grid). */
bounce_status bounce_sync(bounce_ctx *ctx);

/* Gradient dE/dq of the selected parts at the current positions into grad_dev
   ([N][3] float64, caller order): BONDED, SHORT = sum_j (1-chi) W'_sf d/r (r<r''),
   LONG = sum_j chi W'_sf d/r (r'<r<rc), FULL = sum_j W'_sf d/r (r<rc), RECIP =
   the smooth-PME reciprocal-space gradient plus that of the excluded pairs'
   -k_e q_i q_j erf(alpha r)/r (Sec. V; needs pme_grid, else BOUNCE_E_ARG),
   STEP = the pair part of F_0 (SHORT for BOUNCE, FULL for BAOAB, Sec. IV.A)
   computed exactly as the next bounce_step will: the integrator's own force
   list and position mirrors as the steps maintain them (rebuilt first only
   where that step would rebuild them), and its pair kernel (with FP32 pair
   arithmetic over the fixed-point position mirror).  The
   other parts use a separate list built at the current positions.
   Synchronous. */
bounce_status bounce_compute_gradient(bounce_ctx *ctx, int32_t which, double *grad_dev);
/* Energies of every replica into out_host[n_replicas][7]:
   E_bond, E_angle, E_coul, E_lj, E_pair (= coul + lj, shifted force, r < rc),
   E_kin, T_kin.  Synchronous. */
bounce_status bounce_compute_energies(bounce_ctx *ctx, double *out_host);
/* Jump counters of one replica (Sec. VI reports proposal rates per particle
   and step): proposals, accepted reflections, bound violations, rebuilds and
   steps.  Synchronous.  Errors: BOUNCE_E_ARG for a replica out of range. */
bounce_status bounce_get_counters(bounce_ctx *ctx, int32_t replica, bounce_counters *out);
/* Copy up to cap logged jump proposals (in no particular order) and their
   total count: each is one thinning proposal of Sec. III.D (step, phase,
   atom, proposal index k, partner, accept decision U < lambda/lambda*).
   Needs log_events; events beyond event_capacity are counted, not kept. */
bounce_status bounce_get_events(bounce_ctx *ctx, bounce_event *host, int64_t cap, int64_t *n_total);
/* Neighbour lists of Sec. V.  The list built last (FORCE: r < r''+s for BOUNCE, r < rc+s for BAOAB; CAND:
   candidate partners r'-s <= r < rc+s) as CSR in caller ids: row_ptr_host[N+1],
   col_host[cap], rows in the library's canonical order (ascending list-grid cell,
   then id).  Synchronous. */
bounce_status bounce_get_list(bounce_ctx *ctx, int32_t which, int64_t *row_ptr_host,
                              int32_t *col_host, int64_t cap);
/* Rate bounds (Sec. IV.A): L_ab_host[n_mech][n_types][n_types] (n_mech = 2 with
   jump_split, mechanism 0 Coulomb and 1 Lennard-Jones, else 1) and
   L_a_host[n_types] = max over mechanisms and partner types (before bound_scale). */
bounce_status bounce_rate_bounds(const bounce_ctx *ctx, double *L_ab_host, double *L_a_host);
/* The bounds the jump step uses (rate_mode, jump_split): integer weights
   Lq_host[n_types][n_mech n_types] and units unit_host[n_types] (bound_scale
   applied); the bound of a partner of type b of an atom of type a under mechanism
   m is Lq[a][m n_types + b] * unit[a].  Synchronous, host only. */
bounce_status bounce_rate_weights(const bounce_ctx *ctx, uint32_t *Lq_host, double *unit_host);
/* Apply one J half-step alone (Sec. IV.B step J) at the current positions with
   the current candidate lists, random stream (step, phase).  Synchronous. */
bounce_status bounce_jump_halfstep(bounce_ctx *ctx, int64_t step, int32_t phase);

/* Reciprocal-space Ewald parts at the current positions (needs pme_grid):
   e3_host = {E_rec (mesh), E_self = -k_e alpha/sqrt(pi) sum q^2, E_excl = -k_e
   sum over excluded pairs q_i q_j erf(alpha r)/r}.  bounce_compute_energies
   adds all three to E_coul.  Synchronous. */
bounce_status bounce_pme_energy(bounce_ctx *ctx, double *e3_host);

/* Pair-structure diagnostic (the radial distribution functions that Sec. VI
   compares between integrators) at the current positions: ordered
   non-excluded pairs (i != j) of every replica with r < r_max, counted per
   type pair and bin into counts_host[n_types][n_types][n_bins]; a pair is in
   bin k when (k dr)^2 <= r^2 < ((k+1) dr)^2, dr = r_max / n_bins, with the
   displacement minimum-imaged and squared in FP64 (the oracle's rule, so the
   counts are exact).  Needs 0 < r_max <= r_cut and n_types^2 n_bins <= 8192
   (BOUNCE_E_ARG otherwise).  Rebuilds the auxiliary list.  Synchronous. */
bounce_status bounce_rdf_counts(bounce_ctx *ctx, double r_max, int32_t n_bins,
                                uint64_t *counts_host);
/* Mean squared displacement from reference positions ref_dev ([N][3] float64,
   caller order, device memory owned by the caller) per replica and atom type:
   out_host[n_replicas][n_types] (0 where a replica has no atom of a type).
   Positions are never wrapped into the box, so this is the unwrapped MSD of
   the Einstein relation.  Synchronous. */
bounce_status bounce_msd(bounce_ctx *ctx, const double *ref_dev, double *out_host);

/* Direct-space energy E = sum_{i<j, not excluded, r<rc} W_sf,ij of replica 0's
   topology at positions pos_dev ([N][3]) with per-type parameters
   params_dev = [charge[nt], eps[nt], sigma[nt]] (device); writes the scalar to
   energy_dev.  Enqueued on the bound stream. */
bounce_status bounce_direct_energy(bounce_ctx *ctx, const double *pos_dev,
                                   const double *params_dev, double *energy_dev);
/* Backward of bounce_direct_energy: grad_pos_dev[N][3] = g dE/dq and
   grad_params_dev[3 nt] = g dE/d(charge, eps, sigma), with g = *grad_out_dev. */
bounce_status bounce_direct_energy_bwd(bounce_ctx *ctx, const double *pos_dev,
                                       const double *params_dev, const double *grad_out_dev,
                                       double *grad_pos_dev, double *grad_params_dev);

/* Kernel timing for measurement, with HIP events on the bound stream; returns
   the mean duration per launch in ms.  Synchronous.
     which = 0: the standalone F_0 pair kernel at the current positions,
     which = 2: the integrator kernel with its kicks, jumps and drifts off
                (bonded terms and random draws; velocities rewritten unchanged),
                both as reps back-to-back launches that leave the trajectory
                unchanged;
     which = 1: the list build, reps times at the current positions (positions
                and velocities stay; the following steps use these lists);
     which = 3: the integrator kernel of reps real steps (advances the
                trajectory by reps + 1 steps; only that kernel is timed);
     which = 4: the reciprocal-space mesh sum (spread, FFT, convolution, FFT
                back, gather) at the current positions, reps times; needs
                pme_grid; the trajectory is unchanged;
     which = 5: a dry step as two launches: the F_0 pair kernel, then the
                integrator with its kicks, jumps and drifts off (trajectory
                unchanged);
     which = 6: the same dry step as one fused launch (needs persistent = 1). */
bounce_status bounce_profile_kernel(bounce_ctx *ctx, int32_t which, int32_t reps, double *avg_ms);

/* Autotuner: time the F_0 pair kernel (reps launches each) with 4, 8, 16 and 32
   lanes per atom at the current positions, keep the fastest in the context and
   return it in *lanes_out; ms_out (NULL or [4]) receives the mean times.
   Synchronous; leaves the trajectory unchanged. */
bounce_status bounce_autotune(bounce_ctx *ctx, int32_t reps, int32_t *lanes_out, double *ms_out);

/* What bounce_autotune_cached chose and measured (ms; -1: not timed). */
typedef struct {
    int32_t pair_lanes;        /* lanes per atom of the F_0 pair kernel                   */
    int32_t persistent;        /* 1: one fused launch per step                            */
    double pair_ms[4];         /* the pair kernel with 4, 8, 16, 32 lanes                 */
    double step_ms[2];         /* a dry step (which = 5, 6 of bounce_profile_kernel):     */
                               /*   two launches with the chosen lanes, one fused launch  */
    int32_t from_cache;        /* 1: read from the cache file, nothing timed              */
    int32_t pad;
} bounce_tuning;

/* Autotuner over the pair kernel's lanes per atom and the launch structure
   (two launches per step, or one fused persistent launch where the schedule
   allows it: bounce_params.persistent).  The choice is kept in the context
   (bit-identical results either way) and, with cache_path non-NULL, in a cache
   file of JSON lines keyed by the device (name, architecture, compute units)
   and the system and parameters the kernels depend on: a later call with the
   same key reads the choice back and times nothing.  The file is appended to
   and never rewritten; concurrent writers are not coordinated.  Synchronous;
   leaves the trajectory unchanged.  BOUNCE_E_ARG: reps < 1, out NULL, or the
   cache file cannot be written. */
bounce_status bounce_autotune_cached(bounce_ctx *ctx, int32_t reps, const char *cache_path,
                                     bounce_tuning *out);

const char *bounce_status_string(int32_t status);
const char *bounce_last_error(const bounce_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
