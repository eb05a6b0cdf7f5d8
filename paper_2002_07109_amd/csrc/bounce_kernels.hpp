// Launch interface between the C-ABI host code and the HIP kernels.
#pragma once
#include "bounce_lists.hpp"

namespace bnc {

enum PairMode { MODE_SHORT = 0, MODE_FULL = 1, MODE_LONG = 2, MODE_ENERGY = 3, MODE_DBWD = 4 };

struct PairArgs {
    int32_t n;
    int32_t mirror_sel;           // -1: parity of step (device counter + step_off), 0/1 fixed
    int32_t step_off;
    int32_t single_rep;           // 1: one replica (its RepInfo read as reps[0])
    int32_t far_gate;             // 1: skip the rows' far parts while st->far_flag is clear
    const RepInfo *reps;
    Topo tp;
    ListSet ls;
    const DevState *st;
    const double *type_params;    // [3][n_types]: charge, eps, sigma
    const TypePair<float> *tab_f; // force modes: precomputed pair constants of type_params
    const TypePair<double> *tab_d;//   (NULL: computed in the kernel)
    PairGlobals pg;
    double *out;                  // gradient [N][3]
    int32_t out_global;           // 1: caller order, 0: sorted order
    int32_t accumulate;           // 1: out += g
    double *atom_out;             // ENERGY: per-atom energies; DBWD: [N][3*MAXT] basis sums
    int32_t pad1;
    int32_t energy_total;         // ENERGY: 1 -> atom_out[g] = coul + lj (stride 1)
    int32_t atom_stride;          // ENERGY with energy_total = 0: (coul, lj) at
    int32_t atom_col;             //   atom_out[g * atom_stride + atom_col + {0,1}]
};

struct StepArgs {
    int32_t n;
    int32_t do_close;             // finish step n-1: J(n-1, JB), B(dt/2)
    int32_t do_open;              // step n: B(dt/2), J(n, JA), A, O, A
    int32_t bounce;               // 1: jumps on
    int32_t pair_fp64;            // jump pair field precision
    int32_t log_events;
    int32_t max_proposals;
    int32_t step_off;             // step n = device counter + step_off
    int32_t single_rep;           // 1: one replica (its RepInfo read as reps[0])
    int32_t f0_pair;              // 1: F_0 includes fpair; 0: the pair force is on the outer step
    const RepInfo *reps;
    Topo tp;
    ListSet ls;
    DevState *st;
    RepCounters *cnt;
    unsigned long long *wave_cnt; // one replica: [wavefronts][3] jump counters
    Event *events;
    int64_t event_cap;
    const double *fpair;          // [N][3] sorted order, pair part of F_0
    double *pos;                  // [N][3] caller order
    double *vel;                  // [N][3] caller order
    const double *ou_c2;          // [N] O-step noise amplitude
    const double *Lunit;          // [MAXT] unit of each atom type's bound weights (bound_scale applied)
    const uint32_t *Lq;           // [MAXT][LQW] integer bound weights of the (mechanism, partner type) classes
    const TypePair<float> *tab_f; // [MAXT][MAXT] pair constants of the jump field
    const TypePair<double> *tab_d;
    PairGlobals pg;
    double dt, half_dt, c1, beta;
    double skin_half2;            // (s/2)^2
    double far_gate2;             // ((s/2 - margin)/2)^2: a displacement at or above it sets st->far_flag
    const double *grec;           // [N][3] sorted: outer-step gradient for the RESPA kicks
    double rec_close, rec_open;   // kick lengths (fs) with grec after the closing B / before the opening B
};

// one periodic box's smooth-PME mesh
struct PmeArgs {
    int32_t K[3];                 // grid points per edge (powers of two)
    int32_t order;                // B-spline order n
    double box[3], inv_box[3];
    double alpha;                 // Ewald splitting (1/A)
    const DevState *st;           // mirror parity: device step counter + step_off
    int32_t step_off;
    int32_t mirror_sel;           // -1: parity of the step, 0/1: fixed mirror
    double qscale, inv_qscale;    // fixed-point scale of the spread charges (2^k)
    int32_t ncell[3];             // the list cell grid (atoms of a cell are contiguous in
    double cw[3];                 //   sorted order) and its cell edges
    double margin;                // how far an atom may be from its cell: s/2 (skin guard)
};

// per-atom mesh data of one evaluation (sorted slots), written by its first
// kernel: floor(u) per axis, the fractions u - floor(u) with the charge, and
// the spread weights M_n(f + j) (axis 0 times q 2^k)
struct PmeAtoms {
    int4 *fl;                     // [N] (fl0, fl1, fl2, 0)
    double4 *f;                   // [N] (f0, f1, f2, q)
    double *w;                    // [3 n][N]: weight k of atom s at w[k N + s]
};

// cluster pairs for the tile form of the F_0 pair force (kernels_cluster.hip)
struct ClusterSet {
    const int4 *clu;              // [ncl] (first sorted atom, end, replica, 0)
    const int32_t *rep_first;     // [n_reps + 1] first cluster of each replica
    int4 *ctr;                    // [ncl] box centre at the build (fixed point; w = replica)
    float4 *half;                 // [ncl] box half extents (A)
    int32_t *cnt;                 // [ncl] listed j-clusters
    int32_t *list;                // [ncl][cap] j-clusters, ascending
    int32_t ncl, cap;
    int32_t cl;                   // atoms per cluster: 4 or 8
    int32_t pad;
};

// the items of a fused step launch (one launch per step for all replicas)
constexpr int PAIR_G = 8;                       // lanes per atom of its pair-force items
constexpr int PAIR_ATOMS = 256 / PAIR_G;        // atoms per pair-force item
constexpr int STEP_ATOMS = 64;                  // atoms per integrator item (4 lanes each)
struct FusedArgs {
    const int4 *items;            // [n_items]: (replica, first sorted atom, end, kind 0 pair / 1 step),
                                  //   every pair item ahead of every integrator item
    const int32_t *need;          // [n_reps] pair items of each replica
    uint32_t *queue;              // [1 + n_reps]: next item, then finished pair items per
                                  //   replica (zero between launches)
    int32_t n_items;
    int32_t n_reps;
};

struct JumpArgs {
    StepArgs s;
    int64_t step;
    int32_t phase;
};

void launch_build(hipStream_t sm, int32_t n, const double *pos, const RepInfo *reps,
                  const int32_t *cell_rep, const Topo &tp, const ListSet &ls, const BuildSpec &bs,
                  DevState *st);
void launch_pair(hipStream_t sm, int mode, int fp64, int lanes, const PairArgs &a);
void launch_bonded_grad(hipStream_t sm, int32_t n, const double *pos, const RepInfo *reps,
                        const Topo &tp, double *out);
void launch_atom_energy(hipStream_t sm, int32_t n, const double *pos, const double *vel,
                        const RepInfo *reps, const Topo &tp, double *atom5);
void launch_segment_sum(hipStream_t sm, int32_t n_seg, const int64_t *seg_off, const double *vals,
                        int32_t width, int32_t stride, int32_t col0, double *out);
void launch_step(hipStream_t sm, const StepArgs &a);
void launch_fused(hipStream_t sm, const StepArgs &a, const PairArgs &p, const FusedArgs &f, int32_t grid);
void launch_cluster_build(hipStream_t sm, const ClusterSet &cs, const ListSet &ls, const RepInfo *reps,
                          DevState *st, int32_t mirror_sel, int32_t step_off, float rl);
void launch_pair_cl(hipStream_t sm, int mode, const PairArgs &a, const ClusterSet &cs);
int32_t fused_resident_groups(int fp64, int bounce);
// device step counter += count (one thread; orders after the preceding launches)
void launch_advance(hipStream_t sm, DevState *st, int32_t count);
// st->far_flag = 0 (after a build of the main list)
void launch_reset_disp(hipStream_t sm, DevState *st);
void launch_jump(hipStream_t sm, const JumpArgs &a);
void launch_rdf(hipStream_t sm, int32_t n, const RepInfo *reps, int32_t single_rep,
                const ListSet &ls, double r_max, int32_t nbins, int32_t nt,
                unsigned long long *counts);
void launch_msd_atom(hipStream_t sm, int32_t n, const double *pos, const double *ref,
                     const int32_t *type, double *vals);
void launch_pme(hipStream_t sm, int32_t n, const ListSet &ls, const double *pos, const double *charge,
                const Topo &tp, const PmeArgs &pa, const PmeAtoms &pm, double2 *grid, const double *theta,
                double *out, int32_t out_global, int32_t accumulate, double *energy_parts);
// number of per-block energy partials launch_pme writes (energy_parts != NULL)
int64_t pme_energy_parts(const PmeArgs &pa);
void launch_pme_excl_energy(hipStream_t sm, int32_t n, const double *pos, const double *charge,
                            const Topo &tp, const PmeArgs &pa, double *atom_out);
void launch_list_to_global(hipStream_t sm, int32_t n, const ListSet &ls, int32_t which,
                           int32_t *cnt_global, int32_t *col_global, int32_t cap);
void launch_dbwd_finish(hipStream_t sm, int32_t n, int32_t n_types, const double *atom_basis,
                        const int32_t *type, const double *type_params, const double *grad_out,
                        double *grad_pos, double *grad_params, double *scratch);

}  // namespace bnc
