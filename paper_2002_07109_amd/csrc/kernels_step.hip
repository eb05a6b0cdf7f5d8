// The integrator kernel: a group of lanes per atom adds the atom's bonded
// terms to the pair part of F_0 at q_n (from the pair kernel), then runs, for
// its own atom,
//   [close step n-1]  J(n-1, JB) and B(dt/2)        (end of B J A O A J B)
//   [open  step n  ]  B(dt/2), J(n, JA), A, O, A    (start of the next step)
// Positions of other atoms are read from the sorted mirror of q_n and the new
// positions q_{n+1} go to the other mirror buffer, so all groups may run the
// step concurrently (Sec. IV.A: at fixed q the per-atom velocity chains are
// independent).  J is the thinned jump chain of Sec. IV.B / Sec. V: one Poisson
// count with mean |C_i| beta |v_i| L dt/2, then for each proposal a uniform
// partner from C_i, an accept test U < lambda/lambda*, and a reflection.
#include "bounce_kernels.hpp"
#include "bounce_bonded.hpp"
#include "bounce_pairrow.hpp"

namespace bnc {

template <typename R>
__device__ __forceinline__ const TypePair<R> *jump_table(const StepArgs &a);
template <>
__device__ __forceinline__ const TypePair<float> *jump_table<float>(const StepArgs &a) { return a.tab_f; }
template <>
__device__ __forceinline__ const TypePair<double> *jump_table<double>(const StepArgs &a) { return a.tab_d; }

// long-range field of jump mechanism mech on i: F_ij = chi(r) W'_sf(r) d/r
// (the combined mechanism), or with separate mechanisms chi_C W'_C d/r
// (mech 0, Coulomb) or chi_V W'_V d/r (mech 1, Lennard-Jones); zero outside
// r'_mech < r < rc
template <typename R>
__device__ __forceinline__ void long_field(const TypePair<R> &tp, const PairGlobals &pg, int mech,
                                           double dx, double dy, double dz, double F[3])
{
    F[0] = F[1] = F[2] = 0.0;
    const R rx = (R)dx, ry = (R)dy, rz = (R)dz;
    const R r2 = rx * rx + ry * ry + rz * rz;
    const R rc = (R)pg.r_cut;
    if (!(r2 < rc * rc)) return;
    R r, rinv, f;
    if (pg.split) {
        R dwc, dwv;
        pair_dw_parts<R>(r2, tp, (R)pg.alpha, pg.coulomb, r, rinv, dwc, dwv);
        const R lo = mech ? (R)pg.r_on_v : (R)pg.r_on, iw = mech ? (R)pg.inv_w_v : (R)pg.inv_w;
        if (!(r > lo)) return;
        f = switch_chi<R>(r, lo, iw) * (mech ? dwv : dwc) * rinv;
    } else {
        const R dw = pair_dw<R>(r2, tp, (R)pg.alpha, pg.coulomb, r, rinv);
        if (!(r > (R)pg.r_on)) return;
        f = switch_chi<R>(r, (R)pg.r_on, (R)pg.inv_w) * dw * rinv;
    }
    F[0] = (double)(f * rx);
    F[1] = (double)(f * ry);
    F[2] = (double)(f * rz);
}

struct JumpTally {
    unsigned long long prop, acc, bound;
};

// An atom's lanes form a group of GS consecutive lanes, running the same code
// on different data; PB of them evaluate jump proposals side by side.
constexpr int PB = 4;

template <int GS>
__device__ __forceinline__ int group_base() { return (int)(threadIdx.x & 63 & ~(GS - 1)); }

template <int GS>
__device__ __forceinline__ double group_get(double v, int src)
{
    return __shfl(v, group_base<GS>() + src, 64);
}

template <int GS>
__device__ __forceinline__ uint64_t group_get_u64(uint64_t v, int src)
{
    return (uint64_t)__shfl((long long)v, group_base<GS>() + src, 64);
}

template <int GS>
__device__ __forceinline__ int32_t group_get_i32(int32_t v, int src)
{
    return __shfl(v, group_base<GS>() + src, 64);
}

// The atom's jump partners: its candidate row holds ncls groups (the
// partner's type when the rate bounds are per type pair or the mechanisms are
// separate, else one group), each in canonical order.  A proposal class b < KC
// is a (mechanism, group) pair, b = mech ncls + group, with c[b] members, each
// with the bound w[b] * unit (integer weight w[b]).
template <int KC>
struct Partners {
    const int32_t *row;     // group g at row + g * cap, in canonical order
    int32_t cap;
    int32_t ncls;           // groups in the row
    int32_t c[KC];
    uint32_t w[KC];
    uint64_t W;             // sum of the members' weights
    double unit;            // bound of one weight unit: bound_scale L_a 2^-20
};

template <int KC>
__device__ __forceinline__ void no_partners(const StepArgs &a, Partners<KC> &P)
{
    P.row = a.ls.clist;
    P.cap = a.ls.ccap;
    P.ncls = a.ls.ncls;
    P.W = 0;
    P.unit = 0.0;
#pragma unroll
    for (int b = 0; b < KC; ++b) {
        P.c[b] = 0;
        P.w[b] = 0;
    }
}

template <int KC>
__device__ __forceinline__ void load_partners(const StepArgs &a, int32_t s, int ti, Partners<KC> &P)
{
    const int32_t nc = a.ls.ncls;
    P.row = a.ls.clist + (int64_t)s * nc * a.ls.ccap;
    P.cap = a.ls.ccap;
    P.ncls = nc;
    // the type's bound unit from the whole (uniform, scalar-loaded) table, so
    // that it does not wait for a load indexed by the atom's type
    P.unit = 0.0;
#pragma unroll
    for (int b = 0; b < MAXT; ++b) {
        const double ub = a.Lunit[b];
        if (b == ti) P.unit = ub;
    }
    P.W = 0;
    const int32_t nw = a.pg.split ? 2 * nc : nc;     // proposal classes
#pragma unroll
    for (int b = 0; b < KC; ++b) {
        const bool on = b < nw;
        const int32_t grp = b >= nc ? b - nc : b;
        P.c[b] = on ? min(a.ls.ccnt[(int64_t)s * nc + grp], a.ls.ccap) : 0;
        P.w[b] = KC == 1 ? (1u << WEIGHT_BITS) : (on ? a.Lq[ti * LQW + b] : 0u);
        P.W += (uint64_t)P.c[b] * P.w[b];
    }
}

// The partner of one proposal: j with probability weight_j / W, from the first
// word of its Philox block (X uniform on [0, W), the class whose weight range
// holds X, the member within it), and that partner's bound.  With one class
// of weight 2^20 this is the uniform draw umulh(w0, c).
template <int KC>
__device__ __forceinline__ void pick_partner(const Partners<KC> &P, uint64_t w0, int32_t &slot,
                                             double &lb, int32_t &mech)
{
    mech = 0;
    if (KC == 1) {
        slot = P.row[(int32_t)__umul64hi(w0, (uint64_t)P.c[0])];
        lb = (double)(1u << WEIGHT_BITS) * P.unit;
        return;
    }
    const uint64_t X = __umul64hi(w0, P.W);
    uint64_t lo = 0;
    uint32_t wb = 1;
    int32_t off = 0;
    bool found = false;
#pragma unroll
    for (int b = 0; b < KC; ++b) {
        const uint64_t hi = lo + (uint64_t)P.c[b] * P.w[b];
        if (!found && X < hi) {
            found = true;
            wb = P.w[b];
            mech = b >= P.ncls;
            off = (b >= P.ncls ? b - P.ncls : b) * P.cap;
        }
        if (!found) lo = hi;
    }
    // X - lo < 2^53 and the quotient is below 2^20, so the FP64 quotient of
    // the two integers floors to the exact integer quotient
    const int32_t idx = (int32_t)floor((double)(X - lo) / (double)wb);
    slot = P.row[off + idx];
    lb = (double)wb * P.unit;
}

// Poisson count of proposals for one atom and J half-step: inversion of the
// CDF of Poisson(beta |v_i| dt/2 sum_j L_ij) with the uniform U (Sec. IV.B,
// Sec. V; the sum is W weight units)
__device__ __forceinline__ int32_t poisson_count(const StepArgs &a, uint64_t W, double v0,
                                                 double unit, double U, bool &capped)
{
    capped = false;
    if (W == 0 || v0 == 0.0 || unit == 0.0) return 0;
    const double mu = (double)W * a.beta * v0 * unit * a.half_dt;
    // e^-mu >= 1 - mu: a uniform below 1 - mu, less 2^-50 (more than the
    // rounding of this bound and of any faithfully rounded exp), is below the
    // first CDF term, so the inversion stops at M = 0 without evaluating exp
    if (U <= (1.0 - mu) - 0x1p-50) return 0;
    // e^-mu <= 1 - mu + mu^2/2 and e^-mu (1 + mu) >= 1 - mu^2/2 (mu >= 0): a
    // uniform above the first bound and below the second, with 2^-45 to spare
    // on each side (far more than the rounding of these bounds, of exp and of
    // the CDF's first two terms), lies between the first two CDF terms, so the
    // inversion stops at M = 1, again without evaluating exp; likewise M = 2
    // between e^-mu (1 + mu) <= 1 - mu^2/2 + mu^3/3 and
    // e^-mu (1 + mu + mu^2/2) >= 1 - mu^3/6 (each difference has a derivative
    // of one sign for mu >= 0)
    const double h = 0.5 * mu * mu, c = mu * h;      // mu^2/2, mu^3/2
    if (a.max_proposals >= 1 && U > ((1.0 - mu) + h) + 0x1p-45 && U <= (1.0 - h) - 0x1p-45) return 1;
    if (a.max_proposals >= 2 && U > ((1.0 - h) + c * (2.0 / 3.0)) + 0x1p-45 &&
        U <= (1.0 - c * (1.0 / 3.0)) - 0x1p-45)
        return 2;
    int32_t M = 0;
    double term = exp(-mu), cdf = term;
    while (U > cdf) {
        ++M;
        if (M > a.max_proposals) {
            capped = true;
            return 0;
        }
        term *= mu / (double)M;
        cdf += term;
    }
    return M;
}

// one proposal: partner and uniform from the Philox block (step, phase, lid, k)
// and the long-range field of that partner on the atom
struct Proposal {
    double F[3];
    double u;
    double lb;      // the rate bound of this partner and mechanism
    int32_t p;
    int32_t mech;   // the jump mechanism (0: Coulomb or combined, 1: Lennard-Jones)
};

// first stage: the partner and the uniform from the proposal's Philox block
template <int KC>
__device__ __forceinline__ void block_proposal(const U4 &w, const Partners<KC> &P, Proposal &o)
{
    pick_partner<KC>(P, w.x, o.p, o.lb, o.mech);
    o.u = u01(w.y);
}

template <int KC>
__device__ __forceinline__ void draw_proposal(const Partners<KC> &P, const RepInfo &ri,
                                              int64_t step, int32_t phase, int32_t lid, int32_t k,
                                              Proposal &o)
{
    block_proposal<KC>(draw(ri, step, phase, lid, (uint64_t)k), P, o);
}

// second stage: the partner's long-range field on the atom
template <typename R>
__device__ __forceinline__ void field_proposal(const StepArgs &a, const TypePair<R> *tab,
                                               const double4 *X, const RepInfo &ri, int ti,
                                               const double q[3], Proposal &o)
{
    const double4 xj = X[o.p];
    double dx = q[0] - xj.x, dy = q[1] - xj.y, dz = q[2] - xj.z;
    BoxReg(ri).apply(dx, dy, dz);
    long_field<R>(tab[ti * a.pg.n_types + mirror_type(xj.w)], a.pg, o.mech, dx, dy, dz, o.F);
}

template <typename R, int KC>
__device__ __forceinline__ void eval_proposal(const StepArgs &a, const TypePair<R> *tab,
                                              const double4 *X, const Partners<KC> &P,
                                              const RepInfo &ri, int ti, const double q[3],
                                              int64_t step, int32_t phase, int32_t lid, int32_t k,
                                              Proposal &o)
{
    draw_proposal<KC>(P, ri, step, phase, lid, k, o);
    field_proposal<R>(a, tab, X, ri, ti, q, o);
}

// One proposal of the chain applied to v (every lane of the group runs the
// same FP64 arithmetic, so the lanes keep identical v); lane 0 keeps the tally
// and the event log.
__device__ __forceinline__ void apply_proposal(const StepArgs &a, const RepInfo &ri, int32_t lid,
                                               int32_t rep, double v[3], double v0, double L,   // L: the partner's bound
                                               int64_t step, int32_t phase, int32_t k, double Fx,
                                               double Fy, double Fz, double ut, int32_t pt,
                                               int32_t mech, int sub, JumpTally &tally)
{
    const double sdot = v[0] * Fx + v[1] * Fy + v[2] * Fz;
    // U < lambda / lambda*  <=>  U |v| L < v.F  (beta cancels)
    const int acc = (ut * v0 * L) < sdot;
    if (acc) {
        const double f2 = Fx * Fx + Fy * Fy + Fz * Fz;
        const double cf = 2.0 * sdot / f2;
        v[0] = v[0] - cf * Fx;
        v[1] = v[1] - cf * Fy;
        v[2] = v[2] - cf * Fz;
    }
    if (sub == 0) {
        if (sdot > v0 * L * (1.0 + 1e-9)) {
            tally.bound++;
            atomicOr(&a.st->status, ST_BOUND);
        }
        tally.acc += acc;
        tally.prop++;
        if (a.log_events) {
            const unsigned long long slot = atomicAdd((unsigned long long *)&a.st->n_events, 1ull);
            if ((int64_t)slot < a.event_cap) {
                Event ev;
                ev.step = step; ev.phase = phase; ev.atom = lid; ev.k = k;
                ev.partner = a.ls.perm[pt] - (int32_t)ri.atom_off;
                ev.accepted = acc; ev.replica = rep;
                ev.mech = mech; ev.pad = 0;
                a.events[slot] = ev;
            }
        }
    }
}

// The velocity chain of one atom over dt/2 at fixed positions, run by the
// atom's GS lanes together.  Positions do not move during J, so the fields of
// all proposals are independent of the chain.  Proposals 1..n_pre (n_pre =
// min(M, M_pre, NPRE), NPRE <= 2) were evaluated ahead: lane pre_lane1 holds
// proposal 1 and lane pre_lane2 proposal 2 in pre.  The others are evaluated PB at a time (lane t < PB takes
// proposal k0 + t).  Every lane then walks the proposals in order k = 1, 2, ...
// applying the accept test and reflection.  Every lane of the wavefront must
// call this (M = 0 for padding lanes).
template <typename R, int GS, int NPRE, int KC>
__device__ void jump_chain(const StepArgs &a, const TypePair<R> *tab, const double4 *X,
                           const Partners<KC> &PT, int32_t lid, int32_t rep,
                           const RepInfo &ri, int ti, const double q[3], double v[3], double v0,
                           int64_t step, int32_t phase, int32_t M, int32_t M_pre,
                           int pre_lane1, int pre_lane2, const Proposal &pre, int sub,
                           JumpTally &tally)
{
    // one class: every partner has the atom's bound, no need to pass it around
    const double L1 = (double)(1u << WEIGHT_BITS) * PT.unit;
    const int32_t n_pre = min(min(M, M_pre), NPRE);
    // (most wavefronts have no proposal at all and skip the exchange)
    if (__any(n_pre > 0)) {
#pragma unroll
        for (int t = 0; t < NPRE; ++t) {
            const int src = t == 0 ? pre_lane1 : pre_lane2;
            const double Fx = group_get<GS>(pre.F[0], src), Fy = group_get<GS>(pre.F[1], src),
                         Fz = group_get<GS>(pre.F[2], src);
            const double ut = group_get<GS>(pre.u, src);
            const double lb = KC == 1 ? L1 : group_get<GS>(pre.lb, src);
            const int32_t pt = group_get_i32<GS>(pre.p, src);
            const int32_t mc = KC == 1 ? 0 : group_get_i32<GS>(pre.mech, src);
            if (t < n_pre)
                apply_proposal(a, ri, lid, rep, v, v0, lb, step, phase, 1 + t, Fx, Fy, Fz, ut, pt, mc, sub,
                               tally);
        }
    }
    for (int32_t k0 = n_pre + 1; __any(k0 <= M); k0 += PB) {
        const int32_t k = k0 + sub;
        Proposal P;
        P.F[0] = P.F[1] = P.F[2] = 0.0;
        P.u = 1.0;
        P.lb = 1.0;
        P.p = 0;
        P.mech = 0;
        if (k <= M && sub < PB) eval_proposal<R, KC>(a, tab, X, PT, ri, ti, q, step, phase, lid, k, P);
#pragma unroll
        for (int t = 0; t < PB; ++t) {
            const double Fx = group_get<GS>(P.F[0], t), Fy = group_get<GS>(P.F[1], t),
                         Fz = group_get<GS>(P.F[2], t);
            const double ut = group_get<GS>(P.u, t);
            const double lb = KC == 1 ? L1 : group_get<GS>(P.lb, t);
            const int32_t pt = group_get_i32<GS>(P.p, t);
            const int32_t mc = KC == 1 ? 0 : group_get_i32<GS>(P.mech, t);
            if (k0 + t <= M)
                apply_proposal(a, ri, lid, rep, v, v0, lb, step, phase, k0 + t, Fx, Fy, Fz, ut, pt, mc,
                               sub, tally);
        }
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

__device__ void flush_tally(const StepArgs &a, int32_t rep, bool active, const JumpTally &t, int32_t slot)
{
    if (!__any(active && (t.prop | t.acc | t.bound))) return;     // nothing to add (uniform)
    if (a.single_rep) {
        // one replica: each wavefront owns a slot of the per-wavefront counters
        // (launches of one stream never overlap), so no atomics are needed
        const unsigned long long p = wave_sum(active ? t.prop : 0), c = wave_sum(active ? t.acc : 0),
                                 b = wave_sum(active ? t.bound : 0);
        if ((threadIdx.x & 63) == 0 && (p | c | b)) {
            unsigned long long *wc = a.wave_cnt + 3 * (int64_t)slot;
            wc[0] += p;
            wc[1] += c;
            wc[2] += b;
        }
        return;
    }
    // this wavefront's copy of the counters
    const int32_t copy = slot & (CNT_SPREAD - 1);
    const int32_t first = __shfl(rep, 0, 64);
    const bool uniform = __all(!active || rep == first);
    if (uniform) {
        unsigned long long p = wave_sum(active ? t.prop : 0), c = wave_sum(active ? t.acc : 0),
                           b = wave_sum(active ? t.bound : 0);
        if ((threadIdx.x & 63) == 0 && (p | c | b)) {
            RepCounters &rc = a.cnt[first * CNT_SPREAD + copy];
            atomicAdd(&rc.proposals, p);
            atomicAdd(&rc.accepted, c);
            if (b) atomicAdd(&rc.bound_violations, b);
        }
    } else if (active && (t.prop | t.acc | t.bound)) {
        RepCounters &rc = a.cnt[rep * CNT_SPREAD + copy];
        atomicAdd(&rc.proposals, t.prop);
        atomicAdd(&rc.accepted, t.acc);
        if (t.bound) atomicAdd(&rc.bound_violations, t.bound);
    }
}

// LPA = 4 lanes per atom.  Each lane draws one Philox block at entry (lane 0:
// the O step, lane 1: the Poisson uniform of J(n-1, JB), lane 2: that of
// J(n, JA), lane 3: proposal 1 of J(n-1, JB), used only if that count is at
// least 1); lanes 0-2 turn the O block into the three Box-Muller normals and
// the lanes share the atom's bonded terms.  Right after the Poisson counts the
// first proposals of both J half-steps are evaluated side by side: J(n-1, JB)
// (count fixed by the velocity at entry) on lanes 3 and 1, J(n, JA) (count
// estimated from the same velocity; proposals depend on positions only, and
// the chain later uses those with k <= the actual count and evaluates any
// others) on lanes 2 and 0.  Then the lanes run the atom's chain (J, kicks, J,
// drifts, O step) together and lane 0 writes the results.  The pair part of
// F_0 at q_n comes from the pair kernel.
constexpr int LPA = 4;
constexpr int JB_L1 = 3, JB_L2 = 1, JA_L1 = 2, JA_L2 = 0;

// RESPA outer half kick (Sec. V): v -= H * grad_out / m at the boundary of an
// outer step (grad_out: the mesh gradient, plus the short-range pair gradient
// when that is on the outer step), read where used (one step in respa_m is a
// boundary)
__device__ __forceinline__ void outer_kick(const StepArgs &a, int32_t s, int32_t g, double H, double *v)
{
    const double k = a.tp.acc_m[g];
    for (int c = 0; c < 3; ++c) v[c] = v[c] - H * (a.grec[3 * (int64_t)s + c] * k);
}

// The integrator for the sorted atoms s = t / LPA < s_end (lane t % LPA);
// slot: this wavefront's slot of the jump counters.
template <typename R, bool BOUNCE, int KC>
__device__ __forceinline__ void step_atoms(const StepArgs &a, int32_t t, int32_t s_end, int32_t slot)
{
    // the jump field's pair constants are read where a proposal needs them
    // (cached global loads): a copy into LDS would put a load and a barrier
    // ahead of every wavefront's work
    const TypePair<R> *__restrict__ ftab = jump_table<R>(a);
    const int64_t n = a.st->step + a.step_off;
    const int32_t par = (int32_t)(n & 1);
    const double4 *__restrict__ X = a.ls.x[par];
    double4 *__restrict__ Y = a.ls.x[par ^ 1];
    double F[3] = {0.0, 0.0, 0.0};

    const int32_t s = t / LPA, sub = t % LPA;
    const bool active = s < s_end;
    JumpTally tally = {0, 0, 0};
    int32_t rep = 0, g = 0, lid = 0;
    double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
    double v[3] = {0.0, 0.0, 0.0}, fb[3] = {0.0, 0.0, 0.0};
    double km = 0.0, c2 = 0.0, disp2 = 0.0;
    const bool far_seen = a.st->far_flag != 0u;     // read once: set at most once per list
    Partners<KC> PT;
    no_partners<KC>(a, PT);
    U4 w = {0, 0, 0, 0};
    if (active) {
        const int2 si = a.ls.sinfo[s];
        g = si.x;
        rep = si.y;
        xi = X[s];
        if (a.f0_pair) {
            F[0] = a.fpair[3 * (int64_t)s];
            F[1] = a.fpair[3 * (int64_t)s + 1];
            F[2] = a.fpair[3 * (int64_t)s + 2];
        }
        const RepInfo ri = load_rep(a.reps, a.single_rep, rep);
        lid = g - (int32_t)ri.atom_off;
        v[0] = a.vel[3 * (int64_t)g];
        v[1] = a.vel[3 * (int64_t)g + 1];
        v[2] = a.vel[3 * (int64_t)g + 2];
        km = a.half_dt * a.tp.acc_m[g];
        c2 = a.ou_c2[g];
        if (BOUNCE) load_partners<KC>(a, s, mirror_type(xi.w), PT);
        // one Philox block per lane, drawn by one call for the whole group:
        // lane 0 the O step (n, O), lane 1 the Poisson uniform of (n-1, JB),
        // lane 2 that of (n, JA), lane 3 proposal 1 of (n-1, JB)
        const int64_t dstep = (sub == 1 || sub == 3) ? n - 1 : n;
        const int32_t dphase = sub == 0 ? 1 : (sub == 2 ? 0 : 2);
        w = draw(ri, dstep, dphase, lid, sub == 3 ? 1 : 0);
    }
    const RepInfo ri = load_rep(a.reps, a.single_rep, rep);
    const int ti = mirror_type(xi.w);
    double q[3] = {xi.x, xi.y, xi.z};
    // this lane's first bonded term and its atoms' positions, loaded ahead of
    // the jump proposals so the two latency chains overlap
    int4 e0 = make_int4(-1, 0, 0, 0);
    double4 ba = make_double4(0.0, 0.0, 0.0, 0.0), bb = ba, bc = ba;
    if (active) {
        e0 = a.ls.bslot[(int64_t)s * BTMAX + sub];
        if (e0.x >= 0) {
            ba = X[e0.y];
            bb = X[e0.z];
            bc = X[(e0.x >> 28) ? e0.w : e0.y];
        }
    }
    const double U_jb = u01(group_get_u64<LPA>(w.x, 1)), U_ja = u01(group_get_u64<LPA>(w.x, 2));
    // Box-Muller on the O block (while the entry loads are in flight): lane 0 cos, lane 1 sin of (w0, w1); lane 2 cos of (w2, w3)
    const uint64_t ow0 = group_get_u64<LPA>(w.x, 0), ow1 = group_get_u64<LPA>(w.y, 0);
    const uint64_t ow2 = group_get_u64<LPA>(w.z, 0), ow3 = group_get_u64<LPA>(w.w, 0);
    double gauss;
    {
        const double ua = u01(sub >= 2 ? ow2 : ow0), ub = u01(sub >= 2 ? ow3 : ow1);
        const double rad = sqrt(-2.0 * log(ua));
        double sn, cs;
        sincos(2.0 * M_PI * ub, &sn, &cs);
        gauss = rad * (sub == 1 ? sn : cs);
    }
    const double G0 = group_get<LPA>(gauss, 0), G1 = group_get<LPA>(gauss, 1), G2 = group_get<LPA>(gauss, 2);
    int32_t M_jb = 0, M_est = 0;
    Proposal pp;     // lanes 3, 1: proposals 1, 2 of J(n-1, JB); lanes 2, 0: 1, 2 of J(n, JA)
    pp.F[0] = pp.F[1] = pp.F[2] = 0.0;
    pp.u = 1.0;
    pp.lb = 1.0;
    pp.p = 0;
    pp.mech = 0;
    bool need = false;
    if (BOUNCE) {
        // both counts at the entry velocity in one evaluation: lanes 0, 1 the
        // count of (n-1, JB), lanes 2, 3 the estimated count of (n, JA)
        const double v0 = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const bool jb_lane = sub < 2;
        bool capped = false;
        int32_t M = 0;
        if (active && (jb_lane ? a.do_close : a.do_open))
            M = poisson_count(a, PT.W, v0, PT.unit, jb_lane ? U_jb : U_ja, capped);
        M_jb = group_get_i32<LPA>(M, 1);
        M_est = group_get_i32<LPA>(M, 2);
        if (capped && sub == 1) atomicOr(&a.st->status, ST_POISSON);
        // the first two proposals of each half-step, one per lane; lane 3's
        // block was drawn at entry, the others take one call together
        need = sub == JB_L1 ? M_jb >= 1
             : sub == JB_L2 ? M_jb >= 2
             : sub == JA_L1 ? M_est >= 1 : M_est >= 2;
        U4 pw = w;
        if (need && sub != JB_L1)
            pw = draw(ri, sub == JB_L2 ? n - 1 : n, sub == JB_L2 ? 2 : 0, lid, sub == JA_L1 ? 1 : 2);
        // the partner from the candidate row; its position is read after the
        // bonded terms, which run while the row entry is in flight
        if (need) block_proposal<KC>(pw, PT, pp);
    }
    if (active && e0.x >= 0) {
        // bonded terms shared by the lanes: k = sub, sub + LPA, ...
        bonded_slot_grad_pos(s, e0, ba, bb, bc, ri, a.tp, fb);
        const int4 *brow = a.ls.bslot + (int64_t)s * BTMAX;
        for (int k = sub + LPA; k < BTMAX; k += LPA) {
            const int4 e = brow[k];
            if (e.x < 0) break;
            bonded_slot_grad(s, e, X, ri, a.tp, fb);
        }
    }
    if (BOUNCE && need) field_proposal<R>(a, ftab, X, ri, ti, q, pp);
#pragma unroll
    for (int m = 1; m < LPA; m <<= 1) {
        fb[0] += __shfl_xor(fb[0], m, LPA);
        fb[1] += __shfl_xor(fb[1], m, LPA);
        fb[2] += __shfl_xor(fb[2], m, LPA);
    }
    F[0] += fb[0];
    F[1] += fb[1];
    F[2] += fb[2];

    // the atom's chain, on every lane of the group
    if (a.do_close) {
        if (BOUNCE) {
            const double v0 = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            jump_chain<R, LPA, 2, KC>(a, ftab, X, PT, lid, rep, ri, ti, q, v, v0, n - 1, 2, M_jb,
                                      M_jb, JB_L1, JB_L2, pp, sub, tally);
        }
        v[0] = v[0] - km * F[0]; v[1] = v[1] - km * F[1]; v[2] = v[2] - km * F[2];
        if (a.rec_close != 0.0 && active) outer_kick(a, s, g, a.rec_close, v);
    }
    if (a.do_open) {
        if (a.rec_open != 0.0 && active) outer_kick(a, s, g, a.rec_open, v);
        v[0] = v[0] - km * F[0]; v[1] = v[1] - km * F[1]; v[2] = v[2] - km * F[2];
        if (BOUNCE) {
            const double v0 = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            bool capped = false;
            const int32_t M = active ? poisson_count(a, PT.W, v0, PT.unit, U_ja, capped) : 0;
            if (capped && sub == 0) atomicOr(&a.st->status, ST_POISSON);
            jump_chain<R, LPA, 2, KC>(a, ftab, X, PT, lid, rep, ri, ti, q, v, v0, n, 0, M, M_est,
                                      JA_L1, JA_L2, pp, sub, tally);
        }
    }
    if (active && sub == 0) {
        if (a.do_open) {
            for (int k = 0; k < 3; ++k) q[k] = q[k] + a.half_dt * v[k];
            v[0] = a.c1 * v[0] + c2 * G0;
            v[1] = a.c1 * v[1] + c2 * G1;
            v[2] = a.c1 * v[2] + c2 * G2;
            for (int k = 0; k < 3; ++k) q[k] = q[k] + a.half_dt * v[k];
            const double *qb = a.ls.q_build + 3 * (int64_t)g;
            const double ddx = q[0] - qb[0], ddy = q[1] - qb[1], ddz = q[2] - qb[2];
            disp2 = ddx * ddx + ddy * ddy + ddz * ddz;
            if (disp2 >= a.skin_half2) atomicOr(&a.st->status, ST_SKIN);
            a.pos[3 * (int64_t)g] = q[0];
            a.pos[3 * (int64_t)g + 1] = q[1];
            a.pos[3 * (int64_t)g + 2] = q[2];
            Y[s] = make_double4(q[0], q[1], q[2], xi.w);
            if (a.ls.xf[0]) a.ls.xf[par ^ 1][s] = fixed_pos(ri, q[0], q[1], q[2], mirror_type(xi.w));
        }
        a.vel[3 * (int64_t)g] = v[0];
        a.vel[3 * (int64_t)g + 1] = v[1];
        a.vel[3 * (int64_t)g + 2] = v[2];
        bool fin = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) && isfinite(q[0]) &&
                   isfinite(q[1]) && isfinite(q[2]);
        if (!fin) atomicOr(&a.st->status, ST_NONFINITE);
    }
    // an atom beyond the far-part gate since the build sets the flag: one atomic
    // per wavefront that has such an atom, only while the flag read at the start
    // was clear (a stale read adds atomics, it never misses one)
    const bool beyond = __ballot(disp2 >= a.far_gate2) != 0ull;
    if (!far_seen && beyond && (threadIdx.x & 63) == 0) atomicOr(&a.st->far_flag, 1u);
    if (BOUNCE) flush_tally(a, rep, active && sub == 0, tally, slot);
}

template <typename R, bool BOUNCE, int KC = 1>
__global__ void __launch_bounds__(256) k_step(StepArgs a)
{
    step_atoms<R, BOUNCE, KC>(a, blockIdx.x * blockDim.x + threadIdx.x, a.n,
                              blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// One launch per step: the F_0 pair force and the integrator of every replica.
// Workgroups take items from a queue: first every replica's pair-force items
// (PAIR_ATOMS atoms each), then the integrator items (64 atoms each).  An
// integrator item of replica r waits until the counter of r's finished pair
// items reaches r's item count; those items were all taken earlier, by
// running workgroups that wait on nothing, so the wait ends.  The workgroup
// that finds the queue empty last (all items are then done) clears the
// counters for the next launch.
template <typename R, bool BOUNCE, int KC, bool FIXED>
__global__ void __launch_bounds__(256) k_fused(StepArgs a, PairArgs p, FusedArgs f)
{
    constexpr int MODE = BOUNCE ? MODE_SHORT : MODE_FULL;
    __shared__ TypePair<R> tab[MAXT * MAXT];
    __shared__ int32_t s_item;
    const TypePair<R> *pre = jump_table<R>(a);     // the same precomputed constants
    for (int k = threadIdx.x; k < p.pg.n_types * p.pg.n_types; k += blockDim.x) tab[k] = pre[k];
    const int32_t slot = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    for (;;) {
        if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(&f.queue[0], 1u);
        __syncthreads();
        const int32_t it = s_item;
        __syncthreads();
        if (it >= f.n_items) {
            if (threadIdx.x == 0 && it == f.n_items + (int32_t)gridDim.x - 1) {
                for (int32_t r = 0; r <= f.n_reps; ++r) f.queue[r] = 0u;
            }
            return;
        }
        const int4 e = f.items[it];     // (replica, first sorted atom, end, kind)
        if (e.w == 0) {
            pair_force_atoms<R, MODE, PAIR_G, false, FIXED>(p, tab, e.y * PAIR_G + (int32_t)threadIdx.x, e.z);
            __syncthreads();
            if (threadIdx.x == 0) {
                __threadfence();
                atomicAdd(&f.queue[1 + e.x], 1u);
            }
        } else {
            if (threadIdx.x == 0) {
                const uint32_t need = (uint32_t)f.need[e.x];
                while (__hip_atomic_load(&f.queue[1 + e.x], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need)
                    __builtin_amdgcn_s_sleep(2);
            }
            __syncthreads();
            __threadfence();
            step_atoms<R, BOUNCE, KC>(a, e.y * LPA + (int32_t)threadIdx.x, e.z, slot);
        }
    }
}

// the device step counter moves once per batch of launched steps, in a kernel
// of its own: kernels of one stream see it in launch order, with no fences
__global__ void k_advance(DevState *st, int32_t count) { st->step += count; }

__global__ void k_reset_disp(DevState *st) { st->far_flag = 0u; }

void launch_reset_disp(hipStream_t sm, DevState *st)
{
    hipLaunchKernelGGL(k_reset_disp, dim3(1), dim3(1), 0, sm, st);
}

void launch_advance(hipStream_t sm, DevState *st, int32_t count)
{
    if (count > 0) hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, sm, st, count);
}

void launch_step(hipStream_t sm, const StepArgs &a)
{
    if (a.n <= 0) return;
    dim3 grid(((int64_t)a.n * LPA + 255) / 256), block(256);
    if (a.bounce) {
        // proposal classes ((mechanism, partner group) pairs) rounded up to 1, 2, 4 or 8
        const int nw = a.ls.ncls * (a.pg.split ? 2 : 1);
        const int kc = nw <= 1 ? 1 : (nw <= 2 ? 2 : (nw <= 4 ? 4 : 8));
        switch (kc * 2 + a.pair_fp64) {
            case 2: hipLaunchKernelGGL((k_step<float, true, 1>), grid, block, 0, sm, a); break;
            case 3: hipLaunchKernelGGL((k_step<double, true, 1>), grid, block, 0, sm, a); break;
            case 4: hipLaunchKernelGGL((k_step<float, true, 2>), grid, block, 0, sm, a); break;
            case 5: hipLaunchKernelGGL((k_step<double, true, 2>), grid, block, 0, sm, a); break;
            case 8: hipLaunchKernelGGL((k_step<float, true, 4>), grid, block, 0, sm, a); break;
            case 9: hipLaunchKernelGGL((k_step<double, true, 4>), grid, block, 0, sm, a); break;
            case 16: hipLaunchKernelGGL((k_step<float, true, 8>), grid, block, 0, sm, a); break;
            default: hipLaunchKernelGGL((k_step<double, true, 8>), grid, block, 0, sm, a); break;
        }
    } else {
        hipLaunchKernelGGL((k_step<float, false>), grid, block, 0, sm, a);
    }
}

void launch_fused(hipStream_t sm, const StepArgs &a, const PairArgs &p, const FusedArgs &f, int32_t grid)
{
    if (a.n <= 0 || f.n_items <= 0) return;
    const dim3 g(grid), block(256);
    const bool fx = p.ls.xf[0] != nullptr;
    if (a.bounce) {
        const int nw = a.ls.ncls * (a.pg.split ? 2 : 1);
        const int kc = nw <= 1 ? 1 : (nw <= 2 ? 2 : (nw <= 4 ? 4 : 8));
        switch (kc * 2 + a.pair_fp64) {
            case 2: if (fx) hipLaunchKernelGGL((k_fused<float, true, 1, true>), g, block, 0, sm, a, p, f);
                    else hipLaunchKernelGGL((k_fused<float, true, 1, false>), g, block, 0, sm, a, p, f); break;
            case 3: hipLaunchKernelGGL((k_fused<double, true, 1, false>), g, block, 0, sm, a, p, f); break;
            case 4: if (fx) hipLaunchKernelGGL((k_fused<float, true, 2, true>), g, block, 0, sm, a, p, f);
                    else hipLaunchKernelGGL((k_fused<float, true, 2, false>), g, block, 0, sm, a, p, f); break;
            case 5: hipLaunchKernelGGL((k_fused<double, true, 2, false>), g, block, 0, sm, a, p, f); break;
            case 8: if (fx) hipLaunchKernelGGL((k_fused<float, true, 4, true>), g, block, 0, sm, a, p, f);
                    else hipLaunchKernelGGL((k_fused<float, true, 4, false>), g, block, 0, sm, a, p, f); break;
            case 9: hipLaunchKernelGGL((k_fused<double, true, 4, false>), g, block, 0, sm, a, p, f); break;
            case 16: if (fx) hipLaunchKernelGGL((k_fused<float, true, 8, true>), g, block, 0, sm, a, p, f);
                     else hipLaunchKernelGGL((k_fused<float, true, 8, false>), g, block, 0, sm, a, p, f); break;
            default: hipLaunchKernelGGL((k_fused<double, true, 8, false>), g, block, 0, sm, a, p, f); break;
        }
    } else if (a.pair_fp64) {
        hipLaunchKernelGGL((k_fused<double, false, 1, false>), g, block, 0, sm, a, p, f);
    } else if (fx) {
        hipLaunchKernelGGL((k_fused<float, false, 1, true>), g, block, 0, sm, a, p, f);
    } else {
        hipLaunchKernelGGL((k_fused<float, false, 1, false>), g, block, 0, sm, a, p, f);
    }
}

// workgroups of one fused launch that can be resident at once (their upper bound)
int32_t fused_resident_groups(int fp64, int bounce)
{
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const void *fn = bounce ? (fp64 ? (const void *)k_fused<double, true, 1, false>
                                    : (const void *)k_fused<float, true, 1, true>)
                            : (fp64 ? (const void *)k_fused<double, false, 1, false>
                                    : (const void *)k_fused<float, false, 1, true>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0) != hipSuccess || per < 1) per = 1;
    return std::max(1, cus) * per;
}

// J half-step alone at the current positions (diagnostics and parity tests)
template <typename R, int KC>
__global__ void __launch_bounds__(256) k_jump(JumpArgs ja)
{
    const StepArgs &a = ja.s;
    const TypePair<R> *tab = jump_table<R>(a);
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t s = t / PB, sub = t % PB;
    const bool active = s < a.n;
    const int32_t par = (int32_t)((a.st->step + a.step_off) & 1);
    const double4 *X = a.ls.x[par];
    JumpTally tally = {0, 0, 0};
    int32_t rep = 0, g = 0, lid = 0, M = 0;
    double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
    double v[3] = {0.0, 0.0, 0.0}, v0 = 0.0;
    Partners<KC> PT;
    no_partners<KC>(a, PT);
    if (active) {
        const int2 si = a.ls.sinfo[s];
        g = si.x;
        rep = si.y;
        lid = g - (int32_t)a.reps[rep].atom_off;
        xi = X[s];
        v[0] = a.vel[3 * (int64_t)g];
        v[1] = a.vel[3 * (int64_t)g + 1];
        v[2] = a.vel[3 * (int64_t)g + 2];
        load_partners<KC>(a, s, mirror_type(xi.w), PT);
        v0 = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        bool capped = false;
        M = poisson_count(a, PT.W, v0, PT.unit, u01(draw(a.reps[rep], ja.step, ja.phase, lid, 0).x),
                          capped);
        if (capped && sub == 0) atomicOr(&a.st->status, ST_POISSON);
    }
    const RepInfo &ri = a.reps[rep];
    const double q[3] = {xi.x, xi.y, xi.z};
    Proposal none;
    none.F[0] = none.F[1] = none.F[2] = 0.0;
    none.u = 1.0;
    none.lb = 1.0;
    none.p = 0;
    none.mech = 0;
    jump_chain<R, PB, 1, KC>(a, tab, X, PT, lid, rep, ri, mirror_type(xi.w), q, v, v0, ja.step,
                             ja.phase, M, 0, 0, 0, none, sub, tally);
    if (active && sub == 0) {
        a.vel[3 * (int64_t)g] = v[0];
        a.vel[3 * (int64_t)g + 1] = v[1];
        a.vel[3 * (int64_t)g + 2] = v[2];
    }
    flush_tally(a, rep, active && sub == 0, tally, blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

void launch_jump(hipStream_t sm, const JumpArgs &a)
{
    if (a.s.n <= 0) return;
    dim3 grid(((int64_t)a.s.n * PB + 255) / 256), block(256);
    const int nc = a.s.ls.ncls * (a.s.pg.split ? 2 : 1);
    const int kc = nc <= 1 ? 1 : (nc <= 2 ? 2 : (nc <= 4 ? 4 : 8));
    switch (kc * 2 + a.s.pair_fp64) {
        case 2: hipLaunchKernelGGL((k_jump<float, 1>), grid, block, 0, sm, a); break;
        case 3: hipLaunchKernelGGL((k_jump<double, 1>), grid, block, 0, sm, a); break;
        case 4: hipLaunchKernelGGL((k_jump<float, 2>), grid, block, 0, sm, a); break;
        case 5: hipLaunchKernelGGL((k_jump<double, 2>), grid, block, 0, sm, a); break;
        case 8: hipLaunchKernelGGL((k_jump<float, 4>), grid, block, 0, sm, a); break;
        case 9: hipLaunchKernelGGL((k_jump<double, 4>), grid, block, 0, sm, a); break;
        case 16: hipLaunchKernelGGL((k_jump<float, 8>), grid, block, 0, sm, a); break;
        default: hipLaunchKernelGGL((k_jump<double, 8>), grid, block, 0, sm, a); break;
    }
}

}  // namespace bnc
