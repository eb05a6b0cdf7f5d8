// The integrator kernel: one thread per atom runs, for its own atom,
//   [close step n-1]  J(n-1, JB) and B(dt/2)        (end of B J A O A J B)
//   [open  step n  ]  B(dt/2), J(n, JA), A, O, A    (start of the next step)
// with F_0 = pair part (from the pair kernel) + bonded terms at q_n.
// Positions of other atoms are read from the sorted mirror of q_n and the new
// positions q_{n+1} go to the other mirror buffer, so all threads may run the
// step concurrently (Sec. IV.A: at fixed q the per-atom velocity chains are
// independent).  J is the thinned jump chain of Sec. IV.B / Sec. V: one Poisson
// count with mean |C_i| beta |v_i| L dt/2, then for each proposal a uniform
// partner from C_i, an accept test U < lambda/lambda*, and a reflection.
#include "bounce_kernels.hpp"
#include "bounce_bonded.hpp"

namespace bnc {

template <typename R>
__device__ __forceinline__ const TypePair<R> *jump_table(const StepArgs &a);
template <>
__device__ __forceinline__ const TypePair<float> *jump_table<float>(const StepArgs &a) { return a.tab_f; }
template <>
__device__ __forceinline__ const TypePair<double> *jump_table<double>(const StepArgs &a) { return a.tab_d; }

// long-range field F_ij = chi(r) W'_sf(r) d/r on i (zero outside r' < r < rc)
template <typename R>
__device__ __forceinline__ void long_field(const TypePair<R> &tp, const PairGlobals &pg, double dx,
                                           double dy, double dz, double F[3])
{
    F[0] = F[1] = F[2] = 0.0;
    const R rx = (R)dx, ry = (R)dy, rz = (R)dz;
    const R r2 = rx * rx + ry * ry + rz * rz;
    const R rc = (R)pg.r_cut;
    if (!(r2 < rc * rc)) return;
    R r, rinv;
    const R dw = pair_dw<R>(r2, tp, (R)pg.alpha, pg.coulomb, r, rinv);
    if (!(r > (R)pg.r_on)) return;
    const R f = switch_chi<R>(r, (R)pg.r_on, (R)pg.inv_w) * dw * rinv;
    F[0] = (double)(f * rx);
    F[1] = (double)(f * ry);
    F[2] = (double)(f * rz);
}

struct JumpTally {
    unsigned long long prop, acc, bound;
};

// Four lanes per atom ("group"), running the same code on different data.
constexpr int LPA = 4;

__device__ __forceinline__ int group_base() { return (int)(threadIdx.x & 63 & ~(LPA - 1)); }

__device__ __forceinline__ double group_get(double v, int src)
{
    return __shfl(v, group_base() + src, 64);
}

__device__ __forceinline__ uint64_t group_get_u64(uint64_t v, int src)
{
    return (uint64_t)__shfl((long long)v, group_base() + src, 64);
}

__device__ __forceinline__ int32_t group_get_i32(int32_t v, int src)
{
    return __shfl(v, group_base() + src, 64);
}

// The velocity chain of one atom over dt/2 at fixed positions, run by the
// atom's LPA lanes together.  Positions do not move during J, so the fields of
// all proposals are independent of the chain: lane t of the group draws and
// evaluates proposals k = k0 + t of a batch in parallel, then every lane walks
// the batch in order k = k0, k0+1, ... applying the accept test and reflection
// (same FP64 arithmetic on every lane, so the lanes keep identical v).
// U: the uniform of the atom's Poisson draw, counter (step, phase, lid, 0).
// Every lane of the wavefront must call this (active = false for padding).
template <typename R>
__device__ void jump_group(const StepArgs &a, const TypePair<R> *tab, const double4 *X, bool active,
                           int32_t s, int32_t lid, int32_t rep, const RepInfo &ri, int ti,
                           const double q[3], double v[3], int64_t step, int32_t phase, double U,
                           int sub, JumpTally &tally)
{
    int32_t M = 0, c = 0;
    double v0 = 0.0, L = 0.0;
    if (active) {
        c = min(a.ls.ccnt[s], a.ls.ccap);
        v0 = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        L = a.L_a[ti];
        if (c > 0 && v0 != 0.0 && L != 0.0) {
            const double mu = (double)c * a.beta * v0 * L * a.half_dt;
            double term = exp(-mu), cdf = term;
            while (U > cdf) {
                ++M;
                if (M > a.max_proposals) break;
                term *= mu / (double)M;
                cdf += term;
            }
            if (M > a.max_proposals) {
                if (sub == 0) atomicOr(&a.st->status, ST_POISSON);
                M = 0;
            }
        }
    }
    const int32_t *crow = a.ls.clist + (int64_t)s * a.ls.ccap;
    const int nt = a.pg.n_types;
    for (int32_t k0 = 1; __any(k0 <= M); k0 += LPA) {
        // this lane's proposal of the batch
        const int32_t k = k0 + sub;
        double F[3] = {0.0, 0.0, 0.0}, u = 1.0;
        int32_t p = 0;
        if (k <= M) {
            const U4 w = draw(ri, step, phase, lid, (uint64_t)k);
            const int32_t J = (int32_t)__umul64hi(w.x, (uint64_t)c);
            p = crow[J];
            u = u01(w.y);
            const double4 xj = X[p];
            double dx = q[0] - xj.x, dy = q[1] - xj.y, dz = q[2] - xj.z;
            BoxReg(ri).apply(dx, dy, dz);
            long_field<R>(tab[ti * nt + mirror_type(xj.w)], a.pg, dx, dy, dz, F);
        }
        // the chain, in order
#pragma unroll
        for (int t = 0; t < LPA; ++t) {
            const double Fx = group_get(F[0], t), Fy = group_get(F[1], t), Fz = group_get(F[2], t);
            const double ut = group_get(u, t);
            const int32_t pt = group_get_i32(p, t);
            if (k0 + t <= M) {
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
                        const unsigned long long slot =
                            atomicAdd((unsigned long long *)&a.st->n_events, 1ull);
                        if ((int64_t)slot < a.event_cap) {
                            Event ev;
                            ev.step = step; ev.phase = phase; ev.atom = lid; ev.k = k0 + t;
                            ev.partner = a.ls.perm[pt] - (int32_t)ri.atom_off;
                            ev.accepted = acc; ev.replica = rep;
                            a.events[slot] = ev;
                        }
                    }
                }
            }
        }
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

__device__ void flush_tally(const StepArgs &a, int32_t rep, bool active, const JumpTally &t)
{
    // this wavefront's copy of the counters
    const int32_t copy = (int32_t)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (CNT_SPREAD - 1));
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

// Each lane of an atom's group draws one Philox block (lane 0: the O step,
// lane 1: the Poisson uniform of J(n-1, JB), lane 2: that of J(n, JA)), lanes
// 0-2 turn the O block into the three Box-Muller normals and the lanes share
// the atom's bonded terms; then the group runs the atom's chain (kicks, jump
// chains, drifts, O step) together and lane 0 writes the results.
template <typename R, bool BOUNCE>
__global__ void __launch_bounds__(256) k_step(StepArgs a)
{
    const TypePair<R> *tab = jump_table<R>(a);
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t s = t / LPA, sub = t % LPA;
    const bool active = s < a.n;
    const int64_t n = a.st->step + a.step_off;
    const int32_t par = (int32_t)(n & 1);
    const double4 *__restrict__ X = a.ls.x[par];
    double4 *__restrict__ Y = a.ls.x[par ^ 1];
    JumpTally tally = {0, 0, 0};
    int32_t rep = 0, g = 0, lid = 0;
    double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
    U4 w = {0, 0, 0, 0};
    double fb[3] = {0.0, 0.0, 0.0};
    if (active) {
        g = a.ls.perm[s];
        rep = a.tp.rep_of[g];
        const RepInfo &ri = a.reps[rep];
        lid = g - (int32_t)ri.atom_off;
        xi = X[s];
        // one Philox block per lane
        const int64_t dstep = sub == 1 ? n - 1 : n;
        const int32_t dphase = sub == 0 ? 1 : (sub == 1 ? 2 : 0);
        w = draw(ri, dstep, dphase, lid, 0);
        // bonded terms shared by the lanes
        const int4 *brow = a.ls.bslot + (int64_t)s * BTMAX;
        for (int k = sub; k < BTMAX; k += LPA) {
            const int4 e = brow[k];
            if (e.x < 0) break;
            bonded_slot_grad(s, e, X, ri, a.tp, fb);
        }
    }
    // Box-Muller on the O block: lane 0 cos, lane 1 sin of (w0, w1); lane 2 cos of (w2, w3)
    const uint64_t ow0 = group_get_u64(w.x, 0), ow1 = group_get_u64(w.y, 0);
    const uint64_t ow2 = group_get_u64(w.z, 0), ow3 = group_get_u64(w.w, 0);
    double gauss;
    {
        const double ua = u01(sub >= 2 ? ow2 : ow0), ub = u01(sub >= 2 ? ow3 : ow1);
        const double rad = sqrt(-2.0 * log(ua));
        double sn, cs;
        sincos(2.0 * M_PI * ub, &sn, &cs);
        gauss = rad * (sub == 1 ? sn : cs);
    }
    const double G0 = group_get(gauss, 0), G1 = group_get(gauss, 1), G2 = group_get(gauss, 2);
    const double U_jb = u01(group_get_u64(w.x, 1)), U_ja = u01(group_get_u64(w.x, 2));
    double B0 = fb[0], B1 = fb[1], B2 = fb[2];
#pragma unroll
    for (int m = 1; m < LPA; m <<= 1) {
        B0 += __shfl_xor(B0, m, LPA);
        B1 += __shfl_xor(B1, m, LPA);
        B2 += __shfl_xor(B2, m, LPA);
    }

    // the atom's chain, on every lane of the group
    const RepInfo &ri = a.reps[rep];
    const int ti = mirror_type(xi.w);
    double q[3] = {xi.x, xi.y, xi.z};
    double F[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    double km = 0.0;
    if (active) {
        F[0] = a.fpair[3 * (int64_t)s] + B0;
        F[1] = a.fpair[3 * (int64_t)s + 1] + B1;
        F[2] = a.fpair[3 * (int64_t)s + 2] + B2;
        v[0] = a.vel[3 * (int64_t)g];
        v[1] = a.vel[3 * (int64_t)g + 1];
        v[2] = a.vel[3 * (int64_t)g + 2];
        km = a.half_dt * a.tp.acc_m[g];
    }
    if (a.do_close) {
        if (BOUNCE)
            jump_group<R>(a, tab, X, active, s, lid, rep, ri, ti, q, v, n - 1, 2, U_jb, sub, tally);
        v[0] = v[0] - km * F[0]; v[1] = v[1] - km * F[1]; v[2] = v[2] - km * F[2];
    }
    if (a.do_open) {
        v[0] = v[0] - km * F[0]; v[1] = v[1] - km * F[1]; v[2] = v[2] - km * F[2];
        if (BOUNCE)
            jump_group<R>(a, tab, X, active, s, lid, rep, ri, ti, q, v, n, 0, U_ja, sub, tally);
    }
    if (active && sub == 0) {
        if (a.do_open) {
            for (int c = 0; c < 3; ++c) q[c] = q[c] + a.half_dt * v[c];
            const double c2 = a.ou_c2[g];
            v[0] = a.c1 * v[0] + c2 * G0;
            v[1] = a.c1 * v[1] + c2 * G1;
            v[2] = a.c1 * v[2] + c2 * G2;
            for (int c = 0; c < 3; ++c) q[c] = q[c] + a.half_dt * v[c];
            const double *qb = a.ls.q_build + 3 * (int64_t)g;
            const double ddx = q[0] - qb[0], ddy = q[1] - qb[1], ddz = q[2] - qb[2];
            if (ddx * ddx + ddy * ddy + ddz * ddz >= a.skin_half2) atomicOr(&a.st->status, ST_SKIN);
            a.pos[3 * (int64_t)g] = q[0];
            a.pos[3 * (int64_t)g + 1] = q[1];
            a.pos[3 * (int64_t)g + 2] = q[2];
            Y[s] = make_double4(q[0], q[1], q[2], xi.w);
        }
        a.vel[3 * (int64_t)g] = v[0];
        a.vel[3 * (int64_t)g + 1] = v[1];
        a.vel[3 * (int64_t)g + 2] = v[2];
        bool fin = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) && isfinite(q[0]) &&
                   isfinite(q[1]) && isfinite(q[2]);
        if (!fin) atomicOr(&a.st->status, ST_NONFINITE);
    }
    if (BOUNCE) flush_tally(a, rep, active && sub == 0, tally);
}

// the device step counter moves once per batch of launched steps, in a kernel
// of its own: kernels of one stream see it in launch order, with no fences
__global__ void k_advance(DevState *st, int32_t count) { st->step += count; }

void launch_advance(hipStream_t sm, DevState *st, int32_t count)
{
    if (count > 0) hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, sm, st, count);
}

void launch_step(hipStream_t sm, const StepArgs &a)
{
    if (a.n <= 0) return;
    dim3 grid(((int64_t)a.n * LPA + 255) / 256), block(256);
    if (a.bounce) {
        if (a.pair_fp64) hipLaunchKernelGGL((k_step<double, true>), grid, block, 0, sm, a);
        else hipLaunchKernelGGL((k_step<float, true>), grid, block, 0, sm, a);
    } else {
        hipLaunchKernelGGL((k_step<float, false>), grid, block, 0, sm, a);
    }
}

// J half-step alone at the current positions (diagnostics and parity tests)
template <typename R>
__global__ void __launch_bounds__(256) k_jump(JumpArgs ja)
{
    const StepArgs &a = ja.s;
    const TypePair<R> *tab = jump_table<R>(a);
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t s = t / LPA, sub = t % LPA;
    const bool active = s < a.n;
    const int32_t par = (int32_t)((a.st->step + a.step_off) & 1);
    const double4 *X = a.ls.x[par];
    JumpTally tally = {0, 0, 0};
    int32_t rep = 0, g = 0, lid = 0;
    double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
    double v[3] = {0.0, 0.0, 0.0};
    double U = 0.0;
    if (active) {
        g = a.ls.perm[s];
        rep = a.tp.rep_of[g];
        lid = g - (int32_t)a.reps[rep].atom_off;
        xi = X[s];
        v[0] = a.vel[3 * (int64_t)g];
        v[1] = a.vel[3 * (int64_t)g + 1];
        v[2] = a.vel[3 * (int64_t)g + 2];
        U = u01(draw(a.reps[rep], ja.step, ja.phase, lid, 0).x);
    }
    const RepInfo &ri = a.reps[rep];
    const double q[3] = {xi.x, xi.y, xi.z};
    jump_group<R>(a, tab, X, active, s, lid, rep, ri, mirror_type(xi.w), q, v, ja.step, ja.phase, U,
                  sub, tally);
    if (active && sub == 0) {
        a.vel[3 * (int64_t)g] = v[0];
        a.vel[3 * (int64_t)g + 1] = v[1];
        a.vel[3 * (int64_t)g + 2] = v[2];
    }
    flush_tally(a, rep, active && sub == 0, tally);
}

void launch_jump(hipStream_t sm, const JumpArgs &a)
{
    if (a.s.n <= 0) return;
    dim3 grid(((int64_t)a.s.n * LPA + 255) / 256), block(256);
    if (a.s.pair_fp64) hipLaunchKernelGGL((k_jump<double>), grid, block, 0, sm, a);
    else hipLaunchKernelGGL((k_jump<float>), grid, block, 0, sm, a);
}

}  // namespace bnc
