// Pair kernels: the short-range pair gradient of F_0 (BOUNCE), the full pair
// gradient (BAOAB), the long-range field (diagnostics), energies, and the
// direct-space energy backward; plus bonded gradients and reductions.
//
// Layout: G = 8 lanes per atom i walk i's list row (sorted partner indices)
// with stride G; positions are gathered from the sorted FP64 mirror (double4),
// the displacement is formed and minimum-imaged in FP64 and the pair field is
// evaluated in R (float or double); each lane accumulates in FP64 and the G
// partial sums are combined by a fixed butterfly, so results are
// run-to-run deterministic.
#include "bounce_kernels.hpp"
#include "bounce_bonded.hpp"
#include "bounce_pairrow.hpp"

namespace bnc {

template <typename R>
struct DbwdConst {
    R fe_rc, dfe_rc;   // eps basis 4[(s/r)^12 - (s/r)^6] and d/dr at rc
    R fs_rc, dfs_rc;   // sigma basis 4 eps [12 s^11/r^12 - 6 s^5/r^6] and d/dr at rc
    R inv_sig;
    R pad[3];
};

// tab: per-type-pair constants in the pair-arithmetic type R; tabc and tabd:
// the cutoff constants of the energy and of the parameter-gradient bases, kept
// in FP64 so that their rounding does not bias sums over millions of pairs
template <typename R>
__device__ void init_tables(TypePair<R> *tab, TypePair<double> *tabc, DbwdConst<double> *tabd,
                            const double *tpar, const PairGlobals &pg)
{
    const int nt = pg.n_types;
    for (int k = threadIdx.x; k < nt * nt; k += blockDim.x) {
        int a = k / nt, b = k % nt;
        double qq = KE * tpar[a] * tpar[b];
        double eps = sqrt(tpar[nt + a] * tpar[nt + b]);
        double sig = 0.5 * (tpar[2 * nt + a] + tpar[2 * nt + b]);
        double rc = pg.r_cut;
        double g, dg;
        coul_g<double>(rc, 1.0 / rc, pg.alpha, pg.coulomb, g, dg);
        double sr = sig / rc, s6 = sr * sr * sr * sr * sr * sr, s12 = s6 * s6;
        double ul = 0.0, dul = 0.0;
        if (eps != 0.0) {
            ul = 4.0 * eps * (s12 - s6);
            dul = 4.0 * eps * (-12.0 * s12 + 6.0 * s6) / rc;
        }
        TypePair<R> t;
        t.qq = (R)qq; t.eps4 = (R)(4.0 * eps); t.sig2 = (R)(sig * sig);
        t.du_rc = (R)(qq * dg + dul); t.u_rc = (R)(qq * g + ul);
        t.pad[0] = (R)dul; t.pad[1] = (R)(qq * dg); t.pad[2] = (R)0;
        tab[k] = t;
        if (tabc) {
            TypePair<double> c;
            c.qq = qq * g; c.eps4 = qq * dg; c.sig2 = ul; c.du_rc = dul;
            c.u_rc = 0.0; c.pad[0] = c.pad[1] = c.pad[2] = 0.0;
            tabc[k] = c;
        }
        if (tabd) {
            DbwdConst<double> d;
            d.fe_rc = 4.0 * (s12 - s6);
            d.dfe_rc = 4.0 * (-12.0 * s12 + 6.0 * s6) / rc;
            d.inv_sig = sig > 0.0 ? 1.0 / sig : 0.0;
            d.fs_rc = sig > 0.0 ? 4.0 * eps * (12.0 * s12 - 6.0 * s6) / sig : 0.0;
            d.dfs_rc = sig > 0.0 ? 4.0 * eps * (-144.0 * s12 + 36.0 * s6) / (sig * rc) : 0.0;
            d.pad[0] = d.pad[1] = d.pad[2] = 0.0;
            tabd[k] = d;
        }
    }
}

template <typename R>
__device__ __forceinline__ const TypePair<R> *pair_table(const PairArgs &a);
template <>
__device__ __forceinline__ const TypePair<float> *pair_table<float>(const PairArgs &a) { return a.tab_f; }
template <>
__device__ __forceinline__ const TypePair<double> *pair_table<double>(const PairArgs &a) { return a.tab_d; }

// G lanes per atom (4, 8, 16 or 32; chosen by the autotuner).  ONE: a single
// replica, whose box the force modes keep in scalar registers.  FIXED: the
// force modes over the fixed-point position mirror (FP32 pair arithmetic); with
// one replica held to 64 VGPRs: eight wavefronts per SIMD hide the gathers.
template <typename R, int MODE, int G, bool ONE = false, bool FIXED = false>
__global__ void __launch_bounds__(256, FIXED && ONE ? 8 : 1) k_pair(PairArgs a)
{
    __shared__ TypePair<R> tab[MAXT * MAXT];
    __shared__ TypePair<double> tabc[MAXT * MAXT];
    __shared__ DbwdConst<double> tabd[MAXT * MAXT];
    __shared__ double gconst[2];
    const TypePair<R> *pre = pair_table<R>(a);
    if ((MODE == MODE_SHORT || MODE == MODE_FULL || MODE == MODE_LONG) && pre) {
        for (int k = threadIdx.x; k < a.pg.n_types * a.pg.n_types; k += blockDim.x) tab[k] = pre[k];
    } else {
        init_tables<R>(tab, MODE == MODE_ENERGY ? tabc : nullptr, MODE == MODE_DBWD ? tabd : nullptr,
                       a.type_params, a.pg);
    }
    if (MODE == MODE_DBWD && threadIdx.x == 0) {
        double g, dg, rc = a.pg.r_cut;
        coul_g<double>(rc, 1.0 / rc, a.pg.alpha, a.pg.coulomb, g, dg);
        gconst[0] = g;
        gconst[1] = dg;
    }
    __syncthreads();

    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (MODE == MODE_SHORT || MODE == MODE_FULL || MODE == MODE_LONG) {
        pair_force_atoms<R, MODE, G, ONE, FIXED>(a, tab, t, a.n);
        return;
    }
    const int32_t s = t / G, lig = t % G;
    const bool valid = s < a.n;
    const int nt = a.pg.n_types;
    const R alpha = (R)a.pg.alpha, r_on = (R)a.pg.r_on, inv_w = (R)a.pg.inv_w;
    const R r_cut = (R)a.pg.r_cut;
    const R lim = MODE == MODE_SHORT ? (R)a.pg.r_short : r_cut;
    const R lim2 = lim * lim;

    double ax = 0.0, ay = 0.0, az = 0.0, ec = 0.0, el = 0.0;
    double bas[3 * MAXT];
    if (MODE == MODE_DBWD) {
#pragma unroll
        for (int k = 0; k < 3 * MAXT; ++k) bas[k] = 0.0;
    }
    int32_t gi = 0;
    if (valid) {
        const int32_t par = a.mirror_sel >= 0 ? a.mirror_sel : (int32_t)((a.st->step + a.step_off) & 1);
        const double4 *__restrict__ X = a.ls.x[par];
        const double4 xi = X[s];
        const int ti = mirror_type(xi.w);
        const int2 si = a.ls.sinfo[s];
        gi = si.x;
        const BoxReg box(ONE ? a.reps[0] : load_rep(a.reps, a.single_rep, si.y));
        const int32_t *row = a.ls.flist + (int64_t)s * a.ls.fcap;
        const int32_t cap = a.ls.fcap;
        const int2 fc = a.ls.fcnt[s];   // the list build keeps fc.x + fc.y <= cap
        // a far partner was at least lim + s/2 away at the build; while every
        // atom has moved less than (s/2)/2 since (the flag clear), none is within lim
        const bool near_only = a.far_gate && a.st->far_flag == 0u;
        const int32_t nn = fc.x, cnt = near_only ? fc.x : fc.x + fc.y;
        const int32_t tail = cap - 1 + nn;
        {
        // energies and parameter-gradient bases: U entries per lane in flight
        constexpr int U = 4;
        for (int32_t e0 = lig; e0 < cnt; e0 += U * G) {
            int32_t pj[U];
            double4 xj[U];
            R px = (R)0, py = (R)0, pz = (R)0;   // partial sum of this block of U pairs
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = e0 + u * G;
                pj[u] = e < cnt ? row[row_slot(e, nn, tail)] : -1;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) xj[u] = X[pj[u] >= 0 ? pj[u] : s];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // every loaded position is used (an empty slot gets r2 = lim2), so
                // the U gathers stay in flight together
                double dx = xi.x - xj[u].x, dy = xi.y - xj[u].y, dz = xi.z - xj[u].z;
                box.apply(dx, dy, dz);
                const R rx = (R)dx, ry = (R)dy, rz = (R)dz;
                const R r2 = pj[u] >= 0 ? rx * rx + ry * ry + rz * rz : lim2;
                if (!(r2 < lim2)) continue;
                const int tj = mirror_type(xj[u].w);
                const TypePair<R> &tp = tab[ti * nt + tj];
                if (MODE == MODE_ENERGY) {
                    // u(r) in R, the shifted-force terms u(rc) + (r - rc) u'(rc) in FP64
                    const R rinv = rsqrt_<R>(r2);
                    const R r = r2 * rinv;
                    R g, dg;
                    coul_g<R>(r, rinv, alpha, a.pg.coulomb, g, dg);
                    const R s2 = tp.sig2 * rinv * rinv;
                    const R s6 = s2 * s2 * s2;
                    const TypePair<double> &c = tabc[ti * nt + tj];
                    const double dr = (double)r - a.pg.r_cut;
                    ec += (double)(tp.qq * g) - (c.qq + dr * c.eps4);
                    el += (double)(tp.eps4 * (s6 * s6 - s6)) - (c.sig2 + dr * c.du_rc);
                    continue;
                }
                R r, rinv;
                R dw = pair_dw<R>(r2, tp, alpha, a.pg.coulomb, r, rinv);
                R f;
                if (MODE == MODE_SHORT) {
                    f = ((R)1 - switch_chi<R>(r, r_on, inv_w)) * dw * rinv;
                } else if (MODE == MODE_LONG) {
                    f = r > r_on ? switch_chi<R>(r, r_on, inv_w) * dw * rinv : (R)0;
                } else {
                    f = dw * rinv;
                }
                px += f * rx;
                py += f * ry;
                pz += f * rz;
                if (MODE == MODE_DBWD) {
                    R gg, dgg;
                    coul_g<R>(r, rinv, alpha, a.pg.coulomb, gg, dgg);
                    const DbwdConst<double> &dc = tabd[ti * nt + tj];
                    const double dr = (double)r - a.pg.r_cut;
                    const R s2 = tp.sig2 * rinv * rinv;
                    const R s6 = s2 * s2 * s2, s12 = s6 * s6;
                    const double gsf = (double)gg - (gconst[0] + dr * gconst[1]);
                    const double fe = (double)((R)4 * (s12 - s6)) - (dc.fe_rc + dr * dc.dfe_rc);
                    const double fs = (double)(tp.eps4 * ((R)12 * s12 - (R)6 * s6) * (R)dc.inv_sig) -
                                      (dc.fs_rc + dr * dc.dfs_rc);
#pragma unroll
                    for (int b = 0; b < MAXT; ++b) {
                        if (b == tj) {
                            bas[3 * b + 0] += gsf;
                            bas[3 * b + 1] += fe;
                            bas[3 * b + 2] += fs;
                        }
                    }
                }
            }
            ax += (double)px;
            ay += (double)py;
            az += (double)pz;
        }
        }
    }
    if (MODE == MODE_ENERGY) {
        ec = group_sum<G>(ec);
        el = group_sum<G>(el);
        if (valid && lig == 0) {
            if (a.energy_total) {
                a.atom_out[gi] = 0.5 * (ec + el);
            } else {
                a.atom_out[(int64_t)gi * a.atom_stride + a.atom_col] = 0.5 * ec;
                a.atom_out[(int64_t)gi * a.atom_stride + a.atom_col + 1] = 0.5 * el;
            }
        }
        return;
    }
    ax = group_sum<G>(ax);
    ay = group_sum<G>(ay);
    az = group_sum<G>(az);
    if (MODE == MODE_DBWD) {
#pragma unroll
        for (int k = 0; k < 3 * MAXT; ++k) bas[k] = group_sum<G>(bas[k]);
        if (valid && lig == 0) {
            double *o = a.atom_out + (int64_t)gi * 3 * MAXT;
            for (int k = 0; k < 3 * nt; ++k) o[k] = bas[k];
        }
    }
    if (valid && lig == 0) {
        const int64_t o = 3 * (int64_t)(a.out_global ? gi : s);
        if (a.accumulate) {
            a.out[o + 0] += ax;
            a.out[o + 1] += ay;
            a.out[o + 2] += az;
        } else {
            a.out[o + 0] = ax;
            a.out[o + 1] = ay;
            a.out[o + 2] = az;
        }
    }
}

template <typename R, int G>
static void launch_pair_g(hipStream_t sm, int mode, const PairArgs &a)
{
    dim3 grid(((int64_t)a.n * G + 255) / 256), block(256);
    if (a.ls.xf[0] && (mode == MODE_SHORT || mode == MODE_FULL)) {
        // the fixed-point mirror exists only with FP32 pair arithmetic
        if (mode == MODE_SHORT) {
            if (a.single_rep) hipLaunchKernelGGL((k_pair<float, MODE_SHORT, G, true, true>), grid, block, 0, sm, a);
            else hipLaunchKernelGGL((k_pair<float, MODE_SHORT, G, false, true>), grid, block, 0, sm, a);
        } else {
            if (a.single_rep) hipLaunchKernelGGL((k_pair<float, MODE_FULL, G, true, true>), grid, block, 0, sm, a);
            else hipLaunchKernelGGL((k_pair<float, MODE_FULL, G, false, true>), grid, block, 0, sm, a);
        }
        return;
    }
    switch (mode) {
        case MODE_SHORT:
            if (a.single_rep) hipLaunchKernelGGL((k_pair<R, MODE_SHORT, G, true>), grid, block, 0, sm, a);
            else hipLaunchKernelGGL((k_pair<R, MODE_SHORT, G>), grid, block, 0, sm, a);
            break;
        case MODE_FULL:
            if (a.single_rep) hipLaunchKernelGGL((k_pair<R, MODE_FULL, G, true>), grid, block, 0, sm, a);
            else hipLaunchKernelGGL((k_pair<R, MODE_FULL, G>), grid, block, 0, sm, a);
            break;
        case MODE_LONG:
            if (a.single_rep) hipLaunchKernelGGL((k_pair<R, MODE_LONG, G, true>), grid, block, 0, sm, a);
            else hipLaunchKernelGGL((k_pair<R, MODE_LONG, G>), grid, block, 0, sm, a);
            break;
        case MODE_ENERGY: hipLaunchKernelGGL((k_pair<R, MODE_ENERGY, G>), grid, block, 0, sm, a); break;
        case MODE_DBWD: hipLaunchKernelGGL((k_pair<R, MODE_DBWD, G>), grid, block, 0, sm, a); break;
    }
}

template <typename R>
static void launch_pair_r(hipStream_t sm, int mode, int lanes, const PairArgs &a)
{
    switch (lanes) {
        case 4: launch_pair_g<R, 4>(sm, mode, a); break;
        case 16: launch_pair_g<R, 16>(sm, mode, a); break;
        case 32: launch_pair_g<R, 32>(sm, mode, a); break;
        default: launch_pair_g<R, 8>(sm, mode, a); break;
    }
}

void launch_pair(hipStream_t sm, int mode, int fp64, int lanes, const PairArgs &a)
{
    if (a.n <= 0) return;
    if (fp64) launch_pair_r<double>(sm, mode, lanes, a);
    else launch_pair_r<float>(sm, mode, lanes, a);
}

__global__ void k_bonded_grad(int32_t n, const double *pos, const RepInfo *reps, Topo tp,
                              double *out)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    double o[3] = {0.0, 0.0, 0.0};
    bonded_grad_atom(g, CallerPos{pos}, reps[tp.rep_of[g]], tp, o);
    out[3 * (int64_t)g + 0] += o[0];
    out[3 * (int64_t)g + 1] += o[1];
    out[3 * (int64_t)g + 2] += o[2];
}

void launch_bonded_grad(hipStream_t sm, int32_t n, const double *pos, const RepInfo *reps,
                        const Topo &tp, double *out)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bonded_grad, dim3((n + 255) / 256), dim3(256), 0, sm, n, pos, reps, tp,
                       out);
}

// per-atom energies [N][5]: bond, angle (terms owned by their first atom),
// coulomb and LJ slots left untouched, kinetic
__global__ void k_atom_energy(int32_t n, const double *pos, const double *vel, const RepInfo *reps,
                              Topo tp, double *atom5)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const RepInfo &ri = reps[tp.rep_of[g]];
    double eb = 0.0, ea = 0.0;
    for (int32_t k = tp.bt_ptr[g]; k < tp.bt_ptr[g + 1]; ++k) {
        int32_t code = tp.bt[k];
        int32_t kind = code >> 28, idx = code & 0x0fffffff;
        if (kind == 0) {
            if (tp.bond_ij[2 * idx] != g) continue;
            double d[3];
            disp_of(ri, CallerPos{pos}, g, tp.bond_ij[2 * idx + 1], d);
            double x = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - tp.bond_kr[2 * idx + 1];
            eb += tp.bond_kr[2 * idx] * x * x;
        } else {
            if (tp.angle_ijk[3 * idx] != g) continue;
            double e1[3], e2[3];
            int32_t v = tp.angle_ijk[3 * idx + 1], y = tp.angle_ijk[3 * idx + 2];
            disp_of(ri, CallerPos{pos}, g, v, e1);
            disp_of(ri, CallerPos{pos}, y, v, e2);
            double cs = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) /
                        sqrt((e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]) *
                             (e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]));
            cs = fmin(1.0, fmax(-1.0, cs));
            double x = acos(cs) - tp.angle_kt[2 * idx + 1];
            ea += tp.angle_kt[2 * idx] * x * x;
        }
    }
    const double *v = vel + 3 * (int64_t)g;
    double ek = 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (tp.acc_m[g]);
    atom5[5 * (int64_t)g + 0] = eb;
    atom5[5 * (int64_t)g + 1] = ea;
    atom5[5 * (int64_t)g + 4] = ek;
}

void launch_atom_energy(hipStream_t sm, int32_t n, const double *pos, const double *vel,
                        const RepInfo *reps, const Topo &tp, double *atom5)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_atom_energy, dim3((n + 255) / 256), dim3(256), 0, sm, n, pos, vel, reps,
                       tp, atom5);
}

// out[seg][c] = sum over rows of segment seg of vals[row * stride + col0 + c],
// c < width <= 8; one 1024-thread block per segment, all columns in one pass,
// wavefront butterflies then a fixed-order sum over the wavefronts
// (deterministic)
constexpr int SEG_B = 1024, SEG_W = 8;

__global__ void __launch_bounds__(SEG_B) k_segment_sum(const int64_t *seg_off, const double *vals,
                                                      int32_t width, int32_t stride, int32_t col0,
                                                      double *out)
{
    __shared__ double red[SEG_B / 64][SEG_W];
    const int32_t seg = blockIdx.x;
    const int64_t b = seg_off[seg], e = seg_off[seg + 1];
    double acc[SEG_W];
#pragma unroll
    for (int c = 0; c < SEG_W; ++c) acc[c] = 0.0;
    for (int64_t r = b + threadIdx.x; r < e; r += SEG_B) {
        const double *row = vals + r * stride + col0;
#pragma unroll
        for (int c = 0; c < SEG_W; ++c)
            if (c < width) acc[c] += row[c];
    }
#pragma unroll
    for (int c = 0; c < SEG_W; ++c) {
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) acc[c] += __shfl_xor(acc[c], m, 64);
    }
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < SEG_W; ++c) red[threadIdx.x >> 6][c] = acc[c];
    __syncthreads();
    if ((int32_t)threadIdx.x < width) {
        double t = 0.0;
        for (int w = 0; w < SEG_B / 64; ++w) t += red[w][threadIdx.x];
        out[(int64_t)seg * width + threadIdx.x] = t;
    }
}

void launch_segment_sum(hipStream_t sm, int32_t n_seg, const int64_t *seg_off, const double *vals,
                        int32_t width, int32_t stride, int32_t col0, double *out)
{
    if (n_seg <= 0 || width > SEG_W) return;
    hipLaunchKernelGGL(k_segment_sum, dim3(n_seg), dim3(SEG_B), 0, sm, seg_off, vals, width, stride,
                       col0, out);
}

// squared displacement |q_g - ref_g|^2 of each atom into its type's column of
// vals[g][MAXT] (the other columns zero), for per-replica sums
__global__ void k_msd_atom(int32_t n, const double *__restrict__ pos, const double *__restrict__ ref,
                           const int32_t *__restrict__ type, double *__restrict__ vals)
{
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const double dx = pos[3 * (int64_t)g] - ref[3 * (int64_t)g];
    const double dy = pos[3 * (int64_t)g + 1] - ref[3 * (int64_t)g + 1];
    const double dz = pos[3 * (int64_t)g + 2] - ref[3 * (int64_t)g + 2];
    const int ty = type[g];
    double *row = vals + (int64_t)g * MAXT;
    for (int c = 0; c < MAXT; ++c) row[c] = c == ty ? dx * dx + dy * dy + dz * dz : 0.0;
}

void launch_msd_atom(hipStream_t sm, int32_t n, const double *pos, const double *ref,
                     const int32_t *type, double *vals)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_msd_atom, dim3((n + 255) / 256), dim3(256), 0, sm, n, pos, ref, type, vals);
}

// lists in caller ids, rows indexed by caller id
__global__ void k_list_to_global(int32_t n, ListSet ls, int32_t which, int32_t *cnt_global,
                                 int32_t *col_global, int32_t cap)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t g = ls.perm[s];
    int32_t *out = col_global + (int64_t)g * cap;
    if (which != 0) {
        // candidate rows: merge the classes (each ascending) into canonical order
        const int32_t *row = ls.clist + (int64_t)s * ls.ncls * ls.ccap;
        const int32_t *cnt = ls.ccnt + (int64_t)s * ls.ncls;
        int32_t head[MAXT], total = 0;
        for (int b = 0; b < ls.ncls; ++b) {
            head[b] = 0;
            total += cnt[b];
        }
        cnt_global[g] = total;
        for (int32_t k = 0; k < total && k < cap; ++k) {
            int best = -1;
            int32_t v = INT32_MAX;
            for (int b = 0; b < ls.ncls; ++b)
                if (head[b] < cnt[b] && row[b * ls.ccap + head[b]] < v) {
                    v = row[b * ls.ccap + head[b]];
                    best = b;
                }
            ++head[best];
            out[k] = ls.perm[v];
        }
        return;
    }
    // force rows: merge the near part (front, ascending) and the far part
    // (back, ascending from the last slot) back into canonical order
    const int32_t *row = ls.flist + (int64_t)s * ls.fcap;
    const int2 c = ls.fcnt[s];
    cnt_global[g] = c.x + c.y;
    int32_t a = 0, b = 0, k = 0;
    while ((a < c.x || b < c.y) && k < cap) {
        const int32_t u = a < c.x ? row[a] : INT32_MAX;
        const int32_t v = b < c.y ? row[ls.fcap - 1 - b] : INT32_MAX;
        if (u < v) { out[k++] = ls.perm[u]; ++a; }
        else { out[k++] = ls.perm[v]; ++b; }
    }
}

void launch_list_to_global(hipStream_t sm, int32_t n, const ListSet &ls, int32_t which,
                           int32_t *cnt_global, int32_t *col_global, int32_t cap)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_list_to_global, dim3((n + 127) / 128), dim3(128), 0, sm, n, ls, which,
                       cnt_global, col_global, cap);
}

// chain rule of the direct energy w.r.t. per-type parameters:
//   D_ab = sum over directed pairs (i of type a, j of type b) of each basis,
//   dE/dq_a = KE sum_b q_b D^g_ab, dE/deps_a = sum_b sqrt(eps_b/eps_a) D^e_ab / 2,
//   dE/dsig_a = sum_b D^s_ab / 2; all times the upstream gradient g.
__global__ void __launch_bounds__(256) k_dbwd_finish(int32_t n, int32_t nt, const double *atom_basis,
                                                     const int32_t *type, const double *tpar,
                                                     const double *grad_out, double *grad_pos,
                                                     double *grad_params)
{
    __shared__ double red[256];
    __shared__ double D[3 * MAXT * MAXT];
    for (int a = 0; a < nt; ++a) {
        for (int k = 0; k < 3 * nt; ++k) {
            double s = 0.0;
            for (int32_t g = threadIdx.x; g < n; g += 256)
                if (type[g] == a) s += atom_basis[(int64_t)g * 3 * MAXT + k];
            red[threadIdx.x] = s;
            __syncthreads();
            for (int32_t off = 128; off > 0; off >>= 1) {
                if ((int32_t)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                int b = k / 3, w = k % 3;
                D[(w * MAXT + a) * MAXT + b] = red[0];
            }
            __syncthreads();
        }
    }
    double go = *grad_out;
    if (threadIdx.x < nt) {
        int a = threadIdx.x;
        double gq = 0.0, ge = 0.0, gs = 0.0;
        for (int b = 0; b < nt; ++b) {
            gq += KE * tpar[b] * D[(0 * MAXT + a) * MAXT + b];
            ge += 0.5 * sqrt(tpar[nt + b] / tpar[nt + a]) * D[(1 * MAXT + a) * MAXT + b];
            gs += 0.5 * D[(2 * MAXT + a) * MAXT + b];
        }
        grad_params[a] = go * gq;
        grad_params[nt + a] = go * ge;
        grad_params[2 * nt + a] = go * gs;
    }
    for (int64_t k = threadIdx.x; k < 3 * (int64_t)n; k += 256) grad_pos[k] *= go;
}

void launch_dbwd_finish(hipStream_t sm, int32_t n, int32_t n_types, const double *atom_basis,
                        const int32_t *type, const double *type_params, const double *grad_out,
                        double *grad_pos, double *grad_params, double *)
{
    hipLaunchKernelGGL(k_dbwd_finish, dim3(1), dim3(256), 0, sm, n, n_types, atom_basis, type,
                       type_params, grad_out, grad_pos, grad_params);
}

}  // namespace bnc
