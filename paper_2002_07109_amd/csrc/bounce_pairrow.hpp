// The pair-force sum of one atom over its list row, walked by a group of G
// lanes (lane lig takes entries lig, lig + G, ...).  A row has nn entries
// from its front and cnt - nn more from its back (slot cap - 1 downwards):
// entry e sits at row_slot(e, nn, cap - 1 + nn).
//
// MODE_SHORT: (1 - chi(r)) W'_sf(r) d/r for r < r''  (F_0 pair part, Sec. IV.A)
// MODE_FULL:  W'_sf(r) d/r for r < rc                 (BAOAB)
// MODE_LONG:  chi(r) W'_sf(r) d/r for r' < r < rc     (the jump fields, summed)
//
// The displacement is formed and minimum-imaged in FP64 and rounded to R; the
// pair field is evaluated in R; each block of U entries is summed in R and
// added to FP64 accumulators.  The caller combines the G partial sums.
#pragma once
#include "bounce_kernels.hpp"

namespace bnc {

__device__ __forceinline__ int32_t row_slot(int32_t e, int32_t nn, int32_t tail)
{
    return e < nn ? e : tail - e;
}

// The pair's scalar s with gradient s d: SHORT (1 - chi) W'_sf / r, LONG
// chi W'_sf / r (r > r'), FULL W'_sf / r; with separate mechanisms (SPLIT) each of
// the Coulomb and Lennard-Jones parts with its own switch.
template <typename R, int MODE, bool SPLIT>
__device__ __forceinline__ R pair_scalar(R r2, const TypePair<R> &tp, const PairGlobals &pg, R alpha,
                                         R r_on, R inv_w, R r_on_v, R inv_w_v)
{
    R r, rinv;
    if (MODE != MODE_FULL && SPLIT) {
        R dwc, dwv;
        pair_dw_parts<R>(r2, tp, alpha, pg.coulomb, r, rinv, dwc, dwv);
        const R cc = switch_chi<R>(r, r_on, inv_w), cv = switch_chi<R>(r, r_on_v, inv_w_v);
        if (MODE == MODE_SHORT) return (((R)1 - cc) * dwc + ((R)1 - cv) * dwv) * rinv;
        return ((r > r_on ? cc * dwc : (R)0) + (r > r_on_v ? cv * dwv : (R)0)) * rinv;
    }
    const R dw = pair_dw<R>(r2, tp, alpha, pg.coulomb, r, rinv);
    if (MODE == MODE_SHORT) return ((R)1 - switch_chi<R>(r, r_on, inv_w)) * dw * rinv;
    if (MODE == MODE_LONG) return r > r_on ? switch_chi<R>(r, r_on, inv_w) * dw * rinv : (R)0;
    return dw * rinv;
}

template <typename R, int MODE, int G, bool SPLIT>
__device__ __forceinline__ void pair_force_row(const double4 *__restrict__ X, const double4 &xi,
                                               const BoxReg &box, const int32_t *__restrict__ row,
                                               int32_t nn, int32_t cnt, int32_t cap, int lig, int32_t self,
                                               const TypePair<R> *tab_i, const PairGlobals &pg,
                                               double &ax, double &ay, double &az)
{
    const R alpha = (R)pg.alpha, r_on = (R)pg.r_on, inv_w = (R)pg.inv_w;
    const R r_on_v = (R)pg.r_on_v, inv_w_v = (R)pg.inv_w_v;
    const R lim = MODE == MODE_SHORT ? (R)pg.r_short : (R)pg.r_cut;
    const R lim2 = lim * lim;
    // U entries per lane in flight: their position gathers are issued together,
    // and the row indices of the next block load during this block's arithmetic
    constexpr int U = 4;
    // the first block is read from the row's front within its capacity
    // without waiting for the lengths, then masked (and, past the near part,
    // read again from the back)
    const int32_t tail = cap - 1 + nn;
    int32_t pn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t e = lig + u * G;
        pn[u] = e < cap ? row[e] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t e = lig + u * G;
        if (e >= cnt) pn[u] = -1;
        else if (e >= nn) pn[u] = row[tail - e];
    }
    for (int32_t e0 = lig; e0 < cnt; e0 += U * G) {
        int32_t pj[U];
        double4 xj[U];
        R px = (R)0, py = (R)0, pz = (R)0;
#pragma unroll
        for (int u = 0; u < U; ++u) pj[u] = pn[u];
#pragma unroll
        for (int u = 0; u < U; ++u) xj[u] = X[pj[u] >= 0 ? pj[u] : self];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = e0 + (U + u) * G;
            pn[u] = e < cnt ? row[row_slot(e, nn, tail)] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // every loaded position is used (an empty slot gets r2 = lim2), so
            // the U gathers stay in flight together
            double dx = xi.x - xj[u].x, dy = xi.y - xj[u].y, dz = xi.z - xj[u].z;
            box.apply(dx, dy, dz);
            const R rx = (R)dx, ry = (R)dy, rz = (R)dz;
            const R r2 = pj[u] >= 0 ? rx * rx + ry * ry + rz * rz : lim2;
            if (!(r2 < lim2)) continue;
            const TypePair<R> &tp = tab_i[mirror_type(xj[u].w)];
            const R f = pair_scalar<R, MODE, SPLIT>(r2, tp, pg, alpha, r_on, inv_w, r_on_v, inv_w_v);
            px += f * rx;
            py += f * ry;
            pz += f * rz;
        }
        ax += (double)px;
        ay += (double)py;
        az += (double)pz;
    }
}

// 16-byte gathers from the fixed-point mirror through a buffer resource (CDNA
// V#: base, no stride, size in bytes; word 3 = 0x00020000, the 32-bit data
// format of the gfx9 family): a 32-bit byte offset per lane instead of a
// 64-bit address, and an offset past the end reads zeros instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t mirror_rsrc(const int4 *XF, int32_t n)
{
    const int64_t bytes = 16 * (int64_t)n;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<int4 *>(XF), (short)0,
                                             (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff), 0x00020000);
}

__device__ __forceinline__ int4 mirror_load(__amdgpu_buffer_rsrc_t r, int32_t i)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, i * 16, 0, 0);
    return make_int4((int32_t)v[0], (int32_t)v[1], (int32_t)v[2], (int32_t)v[3]);
}

// The same sum in FP32 pair arithmetic over the fixed-point position mirror:
// the displacement is the 32-bit difference of two fixed-point positions
// (minimum image by two's-complement wrap in a periodic box), exact to their
// rounding, and is converted to A by one FP32 rounding per axis.  Per entry:
// the index load, one 16-byte gather, integer and FP32 arithmetic only.  An
// empty slot gathers the atom itself (self), whose zero displacement drops out
// of the r^2 > 0 test.  NEAR: only the row's near part is walked (cnt = nn),
// so an entry's slot is its index.  ISO (one mirror unit on all three axes):
// r^2 is formed in mirror units and scaled once, and the unit goes into the
// pair scalar instead of into each displacement component.
template <int MODE, int G, bool SPLIT, bool NEAR, bool ISO>
__device__ __forceinline__ void pair_force_row_fixed(__amdgpu_buffer_rsrc_t XF, const int4 &xi,
                                                     const float fu[3],
                                                     const int32_t *__restrict__ row, int32_t nn,
                                                     int32_t cnt, int32_t cap, int lig, int32_t self,
                                                     const TypePair<float> *tab_i,
                                                     const PairGlobals &pg, double &ax, double &ay,
                                                     double &az)
{
    const float alpha = (float)pg.alpha, r_on = (float)pg.r_on, inv_w = (float)pg.inv_w;
    const float r_on_v = (float)pg.r_on_v, inv_w_v = (float)pg.inv_w_v;
    const float lim = MODE == MODE_SHORT ? (float)pg.r_short : (float)pg.r_cut;
    const float lim2 = lim * lim;
    const float fu2 = fu[0] * fu[0], lim2u = lim2 / fu2;
    constexpr int U = 4;
    const int32_t tail = cap - 1 + nn;
    int32_t pn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t e = lig + u * G;
        pn[u] = e < cap ? row[e] : self;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t e = lig + u * G;
        if (e >= cnt) pn[u] = self;
        else if (!NEAR && e >= nn) pn[u] = row[tail - e];
    }
    for (int32_t e0 = lig; e0 < cnt; e0 += U * G) {
        int4 xj[U];
        float px = 0.0f, py = 0.0f, pz = 0.0f;
#pragma unroll
        for (int u = 0; u < U; ++u) xj[u] = mirror_load(XF, pn[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = e0 + (U + u) * G;
            pn[u] = e < cnt ? row[NEAR ? e : row_slot(e, nn, tail)] : self;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t dxf = (int32_t)((uint32_t)xi.x - (uint32_t)xj[u].x);
            const int32_t dyf = (int32_t)((uint32_t)xi.y - (uint32_t)xj[u].y);
            const int32_t dzf = (int32_t)((uint32_t)xi.z - (uint32_t)xj[u].z);
            float rx, ry, rz, r2;
            if constexpr (ISO) {
                rx = (float)dxf;
                ry = (float)dyf;
                rz = (float)dzf;
                const float r2u = rx * rx + ry * ry + rz * rz;
                if (!(r2u < lim2u && r2u > 0.0f)) continue;
                r2 = r2u * fu2;
            } else {
                rx = (float)dxf * fu[0];
                ry = (float)dyf * fu[1];
                rz = (float)dzf * fu[2];
                r2 = rx * rx + ry * ry + rz * rz;
                if (!(r2 < lim2 && r2 > 0.0f)) continue;
            }
            const TypePair<float> &tp = tab_i[xj[u].w];
            float f = pair_scalar<float, MODE, SPLIT>(r2, tp, pg, alpha, r_on, inv_w, r_on_v, inv_w_v);
            if constexpr (ISO) f *= fu[0];
            px += f * rx;
            py += f * ry;
            pz += f * rz;
        }
        ax += (double)px;
        ay += (double)py;
        az += (double)pz;
    }
}

// pair_force_row_fixed with the near-part gate and the unit shape as template
// arguments
template <int MODE, int G, bool SPLIT>
__device__ __forceinline__ void pair_row_fixed_by(bool near_only, bool iso, __amdgpu_buffer_rsrc_t XF,
                                                  const int4 &xi, const float fu[3],
                                                  const int32_t *__restrict__ row, int32_t nn, int32_t cnt,
                                                  int32_t cap, int lig, int32_t self,
                                                  const TypePair<float> *tab_i, const PairGlobals &pg,
                                                  double &ax, double &ay, double &az)
{
    if (near_only) {
        if (iso)
            pair_force_row_fixed<MODE, G, SPLIT, true, true>(XF, xi, fu, row, nn, cnt, cap, lig, self, tab_i, pg, ax, ay, az);
        else
            pair_force_row_fixed<MODE, G, SPLIT, true, false>(XF, xi, fu, row, nn, cnt, cap, lig, self, tab_i, pg, ax, ay, az);
    } else if (iso) {
        pair_force_row_fixed<MODE, G, SPLIT, false, true>(XF, xi, fu, row, nn, cnt, cap, lig, self, tab_i, pg, ax, ay, az);
    } else {
        pair_force_row_fixed<MODE, G, SPLIT, false, false>(XF, xi, fu, row, nn, cnt, cap, lig, self, tab_i, pg, ax, ay, az);
    }
}

// sum over the G lanes of a group (fixed butterfly: deterministic)
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
    return v;
}

// The pair force of the sorted atoms s = t / G < s_end (G lanes each, lane
// t % G), MODE_SHORT / MODE_FULL / MODE_LONG, into a.out (sorted or caller
// order, stored or added).  tab: the n_types x n_types pair constants.
// FIXED: FP32 arithmetic over the fixed-point mirror.
template <typename R, int MODE, int G, bool ONE, bool FIXED>
__device__ __forceinline__ void pair_force_atoms(const PairArgs &a, const TypePair<R> *tab, int32_t t,
                                                 int32_t s_end)
{
    const int32_t s = t / G, lig = t % G;
    const bool valid = s < s_end;
    const int nt = a.pg.n_types;
    double ax = 0.0, ay = 0.0, az = 0.0;
    int32_t gi = 0;
    if (valid) {
        const int32_t par = a.mirror_sel >= 0 ? a.mirror_sel : (int32_t)((a.st->step + a.step_off) & 1);
        const double4 *__restrict__ X = a.ls.x[par];
        const int2 si = a.ls.sinfo[s];
        gi = si.x;
        const int32_t *row = a.ls.flist + (int64_t)s * a.ls.fcap;
        const int32_t cap = a.ls.fcap;
        const int2 fc = a.ls.fcnt[s];   // the list build keeps fc.x + fc.y <= cap
        // a far partner was at least lim + s/2 away at the build; while every
        // atom has moved less than (s/2)/2 since (the flag clear), none is within lim
        const bool near_only = a.far_gate && a.st->far_flag == 0u;
        const int32_t nn = fc.x, cnt = near_only ? fc.x : fc.x + fc.y;
        if constexpr (FIXED) {
            const RepInfo &rp = ONE ? a.reps[0] : a.reps[si.y];
            const float fu[3] = {rp.funit[0], rp.funit[1], rp.funit[2]};
            const int4 *__restrict__ XFp = a.ls.xf[par];
            const int4 xfi = XFp[s];
            const __amdgpu_buffer_rsrc_t XF = mirror_rsrc(XFp, a.n);
            const TypePair<float> *tf = reinterpret_cast<const TypePair<float> *>(tab) + xfi.w * nt;
            // the separate-mechanism flag, the near-part gate and the unit
            // shape are uniform (per launch, per replica): branches outside the loop
            const bool iso = fu[0] == fu[1] && fu[1] == fu[2];
            if (MODE != MODE_FULL && a.pg.split)
                pair_row_fixed_by<MODE, G, true>(near_only, iso, XF, xfi, fu, row, nn, cnt, cap, lig, s, tf, a.pg, ax, ay, az);
            else
                pair_row_fixed_by<MODE, G, false>(near_only, iso, XF, xfi, fu, row, nn, cnt, cap, lig, s, tf, a.pg, ax, ay, az);
        } else {
            const double4 xi = X[s];
            const TypePair<R> *ti = tab + mirror_type(xi.w) * nt;
            const BoxReg box(ONE ? a.reps[0] : load_rep(a.reps, a.single_rep, si.y));
            if (MODE != MODE_FULL && a.pg.split)
                pair_force_row<R, MODE, G, true>(X, xi, box, row, nn, cnt, cap, lig, s, ti, a.pg, ax, ay, az);
            else
                pair_force_row<R, MODE, G, false>(X, xi, box, row, nn, cnt, cap, lig, s, ti, a.pg, ax, ay, az);
        }
    }
    ax = group_sum<G>(ax);
    ay = group_sum<G>(ay);
    az = group_sum<G>(az);
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

}  // namespace bnc
