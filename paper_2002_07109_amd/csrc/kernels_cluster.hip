// Cluster-pair (tile) form of the F_0 pair force, FP32 over the fixed-point
// mirror: an alternative to the atom-row kernel, selected by
// bounce_params.pair_kernel.  The pair set and the pair arithmetic are those
// of the atom-row kernel (Sec. IV.A: (1 - chi) W'_sf d/r for r < r'', or the
// full W'_sf d/r for r < rc, over non-excluded pairs); only the way partners
// are found and the summation order differ.
//
// A cluster is CL consecutive sorted atoms of one replica (cell order, so a
// cluster spans one to three neighbouring cells).  At each list build the
// clusters get a bounding box of their build positions, and every cluster I
// a list of the clusters J of its replica whose boxes come within lim + s of
// its own (lim = r'' or rc, s the skin): every atom has moved less than s/2
// since, so the list holds every pair within lim until the next build.  The
// force kernel gives one wavefront to an i-cluster; its 64 lanes cover
// 64 / CL^2 tiles (i-cluster x j-cluster) at a time, one pair per lane: the
// j positions of a tile are one contiguous load, with no per-pair index and no
// per-pair image shift (the 32-bit fixed-point difference is the minimum image).
#include "bounce_kernels.hpp"
#include "bounce_pairrow.hpp"

namespace bnc {

// bounding box of each cluster at the build: centre (fixed point, modulo 2^32
// in a periodic box) and half extents in A
__global__ void __launch_bounds__(256) k_cl_bbox(ClusterSet cs, ListSet ls, const RepInfo *__restrict__ reps,
                                                 const DevState *st, int32_t mirror_sel, int32_t step_off)
{
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cs.ncl) return;
    const int4 c = cs.clu[k];
    const int32_t par = mirror_sel >= 0 ? mirror_sel : (int32_t)((st->step + step_off) & 1);
    const int4 *__restrict__ XF = ls.xf[par];
    const int4 x0 = XF[c.x];
    int32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int32_t s = c.x + 1; s < c.y; ++s) {
        const int4 x = XF[s];
        const int32_t d[3] = {(int32_t)((uint32_t)x.x - (uint32_t)x0.x), (int32_t)((uint32_t)x.y - (uint32_t)x0.y),
                              (int32_t)((uint32_t)x.z - (uint32_t)x0.z)};
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], d[a]);
            hi[a] = max(hi[a], d[a]);
        }
    }
    const RepInfo &ri = reps[c.z];
    int4 ctr;
    float4 h;
    ctr.x = (int32_t)((uint32_t)x0.x + (uint32_t)(int32_t)(((int64_t)lo[0] + hi[0]) / 2));
    ctr.y = (int32_t)((uint32_t)x0.y + (uint32_t)(int32_t)(((int64_t)lo[1] + hi[1]) / 2));
    ctr.z = (int32_t)((uint32_t)x0.z + (uint32_t)(int32_t)(((int64_t)lo[2] + hi[2]) / 2));
    ctr.w = c.z;
    // half extent plus one unit for the halving, and a relative margin for the
    // FP32 rounding of the distance test
    h.x = (float)(((double)hi[0] - lo[0]) * 0.5 + 1.0) * ri.funit[0] * 1.0001f;
    h.y = (float)(((double)hi[1] - lo[1]) * 0.5 + 1.0) * ri.funit[1] * 1.0001f;
    h.z = (float)(((double)hi[2] - lo[2]) * 0.5 + 1.0) * ri.funit[2] * 1.0001f;
    h.w = 0.0f;
    cs.ctr[k] = ctr;
    cs.half[k] = h;
}

// the cluster list: one wavefront per i-cluster, the j-clusters of its replica
// in ascending order whose boxes come within rl (ballot-ordered appends)
__global__ void __launch_bounds__(256) k_cl_list(ClusterSet cs, const RepInfo *__restrict__ reps, float rl,
                                                 DevState *st)
{
    const int lane = threadIdx.x & 63;
    const int32_t I = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (I >= cs.ncl) return;                       // uniform per wavefront
    const int4 ci = cs.ctr[I];
    const float4 hi = cs.half[I];
    const RepInfo &ri = reps[ci.w];
    const int32_t j0 = cs.rep_first[ci.w], j1 = cs.rep_first[ci.w + 1];
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int32_t *row = cs.list + (int64_t)I * cs.cap;
    int32_t n = 0;
    const float rl2 = rl * rl;
    for (int32_t b = j0; b < j1; b += 64) {
        const int32_t J = b + lane;
        bool hit = false;
        if (J < j1) {
            const int4 cj = cs.ctr[J];
            const float4 hj = cs.half[J];
            const float dx = fabsf((float)(int32_t)((uint32_t)ci.x - (uint32_t)cj.x) * ri.funit[0]);
            const float dy = fabsf((float)(int32_t)((uint32_t)ci.y - (uint32_t)cj.y) * ri.funit[1]);
            const float dz = fabsf((float)(int32_t)((uint32_t)ci.z - (uint32_t)cj.z) * ri.funit[2]);
            const float gx = fmaxf(dx - hi.x - hj.x, 0.0f), gy = fmaxf(dy - hi.y - hj.y, 0.0f),
                        gz = fmaxf(dz - hi.z - hj.z, 0.0f);
            hit = gx * gx + gy * gy + gz * gz < rl2;
        }
        const uint64_t m = __ballot(hit);
        if (hit) {
            const int32_t q = n + __popcll(m & below);
            if (q < cs.cap) row[q] = J;
        }
        n += __popcll(m);
    }
    if (lane == 0) {
        cs.cnt[I] = min(n, cs.cap);
        if (n > cs.cap) atomicOr(&st->status, ST_CAPACITY);
    }
}

// The pair force of the CL atoms of an i-cluster over its j-clusters, T tiles
// at a time (lane = t CL^2 + a CL + b: tile t, i-atom a, j-atom b).
template <int MODE, int CL>
__global__ void __launch_bounds__(256) k_pair_cl(PairArgs a, ClusterSet cs)
{
    constexpr int T = 64 / (CL * CL);
    __shared__ TypePair<float> tab[MAXT * MAXT];
    const TypePair<float> *pre = a.tab_f;
    for (int k = threadIdx.x; k < a.pg.n_types * a.pg.n_types; k += blockDim.x) tab[k] = pre[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int32_t I = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (I >= cs.ncl) return;                       // uniform per wavefront; no barrier below
    const int t = lane / (CL * CL), ia = (lane / CL) % CL, jb = lane % CL;
    const int4 c = cs.clu[I];
    const int32_t si = c.x + ia;
    const bool ivalid = si < c.y;
    const int32_t par = a.mirror_sel >= 0 ? a.mirror_sel : (int32_t)((a.st->step + a.step_off) & 1);
    const int4 *__restrict__ XF = a.ls.xf[par];
    const RepInfo &rp = a.reps[c.z];
    const float fu[3] = {rp.funit[0], rp.funit[1], rp.funit[2]};
    const int4 xi = XF[ivalid ? si : c.x];
    const int32_t gi = a.ls.sinfo[ivalid ? si : c.x].x;
    // the atom's excluded partners (caller ids), checked for pairs in range
    int32_t ex_id[8];
    {
        const int32_t e_b = a.tp.excl_ptr[gi], e_n = a.tp.excl_ptr[gi + 1] - e_b;
#pragma unroll
        for (int q = 0; q < 8; ++q) ex_id[q] = q < e_n ? a.tp.excl_idx[e_b + q] : -1;
    }
    const TypePair<float> *tab_i = tab + xi.w * a.pg.n_types;
    const float alpha = (float)a.pg.alpha, r_on = (float)a.pg.r_on, inv_w = (float)a.pg.inv_w;
    const float r_on_v = (float)a.pg.r_on_v, inv_w_v = (float)a.pg.inv_w_v;
    const float lim = MODE == MODE_SHORT ? (float)a.pg.r_short : (float)a.pg.r_cut;
    const float lim2 = lim * lim;
    const int32_t nJ = cs.cnt[I];
    const int32_t *row = cs.list + (int64_t)I * cs.cap;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int32_t k0 = 0; k0 < nJ; k0 += T) {
        const int32_t k = k0 + t;
        float px = 0.0f, py = 0.0f, pz = 0.0f;
        if (k < nJ) {
            const int4 cj = cs.clu[row[k]];
            const int32_t sj = cj.x + jb;
            if (ivalid && sj < cj.y && sj != si) {
                const int4 xj = XF[sj];
                const int32_t dxf = (int32_t)((uint32_t)xi.x - (uint32_t)xj.x);
                const int32_t dyf = (int32_t)((uint32_t)xi.y - (uint32_t)xj.y);
                const int32_t dzf = (int32_t)((uint32_t)xi.z - (uint32_t)xj.z);
                const float rx = (float)dxf * fu[0], ry = (float)dyf * fu[1], rz = (float)dzf * fu[2];
                const float r2 = rx * rx + ry * ry + rz * rz;
                if (r2 < lim2) {
                    const int32_t gj = a.ls.sinfo[sj].x;
                    bool ex = false;
#pragma unroll
                    for (int q = 0; q < 8; ++q) ex |= ex_id[q] == gj;
                    if (!ex) {
                        const TypePair<float> &tp = tab_i[xj.w];
                        const float f = a.pg.split && MODE != MODE_FULL
                                            ? pair_scalar<float, MODE, true>(r2, tp, a.pg, alpha, r_on, inv_w, r_on_v, inv_w_v)
                                            : pair_scalar<float, MODE, false>(r2, tp, a.pg, alpha, r_on, inv_w, r_on_v, inv_w_v);
                        px = f * rx;
                        py = f * ry;
                        pz = f * rz;
                    }
                }
            }
        }
        ax += (double)px;
        ay += (double)py;
        az += (double)pz;
    }
    // the lanes of one i-atom: b over CL, then t over T (fixed order)
#pragma unroll
    for (int m = 1; m < CL; m <<= 1) {
        ax += __shfl_xor(ax, m, 64);
        ay += __shfl_xor(ay, m, 64);
        az += __shfl_xor(az, m, 64);
    }
#pragma unroll
    for (int m = CL * CL; m < 64; m <<= 1) {
        ax += __shfl_xor(ax, m, 64);
        ay += __shfl_xor(ay, m, 64);
        az += __shfl_xor(az, m, 64);
    }
    if (ivalid && t == 0 && jb == 0) {
        const int64_t o = 3 * (int64_t)(a.out_global ? gi : si);
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

void launch_cluster_build(hipStream_t sm, const ClusterSet &cs, const ListSet &ls, const RepInfo *reps,
                          DevState *st, int32_t mirror_sel, int32_t step_off, float rl)
{
    if (cs.ncl <= 0) return;
    hipLaunchKernelGGL(k_cl_bbox, dim3((cs.ncl + 255) / 256), dim3(256), 0, sm, cs, ls, reps, st, mirror_sel,
                       step_off);
    hipLaunchKernelGGL(k_cl_list, dim3((cs.ncl + 3) / 4), dim3(256), 0, sm, cs, reps, rl, st);
}

void launch_pair_cl(hipStream_t sm, int mode, const PairArgs &a, const ClusterSet &cs)
{
    if (cs.ncl <= 0) return;
    const dim3 grid((cs.ncl + 3) / 4), block(256);
    if (cs.cl == 4) {
        if (mode == MODE_SHORT) hipLaunchKernelGGL((k_pair_cl<MODE_SHORT, 4>), grid, block, 0, sm, a, cs);
        else hipLaunchKernelGGL((k_pair_cl<MODE_FULL, 4>), grid, block, 0, sm, a, cs);
    } else {
        if (mode == MODE_SHORT) hipLaunchKernelGGL((k_pair_cl<MODE_SHORT, 8>), grid, block, 0, sm, a, cs);
        else hipLaunchKernelGGL((k_pair_cl<MODE_FULL, 8>), grid, block, 0, sm, a, cs);
    }
}

}  // namespace bnc
