// Pair-list build on the GPU: cell binning, counting sort into canonical
// order (ascending cell, then caller id), and per-atom rows of the force list
// and of the jump-candidate list.
//
// This translation unit is compiled with -ffp-contract=off: the cell index
// and the list predicate |d|^2 < R^2 (minimum image, FP64) are evaluated with
// exactly the roundings written, so the lists are reproducible bit for bit by
// any implementation of the same definition.
#include "bounce_kernels.hpp"

namespace bnc {

// cell of a position on replica ri's grid; -1 if a droplet atom is off-grid
__device__ __forceinline__ int32_t cell_index(const RepInfo &ri, const double *x)
{
    int32_t c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (ri.periodic) {
            double xw = x[k] - ri.box[k] * floor(x[k] * ri.inv_box[k]);
            double f = floor(xw * ri.cinv[k]);
            int32_t ck = (int32_t)f;
            ck = ck < 0 ? 0 : (ck > ri.ncell[k] - 1 ? ri.ncell[k] - 1 : ck);
            c[k] = ck;
        } else {
            double f = floor((x[k] - ri.origin[k]) * ri.inv_cell);
            if (!(f >= 0.0) || f >= (double)ri.ncell[k]) return -1;
            c[k] = (int32_t)f;
        }
    }
    return (c[0] * ri.ncell[1] + c[1]) * ri.ncell[2] + c[2];
}

__global__ void k_bin(int32_t n, const double *__restrict__ pos, const RepInfo *__restrict__ reps,
                      Topo tp, ListSet ls, DevState *st)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const RepInfo &ri = reps[tp.rep_of[g]];
    const double *x = pos + 3 * (int64_t)g;
    int32_t c = cell_index(ri, x);
    if (c < 0) {
        atomicOr(&st->status, ST_GRID);
        c = 0;
    }
    c += ri.cell_off;
    ls.cell_of[g] = c;
    ls.slot[g] = atomicAdd(&ls.cell_count[c], 1);
    ls.q_build[3 * (int64_t)g + 0] = x[0];
    ls.q_build[3 * (int64_t)g + 1] = x[1];
    ls.q_build[3 * (int64_t)g + 2] = x[2];
}

// exclusive scan of the cell counts in one workgroup; clears the counts
__global__ void __launch_bounds__(1024) k_scan(int32_t n_cells, ListSet ls)
{
    __shared__ int32_t part[1024];
    int32_t t = threadIdx.x;
    int32_t chunk = (n_cells + 1023) / 1024;
    int32_t b = t * chunk, e = min(n_cells, b + chunk);
    int32_t s = 0;
    for (int32_t k = b; k < e; ++k) s += ls.cell_count[k];
    part[t] = s;
    __syncthreads();
    for (int32_t off = 1; off < 1024; off <<= 1) {
        int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - s;
    for (int32_t k = b; k < e; ++k) {
        ls.cell_start[k] = run;
        run += ls.cell_count[k];
        ls.cell_count[k] = 0;
    }
    if (t == 1023) ls.cell_start[n_cells] = part[1023];
}

__global__ void k_scatter(int32_t n, ListSet ls)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    ls.perm[ls.cell_start[ls.cell_of[g]] + ls.slot[g]] = g;
}

// one thread per cell: order the cell's atoms by caller id, fill the mirror
__global__ void k_cellsort(int32_t n_cells, const double *__restrict__ pos, Topo tp, ListSet ls,
                           const DevState *st, int32_t mirror_sel)
{
    int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int32_t b = ls.cell_start[c], e = ls.cell_start[c + 1];
    int32_t *p = ls.perm;
    for (int32_t i = b + 1; i < e; ++i) {
        int32_t v = p[i], j = i - 1;
        while (j >= b && p[j] > v) { p[j + 1] = p[j]; --j; }
        p[j + 1] = v;
    }
    int32_t par = mirror_sel >= 0 ? mirror_sel : (int32_t)(st->step & 1);
    double4 *X = ls.x[par];
    for (int32_t i = b; i < e; ++i) {
        int32_t g = p[i];
        ls.inv_perm[g] = i;
        const double *x = pos + 3 * (int64_t)g;
        X[i] = make_double4(x[0], x[1], x[2], (double)tp.type[g]);
    }
}

// distance between cell intervals ci and cj along one dimension (cyclic index
// distance for periodic boxes); a lower bound of any atom-atom distance there
__device__ __forceinline__ double cell_gap(int32_t ci, int32_t cj, int32_t n, double w, int periodic)
{
    int32_t d = ci > cj ? ci - cj : cj - ci;
    if (periodic && n - d < d) d = n - d;
    return d > 1 ? (double)(d - 1) * w : 0.0;
}

// One wavefront per cell: lanes (a, b) = (lane / 8, lane % 8) test i = i0 + a
// of the cell against j = j0 + b of each candidate cell.  Candidate cells are
// visited in ascending cell index and atoms inside a cell in ascending id, and
// the hits of each i are appended in lane order through a ballot, so every row
// comes out in canonical order without a sort.
__global__ void __launch_bounds__(256) k_lists(int32_t n_cells, const RepInfo *__restrict__ reps,
                                               const int32_t *__restrict__ cell_rep, Topo tp,
                                               ListSet ls, BuildSpec bs, DevState *st)
{
    const int lane = threadIdx.x & 63;
    const int32_t ci = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (ci >= n_cells) return;                       // uniform per wavefront
    const int32_t bi = ls.cell_start[ci], ei = ls.cell_start[ci + 1];
    if (bi == ei) return;                            // uniform per wavefront
    const RepInfo &ri = reps[cell_rep[ci]];
    const int32_t par = bs.mirror_sel >= 0 ? bs.mirror_sel : (int32_t)(st->step & 1);
    const double4 *__restrict__ X = ls.x[par];
    const int32_t nx = ri.ncell[0], ny = ri.ncell[1], nz = ri.ncell[2];
    const int32_t loc = ci - ri.cell_off;
    const int32_t cx = loc / (ny * nz), cy = (loc / nz) % ny, cz = loc % nz;
    const double R = bs.rsearch * (1.0 + 1e-12) + 1e-9;
    const double R2 = R * R;
    const double rmax2 = fmax(bs.want_force ? bs.rf2 : 0.0, bs.want_cand ? bs.rcmax2 : 0.0);
    const int a = lane >> 3, b = lane & 7;
    const uint32_t below = (1u << b) - 1u;
    bool overflow = false;
    for (int32_t i0 = bi; i0 < ei; i0 += 8) {
        const int32_t i = i0 + a;
        const bool ivalid = i < ei;
        double4 xi = make_double4(0.0, 0.0, 0.0, 0.0);
        int32_t gi = -1, e_b = 0, e_e = 0;
        if (ivalid) {
            xi = X[i];
            gi = ls.perm[i];
            e_b = tp.excl_ptr[gi];
            e_e = tp.excl_ptr[gi + 1];
        }
        int32_t nf = 0, ncand = 0;
        int32_t *frow = ls.flist + (int64_t)(ivalid ? i : 0) * ls.fcap;
        int32_t *crow = ls.clist + (int64_t)(ivalid ? i : 0) * ls.ccap;
        for (int32_t jx = 0; jx < nx; ++jx) {
            const double gx = cell_gap(cx, jx, nx, ri.cw[0], ri.periodic);
            if (gx >= R) continue;
            for (int32_t jy = 0; jy < ny; ++jy) {
                const double gy = cell_gap(cy, jy, ny, ri.cw[1], ri.periodic);
                const double gxy = gx * gx + gy * gy;
                if (gxy >= R2) continue;
                for (int32_t jz = 0; jz < nz; ++jz) {
                    const double gz = cell_gap(cz, jz, nz, ri.cw[2], ri.periodic);
                    if (gxy + gz * gz >= R2) continue;
                    const int32_t cj = ri.cell_off + (jx * ny + jy) * nz + jz;
                    const int32_t bj = ls.cell_start[cj], ej = ls.cell_start[cj + 1];
                    for (int32_t j0 = bj; j0 < ej; j0 += 8) {
                        const int32_t j = j0 + b;
                        bool f = false, c = false;
                        if (ivalid && j < ej && j != i) {
                            const double4 xj = X[j];
                            double dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
                            min_image(ri, dx, dy, dz);
                            const double r2 = norm2_exact(dx, dy, dz);
                            if (r2 < rmax2) {
                                const int32_t gj = ls.perm[j];
                                bool ex = false;
                                for (int32_t k = e_b; k < e_e; ++k) ex |= (tp.excl_idx[k] == gj);
                                if (!ex) {
                                    f = bs.want_force && r2 < bs.rf2;
                                    c = bs.want_cand && r2 < bs.rcmax2 &&
                                        !(bs.rcmin2 > 0.0 && r2 < bs.rcmin2);
                                }
                            }
                        }
                        const uint32_t mf = (uint32_t)(__ballot(f) >> (8 * a)) & 0xffu;
                        const uint32_t mc = (uint32_t)(__ballot(c) >> (8 * a)) & 0xffu;
                        if (f) {
                            const int32_t k = nf + __popc(mf & below);
                            if (k < ls.fcap) frow[k] = j;
                        }
                        if (c) {
                            const int32_t k = ncand + __popc(mc & below);
                            if (k < ls.ccap) crow[k] = j;
                        }
                        nf += __popc(mf);
                        ncand += __popc(mc);
                    }
                }
            }
        }
        if (ivalid && b == 0) {
            if (bs.want_force) ls.fcnt[i] = min(nf, ls.fcap);
            if (bs.want_cand) ls.ccnt[i] = min(ncand, ls.ccap);
        }
        overflow |= ivalid && (nf > ls.fcap || ncand > ls.ccap);
    }
    if (overflow) atomicOr(&st->status, ST_CAPACITY);
}

void launch_build(hipStream_t sm, int32_t n, const double *pos, const RepInfo *reps,
                  const int32_t *cell_rep, const Topo &tp, const ListSet &ls, const BuildSpec &bs,
                  DevState *st)
{
    if (n <= 0) return;
    int32_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_bin, dim3(nb), dim3(256), 0, sm, n, pos, reps, tp, ls, st);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, sm, ls.n_cells, ls);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, sm, n, ls);
    hipLaunchKernelGGL(k_cellsort, dim3((ls.n_cells + 127) / 128), dim3(128), 0, sm, ls.n_cells,
                       pos, tp, ls, st, bs.mirror_sel);
    hipLaunchKernelGGL(k_lists, dim3((ls.n_cells + 3) / 4), dim3(256), 0, sm, ls.n_cells, reps,
                       cell_rep, tp, ls, bs, st);
}

}  // namespace bnc
