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

// Exclusive scan of the cell counts into cell_start (and the counts cleared
// for the next build), in two launches: the totals of blocks of 1024 cells,
// then the scan inside each block offset by the totals of the blocks before it.
// The same two passes scan the flags "cell holds an atom" into the list of
// occupied cells (busy), which the later build kernels walk instead of the
// whole grid (a droplet's grid is mostly empty).
constexpr int SCAN_B = 1024;

__device__ __forceinline__ int32_t block_incl_scan(int32_t v, int32_t *wsum)
{
    // inclusive scan over a 1024-thread workgroup: wavefront scans + their totals
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        int32_t t = lane < SCAN_B / 64 ? wsum[lane] : 0;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const int32_t o = __shfl_up(t, off, 64);
            if (lane >= off) t += o;
        }
        if (lane < SCAN_B / 64) wsum[lane] = t;
    }
    __syncthreads();
    return v + (w > 0 ? wsum[w - 1] : 0);
}

// scan_part[b]: atoms in block b of cells; scan_part[nsb + b]: occupied cells there
__global__ void __launch_bounds__(SCAN_B) k_scan_part(int32_t n_cells, ListSet ls)
{
    __shared__ int32_t wsum[SCAN_B / 64], wsum_b[SCAN_B / 64];
    const int32_t nsb = (n_cells + SCAN_B - 1) / SCAN_B;
    const int32_t k = blockIdx.x * SCAN_B + threadIdx.x;
    const int32_t v = k < n_cells ? ls.cell_count[k] : 0;
    const int32_t incl = block_incl_scan(v, wsum);
    const int32_t incl_b = block_incl_scan(v > 0 ? 1 : 0, wsum_b);
    if (threadIdx.x == SCAN_B - 1) {
        ls.scan_part[blockIdx.x] = incl;
        ls.scan_part[nsb + blockIdx.x] = incl_b;
    }
}

// the scan inside each block, offset by the sum of the earlier blocks' totals
__global__ void __launch_bounds__(SCAN_B) k_scan_fin(int32_t n_cells, ListSet ls)
{
    __shared__ int32_t wsum[SCAN_B / 64], wsum_b[SCAN_B / 64];
    __shared__ int32_t s_off, s_off_b;
    const int32_t nsb = (n_cells + SCAN_B - 1) / SCAN_B;
    int32_t o = 0, ob = 0;
    for (int32_t b = threadIdx.x; b < (int32_t)blockIdx.x; b += SCAN_B) {
        o += ls.scan_part[b];
        ob += ls.scan_part[nsb + b];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        o += __shfl_xor(o, m, 64);
        ob += __shfl_xor(ob, m, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        wsum[threadIdx.x >> 6] = o;
        wsum_b[threadIdx.x >> 6] = ob;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0, tb = 0;
        for (int w = 0; w < SCAN_B / 64; ++w) {
            t += wsum[w];
            tb += wsum_b[w];
        }
        s_off = t;
        s_off_b = tb;
    }
    __syncthreads();
    const int32_t k = blockIdx.x * SCAN_B + threadIdx.x;
    const int32_t v = k < n_cells ? ls.cell_count[k] : 0;
    const int32_t incl = block_incl_scan(v, wsum) + s_off;
    const int32_t incl_b = block_incl_scan(v > 0 ? 1 : 0, wsum_b) + s_off_b;
    if (k < n_cells) {
        ls.cell_start[k] = incl - v;
        ls.cell_count[k] = 0;
        if (v > 0) ls.busy[incl_b] = k;          // busy[1 + rank among occupied cells]
    }
    if (k == n_cells - 1) {
        ls.cell_start[n_cells] = incl;
        ls.busy[0] = incl_b;
    }
}

__global__ void k_scatter(int32_t n, ListSet ls)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    ls.perm[ls.cell_start[ls.cell_of[g]] + ls.slot[g]] = g;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront per occupied cell (grid-stride over the busy list): order the
// cell's atoms by caller id (rank sort over the lanes; a serial insertion sort
// above 64 atoms) and fill the mirror.
__global__ void __launch_bounds__(256) k_cellsort(const double *__restrict__ pos,
                                                  const RepInfo *__restrict__ reps, Topo tp,
                                                  ListSet ls, const DevState *st,
                                                  int32_t mirror_sel, int32_t step_off)
{
    const int lane = threadIdx.x & 63;
    const int32_t nbusy = ls.busy[0];
    const int32_t waves = gridDim.x * (blockDim.x >> 6);
    const int32_t par = mirror_sel >= 0 ? mirror_sel : (int32_t)((st->step + step_off) & 1);
    double4 *X = ls.x[par];
    int32_t *p = ls.perm;
    for (int32_t idx = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); idx < nbusy; idx += waves) {
        const int32_t c = ls.busy[1 + idx];             // uniform per wavefront
        const int32_t b = ls.cell_start[c], e = ls.cell_start[c + 1], m = e - b;
        if (m <= 64) {
            const int32_t mine = lane < m ? p[b + lane] : 0x7fffffff;
            int32_t rank = 0;
            for (int32_t k = 0; k < m; ++k) rank += __shfl(mine, k, 64) < mine;
            wave_sync();
            if (lane < m) p[b + rank] = mine;
        } else if (lane == 0) {
            for (int32_t i = b + 1; i < e; ++i) {
                int32_t v = p[i], j = i - 1;
                while (j >= b && p[j] > v) { p[j + 1] = p[j]; --j; }
                p[j + 1] = v;
            }
        }
        __threadfence_block();
        wave_sync();
        for (int32_t i = b + lane; i < e; i += 64) {
            const int32_t g = p[i];
            ls.inv_perm[g] = i;
            ls.sinfo[i] = make_int2(g, tp.rep_of[g]);
            const double *x = pos + 3 * (int64_t)g;
            X[i] = make_double4(x[0], x[1], x[2], mirror_w(g, tp.type[g]));
            if (ls.xf[par]) ls.xf[par][i] = fixed_pos(reps[tp.rep_of[g]], x[0], x[1], x[2], tp.type[g]);
        }
    }
}

// the bonded terms of the atom at sorted position sl (caller id g) with their
// atoms as sorted positions (needs the whole sort done)
__device__ void bslot_row(int32_t g, int32_t sl, const Topo &tp, const ListSet &ls)
{
    int4 *row = ls.bslot + (int64_t)sl * BTMAX;
    const int32_t b = tp.bt_ptr[g], e = tp.bt_ptr[g + 1];
    for (int32_t k = 0; k < BTMAX; ++k) {
        int4 t = make_int4(-1, 0, 0, 0);
        if (b + k < e) {
            const int32_t code = tp.bt[b + k], idx = code & 0x0fffffff;
            t.x = code;
            if ((code >> 28) == 0) {
                t.y = ls.inv_perm[tp.bond_ij[2 * idx]];
                t.z = ls.inv_perm[tp.bond_ij[2 * idx + 1]];
            } else {
                t.y = ls.inv_perm[tp.angle_ijk[3 * idx]];
                t.z = ls.inv_perm[tp.angle_ijk[3 * idx + 1]];
                t.w = ls.inv_perm[tp.angle_ijk[3 * idx + 2]];
            }
        }
        row[k] = t;
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

constexpr int LB = 4;          // wavefronts per cell
constexpr int LCAP = 512;      // candidate atoms staged in LDS per batch
static_assert(LCAP % 64 == 0, "a wavefront's 64 lanes test whole chunks of the staged batch");
constexpr int LMAXI = 64;      // atoms per cell handled
constexpr int LDIM = 12;       // candidate cells per dimension
constexpr int LCELLS = 352;    // candidate cells kept per cell
constexpr int LEXCL = 8;       // exclusions per atom held in registers
constexpr int LGRID = 4096;    // workgroups of the list kernel (it strides over further cells)

// Workgroups walk the occupied cells (grid-stride over the busy list), one
// cell at a time.  (1) Wavefront 0 enumerates the candidate cells
// (cell gap below the search radius) in ascending cell index, fetching their
// atom ranges in parallel and compacting them by ballots, and prefix-sums the
// range sizes.  (2) The workgroup stages a batch of candidate atoms (slot,
// FP64 position, caller id), in ascending cell and id order, in LDS.  (3) Each
// wavefront takes every LB-th atom i of the cell; its 64 lanes test 64
// consecutive staged candidates at a time and a ballot appends the hits in
// candidate order, so every row comes out in canonical order.
template <int KC>
__global__ void __launch_bounds__(64 * LB) k_lists(int32_t n_cells, const RepInfo *__restrict__ reps,
                                                   const int32_t *__restrict__ cell_rep,
                                                   const double *__restrict__ pos, Topo tp,
                                                   ListSet ls, BuildSpec bs, DevState *st)
{
    __shared__ double cx[LCAP], cy[LCAP], cz[LCAP];
    __shared__ int32_t cj[LCAP];
    __shared__ uint8_t ct[KC > 1 ? LCAP : 1];
    __shared__ int32_t rowf[LMAXI], rowg[LMAXI], rowc[LMAXI * KC];
    __shared__ double iexr2[LMAXI];
    __shared__ int32_t dcell[3][LDIM];
    __shared__ double dgap[3][LDIM];
    __shared__ int32_t cbeg[LCELLS], cnum[LCELLS], cpre[LCELLS + 1];
    __shared__ double4 ipos[LMAXI];
    __shared__ int32_t iex[LMAXI][LEXCL];
    __shared__ int32_t s_ncells;
    // (the wavefront index as a scalar: the row pointers of the atom a wavefront
    // handles are then scalar too, as the buffer resources of its stores need)
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t nbusy = ls.busy[0];
    for (int32_t idx = blockIdx.x; idx < nbusy; idx += gridDim.x) {
    const int32_t ci = ls.busy[1 + idx];              // uniform per workgroup
    const int32_t bi = ls.cell_start[ci], ei_all = ls.cell_start[ci + 1];
    const int32_t ei = min(ei_all, bi + LMAXI), ni = ei - bi;
    if (ls.bslot)     // this cell's rows of the bonded-term table
        for (int32_t k = threadIdx.x; k < ei_all - bi; k += 64 * LB)
            bslot_row(ls.perm[bi + k], bi + k, tp, ls);
    for (int32_t i = ei + threadIdx.x; i < ei_all; i += 64 * LB) {   // atoms beyond the limit
        ls.fcnt[i] = make_int2(0, 0);
        if (bs.want_cand)
            for (int b = 0; b < ls.ncls; ++b) ls.ccnt[(int64_t)i * ls.ncls + b] = 0;
    }
    if (ni == 0) continue;                           // uniform per workgroup
    const RepInfo &ri = reps[cell_rep[ci]];
    const BoxReg box(ri);
    const int32_t par = bs.mirror_sel >= 0 ? bs.mirror_sel : (int32_t)((st->step + bs.step_off) & 1);
    const double4 *__restrict__ X = ls.x[par];
    const double rmax2 = fmax(bs.want_force ? bs.rf2 : 0.0, bs.want_cand ? bs.rcmax2 : 0.0);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    bool overflow = ei_all > ei;
    // the cell's own atoms (on the last wavefront, while the first enumerates
    // the candidate cells): positions, exclusions, and the largest squared
    // distance to the atom itself or an excluded partner, computed exactly as
    // the predicate below computes it (the mirror holds the caller's positions
    // bit for bit); no candidate farther than that can be excluded, so the
    // exclusion test runs only at or below it
    if (w == LB - 1) {
        for (int32_t k = lane; k < ni; k += 64) {
            rowf[k] = rowg[k] = 0;
            for (int b = 0; b < KC; ++b) rowc[k * KC + b] = 0;
            const int32_t g = ls.perm[bi + k];
            const double4 x = make_double4(pos[3 * (int64_t)g], pos[3 * (int64_t)g + 1],
                                           pos[3 * (int64_t)g + 2], 0.0);
            ipos[k] = x;
            const int32_t e_b = tp.excl_ptr[g], e_n = tp.excl_ptr[g + 1] - e_b;
            double m2 = 0.0;
            for (int32_t t = 0; t < LEXCL; ++t) {
                const int32_t ge = t < e_n ? tp.excl_idx[e_b + t] : -1;
                iex[k][t] = ge;     // excluded partners' caller ids
                if (ge >= 0) {
                    const double *xe = pos + 3 * (int64_t)ge;
                    double dx = x.x - xe[0], dy = x.y - xe[1], dz = x.z - xe[2];
                    box.apply(dx, dy, dz);
                    m2 = fmax(m2, norm2_exact(dx, dy, dz));
                }
            }
            iexr2[k] = m2;
            if (e_n > LEXCL) overflow = true;
        }
    }
    if (w == 0) {
        const int32_t loc = ci - ri.cell_off;
        const int32_t cc[3] = {loc / (ri.ncell[1] * ri.ncell[2]), (loc / ri.ncell[2]) % ri.ncell[1],
                               loc % ri.ncell[2]};
        const double R = bs.rsearch * (1.0 + 1e-12) + 1e-9;
        const double R2 = R * R;
        // (1a) candidate cell indices per dimension, ascending
        int32_t nd[3];
        for (int d = 0; d < 3; ++d) {
            int32_t cnt = 0;
            for (int32_t j0 = 0; j0 < ri.ncell[d]; j0 += 64) {
                const int32_t j = j0 + lane;
                double gp = 0.0;
                bool ok = false;
                if (j < ri.ncell[d]) {
                    gp = cell_gap(cc[d], j, ri.ncell[d], ri.cw[d], ri.periodic);
                    ok = gp < R;
                }
                const uint64_t m = __ballot(ok);
                const int32_t k = cnt + __popcll(m & below);
                if (ok && k < LDIM) {
                    dcell[d][k] = j;
                    dgap[d][k] = gp * gp;
                }
                cnt += __popcll(m);
            }
            if (cnt > LDIM) overflow = true;
            nd[d] = min(cnt, LDIM);
        }
        wave_sync();
        // (1b) candidate cells in ascending index with their atom ranges: each
        // lane takes TPL triples per pass, so their range loads are in flight together
        const int32_t ntrip = nd[0] * nd[1] * nd[2];
        int32_t ncells = 0;
        constexpr int TPL = 6;
        for (int32_t t0 = 0; t0 < ntrip; t0 += 64 * TPL) {
            int32_t jb[TPL], je[TPL];
#pragma unroll
            for (int u = 0; u < TPL; ++u) {
                const int32_t t = t0 + 64 * u + lane;
                jb[u] = je[u] = 0;
                if (t < ntrip) {
                    const int32_t a = t / (nd[1] * nd[2]), b = (t / nd[2]) % nd[1], c = t % nd[2];
                    if (dgap[0][a] + dgap[1][b] + dgap[2][c] < R2) {
                        const int32_t cjx = ri.cell_off +
                                            (dcell[0][a] * ri.ncell[1] + dcell[1][b]) * ri.ncell[2] +
                                            dcell[2][c];
                        jb[u] = ls.cell_start[cjx];
                        je[u] = ls.cell_start[cjx + 1];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < TPL; ++u) {
                const bool ok = je[u] > jb[u];
                const uint64_t m = __ballot(ok);
                const int32_t k = ncells + __popcll(m & below);
                if (ok && k < LCELLS) {
                    cbeg[k] = jb[u];
                    cnum[k] = je[u] - jb[u];
                }
                ncells += __popcll(m);
            }
        }
        if (ncells > LCELLS) overflow = true;
        ncells = min(ncells, LCELLS);
        wave_sync();
        // prefix sum of the cell sizes (fixed order, wave scan in chunks of 64)
        int32_t run = 0;
        for (int32_t k0 = 0; k0 < ncells; k0 += 64) {
            const int32_t k = k0 + lane;
            const int32_t v = k < ncells ? cnum[k] : 0;
            int32_t incl = v;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int32_t o = __shfl_up(incl, off, 64);
                if (lane >= off) incl += o;
            }
            if (k < ncells) cpre[k] = run + incl - v;
            run += __shfl(incl, 63, 64);
        }
        if (lane == 0) {
            cpre[ncells] = run;
            s_ncells = ncells;
        }
    }
    __syncthreads();
    const int32_t ncells = s_ncells;
    const int32_t total = cpre[ncells];

    for (int32_t lo = 0; lo < total; lo += LCAP) {
        const int32_t nb = min(LCAP, total - lo);
        // (2a) slots of candidates [lo, lo + nb) of the flat sequence
        for (int32_t k = threadIdx.x; k < ncells; k += 64 * LB) {
            const int32_t p0 = cpre[k], jb = cbeg[k], jn = cnum[k];
            const int32_t t_lo = max(0, lo - p0), t_hi = min(jn, lo + nb - p0);
            for (int32_t t = t_lo; t < t_hi; ++t) cj[p0 + t - lo] = jb + t;
        }
        __syncthreads();
        // (2b) their positions and types
        for (int32_t f = threadIdx.x; f < nb; f += 64 * LB) {
            const double4 x = X[cj[f]];
            cx[f] = x.x;
            cy[f] = x.y;
            cz[f] = x.z;
            if (KC > 1) ct[f] = (uint8_t)mirror_type(x.w);
        }
        __syncthreads();
        // (3) this wavefront's atoms of the cell against the batch
        for (int32_t k = w; k < ni; k += LB) {
            const int32_t i = bi + k;
            const double4 xi = ipos[k];
            const double exr2 = iexr2[k];
            int32_t ex_id[LEXCL];
#pragma unroll
            for (int t = 0; t < LEXCL; ++t) ex_id[t] = iex[k][t];
            int32_t nf = rowf[k], ng = rowg[k], nc[KC];
#pragma unroll
            for (int b = 0; b < KC; ++b) nc[b] = rowc[k * KC + b];
            int32_t *frow = ls.flist + (int64_t)i * ls.fcap;
            int32_t *crow = ls.clist + (int64_t)i * ls.ncls * ls.ccap;
            // the row stores go through buffer resources of this atom's rows
            // (uniform across the wavefront; word 3 = 0x00020000, the 32-bit
            // data format of the gfx9 family): 32-bit offsets, and an entry past
            // a row's capacity is dropped by the hardware's range check (the
            // counts still take it, and the build reports the overflow)
            const __amdgpu_buffer_rsrc_t rsf = __builtin_amdgcn_make_buffer_rsrc(frow, (short)0, 4 * ls.fcap, 0x00020000);
            const __amdgpu_buffer_rsrc_t rsc = __builtin_amdgcn_make_buffer_rsrc(crow, (short)0, 4 * ls.ncls * ls.ccap, 0x00020000);
            for (int32_t f0 = 0; f0 < nb; f0 += 64) {
                // every lane reads a staged entry (f < LCAP: f0 < nb <= LCAP and
                // f0 is a multiple of 64, as LCAP is), and a lane past the batch
                // takes r2 = +inf, which no test below accepts: the predicates are
                // computed without branches
                const int32_t f = f0 + lane;
                const int32_t j = cj[f];
                double dx = xi.x - cx[f], dy = xi.y - cy[f], dz = xi.z - cz[f];
                box.apply(dx, dy, dz);
                const double r2 = f < nb ? norm2_exact(dx, dy, dz) : __builtin_huge_val();
                bool ex = false;
                if (r2 <= exr2) {      // the atom itself or possibly excluded (never past the batch)
                    const int32_t gj = ls.perm[j];
                    ex = j == i;
#pragma unroll
                    for (int t = 0; t < LEXCL; ++t) ex |= ex_id[t] == gj;
                }
                const bool in = r2 < rmax2 && !ex;
                const bool in_f = in && bs.want_force && r2 < bs.rf2;
                const bool hf = in_f && r2 < bs.rfn2;
                const bool hg = in_f && !(r2 < bs.rfn2);
                const bool hc = in && bs.want_cand && r2 < bs.rcmax2 && !(bs.rcmin2 > 0.0 && r2 < bs.rcmin2);
                const uint64_t mf = __ballot(hf), mg = __ballot(hg);
                if (hf) {      // near: from the front of the row
                    const int32_t q = nf + __popcll(mf & below);
                    __builtin_amdgcn_raw_buffer_store_b32(j, rsf, 4 * q, 0, 0);
                }
                if (hg) {      // far: from the back (past the capacity: a negative
                               // index, i.e. an offset beyond the range, dropped)
                    const int32_t q = ng + __popcll(mg & below);
                    __builtin_amdgcn_raw_buffer_store_b32(j, rsf, 4 * (ls.fcap - 1 - q), 0, 0);
                }
                // candidates by class (the partner's type when the rate
                // bounds are per type pair, else one class), each in candidate order
                const int cls = KC > 1 && f < nb ? (int)ct[f] : 0;
#pragma unroll
                for (int b = 0; b < KC; ++b) {
                    if (b >= ls.ncls) break;
                    const bool hb = hc && cls == b;
                    const uint64_t mb = __ballot(hb);
                    if (hb) {
                        const int32_t q = nc[b] + __popcll(mb & below);
                        // one class: the range check drops what is past the row;
                        // several: a class must not spill into the next one
                        if (KC == 1 || q < ls.ccap)
                            __builtin_amdgcn_raw_buffer_store_b32(j, rsc, 4 * (b * ls.ccap + q), 0, 0);
                    }
                    nc[b] += __popcll(mb);
                }
                nf += __popcll(mf);
                ng += __popcll(mg);
            }
            if (lane == 0) {
                rowf[k] = nf;
                rowg[k] = ng;
#pragma unroll
                for (int b = 0; b < KC; ++b) rowc[k * KC + b] = nc[b];
            }
        }
        __syncthreads();
    }
    for (int32_t k = threadIdx.x; k < ni; k += 64 * LB) {
        const int32_t nf = rowf[k], ng = rowg[k];
        const bool full = nf + ng > ls.fcap;     // the two ends met
        if (bs.want_force) ls.fcnt[bi + k] = full ? make_int2(0, 0) : make_int2(nf, ng);
        if (full) overflow = true;
        if (bs.want_cand)
            for (int b = 0; b < ls.ncls; ++b) {
                const int32_t nc = rowc[k * KC + b];
                ls.ccnt[(int64_t)(bi + k) * ls.ncls + b] = min(nc, ls.ccap);
                if (nc > ls.ccap) overflow = true;
            }
    }
    // (the barrier also ends every use of this cell's shared arrays)
    if (__syncthreads_or(overflow) && threadIdx.x == 0) atomicOr(&st->status, ST_CAPACITY);
    }
}

// Pair-structure histogram over the rows of a list set built at or beyond
// r_max: each ordered pair (i, j) with r^2 < r_max^2 counted in bin k with
// (k dr)^2 <= r^2 < ((k+1) dr)^2 of its type pair, the displacement
// minimum-imaged and squared in FP64 as the list predicate is (this unit is
// compiled without contraction).  RG lanes per atom, a workgroup histogram
// in LDS flushed with 64-bit atomics.
constexpr int RG = 16;

__global__ void __launch_bounds__(256) k_rdf(int32_t n, const RepInfo *__restrict__ reps,
                                             int32_t single_rep, ListSet ls, double rmax2, double dr,
                                             int32_t nbins, int32_t nt,
                                             unsigned long long *__restrict__ counts)
{
    extern __shared__ uint32_t hist[];
    const int32_t nh = nt * nt * nbins;
    for (int32_t k = threadIdx.x; k < nh; k += blockDim.x) hist[k] = 0u;
    __syncthreads();
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t s = t / RG, lig = t % RG;
    if (s < n) {
        const double4 *__restrict__ X = ls.x[0];
        const double4 xi = X[s];
        const int ti = mirror_type(xi.w);
        const BoxReg box(load_rep(reps, single_rep, ls.sinfo[s].y));
        const int32_t *row = ls.flist + (int64_t)s * ls.fcap;
        const int2 fc = ls.fcnt[s];
        const int32_t nn = fc.x, cnt = fc.x + fc.y, tail = ls.fcap - 1 + nn;
        for (int32_t e = lig; e < cnt; e += RG) {
            const double4 xj = X[row[e < nn ? e : tail - e]];
            double dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
            box.apply(dx, dy, dz);
            const double r2 = norm2_exact(dx, dy, dz);
            if (!(r2 < rmax2)) continue;
            int32_t k = min(max((int32_t)(sqrt(r2) / dr), 0), nbins - 1);
            while (k > 0 && ((double)k * dr) * ((double)k * dr) > r2) --k;
            while (k + 1 < nbins && ((double)(k + 1) * dr) * ((double)(k + 1) * dr) <= r2) ++k;
            atomicAdd(&hist[(ti * nt + mirror_type(xj.w)) * nbins + k], 1u);
        }
    }
    __syncthreads();
    for (int32_t k = threadIdx.x; k < nh; k += blockDim.x)
        if (hist[k]) atomicAdd(&counts[k], (unsigned long long)hist[k]);
}

void launch_rdf(hipStream_t sm, int32_t n, const RepInfo *reps, int32_t single_rep,
                const ListSet &ls, double r_max, int32_t nbins, int32_t nt,
                unsigned long long *counts)
{
    if (n <= 0) return;
    const double dr = r_max / (double)nbins;
    const size_t lds = sizeof(uint32_t) * (size_t)nt * nt * nbins;
    hipLaunchKernelGGL(k_rdf, dim3(((int64_t)n * RG + 255) / 256), dim3(256), lds, sm, n, reps,
                       single_rep, ls, r_max * r_max, dr, nbins, nt, counts);
}

void launch_build(hipStream_t sm, int32_t n, const double *pos, const RepInfo *reps,
                  const int32_t *cell_rep, const Topo &tp, const ListSet &ls, const BuildSpec &bs,
                  DevState *st)
{
    if (n <= 0) return;
    int32_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_bin, dim3(nb), dim3(256), 0, sm, n, pos, reps, tp, ls, st);
    const int32_t nsb = (ls.n_cells + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_part, dim3(nsb), dim3(SCAN_B), 0, sm, ls.n_cells, ls);
    hipLaunchKernelGGL(k_scan_fin, dim3(nsb), dim3(SCAN_B), 0, sm, ls.n_cells, ls);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, sm, n, ls);
    // occupied cells: at most min(n_cells, n); the grids are sized for one
    // pass over the occupied cells of a dense box and stride over the rest
    const int32_t maxbusy = std::min(ls.n_cells, n);
    hipLaunchKernelGGL(k_cellsort, dim3(std::min((maxbusy + 3) / 4, 2048)), dim3(256), 0, sm,
                       pos, reps, tp, ls, st, bs.mirror_sel, bs.step_off);
    // candidate classes rounded up to 1, 2, 4 or 8 (one class: no per-class appends)
    const int nc = bs.want_cand ? ls.ncls : 1;
    const dim3 grid(std::min(maxbusy, LGRID)), block(64 * LB);
    if (nc <= 1)
        hipLaunchKernelGGL(k_lists<1>, grid, block, 0, sm, ls.n_cells, reps, cell_rep, pos, tp, ls, bs, st);
    else if (nc <= 2)
        hipLaunchKernelGGL(k_lists<2>, grid, block, 0, sm, ls.n_cells, reps, cell_rep, pos, tp, ls, bs, st);
    else if (nc <= 4)
        hipLaunchKernelGGL(k_lists<4>, grid, block, 0, sm, ls.n_cells, reps, cell_rep, pos, tp, ls, bs, st);
    else
        hipLaunchKernelGGL(k_lists<8>, grid, block, 0, sm, ls.n_cells, reps, cell_rep, pos, tp, ls, bs, st);
}

}  // namespace bnc
