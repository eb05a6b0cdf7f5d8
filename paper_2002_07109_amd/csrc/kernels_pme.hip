// Reciprocal-space Ewald by smooth particle-mesh Ewald (Sec. V: the
// reciprocal part of the Coulomb sum; Essmann et al., J. Chem. Phys. 103,
// 8577 (1995)).  One periodic box; FP64 throughout.
//
//   spread:   Q(l) = sum_i q_i prod_c M_n(u_ic - l_c), u = K x / L, summed
//             per mesh brick in LDS as 64-bit integers in fixed point (2^k:
//             no overflow, and the sum does not depend on the order of the
//             atomics, so every run gives the same bits)
//   FFT:      F(Q)(k) = sum_l Q(l) exp(+2 pi i k.l / K), one kernel per axis
//   convolve: F(Q)(k) *= theta(k) = k_e/(pi V) exp(-pi^2 m^2/alpha^2)/m^2 B(k),
//             fused with the last forward and the first backward axis
//   FFT back: phi(l) = Re sum_k ... exp(-2 pi i k.l / K)
//   gather:   dE/dx_ic = q_i sum_l phi(l) dQ_i(l)/dx_ic, plus the gradient of
//             the excluded pairs' correction -k_e q_i q_j erf(alpha r)/r
#include "bounce_kernels.hpp"

namespace bnc {

// B-spline weights of one coordinate: for the fraction f = u - floor(u), the
// values M_n(f + j) and (D) derivatives M_n'(f + j), j = 0..n-1, by the order
// recursion M_k(x) = (x M_{k-1}(x) + (k - x) M_{k-1}(x - 1)) / (k - 1)
// applied to the whole array at once (grid point of weight j: floor(u) - j)
template <int n, bool D>
__device__ __forceinline__ void spline_weights(double f, double *w, double *dw)
{
    double a[n];
    a[0] = f;
    a[1] = 1.0 - f;                           // order 2
#pragma unroll
    for (int j = 2; j < n; ++j) a[j] = 0.0;
#pragma unroll
    for (int k = 3; k <= n; ++k) {
        if (D && k == n)                      // derivatives from order n - 1
#pragma unroll
            for (int j = 0; j < n; ++j) dw[j] = (j < n - 1 ? a[j] : 0.0) - (j > 0 ? a[j - 1] : 0.0);
        double prev = 0.0;
#pragma unroll
        for (int j = 0; j < k; ++j) {
            const double cur = j < k - 1 ? a[j] : 0.0;
            a[j] = ((f + j) * cur + ((double)k - f - j) * prev) / (double)(k - 1);
            prev = cur;
        }
    }
#pragma unroll
    for (int j = 0; j < n; ++j) w[j] = a[j];
}

// mesh coordinate of a position: u = K x / L with x wrapped into [0, L);
// fl = floor(u) reduced into [0, K) (the wrapped x may round to L or to just
// below 0), f = u - floor(u)
__device__ __forceinline__ void grid_coord(double x, double L, int K, int &fl, double &f)
{
    const double xw = x - L * floor(x / L);
    const double u = (double)K * xw / L;
    const double flr = floor(u);
    f = u - flr;
    fl = (int)flr;
    if (fl >= K) fl -= K;
    if (fl < 0) fl += K;
}

__device__ __forceinline__ const double4 *pme_mirror(const ListSet &ls, const PmeArgs &pa)
{
    const int32_t par = pa.mirror_sel >= 0 ? pa.mirror_sel : (int32_t)((pa.st->step + pa.step_off) & 1);
    return ls.x[par];
}

// Owner-computes bricks.  The spread and the gather give each workgroup a
// brick of mesh points, P <= l < P + B on every axis (B = SB for the spread,
// GB for the gather, or K along an axis with fewer points).
// The atoms a brick needs have u = K x / L in [P, P + B + hi) on every axis
// (hi = n - 1 for the spread: an atom at u reaches the points floor(u) - j,
// j < n; hi = 0 for the gather, which takes the atoms whose floor(u) lies in
// the brick).  They come from the list cells that overlap that slab widened by
// the skin margin (an atom is at most s/2 from the cell it was listed in);
// the atoms of a (c0, c1) row of cells are contiguous in sorted order, the
// rows' runs are laid end to end, and the workgroup's NT threads take NT
// candidates at a time, so their loads are all in flight together.
constexpr int SB = 8;                 // brick edge of the spread
constexpr int GB = 8;                 // brick edge of the gather
constexpr int ST = 512;               // threads of a spread workgroup
constexpr int GT = 256;               // threads of a gather workgroup
constexpr int BROWS = 256;            // most cell rows per batch (one per thread)
constexpr int MAXNW = ST / 64;

struct Brick {
    int B[3], P[3];
};

template <int BE>
__device__ __forceinline__ Brick brick_of(const PmeArgs &pa, int64_t bid)
{
    Brick bk;
    for (int c = 2; c >= 0; --c) {
        bk.B[c] = pa.K[c] < BE ? pa.K[c] : BE;
        const int nb = pa.K[c] / bk.B[c];
        bk.P[c] = (int)(bid % nb) * bk.B[c];
        bid /= nb;
    }
    return bk;
}

struct WalkLds {
    int32_t seg_s[2 * BROWS], seg_p[2 * BROWS];
    int wsum[MAXNW];
};

// body(s) for each candidate (s = its sorted slot, or -1 for a thread without
// one), NT per call; every thread of the workgroup makes the same calls, so
// body may synchronise the workgroup.
template <int NT, class F>
__device__ __forceinline__ void walk_candidates(const ListSet &ls, const PmeArgs &pa, const Brick &bk, int hi,
                                                WalkLds &wl, F &&body)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int lo[3], cnt[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int nc = pa.ncell[c];
        const double h = pa.box[c] / (double)pa.K[c];
        const double xl = (double)bk.P[c] * h - pa.margin, xh = (double)(bk.P[c] + bk.B[c] + hi) * h + pa.margin;
        int a = (int)floor(xl / pa.cw[c]);
        const int b = (int)floor(xh / pa.cw[c]);
        int m = b - a + 1;
        if (m >= nc) {
            a = 0;
            m = nc;
        } else {
            a %= nc;
            if (a < 0) a += nc;
        }
        lo[c] = a;
        cnt[c] = m;
    }
    const int nrow = cnt[0] * cnt[1];
    const int n2 = pa.ncell[2];
    constexpr int ROWS = NT < BROWS ? NT : BROWS;
    for (int rb = 0; rb < nrow; rb += ROWS) {
        const int nr = nrow - rb < ROWS ? nrow - rb : ROWS;
        // this thread's row: the run of cells lo2 .. up to the row's end, then the wrapped part
        int32_t s0 = 0, s1 = 0, len0 = 0, len1 = 0;
        if (tid < nr) {
            const int pr = rb + tid;
            const int c0 = (lo[0] + pr / cnt[1]) % pa.ncell[0], c1 = (lo[1] + pr % cnt[1]) % pa.ncell[1];
            const int rowbase = (c0 * pa.ncell[1] + c1) * n2;
            const int e2 = lo[2] + cnt[2];
            s0 = ls.cell_start[rowbase + lo[2]];
            len0 = ls.cell_start[rowbase + (e2 < n2 ? e2 : n2)] - s0;
            if (e2 > n2) {
                s1 = ls.cell_start[rowbase];
                len1 = ls.cell_start[rowbase + e2 - n2] - s1;
            }
        }
        // exclusive scan of the run lengths over the threads
        int v = len0 + len1;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(v, o, 64);
            if (lane >= o) v += y;
        }
        if (lane == 63) wl.wsum[wv] = v;
        __syncthreads();
        int off = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            off += w < wv ? wl.wsum[w] : 0;
            total += wl.wsum[w];
        }
        const int excl = off + v - (len0 + len1);
        if (tid < nr) {
            wl.seg_s[2 * tid] = s0;
            wl.seg_s[2 * tid + 1] = s1;
            wl.seg_p[2 * tid] = excl;
            wl.seg_p[2 * tid + 1] = excl + len0;
        }
        __syncthreads();
        for (int cb = 0; cb < total; cb += NT) {
            const int idx = cb + tid;
            int32_t s = -1;
            if (idx < total) {
                // the run holding idx: the last k with seg_p[k] <= idx (empty runs share a start)
                int a = 0, b = 2 * nr - 1;
                while (a < b) {
                    const int mid = (a + b + 1) >> 1;
                    if (wl.seg_p[mid] <= idx) a = mid;
                    else b = mid - 1;
                }
                s = wl.seg_s[a] + (idx - wl.seg_p[a]);
            }
            body(s);
        }
        __syncthreads();
    }
}

// compaction of the threads with flag set: returns this thread's slot (if
// flag) and the workgroup's count; synchronises the workgroup
template <int NT>
__device__ __forceinline__ int compact_slot(bool flag, int *wq, int &count)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(flag);
    if (lane == 0) wq[wv] = __popcll(bal);
    __syncthreads();
    int off = 0;
    count = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        off += w < wv ? wq[w] : 0;
        count += wq[w];
    }
    return off + __popcll(bal & ((1ull << lane) - 1ull));
}

// Per atom, once per evaluation: floor(u) per axis, the fractions with the
// charge, and the spread weights (axis 0 times q 2^k), weight k of atom s at
// w[k N + s] so that the stores of a wave are contiguous.
template <int NO>
__global__ void __launch_bounds__(256) k_pme_prep(int32_t n, ListSet ls, const double *__restrict__ charge,
                                                  PmeArgs pa, PmeAtoms pm)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double4 x = pme_mirror(ls, pa)[s];
    const double qi = charge[mirror_type(x.w)];
    const double xc[3] = {x.x, x.y, x.z};
    int fl[3];
    double f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        grid_coord(xc[c], pa.box[c], pa.K[c], fl[c], f[c]);
        double wc[NO], dw[NO];
        spline_weights<NO, false>(f[c], wc, dw);
#pragma unroll
        for (int j = 0; j < NO; ++j) pm.w[(int64_t)(c * NO + j) * n + s] = c == 0 ? qi * pa.qscale * wc[j] : wc[j];
    }
    pm.fl[s] = make_int4(fl[0], fl[1], fl[2], 0);
    pm.f[s] = make_double4(f[0], f[1], f[2], qi);
}

// exact round-to-nearest of |v| < 2^51 to an integer: adding 1.5 2^52 leaves
// the integer in the low mantissa bits
__device__ __forceinline__ long long round_small(double v)
{
    const double M = 6755399441055744.0;
    return __double_as_longlong(v + M) - __double_as_longlong(M);
}

// Spread: each candidate that reaches the brick is compacted into LDS with its
// spline weights (charge and scale folded into axis 0), then the threads share
// out the (j0, j1) stencil rows.  The sums are 64-bit integers in fixed point
// (scale 2^k, each term below 2^51 and rounded to nearest), so their value
// does not depend on the order of the LDS atomics; rows of the LDS brick are
// padded to SB + 1 entries so that the rows of one atom fall in different
// banks.  The brick is then stored with plain writes (imaginary part 0), each
// mesh point by the one workgroup that owns it.
template <int NO>
__global__ void __launch_bounds__(ST) k_pme_spread(PmeArgs pa, ListSet ls, PmeAtoms pm, int32_t n,
                                                   double2 *__restrict__ grid)
{
    constexpr int RS = SB + 1;
    __shared__ unsigned long long acc[SB * SB * RS];
    __shared__ WalkLds wl;
    __shared__ double qw[ST][3 * NO];
    __shared__ int qr[ST][3];
    __shared__ int qm[ST];
    __shared__ int wq[ST / 64];
    const int tid = threadIdx.x;
    const Brick bk = brick_of<SB>(pa, blockIdx.x);
    for (int k = tid; k < SB * SB * RS; k += ST) acc[k] = 0ull;
    __syncthreads();
    walk_candidates<ST>(ls, pa, bk, NO - 1, wl, [&](int32_t s) {
        bool touch = false;
        int r[3] = {0, 0, 0}, m[3] = {0, 0, 0};
        if (s >= 0) {
            const int4 fq = pm.fl[s];
            const int flc[3] = {fq.x, fq.y, fq.z};
            touch = true;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int rr = flc[c] - bk.P[c];
                if (rr < 0) rr += pa.K[c];
                int mm = 0;
#pragma unroll
                for (int j = 0; j < NO; ++j) {
                    int t = rr - j;
                    if (t < 0) t += pa.K[c];
                    if (t < bk.B[c]) mm |= 1 << j;
                }
                r[c] = rr;
                m[c] = mm;
                touch = touch && mm != 0;
            }
        }
        int nq;
        const int slot = compact_slot<ST>(touch, wq, nq);
        if (touch) {
#pragma unroll
            for (int k = 0; k < 3 * NO; ++k) qw[slot][k] = pm.w[(int64_t)k * n + s];
#pragma unroll
            for (int c = 0; c < 3; ++c) qr[slot][c] = r[c];
            qm[slot] = m[0] | (m[1] << 8) | (m[2] << 16);
        }
        __syncthreads();
        for (int it = tid; it < nq * NO * NO; it += ST) {
            const int e = it / (NO * NO), j0 = (it / NO) % NO, j1 = it % NO;
            const int mk = qm[e];
            if (!((mk >> j0) & 1) || !((mk >> (8 + j1)) & 1)) continue;
            int t0 = qr[e][0] - j0;
            if (t0 < 0) t0 += pa.K[0];
            int t1 = qr[e][1] - j1;
            if (t1 < 0) t1 += pa.K[1];
            const double w01 = qw[e][j0] * qw[e][NO + j1];
            unsigned long long *row = acc + (t0 * SB + t1) * RS;
            const int r2 = qr[e][2];
#pragma unroll
            for (int j2 = 0; j2 < NO; ++j2) {
                if (!((mk >> (16 + j2)) & 1)) continue;
                int t2 = r2 - j2;
                if (t2 < 0) t2 += pa.K[2];
                atomicAdd(&row[t2], (unsigned long long)round_small(w01 * qw[e][2 * NO + j2]));
            }
        }
        __syncthreads();
    });
    const int nbrick = bk.B[0] * bk.B[1] * bk.B[2];
    for (int k = tid; k < nbrick; k += ST) {
        const int t2 = k % bk.B[2], t1 = (k / bk.B[2]) % bk.B[1], t0 = k / (bk.B[1] * bk.B[2]);
        const int64_t g = ((int64_t)(bk.P[0] + t0) * pa.K[1] + (bk.P[1] + t1)) * pa.K[2] + (bk.P[2] + t2);
        grid[g] = make_double2((double)(long long)acc[(t0 * SB + t1) * RS + t2] * pa.inv_qscale, 0.0);
    }
}

// Radix-2 Stockham transform of lines along one axis, LPB lines of length
// len per workgroup (blockDim = LPB len / 2 = 256, one butterfly per thread
// per pass), in LDS, with the len/2 twiddles exp(sign 2 pi i m / len) in a
// table; sign +1: exp(+2 pi i kl/len).  Lines along the contiguous axis are
// loaded element-fastest, the others line-fastest (neighbouring lines are
// neighbours in memory), so both stay coalesced.
//
// theta != NULL (the last forward axis): after the forward transform each
// point is multiplied by theta (with energy != NULL, the block's sum of
// theta |F(Q)|^2 / 2 taken before that goes to energy[block]), and with
// inverse != 0 the line is transformed back (sign -1) before it is stored.
__device__ __forceinline__ void fft_passes(double2 *&x, double2 *&y, const double2 *tw, int len, int l, int j,
                                           double conj)
{
    const int half = len / 2;
    for (int ns = 1; ns < len; ns *= 2) {
        const double2 *xl = x + l * len;
        double2 *yl = y + l * len;
        const int k = j % ns;
        const double2 t = tw[k * (half / ns)];
        const double cs = t.x, sn = conj * t.y;
        const double2 v0 = xl[j], a = xl[j + half];
        const double2 v1 = make_double2(a.x * cs - a.y * sn, a.x * sn + a.y * cs);
        const int d = (j / ns) * 2 * ns + k;
        yl[d] = make_double2(v0.x + v1.x, v0.y + v1.y);
        yl[d + ns] = make_double2(v0.x - v1.x, v0.y - v1.y);
        __syncthreads();
        double2 *tt = x;
        x = y;
        y = tt;
    }
}

__global__ void __launch_bounds__(256) k_pme_fft(double2 *__restrict__ grid, PmeArgs pa, int ax, double sign,
                                                 const double *__restrict__ theta, double *__restrict__ energy,
                                                 int inverse)
{
    extern __shared__ double2 buf[];
    __shared__ double red[4];
    const int len = pa.K[ax], half = len / 2;
    const int lpb = blockDim.x / half;
    const int64_t stride = ax == 2 ? 1 : (ax == 1 ? pa.K[2] : (int64_t)pa.K[1] * pa.K[2]);
    const int64_t nlines = (int64_t)pa.K[0] * pa.K[1] * pa.K[2] / len;
    const int64_t line0 = (int64_t)blockIdx.x * lpb;
    auto base = [&](int64_t L) -> int64_t {
        if (ax == 2) return L * len;
        if (ax == 1) return (L / pa.K[2]) * (int64_t)pa.K[1] * pa.K[2] + L % pa.K[2];
        return L;                                     // ax == 0: (i1, i2) = L
    };
    double2 *x = buf, *y = buf + lpb * len, *tw = buf + 2 * lpb * len;
    for (int m = threadIdx.x; m < half; m += blockDim.x) {
        double sn, cs;
        sincospi(sign * 2.0 * (double)m / (double)len, &sn, &cs);
        tw[m] = make_double2(cs, sn);
    }
    for (int t = threadIdx.x; t < lpb * len; t += blockDim.x) {
        const int l = ax == 2 ? t / len : t % lpb, e = ax == 2 ? t % len : t / lpb;
        const int64_t L = line0 + l;
        x[l * len + e] = L < nlines ? grid[base(L) + e * stride] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int l = threadIdx.x / half, j = threadIdx.x % half;
    fft_passes(x, y, tw, len, l, j, 1.0);
    if (theta) {
        double e = 0.0;
        for (int t = threadIdx.x; t < lpb * len; t += blockDim.x) {
            const int ll = ax == 2 ? t / len : t % lpb, el = ax == 2 ? t % len : t / lpb;
            const int64_t L = line0 + ll;
            if (L >= nlines) continue;
            const double th = theta[base(L) + el * stride];
            const double2 g = x[ll * len + el];
            e += 0.5 * th * (g.x * g.x + g.y * g.y);
            x[ll * len + el] = make_double2(g.x * th, g.y * th);
        }
        if (energy) {
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) e += __shfl_xor(e, m, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
        }
        __syncthreads();
        if (energy && threadIdx.x == 0) energy[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
        if (inverse) fft_passes(x, y, tw, len, l, j, -1.0);
    }
    for (int t = threadIdx.x; t < lpb * len; t += blockDim.x) {
        const int ll = ax == 2 ? t / len : t % lpb, e = ax == 2 ? t % len : t / lpb;
        const int64_t L = line0 + ll;
        if (L < nlines) grid[base(L) + e * stride] = x[ll * len + e];
    }
}

static int fft_lines_per_block(int len)
{
    return len / 2 >= 256 ? 1 : 512 / len;
}

int64_t pme_energy_parts(const PmeArgs &pa)
{
    const int64_t nlines = (int64_t)pa.K[0] * pa.K[1];
    const int lpb = fft_lines_per_block(pa.K[2]);
    return (nlines + lpb - 1) / lpb;
}

// dE/dx of the mesh energy and of the excluded pairs' correction, for the
// atoms whose floor(u) lies in the workgroup's brick (each atom has one such
// brick).  The brick and the n - 1 mesh points below it on every axis (the
// points its atoms' stencils reach) are staged in LDS; owned candidates are
// queued and taken GT at a time, one thread per atom.  out[s] (sorted order)
// or out[g] (caller order).
template <int NO>
__device__ __forceinline__ void gather_atom(int32_t s, const double4 *X, const PmeAtoms &pm, const ListSet &ls,
                                            const double *pos, const double *charge, const Topo &tp,
                                            const PmeArgs &pa, const Brick &bk, const double *ph,
                                            double *out, int32_t out_global, int32_t accumulate)
{
    const int4 fq = pm.fl[s];
    const double4 fx = pm.f[s];
    const double qi = fx.w;
    const int flc[3] = {fq.x, fq.y, fq.z};
    const double fc[3] = {fx.x, fx.y, fx.z};
    int r[3];
    double w[3][NO], dw[3][NO];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        spline_weights<NO, true>(fc[c], w[c], dw[c]);
        r[c] = flc[c] - bk.P[c];
        if (r[c] < 0) r[c] += pa.K[c];
    }
    const double4 x = X[s];
    const double xc[3] = {x.x, x.y, x.z};
    const int E1 = bk.B[1] + NO - 1, E2 = bk.B[2] + NO - 1;
    // separable sums: g0 = sum dw0 w1 w2 phi, g1 = sum w0 dw1 w2 phi, g2 = sum w0 w1 dw2 phi
    double g[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j0 = 0; j0 < NO; ++j0) {
        double t = 0.0, u = 0.0, v = 0.0;
#pragma unroll
        for (int j1 = 0; j1 < NO; ++j1) {
            const double *row = ph + ((r[0] + NO - 1 - j0) * E1 + (r[1] + NO - 1 - j1)) * E2 + (r[2] + NO - 1);
            double sw = 0.0, sd = 0.0;
#pragma unroll
            for (int j2 = 0; j2 < NO; ++j2) {
                const double p = row[-j2];
                sw += w[2][j2] * p;
                sd += dw[2][j2] * p;
            }
            t += w[1][j1] * sw;
            u += dw[1][j1] * sw;
            v += w[1][j1] * sd;
        }
        g[0] += dw[0][j0] * t;
        g[1] += w[0][j0] * u;
        g[2] += w[0][j0] * v;
    }
    for (int c = 0; c < 3; ++c) g[c] *= qi * (double)pa.K[c] / pa.box[c];
    // excluded partners: -k_e q_i q_j erf(alpha r)/r (minimum image)
    const int32_t gi = ls.sinfo[s].x;
    for (int32_t e = tp.excl_ptr[gi]; e < tp.excl_ptr[gi + 1]; ++e) {
        const int32_t gj = tp.excl_idx[e];
        double d[3];
        for (int c = 0; c < 3; ++c) {
            d[c] = xc[c] - pos[3 * (int64_t)gj + c];
            d[c] = d[c] - pa.box[c] * rint(d[c] * pa.inv_box[c]);
        }
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double rr = sqrt(r2), ar = pa.alpha * rr;
        const double qq = KE * qi * charge[tp.type[gj]];
        const double dfdr = (TWO_OVER_SQRTPI * pa.alpha * exp(-ar * ar) * rr - erf(ar)) / r2;
        for (int c = 0; c < 3; ++c) g[c] -= qq * dfdr * d[c] / rr;
    }
    double *o = out + 3 * (int64_t)(out_global ? gi : s);
    for (int c = 0; c < 3; ++c) o[c] = accumulate ? o[c] + g[c] : g[c];
}

template <int NO>
__global__ void __launch_bounds__(GT) k_pme_gather(ListSet ls, const double *__restrict__ pos,
                                                   const double *__restrict__ charge, Topo tp, PmeArgs pa,
                                                   PmeAtoms pm, const double2 *__restrict__ grid,
                                                   double *__restrict__ out, int32_t out_global, int32_t accumulate)
{
    constexpr int E = GB + NO - 1;
    __shared__ double ph[E * E * E];
    __shared__ WalkLds wl;
    __shared__ int32_t own[2 * GT];
    __shared__ int wq[GT / 64];
    const int tid = threadIdx.x;
    const Brick bk = brick_of<GB>(pa, blockIdx.x);
    const int E0 = bk.B[0] + NO - 1, E1 = bk.B[1] + NO - 1, E2 = bk.B[2] + NO - 1;
    // local a_c <-> mesh point (P_c - (n - 1) + a_c) mod K_c
    for (int k = tid; k < E0 * E1 * E2; k += GT) {
        const int a2 = k % E2, a1 = (k / E2) % E1, a0 = k / (E1 * E2);
        int l[3] = {bk.P[0] - (NO - 1) + a0, bk.P[1] - (NO - 1) + a1, bk.P[2] - (NO - 1) + a2};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            l[c] %= pa.K[c];
            if (l[c] < 0) l[c] += pa.K[c];
        }
        ph[k] = grid[((int64_t)l[0] * pa.K[1] + l[1]) * pa.K[2] + l[2]].x;
    }
    __syncthreads();
    const double4 *X = pme_mirror(ls, pa);
    int queued = 0;                       // uniform: owned atoms waiting in own[]
    walk_candidates<GT>(ls, pa, bk, 0, wl, [&](int32_t s) {
        bool mine = false;
        if (s >= 0) {
            const int4 fq = pm.fl[s];
            const int flc[3] = {fq.x, fq.y, fq.z};
            mine = true;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                int rr = flc[c] - bk.P[c];
                if (rr < 0) rr += pa.K[c];
                mine = mine && rr < bk.B[c];
            }
        }
        int nq;
        const int slot = compact_slot<GT>(mine, wq, nq);
        if (mine) own[queued + slot] = s;
        queued += nq;
        __syncthreads();
        if (queued >= GT) {               // a full round: every thread takes one atom
            gather_atom<NO>(own[tid], X, pm, ls, pos, charge, tp, pa, bk, ph, out, out_global, accumulate);
            const int rest = queued - GT;
            const int moved = tid < rest ? own[GT + tid] : 0;
            __syncthreads();
            if (tid < rest) own[tid] = moved;
            queued = rest;
            __syncthreads();
        }
    });
    if (tid < queued)
        gather_atom<NO>(own[tid], X, pm, ls, pos, charge, tp, pa, bk, ph, out, out_global, accumulate);
}

void launch_pme(hipStream_t sm, int32_t n, const ListSet &ls, const double *pos, const double *charge,
                const Topo &tp, const PmeArgs &pa, const PmeAtoms &pm, double2 *grid, const double *theta,
                double *out, int32_t out_global, int32_t accumulate, double *energy_parts)
{
    if (n <= 0) return;
    int64_t nbricks = 1, gbricks = 1;
    for (int c = 0; c < 3; ++c) {
        nbricks *= pa.K[c] / (pa.K[c] < SB ? pa.K[c] : SB);
        gbricks *= pa.K[c] / (pa.K[c] < GB ? pa.K[c] : GB);
    }
    const dim3 gs((unsigned)nbricks), bs(ST), gg((unsigned)gbricks), bg(GT), gp((n + 255) / 256), bp(256);
    switch (pa.order) {
        case 4:
            hipLaunchKernelGGL(k_pme_prep<4>, gp, bp, 0, sm, n, ls, charge, pa, pm);
            hipLaunchKernelGGL(k_pme_spread<4>, gs, bs, 0, sm, pa, ls, pm, n, grid);
            break;
        case 6:
            hipLaunchKernelGGL(k_pme_prep<6>, gp, bp, 0, sm, n, ls, charge, pa, pm);
            hipLaunchKernelGGL(k_pme_spread<6>, gs, bs, 0, sm, pa, ls, pm, n, grid);
            break;
        default:
            hipLaunchKernelGGL(k_pme_prep<5>, gp, bp, 0, sm, n, ls, charge, pa, pm);
            hipLaunchKernelGGL(k_pme_spread<5>, gs, bs, 0, sm, pa, ls, pm, n, grid);
            break;
    }
    const int64_t KK = (int64_t)pa.K[0] * pa.K[1] * pa.K[2];
    auto fft = [&](int ax, double sign, const double *th, double *en, int inv) {
        const int len = pa.K[ax];
        const int lpb = fft_lines_per_block(len);
        const int64_t nlines = KK / len;
        const size_t lds = sizeof(double2) * ((size_t)2 * lpb * len + len / 2);
        hipLaunchKernelGGL(k_pme_fft, dim3((unsigned)((nlines + lpb - 1) / lpb)), dim3(lpb * len / 2), lds, sm,
                           grid, pa, ax, sign, th, en, inv);
    };
    fft(0, 1.0, nullptr, nullptr, 0);
    fft(1, 1.0, nullptr, nullptr, 0);
    fft(2, 1.0, theta, energy_parts, out ? 1 : 0);      // forward, theta, and back along the last axis
    if (!out) return;
    fft(1, -1.0, nullptr, nullptr, 0);
    fft(0, -1.0, nullptr, nullptr, 0);
    switch (pa.order) {
        case 4: hipLaunchKernelGGL(k_pme_gather<4>, gg, bg, 0, sm, ls, pos, charge, tp, pa, pm, grid, out,
                                   out_global, accumulate); break;
        case 6: hipLaunchKernelGGL(k_pme_gather<6>, gg, bg, 0, sm, ls, pos, charge, tp, pa, pm, grid, out,
                                   out_global, accumulate); break;
        default: hipLaunchKernelGGL(k_pme_gather<5>, gg, bg, 0, sm, ls, pos, charge, tp, pa, pm, grid, out,
                                    out_global, accumulate); break;
    }
}

// per atom: half the excluded pairs' correction -k_e q_i q_j erf(alpha r)/r
// over its exclusion list (each pair is seen from both atoms), caller order
__global__ void k_pme_excl_energy(int32_t n, const double *__restrict__ pos,
                                  const double *__restrict__ charge, Topo tp, PmeArgs pa,
                                  double *__restrict__ atom_out)
{
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const double qi = charge[tp.type[g]];
    double e = 0.0;
    for (int32_t k = tp.excl_ptr[g]; k < tp.excl_ptr[g + 1]; ++k) {
        const int32_t j = tp.excl_idx[k];
        double r2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            double d = pos[3 * (int64_t)g + c] - pos[3 * (int64_t)j + c];
            d = d - pa.box[c] * rint(d * pa.inv_box[c]);
            r2 += d * d;
        }
        const double r = sqrt(r2);
        e -= 0.5 * KE * qi * charge[tp.type[j]] * erf(pa.alpha * r) / r;
    }
    atom_out[g] = e;
}

void launch_pme_excl_energy(hipStream_t sm, int32_t n, const double *pos, const double *charge,
                            const Topo &tp, const PmeArgs &pa, double *atom_out)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pme_excl_energy, dim3((n + 255) / 256), dim3(256), 0, sm, n, pos, charge, tp,
                       pa, atom_out);
}

}  // namespace bnc
