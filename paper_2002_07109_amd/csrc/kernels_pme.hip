// Reciprocal-space Ewald by smooth particle-mesh Ewald (Sec. V: the
// reciprocal part of the Coulomb sum; Essmann et al., J. Chem. Phys. 103,
// 8577 (1995)).  One periodic box; FP64 throughout.
//
//   spread:   Q(l) = sum_i q_i prod_c M_n(u_ic - l_c), u = K x / L, summed
//             by 64-bit integer atomics in fixed point (2^k with k set so that
//             sum_i |q_i| 2^k < 2^62: no overflow, and the sum does not depend
//             on the order of the atomics, so every run gives the same bits)
//   FFT:      F(Q)(k) = sum_l Q(l) exp(+2 pi i k.l / K), one kernel per axis
//   convolve: F(Q)(k) *= theta(k) = k_e/(pi V) exp(-pi^2 m^2/alpha^2)/m^2 B(k)
//   FFT back: phi(l) = Re sum_k ... exp(-2 pi i k.l / K)
//   gather:   dE/dx_ic = q_i sum_l phi(l) dQ_i(l)/dx_ic, plus the gradient of
//             the excluded pairs' correction -k_e q_i q_j erf(alpha r)/r
#include "bounce_kernels.hpp"

namespace bnc {

// B-spline weights of one coordinate: for the fraction f = u - floor(u), the
// values M_n(f + j) and derivatives M_n'(f + j), j = 0..n-1, by the order
// recursion M_k(x) = (x M_{k-1}(x) + (k - x) M_{k-1}(x - 1)) / (k - 1)
// applied to the whole array at once (grid point of weight j: floor(u) - j)
template <int n>
__device__ __forceinline__ void spline_weights(double f, double *w, double *dw)
{
    double a[n];
    a[0] = f;
    a[1] = 1.0 - f;                           // order 2
#pragma unroll
    for (int j = 2; j < n; ++j) a[j] = 0.0;
#pragma unroll
    for (int k = 3; k <= n; ++k) {
        if (k == n)                           // derivatives from order n - 1
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

__device__ __forceinline__ void grid_coord(double x, double L, int K, int &fl, double &f)
{
    const double xw = x - L * floor(x / L);
    const double u = (double)K * xw / L;
    const double flr = floor(u);
    f = u - flr;
    fl = (int)flr;
}

__global__ void k_pme_zero(double2 *__restrict__ grid, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) grid[k] = make_double2(0.0, 0.0);
}

__device__ __forceinline__ const double4 *pme_mirror(const ListSet &ls, const PmeArgs &pa)
{
    const int32_t par = pa.mirror_sel >= 0 ? pa.mirror_sel : (int32_t)((pa.st->step + pa.step_off) & 1);
    return ls.x[par];
}

// one thread per atom (sorted slot); charges from the mirror's type word;
// each term rounded to the nearest multiple of 2^-k and added as an integer
// into the real part of its grid point
template <int NO>
__global__ void k_pme_spread(int32_t n, ListSet ls, const double *__restrict__ charge, PmeArgs pa,
                             double2 *__restrict__ grid)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double4 x = pme_mirror(ls, pa)[s];
    const double qi = charge[mirror_type(x.w)];
    int fl[3];
    double w[3][NO], dw[3][NO];
    const double xc[3] = {x.x, x.y, x.z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double f;
        grid_coord(xc[c], pa.box[c], pa.K[c], fl[c], f);
        spline_weights<NO>(f, w[c], dw[c]);
    }
#pragma unroll
    for (int j0 = 0; j0 < NO; ++j0) {
        const int l0 = (fl[0] - j0 + pa.K[0]) % pa.K[0];
#pragma unroll
        for (int j1 = 0; j1 < NO; ++j1) {
            const int l1 = (fl[1] - j1 + pa.K[1]) % pa.K[1];
            const double w01 = qi * w[0][j0] * w[1][j1];
            double2 *row = grid + ((int64_t)l0 * pa.K[1] + l1) * pa.K[2];
#pragma unroll
            for (int j2 = 0; j2 < NO; ++j2) {
                const int l2 = (fl[2] - j2 + pa.K[2]) % pa.K[2];
                const long long t = __double2ll_rn(w01 * w[2][j2] * pa.qscale);
                atomicAdd(reinterpret_cast<unsigned long long *>(&row[l2].x), (unsigned long long)t);
            }
        }
    }
}

// Radix-2 Stockham transform of lines along one axis, LPB lines of length
// len per workgroup (blockDim = LPB len / 2, one butterfly per thread per
// pass), in LDS; sign +1: exp(+2 pi i kl/len).  Lines along the contiguous
// axis are loaded element-fastest, the others line-fastest (neighbouring
// lines are neighbours in memory), so both stay coalesced.  from_fixed: the
// real parts hold the spread's fixed-point integers (first pass only).
__global__ void k_pme_fft(double2 *__restrict__ grid, PmeArgs pa, int ax, double sign, int from_fixed)
{
    extern __shared__ double2 buf[];
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
    double2 *x = buf, *y = buf + lpb * len;
    for (int t = threadIdx.x; t < lpb * len; t += blockDim.x) {
        const int l = ax == 2 ? t / len : t % lpb, e = ax == 2 ? t % len : t / lpb;
        const int64_t L = line0 + l;
        double2 v = L < nlines ? grid[base(L) + e * stride] : make_double2(0.0, 0.0);
        if (from_fixed) v = make_double2((double)__double_as_longlong(v.x) * pa.inv_qscale, 0.0);
        x[l * len + e] = v;
    }
    __syncthreads();
    const int l = threadIdx.x / half, j = threadIdx.x % half;
    for (int ns = 1; ns < len; ns *= 2) {
        const double2 *xl = x + l * len;
        double2 *yl = y + l * len;
        const int k = j % ns;
        double sn, cs;
        sincospi(sign * (double)k / (double)ns, &sn, &cs);
        const double2 v0 = xl[j], a = xl[j + half];
        const double2 v1 = make_double2(a.x * cs - a.y * sn, a.x * sn + a.y * cs);
        const int d = (j / ns) * 2 * ns + k;
        yl[d] = make_double2(v0.x + v1.x, v0.y + v1.y);
        yl[d + ns] = make_double2(v0.x - v1.x, v0.y - v1.y);
        __syncthreads();
        double2 *t = x;
        x = y;
        y = t;
    }
    for (int t = threadIdx.x; t < lpb * len; t += blockDim.x) {
        const int ll = ax == 2 ? t / len : t % lpb, e = ax == 2 ? t % len : t / lpb;
        const int64_t L = line0 + ll;
        if (L < nlines) grid[base(L) + e * stride] = x[ll * len + e];
    }
}

// F(Q)(k) *= theta(k); with energy != NULL also the per-block partial sums of
// theta |F(Q)|^2 / 2 (before the multiplication)
__global__ void __launch_bounds__(256) k_pme_convolve(double2 *__restrict__ grid,
                                                       const double *__restrict__ theta, int64_t n,
                                                       double *__restrict__ energy)
{
    __shared__ double red[4];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (k < n) {
        const double2 g = grid[k];
        const double th = theta[k];
        e = 0.5 * th * (g.x * g.x + g.y * g.y);
        grid[k] = make_double2(g.x * th, g.y * th);
    }
    if (!energy) return;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) e += __shfl_xor(e, m, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) energy[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// dE/dx of the mesh energy and of the excluded pairs' correction for the
// atom at sorted slot s; out[s] (sorted order) or out[g] (caller order)
template <int NO>
__global__ void k_pme_gather(int32_t n, ListSet ls, const double *__restrict__ pos,
                             const double *__restrict__ charge, Topo tp, PmeArgs pa,
                             const double2 *__restrict__ grid, double *__restrict__ out,
                             int32_t out_global, int32_t accumulate)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double4 x = pme_mirror(ls, pa)[s];
    const double qi = charge[mirror_type(x.w)];
    int fl[3];
    double w[3][NO], dw[3][NO];
    const double xc[3] = {x.x, x.y, x.z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double f;
        grid_coord(xc[c], pa.box[c], pa.K[c], fl[c], f);
        spline_weights<NO>(f, w[c], dw[c]);
    }
    double g[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j0 = 0; j0 < NO; ++j0) {
        const int l0 = (fl[0] - j0 + pa.K[0]) % pa.K[0];
#pragma unroll
        for (int j1 = 0; j1 < NO; ++j1) {
            const int l1 = (fl[1] - j1 + pa.K[1]) % pa.K[1];
            const double2 *row = grid + ((int64_t)l0 * pa.K[1] + l1) * pa.K[2];
#pragma unroll
            for (int j2 = 0; j2 < NO; ++j2) {
                const double phi = row[(fl[2] - j2 + pa.K[2]) % pa.K[2]].x;
                g[0] += phi * dw[0][j0] * w[1][j1] * w[2][j2];
                g[1] += phi * w[0][j0] * dw[1][j1] * w[2][j2];
                g[2] += phi * w[0][j0] * w[1][j1] * dw[2][j2];
            }
        }
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
        const double r = sqrt(r2), ar = pa.alpha * r;
        const double qq = KE * qi * charge[tp.type[gj]];
        const double dfdr = (TWO_OVER_SQRTPI * pa.alpha * exp(-ar * ar) * r - erf(ar)) / r2;
        for (int c = 0; c < 3; ++c) g[c] -= qq * dfdr * d[c] / r;
    }
    double *o = out + 3 * (int64_t)(out_global ? gi : s);
    for (int c = 0; c < 3; ++c) o[c] = accumulate ? o[c] + g[c] : g[c];
}

void launch_pme(hipStream_t sm, int32_t n, const ListSet &ls, const double *pos, const double *charge,
                const Topo &tp, const PmeArgs &pa, double2 *grid, const double *theta, double *out,
                int32_t out_global, int32_t accumulate, double *energy_parts)
{
    if (n <= 0) return;
    const int64_t KK = (int64_t)pa.K[0] * pa.K[1] * pa.K[2];
    hipLaunchKernelGGL(k_pme_zero, dim3((KK + 255) / 256), dim3(256), 0, sm, grid, KK);
    const dim3 ga((n + 127) / 128), ba(128);
    switch (pa.order) {
        case 4: hipLaunchKernelGGL(k_pme_spread<4>, ga, ba, 0, sm, n, ls, charge, pa, grid); break;
        case 6: hipLaunchKernelGGL(k_pme_spread<6>, ga, ba, 0, sm, n, ls, charge, pa, grid); break;
        default: hipLaunchKernelGGL(k_pme_spread<5>, ga, ba, 0, sm, n, ls, charge, pa, grid); break;
    }
    auto fft = [&](double sign) {
        for (int ax = 0; ax < 3; ++ax) {
            const int len = pa.K[ax], half = len / 2;
            const int lpb = half >= 256 ? 1 : 256 / half;
            const int64_t nlines = KK / len;
            const size_t lds = 2 * sizeof(double2) * (size_t)lpb * len;
            hipLaunchKernelGGL(k_pme_fft, dim3((nlines + lpb - 1) / lpb), dim3(lpb * half), lds, sm,
                               grid, pa, ax, sign, (int)(sign > 0.0 && ax == 0));
        }
    };
    fft(1.0);
    hipLaunchKernelGGL(k_pme_convolve, dim3((KK + 255) / 256), dim3(256), 0, sm, grid, theta, KK,
                       energy_parts);
    if (!out) return;
    fft(-1.0);
    switch (pa.order) {
        case 4: hipLaunchKernelGGL(k_pme_gather<4>, ga, ba, 0, sm, n, ls, pos, charge, tp, pa, grid, out,
                                   out_global, accumulate); break;
        case 6: hipLaunchKernelGGL(k_pme_gather<6>, ga, ba, 0, sm, n, ls, pos, charge, tp, pa, grid, out,
                                   out_global, accumulate); break;
        default: hipLaunchKernelGGL(k_pme_gather<5>, ga, ba, 0, sm, n, ls, pos, charge, tp, pa, grid,
                                    out, out_global, accumulate); break;
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
