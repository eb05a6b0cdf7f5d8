// Device-side building blocks of the BOUNCE library: the Philox4x64-10
// stream, the shifted-force pair field and the switch, shared by the
// list-build, pair, step and gradient kernels.  gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bnc {

constexpr double KE = 332.0637;        // kcal A / (mol e^2)
constexpr double KB = 0.0019872041;    // kcal / (mol K)
constexpr double ACC = 4.184e-4;       // (kcal/mol/A)/amu -> A/fs^2
constexpr double TWO_OVER_SQRTPI = 1.1283791670955126;
constexpr int MAXT = 8;
// jump bounds as integer weights: 2^WEIGHT_BITS units make the bound of an atom type
constexpr int WEIGHT_BITS = 20;
constexpr double WEIGHT_SLACK = 1e-4;
// row stride of the bound-weight table: (mechanism, partner type) classes per atom type
constexpr int LQW = 2 * MAXT;
// pair-structure histogram: at most this many (type pair, bin) counters
constexpr int RDF_MAX_BINS = 8192;
// smooth-PME B-spline order limit
constexpr int PME_MAX_ORDER = 8;

// latched device conditions
enum : uint32_t {
    ST_CAPACITY = 1u, ST_SKIN = 2u, ST_BOUND = 4u, ST_POISSON = 8u, ST_NONFINITE = 16u,
    ST_GRID = 32u
};

// per-replica geometry of the list grid
struct RepInfo {
    double box[3], inv_box[3];
    double cinv[3];        // periodic: ncell / box
    double cw[3];          // cell edge
    double origin[3];      // droplet grid origin
    double inv_cell;       // droplet: 1 / cell_size
    int32_t ncell[3];
    int32_t periodic;
    int64_t atom_off;
    int32_t n_atoms;
    int32_t cell_off;
    uint64_t key0, key1;   // Philox key (seed, replica)
    // fixed-point position mirror (FP32 pair arithmetic): x = forigin + n funit,
    // finv = 1 / funit; periodic: funit = edge / 2^32, forigin = 0
    double finv[3], forigin[3];
    float funit[3];
    float pad_f;
};

// small device-resident state: step counter, latched status, counters
struct DevState {
    int64_t step;
    int64_t n_events;
    uint32_t status;
    uint32_t far_flag;            // an atom has moved (s/2 - margin)/2 or more since the main
                                  //   list's build: the force rows' far parts may be in range
    uint64_t pad;
};

// jump counters of one replica, held in CNT_SPREAD copies (one 128-byte line
// each) so that the wavefronts' atomic adds spread over many addresses; a read
// sums the copies
constexpr int CNT_SPREAD = 64;
struct RepCounters {
    unsigned long long proposals, accepted, bound_violations, pad[13];
};

struct Event {
    int64_t step;
    int32_t phase, atom, k, partner, accepted, replica;
    int32_t mech, pad;
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): 10 rounds, Weyl key schedule.
// ---------------------------------------------------------------------------
struct U4 { uint64_t x, y, z, w; };

// the full 128-bit product a b as (hi, lo) from four 32 x 32 -> 64 products
// with 64-bit accumulation (each maps to one v_mad_u64_u32); none of the
// partial sums can overflow 64 bits
__device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t t = (uint64_t)a0 * b0;
    const uint64_t u = (uint64_t)a1 * b0 + (t >> 32);
    const uint64_t v = (uint64_t)a0 * b1 + (uint32_t)u;
    const uint64_t w = (uint64_t)a1 * b1 + (u >> 32);
    hi = w + (v >> 32);
    lo = (v << 32) | (uint32_t)t;
}

__device__ __forceinline__ U4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, c0, hi0, lo0);
        mul128(M1, c2, hi1, lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(const RepInfo &ri, int64_t step, int32_t phase, int32_t atom,
                                   uint64_t k)
{
    return philox4x64_10((uint64_t)step, ((uint64_t)(uint32_t)phase << 32) | (uint32_t)atom, k, 0,
                         ri.key0, ri.key1);
}

// uniform in (0,1): top 52 bits plus one half, times 2^-52 (exact)
__device__ __forceinline__ double u01(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

// ---------------------------------------------------------------------------
// Type-pair constants of the shifted-force potential (Lorentz-Berthelot).
// ---------------------------------------------------------------------------
template <typename R>
struct TypePair {
    R qq;      // KE q_a q_b
    R eps4;    // 4 eps_ab
    R sig2;    // sigma_ab^2
    R du_rc;   // u'(rc)
    R u_rc;    // u(rc)
    R pad[3];  // [0]: the Lennard-Jones part of u'(rc), [1]: its Coulomb part
};

struct PairGlobals {
    double alpha;     // Ewald splitting (1/A)
    double r_on, r_off, inv_w;  // switch window and 1/(r'' - r') (Coulomb, or both parts)
    double r_on_v, inv_w_v;     // separate mechanisms: the Lennard-Jones window
    double r_short;             // the short-range force's reach: r'' (the larger one when split)
    double r_cut;
    int32_t coulomb;  // 0 bare, 1 erfc
    int32_t n_types;
    int32_t split;    // 1: separate Coulomb and Lennard-Jones jump mechanisms
    int32_t pad_i;
};

// Coulomb kernel g(r) and g'(r)
template <typename R>
__device__ __forceinline__ void coul_g(R r, R rinv, R alpha, int coulomb, R &g, R &dg);

// FP32: erfc(x) = exp(-x^2) Q(t), t = 1 / (1 + 0.4 x), with Q the degree-9
// polynomial fitted to erfc(x) exp(x^2) on 0 <= x <= 8 (relative error 1.9e-8;
// about 4e-7 in FP32; paper_2002_07109_amd/fit_erfc.py computes the
// coefficients).  This returns Q; the caller multiplies by exp(-x^2), which it
// shares with g'(r).  Beyond x = 8 that product is below 1e-27.
__device__ __forceinline__ float erfcx_fit(float x)
{
    const float t = __builtin_amdgcn_rcpf(fmaf(0.4f, x, 1.0f));
    float q = 0.020177293568849564f;
    q = fmaf(q, t, -0.028550047427415848f);
    q = fmaf(q, t, -0.17227867245674133f);
    q = fmaf(q, t, 0.4207404553890228f);
    q = fmaf(q, t, -0.18945305049419403f);
    q = fmaf(q, t, 0.33385446667671204f);
    q = fmaf(q, t, 0.15468838810920715f);
    q = fmaf(q, t, 0.23628339171409607f);
    q = fmaf(q, t, 0.22447969019412994f);
    q = fmaf(q, t, 5.809841604786925e-05f);
    return q;
}

template <>
__device__ __forceinline__ void coul_g<float>(float r, float rinv, float alpha, int coulomb,
                                              float &g, float &dg)
{
    if (coulomb) {
        const float ar = alpha * r;
        const float ex = __expf(-ar * ar);
        const float q = erfcx_fit(ar);          // erfc(ar) = ex q
        g = ex * q * rinv;
        dg = -(ex * fmaf(q, rinv, (float)TWO_OVER_SQRTPI * alpha)) * rinv;
    } else {
        g = rinv;
        dg = -rinv * rinv;
    }
}

template <>
__device__ __forceinline__ void coul_g<double>(double r, double rinv, double alpha, int coulomb,
                                               double &g, double &dg)
{
    if (coulomb) {
        double ar = alpha * r;
        double e = erfc(ar);
        double ex = exp(-ar * ar);
        g = e * rinv;
        dg = -(g + TWO_OVER_SQRTPI * alpha * ex) * rinv;
    } else {
        g = rinv;
        dg = -rinv * rinv;
    }
}

template <typename R>
__device__ __forceinline__ R rsqrt_(R x);
template <>
__device__ __forceinline__ float rsqrt_<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double rsqrt_<double>(double x) { return 1.0 / sqrt(x); }

// W'_sf(r) = u'(r) - u'(rc) (requires r < rc); also returns 1/r
template <typename R>
__device__ __forceinline__ R pair_dw(R r2, const TypePair<R> &tp, R alpha, int coulomb, R &r_out,
                                     R &rinv_out)
{
    R rinv = rsqrt_<R>(r2);
    R r = r2 * rinv;
    R g, dg;
    coul_g<R>(r, rinv, alpha, coulomb, g, dg);
    R rinv2 = rinv * rinv;
    R s2 = tp.sig2 * rinv2;
    R s6 = s2 * s2 * s2;
    R dlj = tp.eps4 * (s6 * ((R)6 - (R)12 * s6)) * rinv;
    r_out = r;
    rinv_out = rinv;
    return tp.qq * dg + dlj - tp.du_rc;
}

// the Coulomb and Lennard-Jones parts of W'_sf(r), qq (g'(r) - g'(rc)) and
// LJ'(r) - LJ'(rc) (requires r < rc); also returns r and 1/r
template <typename R>
__device__ __forceinline__ void pair_dw_parts(R r2, const TypePair<R> &tp, R alpha, int coulomb,
                                              R &r_out, R &rinv_out, R &dwc, R &dwv)
{
    R rinv = rsqrt_<R>(r2);
    R r = r2 * rinv;
    R g, dg;
    coul_g<R>(r, rinv, alpha, coulomb, g, dg);
    R rinv2 = rinv * rinv;
    R s2 = tp.sig2 * rinv2;
    R s6 = s2 * s2 * s2;
    R dlj = tp.eps4 * (s6 * ((R)6 - (R)12 * s6)) * rinv;
    r_out = r;
    rinv_out = rinv;
    dwc = tp.qq * dg - tp.pad[1];
    dwv = dlj - tp.pad[0];
}

// quintic smoothstep switch on [r', r'']
template <typename R>
__device__ __forceinline__ R switch_chi(R r, R r_on, R inv_w)
{
    R x = (r - r_on) * inv_w;
    x = x < (R)0 ? (R)0 : (x > (R)1 ? (R)1 : x);
    return x * x * x * ((R)10 + x * ((R)6 * x - (R)15));
}

// FP32 (the pair kernels' hot loop): the clamp to [0, 1] as one median of three
template <>
__device__ __forceinline__ float switch_chi<float>(float r, float r_on, float inv_w)
{
    const float x = __builtin_amdgcn_fmed3f(fmaf(r, inv_w, -r_on * inv_w), 0.0f, 1.0f);
    return x * x * x * fmaf(x, fmaf(6.0f, x, -15.0f), 10.0f);
}

// The sorted position mirror stores (x, y, z, w) with w = 16 id + type, an
// integer exactly representable in FP64, so one 32-byte load gives a partner's
// position, type and caller id.
__device__ __forceinline__ double mirror_w(int32_t id, int32_t type) { return (double)(id * 16 + type); }
__device__ __forceinline__ int32_t mirror_type(double w) { return (int32_t)w & 15; }
__device__ __forceinline__ int32_t mirror_id(double w) { return (int32_t)w >> 4; }

// minimum-image displacement in FP64.  The list-build translation unit is
// compiled without FMA contraction, so there these expressions round exactly
// where written (the list predicate must be reproducible bit for bit).
__device__ __forceinline__ void min_image(const RepInfo &ri, double &dx, double &dy, double &dz)
{
    if (ri.periodic) {
        dx = dx - ri.box[0] * rint(dx * ri.inv_box[0]);
        dy = dy - ri.box[1] * rint(dy * ri.inv_box[1]);
        dz = dz - ri.box[2] * rint(dz * ri.inv_box[2]);
    }
}

// a replica's parameters; with one replica the index is the constant 0, so the
// load is uniform and need not wait for the per-atom replica index
__device__ __forceinline__ RepInfo load_rep(const RepInfo *reps, int single, int32_t rep)
{
    RepInfo r;
    if (single) r = reps[0];
    else r = reps[rep];
    return r;
}

// the periodic box of one replica, held in registers by the pair loops
struct BoxReg {
    double L[3], iL[3];
    int periodic;
    __device__ __forceinline__ explicit BoxReg(const RepInfo &ri)
    {
        periodic = ri.periodic;
        for (int k = 0; k < 3; ++k) { L[k] = ri.box[k]; iL[k] = ri.inv_box[k]; }
    }
    __device__ __forceinline__ void apply(double &dx, double &dy, double &dz) const
    {
        if (periodic) {
            dx = dx - L[0] * rint(dx * iL[0]);
            dy = dy - L[1] * rint(dy * iL[1]);
            dz = dz - L[2] * rint(dz * iL[2]);
        }
    }
};

__device__ __forceinline__ double norm2_exact(double dx, double dy, double dz)
{
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ uint32_t atomic_or_status(DevState *st, uint32_t bits)
{
    return atomicOr(&st->status, bits);
}

}  // namespace bnc
