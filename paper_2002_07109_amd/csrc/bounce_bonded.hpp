// Bonded terms of F_0: E = k (r - r0)^2 per bond, E = k (theta - theta0)^2 per
// angle (vertex in the middle).  Each atom sums the gradient of the terms that
// touch it, so no atomics are needed.
#pragma once
#include "bounce_lists.hpp"

namespace bnc {

// positions in caller order
struct CallerPos {
    const double *p;
    __device__ __forceinline__ void operator()(int32_t g, double x[3]) const
    {
        x[0] = p[3 * (int64_t)g]; x[1] = p[3 * (int64_t)g + 1]; x[2] = p[3 * (int64_t)g + 2];
    }
};

// positions from a sorted mirror
struct MirrorPos {
    const double4 *X;
    const int32_t *inv_perm;
    __device__ __forceinline__ void operator()(int32_t g, double x[3]) const
    {
        double4 v = X[inv_perm[g]];
        x[0] = v.x; x[1] = v.y; x[2] = v.z;
    }
};

template <class PosF>
__device__ __forceinline__ void disp_of(const RepInfo &ri, const PosF &pf, int32_t a, int32_t b,
                                        double d[3])
{
    double xa[3], xb[3];
    pf(a, xa);
    pf(b, xb);
    double dx = xa[0] - xb[0], dy = xa[1] - xb[1], dz = xa[2] - xb[2];
    min_image(ri, dx, dy, dz);
    d[0] = dx; d[1] = dy; d[2] = dz;
}

// gradient on atom g of one bonded term (code = kind << 28 | index)
template <class PosF>
__device__ __forceinline__ void bonded_term_grad(int32_t g, int32_t code, const PosF &pf,
                                                 const RepInfo &ri, const Topo &tp, double out[3])
{
    const int32_t kind = code >> 28, idx = code & 0x0fffffff;
    if (kind == 0) {
        const int32_t a0 = tp.bond_ij[2 * idx], a1 = tp.bond_ij[2 * idx + 1];
        double d[3];
        disp_of(ri, pf, a0, a1, d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double c = 2.0 * tp.bond_kr[2 * idx] * (r - tp.bond_kr[2 * idx + 1]) / r;
        const double sg = (g == a0) ? c : -c;
        out[0] += sg * d[0]; out[1] += sg * d[1]; out[2] += sg * d[2];
    } else {
        const int32_t x = tp.angle_ijk[3 * idx], v = tp.angle_ijk[3 * idx + 1],
                      y = tp.angle_ijk[3 * idx + 2];
        double e1[3], e2[3];
        disp_of(ri, pf, x, v, e1);
        disp_of(ri, pf, y, v, e2);
        const double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        const double l2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        const double il = 1.0 / (l1 * l2);
        double cs = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) * il;
        cs = fmin(1.0, fmax(-1.0, cs));
        const double th = acos(cs);
        const double sn = sqrt(1.0 - cs * cs);
        // dE/dtheta * dtheta/dcos, with dtheta/dcos = -1/sin
        const double w = -2.0 * tp.angle_kt[2 * idx] * (th - tp.angle_kt[2 * idx + 1]) / sn;
        for (int c = 0; c < 3; ++c) {
            const double gx = w * (e2[c] * il - cs * e1[c] / (l1 * l1));
            const double gy = w * (e1[c] * il - cs * e2[c] / (l2 * l2));
            if (g == x) out[c] += gx;
            if (g == y) out[c] += gy;
            if (g == v) out[c] -= gx + gy;
        }
    }
}

// the same gradient from a resolved term e = (code, slot of each atom) of the
// atom at sorted position s, with the positions of the term's atoms given
// (xa, xb, xc: slots e.y, e.z, e.w; xc unused for a bond)
__device__ __forceinline__ void bonded_slot_grad_pos(int32_t s, int4 e, const double4 &xa,
                                                     const double4 &xb, const double4 &xc,
                                                     const RepInfo &ri, const Topo &tp, double out[3])
{
    const int32_t kind = e.x >> 28, idx = e.x & 0x0fffffff;
    auto disp = [&](const double4 &p, const double4 &r, double d[3]) {
        double dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z;
        min_image(ri, dx, dy, dz);
        d[0] = dx; d[1] = dy; d[2] = dz;
    };
    if (kind == 0) {
        double d[3];
        disp(xa, xb, d);
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double c = 2.0 * tp.bond_kr[2 * idx] * (r - tp.bond_kr[2 * idx + 1]) / r;
        const double sg = (s == e.y) ? c : -c;
        out[0] += sg * d[0]; out[1] += sg * d[1]; out[2] += sg * d[2];
    } else {
        double e1[3], e2[3];
        disp(xa, xb, e1);
        disp(xc, xb, e2);
        const double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        const double l2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        const double il = 1.0 / (l1 * l2);
        double cs = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) * il;
        cs = fmin(1.0, fmax(-1.0, cs));
        const double th = acos(cs);
        const double sn = sqrt(1.0 - cs * cs);
        // dE/dtheta * dtheta/dcos, with dtheta/dcos = -1/sin
        const double w = -2.0 * tp.angle_kt[2 * idx] * (th - tp.angle_kt[2 * idx + 1]) / sn;
        for (int c = 0; c < 3; ++c) {
            const double gx = w * (e2[c] * il - cs * e1[c] / (l1 * l1));
            const double gy = w * (e1[c] * il - cs * e2[c] / (l2 * l2));
            if (s == e.y) out[c] += gx;
            if (s == e.w) out[c] += gy;
            if (s == e.z) out[c] -= gx + gy;
        }
    }
}

// the same, loading the term's positions from the sorted mirror X
__device__ __forceinline__ void bonded_slot_grad(int32_t s, int4 e, const double4 *X,
                                                 const RepInfo &ri, const Topo &tp, double out[3])
{
    const double4 xa = X[e.y], xb = X[e.z], xc = X[(e.x >> 28) ? e.w : e.y];
    bonded_slot_grad_pos(s, e, xa, xb, xc, ri, tp, out);
}

template <class PosF>
__device__ void bonded_grad_atom(int32_t g, const PosF &pf, const RepInfo &ri, const Topo &tp,
                                 double out[3])
{
    for (int32_t k = tp.bt_ptr[g]; k < tp.bt_ptr[g + 1]; ++k)
        bonded_term_grad(g, tp.bt[k], pf, ri, tp, out);
}

}  // namespace bnc
