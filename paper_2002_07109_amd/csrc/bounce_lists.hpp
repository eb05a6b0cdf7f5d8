// Host/device view of one set of sorted atom arrays and pair lists.
#pragma once
#include "bounce_device.hpp"

namespace bnc {

struct ListSet {
    int32_t *perm;        // sorted position -> caller id
    int32_t *inv_perm;    // caller id -> sorted position
    int32_t *cell_of;     // caller id -> global cell
    int32_t *slot;        // caller id -> arrival slot in its cell
    int32_t *cell_count;  // [n_cells]
    int32_t *cell_start;  // [n_cells + 1]
    int32_t *scan_part;   // [2 ceil(n_cells / 1024)] block sums of the cell-count scan
                          //   and of the occupied-cell count
    int32_t *busy;        // [n_cells + 1] occupied cells: [0] their number, then their
                          //   indices in ascending order
    int2 *sinfo;          // sorted position -> (caller id, replica)
    double4 *x[2];        // sorted positions (x, y, z, type), double-buffered by step parity
    double *q_build;      // [N][3] positions at the build (skin guard)
    int2 *fcnt;           // force list: (near, far) entries of each sorted atom's row
    int32_t *flist;       // [N][fcap] sorted partner positions: the near entries fill
                          //   the row from the front, the far ones from the back
                          //   (each part ascending in canonical order from its end)
    int32_t *ccnt;        // candidate list (jump partners): [N][ncls] members per class
    int32_t *clist;       // [N][ncls][ccap], each class in canonical order
    int4 *bslot;          // [N][BTMAX] bonded terms of each sorted atom with their
                          //   atoms as sorted positions (x = term code, -1: none); or NULL
    // FP32 pair arithmetic: the positions of x[] again as fixed-point integers
    // (x, y, z, type), one unit = funit of the atom's replica, taken modulo 2^32
    // in a periodic box whose edge is 2^32 units: the difference of two such
    // integers in 32-bit two's complement is the minimum-image displacement,
    // exact to the rounding of the two positions (NULL when not kept)
    int4 *xf[2];
    int32_t fcap, ccap;
    int32_t n_cells;
    int32_t ncls;         // candidate classes: the partner's type (per-type-pair bounds) or one
};

// fixed-point position of an atom on its replica: periodic, round(x / u) mod 2^32
// with u = edge / 2^32; droplet, round((x - origin) / u) with u = grid extent / 2^30
__device__ __forceinline__ int4 fixed_pos(const RepInfo &ri, double x, double y, double z, int32_t type)
{
    const int64_t fx = (int64_t)rint((x - ri.forigin[0]) * ri.finv[0]);
    const int64_t fy = (int64_t)rint((y - ri.forigin[1]) * ri.finv[1]);
    const int64_t fz = (int64_t)rint((z - ri.forigin[2]) * ri.finv[2]);
    return make_int4((int32_t)(uint32_t)(uint64_t)fx, (int32_t)(uint32_t)(uint64_t)fy,
                     (int32_t)(uint32_t)(uint64_t)fz, type);
}

// most bonded terms (bonds + angles) touching one atom
constexpr int BTMAX = 8;

// what one build produces
// A force-list row holds every partner within the list radius.  Partners
// beyond the near radius (the force cutoff plus half the skin) at build time
// come within the cutoff only if the pair closes by more than half the skin
// before the next build, which is rare; a pair kernel that walks the near
// entries first therefore finds the wavefront blocks over far entries
// almost always out of range and skips their pair arithmetic.  Every entry is
// still tested, so the order is a matter of speed only.
struct BuildSpec {
    double rf2;           // force-list radius squared
    double rfn2;          // force-list entries with r^2 < rfn2 are near, the others far
    double rcmin2;        // candidate lower radius squared (0: none)
    double rcmax2;        // candidate upper radius squared
    double rsearch;       // cell-search radius (max of the radii)
    int32_t want_force;
    int32_t want_cand;
    int32_t mirror_sel;   // -1: mirror of the parity of step (device counter + step_off), 0/1: fixed
    int32_t step_off;
};

// static per-atom topology on the device
struct Topo {
    const int32_t *type;       // [N]
    const int32_t *rep_of;     // [N]
    const double *acc_m;       // [N] ACC / m
    const double *inv_mass;    // [N] 1 / m
    const int32_t *excl_ptr;   // [N+1]
    const int32_t *excl_idx;   // caller ids
    const int32_t *bt_ptr;     // [N+1] bonded terms touching each atom
    const int32_t *bt;         // term code: (kind << 28) | index
    const int32_t *bond_ij;    // [nb][2]
    const double *bond_kr;     // [nb][2] (k, r0)
    const int32_t *angle_ijk;  // [na][3]
    const double *angle_kt;    // [na][2] (k, theta0)
};

}  // namespace bnc
