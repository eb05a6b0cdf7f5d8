// C-ABI host side of the BOUNCE library: context, workspace binding, rate
// bounds, list-build schedule, step orchestration (direct launches or replayed
// HIP graphs), diagnostics and the differentiable direct energy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/bounce.h"
#include "bounce_kernels.hpp"

using namespace bnc;

namespace {

// ---------------------------------------------------------------------------
// host-side pair potential, used only for the rate bounds (Sec. IV.A: the bound
// L >= |chi W'|_inf is computed numerically once from the 1-D function)
// ---------------------------------------------------------------------------
struct HostFF {
    int nt;
    double q[MAXT], eps[MAXT], sig[MAXT];
    int coulomb;
    double alpha, r_on, r_off, r_cut;
    int split;                    // separate Coulomb and Lennard-Jones mechanisms
    double r_on_v, r_off_v;       // the Lennard-Jones window

    // the Coulomb and Lennard-Jones parts of u'(r)
    void du_parts(int a, int b, double r, double &dc, double &dv) const
    {
        double qq = KE * q[a] * q[b];
        double e = std::sqrt(eps[a] * eps[b]);
        double s = 0.5 * (sig[a] + sig[b]);
        double dg;
        if (coulomb) {
            double ar = alpha * r;
            dg = -std::erfc(ar) / (r * r) - TWO_OVER_SQRTPI * alpha * std::exp(-ar * ar) / r;
        } else {
            dg = -1.0 / (r * r);
        }
        double dl = 0.0;
        if (e != 0.0) {
            double x = s / r, x6 = x * x * x * x * x * x;
            dl = 4.0 * e * (6.0 * x6 - 12.0 * x6 * x6) / r;
        }
        dc = qq * dg;
        dv = dl;
    }
    void du(int a, int b, double r, double &d) const
    {
        double dc, dv;
        du_parts(a, b, r, dc, dv);
        d = dc + dv;
    }
    static double smooth(double lo, double hi, double r)
    {
        double x = (r - lo) / (hi - lo);
        x = std::min(1.0, std::max(0.0, x));
        return x * x * x * (10.0 + x * (6.0 * x - 15.0));
    }
    double chi(double r) const { return smooth(r_on, r_off, r); }
    // (1 + 1e-3) * max over the grid r'_m + k 1e-4 < rc of |chi_m(r) W'_m(r)| for
    // mechanism m: the combined one (chi (u'(r) - u'(rc))), or with split
    // mechanisms Coulomb (m = 0) and Lennard-Jones (m = 1) each with its window
    double bound(int m, int a, int b) const
    {
        double drc, dcc, dvc;
        du(a, b, r_cut, drc);
        du_parts(a, b, r_cut, dcc, dvc);
        const double lo = split && m == 1 ? r_on_v : r_on, hi = split && m == 1 ? r_off_v : r_off;
        double mx = 0.0;
        for (long k = 0;; ++k) {
            double r = lo + (double)k * 1e-4;
            if (r >= r_cut) break;
            double w;
            if (!split) {
                double d;
                du(a, b, r, d);
                w = d - drc;
            } else {
                double dc, dv;
                du_parts(a, b, r, dc, dv);
                w = m == 1 ? dv - dvc : dc - dcc;
            }
            mx = std::max(mx, std::fabs(smooth(lo, hi, r) * w));
        }
        return mx * (1.0 + 1e-3);
    }
};

struct Region {
    size_t off, bytes;
};

// the short-range force reaches to r'' (the larger window end of the two
// mechanisms when they are separate); the jump fields start at r' (the smaller)
static double r_short(const bounce_params &p) { return p.jump_split ? std::max(p.r_off, p.r_off_lj) : p.r_off; }
static double r_long(const bounce_params &p) { return p.jump_split ? std::min(p.r_on, p.r_on_lj) : p.r_on; }

}  // namespace

struct bounce_ctx {
    bounce_params p{};
    bool have_system = false, bound = false;
    int static_dev = -1;          // device whose static workspace this context uses, or -1
    std::string err;
    // system (host copies)
    int32_t n = 0, R = 0, nt = 0;
    std::vector<int64_t> rep_off;
    std::vector<RepInfo> reps;
    std::vector<int32_t> type, rep_of, excl_ptr, excl_idx, bt_ptr, bt, bond_ij, angle_ijk;
    std::vector<double> mass, acc_m, inv_mass, ou_c2, bond_kr, angle_kt, tparams;
    std::vector<double> L_ab, L_a;
    std::vector<uint32_t> Lq;     // [MAXT][LQW] integer bound weights of the jump step
    int32_t ncls = 1;             // candidate classes: n_types for BOUNCE_RATE_PAIR or split mechanisms, else 1
    int32_t nmech = 1;            // jump mechanisms per pair: 2 with jump_split
    std::vector<TypePair<float>> tab_f;     // jump-field pair constants per type pair
    std::vector<TypePair<double>> tab_d;
    int32_t n_cells = 0, fcap = 0, ccap = 0, acap = 0, xcap = 0;
    bool fixed = false;           // FP32 pair arithmetic: keep the fixed-point position mirror
    // workspace
    char *ws = nullptr;
    uint64_t ws_bytes = 0;
    double *pos = nullptr, *vel = nullptr;
    hipStream_t stream = nullptr;
    Topo tp{};
    ListSet main{}, aux{};
    RepInfo *d_reps = nullptr;
    DevState *d_st = nullptr;
    RepCounters *d_cnt = nullptr;
    unsigned long long *d_wave_cnt = nullptr;
    Event *d_events = nullptr;
    const TypePair<float> *d_tab_f = nullptr;
    const TypePair<double> *d_tab_d = nullptr;
    double *d_unit = nullptr, *d_tparams = nullptr, *d_fpair = nullptr, *d_atom = nullptr,
           *d_seg = nullptr, *d_ou_c2 = nullptr;
    int64_t *d_rep_off = nullptr, *d_one_seg = nullptr;
    int32_t *d_cell_rep = nullptr;
    uint32_t *d_Lq = nullptr;
    unsigned long long *d_rdf = nullptr;
    // smooth PME: mesh, influence function theta(k) (host-computed), RESPA gradient
    bool pme = false;
    bool out_pair = false;        // the short-range pair force is on the RESPA outer step
    bool outer = false;           // there is an outer step (mesh and/or pair force on it)
    int64_t pme_points = 0;
    double pme_qscale = 1.0;
    std::vector<double> theta;
    double2 *d_grid = nullptr;
    double *d_theta = nullptr, *d_grec = nullptr, *d_pme_e = nullptr, *d_charge = nullptr;
    PmeAtoms pme_atoms{};
    std::vector<int32_t> cell_rep;
    int32_t *d_xcnt = nullptr, *d_xcol = nullptr;
    // fused step launch: items (replica, first sorted atom, end, kind), pair
    // items per replica, the queue counters, and the launch's workgroups
    std::vector<int4> fitems;
    std::vector<int32_t> fneed;
    FusedArgs fused{};
    int32_t fused_grid = 0;
    // cluster pairs (pair_kernel = 4 or 8)
    std::vector<int4> clu;
    std::vector<int32_t> cl_first;
    ClusterSet cs{};
    int32_t cl_cap = 0;
    // schedule
    int64_t step = 0;             // host view: device counter + pending
    int32_t pending = 0;          // steps opened since the device counter last moved
    int64_t built_step = -1;
    int64_t host_steps = 0, host_rebuilds = 0;
    // graphs of K steps
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
};

static bounce_status fail(bounce_ctx *c, bounce_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIPCHK(ctx, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, BOUNCE_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// API functions: C linkage comes from their declarations in bounce.h

const char *bounce_status_string(int32_t s)
{
    switch (s) {
        case BOUNCE_OK: return "ok";
        case BOUNCE_E_ARG: return "invalid argument";
        case BOUNCE_E_HIP: return "HIP runtime error";
        case BOUNCE_E_CAPACITY: return "pair-list or cell capacity exceeded";
        case BOUNCE_E_SKIN: return "an atom moved half the Verlet skin since the list build";
        case BOUNCE_E_BOUND: return "a jump proposal exceeded the rate bound";
        case BOUNCE_E_POISSON_CAP: return "Poisson proposal count above max_proposals";
        case BOUNCE_E_NONFINITE: return "non-finite position or velocity";
        case BOUNCE_E_STATE: return "context not ready (system not set or not bound)";
        case BOUNCE_E_GRID: return "a droplet atom left its cell grid";
        case BOUNCE_E_WORKSPACE: return "workspace too small";
        default: return "unknown status";
    }
}

const char *bounce_last_error(const bounce_ctx *c) { return c ? c->err.c_str() : "null context"; }

bounce_status bounce_create(const bounce_params *p, bounce_ctx **out)
{
    if (!p || !out) return BOUNCE_E_ARG;
    *out = nullptr;
    if (p->integrator != BOUNCE_BJAOAJB && p->integrator != BOUNCE_BAOAB) return BOUNCE_E_ARG;
    if (!(p->dt > 0) || !(p->gamma >= 0) || !(p->temperature > 0)) return BOUNCE_E_ARG;
    if (!(p->r_cut > 0) || !(p->skin >= 0) || !(p->cell_size > 0)) return BOUNCE_E_ARG;
    if (p->integrator == BOUNCE_BJAOAJB && !(p->r_on > 0 && p->r_off > p->r_on)) return BOUNCE_E_ARG;
    if (p->rebuild_interval < 1 || p->max_proposals < 1) return BOUNCE_E_ARG;
    if (!(p->bound_scale > 0)) return BOUNCE_E_ARG;
    if (p->rate_mode != BOUNCE_RATE_ATOM && p->rate_mode != BOUNCE_RATE_PAIR) return BOUNCE_E_ARG;
    if (p->pme_grid[0] || p->pme_grid[1] || p->pme_grid[2]) {
        for (int k = 0; k < 3; ++k) {
            const int32_t g = p->pme_grid[k];
            if (g < 8 || g > 512 || (g & (g - 1))) return BOUNCE_E_ARG;
        }
        if (p->pme_order < 4 || p->pme_order > 6 || !p->periodic) return BOUNCE_E_ARG;
    }
    if (p->respa_m < 0 || (p->respa_m > 0 && p->rebuild_interval % p->respa_m)) return BOUNCE_E_ARG;
    if (p->respa_outer != BOUNCE_OUTER_RECIP && p->respa_outer != BOUNCE_OUTER_NONBONDED) return BOUNCE_E_ARG;
    if (p->respa_outer == BOUNCE_OUTER_NONBONDED && p->respa_m < 1) return BOUNCE_E_ARG;
    if (p->persistent != 0 && p->persistent != 1) return BOUNCE_E_ARG;
    if (p->pair_kernel != 0 && p->pair_kernel != 4 && p->pair_kernel != 8) return BOUNCE_E_ARG;
    if (p->pair_kernel != 0 && p->pair_precision != BOUNCE_PAIR_FP32) return BOUNCE_E_ARG;
    if (p->pair_lanes != 0 && p->pair_lanes != 4 && p->pair_lanes != 8 && p->pair_lanes != 16 &&
        p->pair_lanes != 32)
        return BOUNCE_E_ARG;
    if (p->jump_split != 0 && p->jump_split != 1) return BOUNCE_E_ARG;
    const bool lj_window = p->r_on_lj != 0.0 || p->r_off_lj != 0.0;
    if (p->jump_split && p->integrator == BOUNCE_BJAOAJB && lj_window &&
        !(p->r_on_lj > 0 && p->r_off_lj > p->r_on_lj && p->r_off_lj < p->r_cut))
        return BOUNCE_E_ARG;
    bounce_ctx *c = new bounce_ctx();
    c->p = *p;
    if (!c->p.jump_split || !lj_window) {      // the Lennard-Jones window defaults to Coulomb's
        c->p.r_on_lj = c->p.r_on;
        c->p.r_off_lj = c->p.r_off;
    }
    if (c->p.pair_lanes == 0) c->p.pair_lanes = 8;
    *out = c;
    return BOUNCE_OK;
}

// The static workspace of bounce_bind_static: one file-scope device array,
// present on every device the library runs on until the process ends.  Host
// code never uses the array's name as an address (on the host it is only a
// stand-in for the symbol): each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) char scratch[BOUNCE_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[STATIC_MAX_DEVICES] = {};
const bounce_ctx *g_static_owner[STATIC_MAX_DEVICES] = {};
}  // namespace

void bounce_destroy(bounce_ctx *c)
{
    if (!c) return;
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
    }
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    delete c;
}

// cardinal B-spline values M_n(1), ..., M_n(n-1) by the order recursion on the
// integer points, for the Euler-spline factors |b(k)|^2 of smooth PME
static std::vector<double> spline_at_integers(int n)
{
    std::vector<double> m(n + 1, 0.0);      // m[j] = M_k(j), k = 2 at start
    m[1] = 1.0;
    for (int k = 3; k <= n; ++k) {
        std::vector<double> nx(n + 1, 0.0);
        for (int j = 1; j < k; ++j)
            nx[j] = ((double)j * m[j] + (double)(k - j) * m[j - 1]) / (double)(k - 1);
        m = nx;
    }
    return m;
}

// theta(k) = k_e / (pi V) exp(-pi^2 m^2 / alpha^2) / m^2 |b_0|^2 |b_1|^2 |b_2|^2,
// theta(0) = 0; |b(k)|^2 = 1 / |sum_{j=0}^{n-2} M_n(j+1) exp(2 pi i k j / K)|^2, and
// where that sum vanishes (odd n, k = K/2) the mean of the neighbouring values
static void make_theta(bounce_ctx *c)
{
    const RepInfo &ri = c->reps[0];
    const int n = c->p.pme_order;
    const std::vector<double> M = spline_at_integers(n);
    std::vector<double> bsq[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int K = c->p.pme_grid[ax];
        bsq[ax].assign(K, 0.0);
        for (int k = 0; k < K; ++k) {
            double re = 0.0, im = 0.0;
            for (int j = 0; j <= n - 2; ++j) {
                const double ph = 2.0 * M_PI * (double)((int64_t)k * j % K) / (double)K;
                re += M[j + 1] * std::cos(ph);
                im += M[j + 1] * std::sin(ph);
            }
            const double d = re * re + im * im;
            bsq[ax][k] = d > 1e-30 ? 1.0 / d : -1.0;
        }
        for (int k = 0; k < K; ++k)
            if (bsq[ax][k] < 0.0) bsq[ax][k] = 0.5 * (bsq[ax][(k + K - 1) % K] + bsq[ax][(k + 1) % K]);
    }
    const int K0 = c->p.pme_grid[0], K1 = c->p.pme_grid[1], K2 = c->p.pme_grid[2];
    const double V = ri.box[0] * ri.box[1] * ri.box[2], a = c->p.ewald_alpha;
    c->pme_points = (int64_t)K0 * K1 * K2;
    c->theta.assign(c->pme_points, 0.0);
    for (int k0 = 0; k0 < K0; ++k0)
        for (int k1 = 0; k1 < K1; ++k1)
            for (int k2 = 0; k2 < K2; ++k2) {
                if (!k0 && !k1 && !k2) continue;
                const int kk[3] = {k0, k1, k2}, KK[3] = {K0, K1, K2};
                double m2 = 0.0;
                for (int ax = 0; ax < 3; ++ax) {
                    const double mc = (double)(kk[ax] <= KK[ax] / 2 ? kk[ax] : kk[ax] - KK[ax]) / ri.box[ax];
                    m2 += mc * mc;
                }
                c->theta[((int64_t)k0 * K1 + k1) * K2 + k2] =
                    KE / (M_PI * V) * std::exp(-M_PI * M_PI * m2 / (a * a)) / m2 * bsq[0][k0] * bsq[1][k1] *
                    bsq[2][k2];
            }
}

static void make_ou(bounce_ctx *c)
{
    double c1 = std::exp(-c->p.gamma * c->p.dt);
    double kt = KB * c->p.temperature;
    c->ou_c2.resize(c->n);
    for (int32_t g = 0; g < c->n; ++g) c->ou_c2[g] = std::sqrt(kt * (1.0 - c1 * c1) * ACC / c->mass[g]);
}

static void make_bounds(bounce_ctx *c)
{
    HostFF ff{};
    ff.nt = c->nt;
    for (int a = 0; a < c->nt; ++a) {
        ff.q[a] = c->tparams[a]; ff.eps[a] = c->tparams[c->nt + a]; ff.sig[a] = c->tparams[2 * c->nt + a];
    }
    ff.coulomb = c->p.coulomb;
    ff.alpha = c->p.ewald_alpha;
    ff.r_on = c->p.r_on; ff.r_off = c->p.r_off; ff.r_cut = c->p.r_cut;
    ff.split = c->p.jump_split;
    ff.r_on_v = c->p.r_on_lj; ff.r_off_v = c->p.r_off_lj;
    const int nt = c->nt, nm = c->p.jump_split ? 2 : 1;
    c->nmech = nm;
    c->L_ab.assign(nm * nt * nt, 0.0);
    c->L_a.assign(nt, 0.0);
    // pair constants of the jump fields: q_a q_b, LJ, u'(rc) and its Coulomb
    // and Lennard-Jones parts (pad[1], pad[0]) for the separate mechanisms
    c->tab_f.assign(MAXT * MAXT, TypePair<float>{});
    c->tab_d.assign(MAXT * MAXT, TypePair<double>{});
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            const double qq = KE * ff.q[a] * ff.q[b], eps = std::sqrt(ff.eps[a] * ff.eps[b]);
            const double sig = 0.5 * (ff.sig[a] + ff.sig[b]);
            double drc, dcc, dvc;
            ff.du(a, b, ff.r_cut, drc);
            ff.du_parts(a, b, ff.r_cut, dcc, dvc);
            TypePair<double> &td = c->tab_d[a * nt + b];
            td.qq = qq; td.eps4 = 4.0 * eps; td.sig2 = sig * sig; td.du_rc = drc;
            td.pad[0] = dvc; td.pad[1] = dcc;
            TypePair<float> &tf = c->tab_f[a * nt + b];
            tf.qq = (float)qq; tf.eps4 = (float)(4.0 * eps); tf.sig2 = (float)(sig * sig);
            tf.du_rc = (float)drc;
            tf.pad[0] = (float)dvc; tf.pad[1] = (float)dcc;
        }
    c->Lq.assign(MAXT * LQW, 1u << WEIGHT_BITS);
    c->ncls = 1;
    if (c->p.integrator != BOUNCE_BJAOAJB) return;
    for (int m = 0; m < nm; ++m)
        for (int a = 0; a < nt; ++a)
            for (int b = a; b < nt; ++b)
                c->L_ab[(m * nt + a) * nt + b] = c->L_ab[(m * nt + b) * nt + a] = ff.bound(m, a, b);
    for (int m = 0; m < nm; ++m)
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < nt; ++b) c->L_a[a] = std::max(c->L_a[a], c->L_ab[(m * nt + a) * nt + b]);
    // per-type-pair (and per-mechanism) bounds as integer weights of the row unit
    // L_a 2^-20, rounded up after a slack of 1e-4 of a unit (bounds that agree
    // to 1e-12 with another computation of them give the same weights); the
    // weight of mechanism m and partner type b of an atom of type a sits at
    // Lq[a LQW + m n_types + b]
    if (c->p.rate_mode == BOUNCE_RATE_PAIR || c->p.jump_split) {
        c->ncls = nt;
        const double one = (double)(1u << WEIGHT_BITS);
        for (int a = 0; a < nt; ++a)
            for (int m = 0; m < nm; ++m)
                for (int b = 0; b < nt; ++b)
                    if (c->L_a[a] > 0.0)
                        c->Lq[a * LQW + m * nt + b] =
                            (uint32_t)std::ceil(c->L_ab[(m * nt + a) * nt + b] / c->L_a[a] * one - WEIGHT_SLACK);
    }
}

// unit of each atom type's bound weights: bound_scale L_a 2^-20
static std::vector<double> bound_units(const bounce_ctx *c)
{
    std::vector<double> u(MAXT, 0.0);
    for (int a = 0; a < c->nt && a < (int)c->L_a.size(); ++a)
        u[a] = c->p.bound_scale * c->L_a[a] / (double)(1u << WEIGHT_BITS);
    return u;
}

bounce_status bounce_set_system(bounce_ctx *c, const bounce_system *s)
{
    if (!c || !s) return BOUNCE_E_ARG;
    if (s->n_replicas < 1 || s->n_atoms < 1 || !s->replica_offset || !s->type || !s->mass)
        return fail(c, BOUNCE_E_ARG, "missing replicas, atoms, types or masses");
    if (s->n_types < 1 || s->n_types > MAXT || !s->charge || !s->eps || !s->sigma)
        return fail(c, BOUNCE_E_ARG, "n_types must be in [1, 8] with charge/eps/sigma");
    if (c->p.jump_split && s->n_types > MAXT / 2)
        return fail(c, BOUNCE_E_ARG, "jump_split needs n_types <= 4");
    if (s->replica_offset[0] != 0 || s->replica_offset[s->n_replicas] != s->n_atoms)
        return fail(c, BOUNCE_E_ARG, "replica_offset must run from 0 to n_atoms");
    if (c->p.periodic && !s->box) return fail(c, BOUNCE_E_ARG, "periodic system needs box");
    if (!c->p.periodic && (!s->grid_origin || !s->grid_dims))
        return fail(c, BOUNCE_E_ARG, "droplet system needs grid_origin and grid_dims");
    const int32_t n = s->n_atoms, R = s->n_replicas, nt = s->n_types;
    c->n = n; c->R = R; c->nt = nt;
    c->rep_off.assign(s->replica_offset, s->replica_offset + R + 1);
    c->type.assign(s->type, s->type + n);
    c->mass.assign(s->mass, s->mass + n);
    for (int32_t g = 0; g < n; ++g) {
        if (c->type[g] < 0 || c->type[g] >= nt) return fail(c, BOUNCE_E_ARG, "atom type out of range");
        if (!(c->mass[g] > 0)) return fail(c, BOUNCE_E_ARG, "masses must be positive");
    }
    c->tparams.resize(3 * nt);
    for (int a = 0; a < nt; ++a) {
        c->tparams[a] = s->charge[a]; c->tparams[nt + a] = s->eps[a]; c->tparams[2 * nt + a] = s->sigma[a];
    }
    c->rep_of.assign(n, 0);
    c->reps.assign(R, RepInfo{});
    int32_t cell_off = 0;
    double max_rho = 0.0;
    const double rsearch = std::max(c->p.r_cut, r_short(c->p)) + c->p.skin;
    for (int32_t r = 0; r < R; ++r) {
        int64_t b = c->rep_off[r], e = c->rep_off[r + 1];
        if (e <= b) return fail(c, BOUNCE_E_ARG, "empty replica");
        for (int64_t g = b; g < e; ++g) c->rep_of[g] = r;
        RepInfo &ri = c->reps[r];
        ri.periodic = c->p.periodic;
        ri.atom_off = b;
        ri.n_atoms = (int32_t)(e - b);
        ri.cell_off = cell_off;
        ri.key0 = c->p.seed;
        ri.key1 = (uint64_t)r;
        double vol = 1.0;
        for (int k = 0; k < 3; ++k) {
            if (c->p.periodic) {
                double L = s->box[3 * r + k];
                if (!(L > 2.0 * rsearch))
                    return fail(c, BOUNCE_E_ARG, "box edge must exceed 2 (max(rc, r'') + skin)");
                ri.box[k] = L;
                ri.inv_box[k] = 1.0 / L;
                int32_t nc = (int32_t)std::floor(L / c->p.cell_size);
                if (nc < 1) nc = 1;
                ri.ncell[k] = nc;
                ri.cinv[k] = (double)nc * ri.inv_box[k];
                ri.cw[k] = L / nc;
                vol *= L;
            } else {
                ri.box[k] = 0.0; ri.inv_box[k] = 0.0;
                ri.origin[k] = s->grid_origin[3 * r + k];
                ri.ncell[k] = s->grid_dims[3 * r + k];
                if (ri.ncell[k] < 1) return fail(c, BOUNCE_E_ARG, "grid_dims must be >= 1");
                ri.cw[k] = c->p.cell_size;
                vol *= ri.ncell[k] * c->p.cell_size;
            }
        }
        ri.inv_cell = 1.0 / c->p.cell_size;
        int64_t nc3 = (int64_t)ri.ncell[0] * ri.ncell[1] * ri.ncell[2];
        if (nc3 > (int64_t)1 << 28) return fail(c, BOUNCE_E_ARG, "cell grid too large");
        cell_off += (int32_t)nc3;
        double rho = c->p.periodic ? (double)(e - b) / vol : 0.12;
        max_rho = std::max(max_rho, rho);
    }
    c->n_cells = cell_off;
    // fixed-point position mirror of the FP32 pair kernels: periodic, unit
    // edge / 2^32 (positions modulo 2^32: the 32-bit difference is the minimum
    // image); droplet, unit grid extent / 2^30 from the grid origin
    c->fixed = c->p.pair_precision == BOUNCE_PAIR_FP32;
    // the FP32 pair kernels gather the mirror through a buffer resource with
    // 32-bit byte offsets (16 bytes an atom)
    if (c->fixed && (int64_t)c->n * 16 > (int64_t)0x7fffffff)
        return fail(c, BOUNCE_E_ARG, "FP32 pair arithmetic supports at most 134,217,727 atoms");
    for (RepInfo &ri : c->reps)
        for (int k = 0; k < 3; ++k) {
            const double u = ri.periodic ? std::ldexp(ri.box[k], -32)
                                         : std::ldexp(ri.cw[k] * ri.ncell[k], -30);
            ri.finv[k] = 1.0 / u;
            ri.forigin[k] = ri.periodic ? 0.0 : ri.origin[k];
            ri.funit[k] = (float)u;
        }
    c->cell_rep.assign(cell_off, 0);
    for (int32_t r = 0; r < R; ++r) {
        int32_t e = r + 1 < R ? c->reps[r + 1].cell_off : cell_off;
        for (int32_t k = c->reps[r].cell_off; k < e; ++k) c->cell_rep[k] = r;
    }
    // fused step items: a replica's atoms occupy its own cells, so in sorted
    // order they are the contiguous range [offset_r, offset_r+1); every pair
    // item ahead of every integrator item
    c->fitems.clear();
    c->fneed.assign(R, 0);
    for (int kind = 0; kind < 2; ++kind)
        for (int32_t r = 0; r < R; ++r) {
            const int32_t tile = kind == 0 ? PAIR_ATOMS : STEP_ATOMS;
            for (int64_t b = c->rep_off[r]; b < c->rep_off[r + 1]; b += tile) {
                const int64_t e = std::min<int64_t>(b + tile, c->rep_off[r + 1]);
                c->fitems.push_back(make_int4(r, (int32_t)b, (int32_t)e, kind));
                if (kind == 0) c->fneed[r]++;
            }
        }
    // clusters of pair_kernel consecutive sorted atoms, per replica
    c->clu.clear();
    c->cl_first.assign(R + 1, 0);
    if (c->p.pair_kernel) {
        const int32_t CL = c->p.pair_kernel;
        int64_t max_cl = 1;
        for (int32_t r = 0; r < R; ++r) {
            c->cl_first[r] = (int32_t)c->clu.size();
            for (int64_t b = c->rep_off[r]; b < c->rep_off[r + 1]; b += CL)
                c->clu.push_back(make_int4((int32_t)b, (int32_t)std::min<int64_t>(b + CL, c->rep_off[r + 1]), r, 0));
            max_cl = std::max<int64_t>(max_cl, (int64_t)c->clu.size() - c->cl_first[r]);
        }
        c->cl_first[R] = (int32_t)c->clu.size();
    }
    // row capacities: 1.5 x the mean count in the list sphere at the densest replica
    auto cap = [&](double r) {
        double m = 1.5 * max_rho * 4.18879020478639 * r * r * r + 64.0;
        return (int32_t)(std::ceil(m / 32.0) * 32.0);
    };
    int64_t max_rep = 0;
    for (int32_t r = 0; r < R; ++r) max_rep = std::max<int64_t>(max_rep, c->rep_off[r + 1] - c->rep_off[r]);
    auto clampcap = [&](int32_t k) { return (int32_t)std::min<int64_t>(k, std::max<int64_t>(32, ((max_rep + 31) / 32) * 32)); };
    bool bounce = c->p.integrator == BOUNCE_BJAOAJB;
    c->fcap = clampcap(cap((bounce ? r_short(c->p) : c->p.r_cut) + c->p.skin));
    c->ccap = bounce ? clampcap(cap(c->p.r_cut + c->p.skin)) : 0;
    c->acap = clampcap(cap(c->p.r_cut + 0.01));
    c->xcap = std::max(c->fcap, std::max(c->ccap, c->acap));
    if (c->p.pair_kernel) {
        // clusters whose boxes (up to ~6 A across) come within the list radius:
        // 1.5 x the mean count in the sphere of radius rl + 6 A, plus 64
        const double rl = (bounce ? r_short(c->p) : c->p.r_cut) + c->p.skin + 6.0;
        int64_t per = 1;
        for (int32_t r = 0; r < R; ++r) per = std::max<int64_t>(per, c->cl_first[r + 1] - c->cl_first[r]);
        const double m = 1.5 * max_rho * 4.18879020478639 * rl * rl * rl / c->p.pair_kernel + 64.0;
        c->cl_cap = (int32_t)std::min<int64_t>((int64_t)(std::ceil(m / 32.0) * 32.0), ((per + 31) / 32) * 32);
        // in a droplet a cluster can run from the end of one column of cells to
        // the start of the next, across the droplet: such boxes meet every
        // cluster of the replica, so the capacity is the replica's cluster count
        if (!c->p.periodic) c->cl_cap = (int32_t)(((per + 31) / 32) * 32);
    } else {
        c->cl_cap = 0;
    }
    // exclusions (both directions) and bonded terms per atom
    std::vector<std::vector<int32_t>> ex(n), bt(n);
    for (int32_t k = 0; k < s->n_excl; ++k) {
        int32_t a = s->excl[2 * k], b = s->excl[2 * k + 1];
        if (a < 0 || b < 0 || a >= n || b >= n) return fail(c, BOUNCE_E_ARG, "exclusion index");
        ex[a].push_back(b);
        ex[b].push_back(a);
    }
    c->bond_ij.assign(s->bonds, s->bonds + 2 * s->n_bonds);
    c->bond_kr.resize(2 * s->n_bonds);
    for (int32_t k = 0; k < s->n_bonds; ++k) {
        c->bond_kr[2 * k] = s->bond_k[k];
        c->bond_kr[2 * k + 1] = s->bond_r0[k];
        for (int j = 0; j < 2; ++j) {
            int32_t a = s->bonds[2 * k + j];
            if (a < 0 || a >= n) return fail(c, BOUNCE_E_ARG, "bond index");
            bt[a].push_back(k);
        }
    }
    c->angle_ijk.assign(s->angles, s->angles + 3 * s->n_angles);
    c->angle_kt.resize(2 * s->n_angles);
    for (int32_t k = 0; k < s->n_angles; ++k) {
        c->angle_kt[2 * k] = s->angle_k[k];
        c->angle_kt[2 * k + 1] = s->angle_t0[k];
        for (int j = 0; j < 3; ++j) {
            int32_t a = s->angles[3 * k + j];
            if (a < 0 || a >= n) return fail(c, BOUNCE_E_ARG, "angle index");
            bt[a].push_back((1 << 28) | k);
        }
    }
    for (int32_t g = 0; g < n; ++g)
        if ((int)bt[g].size() > BTMAX) return fail(c, BOUNCE_E_ARG, "more than 8 bonded terms on one atom");
    c->excl_ptr.assign(n + 1, 0);
    c->bt_ptr.assign(n + 1, 0);
    c->excl_idx.clear();
    c->bt.clear();
    for (int32_t g = 0; g < n; ++g) {
        c->excl_idx.insert(c->excl_idx.end(), ex[g].begin(), ex[g].end());
        c->bt.insert(c->bt.end(), bt[g].begin(), bt[g].end());
        c->excl_ptr[g + 1] = (int32_t)c->excl_idx.size();
        c->bt_ptr[g + 1] = (int32_t)c->bt.size();
    }
    c->acc_m.resize(n);
    c->inv_mass.resize(n);
    for (int32_t g = 0; g < n; ++g) {
        c->acc_m[g] = ACC / c->mass[g];
        c->inv_mass[g] = 1.0 / c->mass[g];
    }
    make_ou(c);
    make_bounds(c);
    c->pme = c->p.pme_grid[0] > 0;
    c->out_pair = c->p.respa_m >= 1 && c->p.respa_outer == BOUNCE_OUTER_NONBONDED;
    c->outer = c->p.respa_m >= 1 && (c->pme || c->out_pair);
    c->pme_points = 0;
    if (c->pme) {
        if (R != 1 || !c->reps[0].periodic)
            return fail(c, BOUNCE_E_ARG, "the PME mesh needs one periodic replica");
        make_theta(c);
        // fixed point of the spread: 2^k with sum_i |q_i| 2^k < 2^61 (a mesh
        // point's sum is at most sum_i |q_i|: the spline weights lie in [0, 1])
        // and every term |q w w w| 2^k < 2^51 (exact integer conversion by one
        // FP64 addition)
        double qabs = 0.0, qmax = 0.0;
        for (int32_t g = 0; g < n; ++g) {
            qabs += std::fabs(c->tparams[c->type[g]]);
            qmax = std::max(qmax, std::fabs(c->tparams[c->type[g]]));
        }
        int e2 = 0, e3 = 0;
        std::frexp(std::max(qabs, 1e-300), &e2);     // qabs < 2^e2
        std::frexp(std::max(qmax, 1e-300), &e3);     // qmax < 2^e3
        c->pme_qscale = std::ldexp(1.0, std::min(std::min(61 - e2, 51 - e3), 60));
    }
    c->have_system = true;
    c->bound = false;
    return BOUNCE_OK;
}

// workspace layout
struct Layout {
    size_t total = 0;
    size_t take(size_t bytes)
    {
        size_t off = (total + 255) & ~(size_t)255;
        total = off + bytes;
        return off;
    }
};

template <typename T>
static T *at(char *base, size_t off) { return reinterpret_cast<T *>(base + off); }

struct Offsets {
    size_t type, rep_of, acc_m, inv_mass, ou_c2, excl_ptr, excl_idx, bt_ptr, bt, bond_ij, bond_kr,
        angle_ijk, angle_kt, reps, unit, Lq, tparams, tab_f, tab_d, wave_cnt, rep_off, one_seg, st, cnt, events, fpair, atom,
        seg, xcnt, xcol, cell_rep, rdf, grid, theta, grec, pme_e, pme_fl, pme_f, pme_w, fitems, fneed,
        fqueue, clu, cl_first, cl_ctr, cl_half, cl_cnt, cl_list;
    size_t ls[2][18];
};

// wavefront slots of the integrator and jump kernels (4 lanes per atom, 64
// atoms per workgroup of 4 wavefronts; the fused launch has at most as many
// workgroups)
static int64_t wave_slots(const bounce_ctx *c) { return 4 * (((int64_t)c->n + 63) / 64) + 4; }

static void plan(const bounce_ctx *c, Layout &L, Offsets &o)
{
    const size_t n = c->n, R = c->R;
    o.type = L.take(4 * n);
    o.rep_of = L.take(4 * n);
    o.acc_m = L.take(8 * n);
    o.inv_mass = L.take(8 * n);
    o.ou_c2 = L.take(8 * n);
    o.excl_ptr = L.take(4 * (n + 1));
    o.excl_idx = L.take(4 * std::max<size_t>(1, c->excl_idx.size()));
    o.bt_ptr = L.take(4 * (n + 1));
    o.bt = L.take(4 * std::max<size_t>(1, c->bt.size()));
    o.bond_ij = L.take(4 * std::max<size_t>(1, c->bond_ij.size()));
    o.bond_kr = L.take(8 * std::max<size_t>(1, c->bond_kr.size()));
    o.angle_ijk = L.take(4 * std::max<size_t>(1, c->angle_ijk.size()));
    o.angle_kt = L.take(8 * std::max<size_t>(1, c->angle_kt.size()));
    o.reps = L.take(sizeof(RepInfo) * R);
    o.unit = L.take(8 * MAXT);
    o.Lq = L.take(4 * MAXT * LQW);
    o.tparams = L.take(8 * 3 * MAXT);
    o.tab_f = L.take(sizeof(TypePair<float>) * MAXT * MAXT);
    o.tab_d = L.take(sizeof(TypePair<double>) * MAXT * MAXT);
    o.rep_off = L.take(8 * (R + 1));
    o.cell_rep = L.take(4 * (size_t)c->n_cells);
    o.one_seg = L.take(16);
    o.st = L.take(sizeof(DevState));
    o.cnt = L.take(sizeof(RepCounters) * CNT_SPREAD * R);
    o.wave_cnt = L.take(8 * 3 * (size_t)wave_slots(c));
    o.events = L.take(sizeof(Event) * std::max<int64_t>(1, c->p.log_events ? c->p.event_capacity : 1));
    o.fpair = L.take(24 * n);
    o.atom = L.take(8 * n * std::max(5, 3 * MAXT));
    o.seg = L.take(8 * 8 * R);
    o.rdf = L.take(8 * (size_t)RDF_MAX_BINS);
    o.grid = L.take(16 * (size_t)std::max<int64_t>(1, c->pme_points));
    o.theta = L.take(8 * (size_t)std::max<int64_t>(1, c->pme_points));
    o.grec = L.take(24 * n);
    o.pme_e = L.take(8 * (size_t)(c->pme_points / 256 + 2));   // >= the fused pass's blocks (K^3 / 512)
    const size_t pn = c->pme ? (size_t)n : 1;
    o.pme_fl = L.take(16 * pn);
    o.pme_f = L.take(32 * pn);
    o.pme_w = L.take(8 * 3 * (size_t)std::max(1, c->p.pme_order) * pn);
    o.xcnt = L.take(4 * n);
    o.xcol = L.take(4 * n * (size_t)c->xcap);
    o.fitems = L.take(16 * std::max<size_t>(1, c->fitems.size()));
    o.fneed = L.take(4 * R);
    o.fqueue = L.take(4 * (R + 1));
    const size_t ncl = c->clu.size();
    o.clu = L.take(16 * std::max<size_t>(1, ncl));
    o.cl_first = L.take(4 * (R + 1));
    o.cl_ctr = L.take(16 * std::max<size_t>(1, ncl));
    o.cl_half = L.take(16 * std::max<size_t>(1, ncl));
    o.cl_cnt = L.take(4 * std::max<size_t>(1, ncl));
    o.cl_list = L.take(4 * std::max<size_t>(1, ncl * (size_t)c->cl_cap));
    for (int k = 0; k < 2; ++k) {
        const size_t fcap = k == 0 ? c->fcap : c->acap, ccap = k == 0 ? c->ccap : 0;
        size_t *q = o.ls[k];
        q[0] = L.take(4 * n);                      // perm
        q[1] = L.take(4 * n);                      // inv_perm
        q[2] = L.take(4 * n);                      // cell_of
        q[3] = L.take(4 * n);                      // slot
        q[4] = L.take(4 * (size_t)c->n_cells);     // cell_count
        q[5] = L.take(4 * ((size_t)c->n_cells + 1));  // cell_start
        q[6] = L.take(32 * n);                     // x[0]
        q[7] = L.take(32 * n);                     // x[1]
        q[8] = L.take(24 * n);                     // q_build
        q[9] = L.take(8 * n);                      // fcnt (near, far)
        q[10] = L.take(4 * n * fcap);              // flist
        const size_t ncls = k == 0 ? (size_t)c->ncls : 1;
        q[11] = L.take(4 * n * ncls * std::max<size_t>(1, ccap) + 4 * n * ncls);  // ccnt + clist
        q[12] = k == 0 ? L.take(sizeof(int4) * BTMAX * n) : 0;       // bslot (main set)
        q[13] = L.take(sizeof(int2) * n);                               // sinfo
        q[14] = L.take(8 * ((size_t)c->n_cells / 1024 + 2));            // scan_part
        q[17] = L.take(4 * ((size_t)c->n_cells + 1));                   // busy
        const bool fx = k == 0 && c->fixed;
        q[15] = fx ? L.take(16 * n) : 0;                                // xf[0]
        q[16] = fx ? L.take(16 * n) : 0;                                // xf[1]
    }
}

bounce_status bounce_workspace_size(const bounce_ctx *c, uint64_t *bytes)
{
    if (!c || !bytes) return BOUNCE_E_ARG;
    if (!c->have_system) return BOUNCE_E_STATE;
    Layout L;
    Offsets o;
    plan(c, L, o);
    *bytes = L.total + 256;
    return BOUNCE_OK;
}

template <typename T>
static hipError_t up(hipStream_t sm, char *ws, size_t off, const std::vector<T> &v)
{
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(ws + off, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, sm);
}

static bounce_status bind_impl(bounce_ctx *c, void *workspace, uint64_t bytes, double *pos,
                               double *vel, void *stream);

bounce_status bounce_bind(bounce_ctx *c, void *workspace, uint64_t bytes, double *pos, double *vel,
                          void *stream)
{
    if (!c || !workspace || !pos || !vel) return BOUNCE_E_ARG;
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
        c->static_dev = -1;
    }
    return bind_impl(c, workspace, bytes, pos, vel, stream);
}

bounce_status bounce_bind_static(bounce_ctx *c, double *pos, double *vel, void *stream)
{
    if (!c || !pos || !vel) return BOUNCE_E_ARG;
    if (!c->have_system) return fail(c, BOUNCE_E_STATE, "bounce_set_system first");
    uint64_t need = 0;
    bounce_status s = bounce_workspace_size(c, &need);
    if (s) return s;
    if (need > BOUNCE_STATIC_WORKSPACE_BYTES)
        return fail(c, BOUNCE_E_WORKSPACE,
                    "the system needs a " + std::to_string(need >> 20) +
                        " MiB workspace; the static workspace holds " +
                        std::to_string(BOUNCE_STATIC_WORKSPACE_BYTES >> 20) + " MiB");
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(c, BOUNCE_E_ARG, "device index");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (!g_static_ptr[dev]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(c, BOUNCE_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                                 hipGetErrorString(e));
            g_static_ptr[dev] = p;
        }
        ptr = g_static_ptr[dev];
        // the device's array now belongs to this context; a context bound to it
        // before is refused from here on (ready() compares owners)
        if (c->static_dev >= 0 && g_static_owner[c->static_dev] == c)
            g_static_owner[c->static_dev] = nullptr;
        g_static_owner[dev] = c;
        c->static_dev = dev;
    }
    return bind_impl(c, ptr, BOUNCE_STATIC_WORKSPACE_BYTES, pos, vel, stream);
}

static bounce_status bind_impl(bounce_ctx *c, void *workspace, uint64_t bytes, double *pos,
                               double *vel, void *stream)
{
    if (!c->have_system) return fail(c, BOUNCE_E_STATE, "bounce_set_system first");
    Layout L;
    Offsets o;
    plan(c, L, o);
    char *ws = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    if ((uint64_t)(ws - (char *)workspace) + L.total > bytes)
        return fail(c, BOUNCE_E_WORKSPACE, "workspace smaller than bounce_workspace_size");
    c->ws = ws;
    c->ws_bytes = bytes;
    c->pos = pos;
    c->vel = vel;
    c->stream = (hipStream_t)stream;
    hipStream_t sm = c->stream;
    HIPCHK(c, up(sm, ws, o.type, c->type));
    HIPCHK(c, up(sm, ws, o.rep_of, c->rep_of));
    HIPCHK(c, up(sm, ws, o.acc_m, c->acc_m));
    HIPCHK(c, up(sm, ws, o.inv_mass, c->inv_mass));
    HIPCHK(c, up(sm, ws, o.ou_c2, c->ou_c2));
    HIPCHK(c, up(sm, ws, o.excl_ptr, c->excl_ptr));
    HIPCHK(c, up(sm, ws, o.excl_idx, c->excl_idx));
    HIPCHK(c, up(sm, ws, o.bt_ptr, c->bt_ptr));
    HIPCHK(c, up(sm, ws, o.bt, c->bt));
    HIPCHK(c, up(sm, ws, o.bond_ij, c->bond_ij));
    HIPCHK(c, up(sm, ws, o.bond_kr, c->bond_kr));
    HIPCHK(c, up(sm, ws, o.angle_ijk, c->angle_ijk));
    HIPCHK(c, up(sm, ws, o.angle_kt, c->angle_kt));
    HIPCHK(c, up(sm, ws, o.reps, c->reps));
    HIPCHK(c, up(sm, ws, o.unit, bound_units(c)));
    HIPCHK(c, up(sm, ws, o.Lq, c->Lq));
    HIPCHK(c, up(sm, ws, o.tparams, c->tparams));
    HIPCHK(c, up(sm, ws, o.tab_f, c->tab_f));
    HIPCHK(c, up(sm, ws, o.tab_d, c->tab_d));
    HIPCHK(c, up(sm, ws, o.rep_off, c->rep_off));
    HIPCHK(c, up(sm, ws, o.cell_rep, c->cell_rep));
    std::vector<int64_t> one = {0, c->n};
    HIPCHK(c, up(sm, ws, o.one_seg, one));
    HIPCHK(c, hipMemsetAsync(ws + o.st, 0, sizeof(DevState), sm));
    HIPCHK(c, hipMemsetAsync(ws + o.cnt, 0, sizeof(RepCounters) * CNT_SPREAD * c->R, sm));
    HIPCHK(c, hipMemsetAsync(ws + o.wave_cnt, 0, 8 * 3 * (size_t)wave_slots(c), sm));
    HIPCHK(c, up(sm, ws, o.fitems, c->fitems));
    HIPCHK(c, up(sm, ws, o.fneed, c->fneed));
    HIPCHK(c, hipMemsetAsync(ws + o.fqueue, 0, 4 * ((size_t)c->R + 1), sm));
    HIPCHK(c, up(sm, ws, o.clu, c->clu));
    HIPCHK(c, up(sm, ws, o.cl_first, c->cl_first));
    c->cs.clu = at<int4>(ws, o.clu);
    c->cs.rep_first = at<int32_t>(ws, o.cl_first);
    c->cs.ctr = at<int4>(ws, o.cl_ctr);
    c->cs.half = at<float4>(ws, o.cl_half);
    c->cs.cnt = at<int32_t>(ws, o.cl_cnt);
    c->cs.list = at<int32_t>(ws, o.cl_list);
    c->cs.ncl = (int32_t)c->clu.size();
    c->cs.cap = c->cl_cap;
    c->cs.cl = c->p.pair_kernel;
    c->fused.items = at<int4>(ws, o.fitems);
    c->fused.need = at<int32_t>(ws, o.fneed);
    c->fused.queue = at<uint32_t>(ws, o.fqueue);
    c->fused.n_items = (int32_t)c->fitems.size();
    c->fused.n_reps = c->R;
    {
        // at most as many workgroups as can be resident, and no more than the
        // integrator items (the one-replica jump counters have a slot per wavefront)
        const int32_t steps = (int32_t)(c->fitems.size()) - [&] { int32_t s = 0; for (int32_t v : c->fneed) s += v; return s; }();
        c->fused_grid = std::max(1, std::min(fused_resident_groups(c->p.pair_precision == BOUNCE_PAIR_FP64,
                                                                   c->p.integrator == BOUNCE_BJAOAJB),
                                             steps));
    }
    Topo &t = c->tp;
    t.type = at<int32_t>(ws, o.type);
    t.rep_of = at<int32_t>(ws, o.rep_of);
    t.acc_m = at<double>(ws, o.acc_m);
    t.inv_mass = at<double>(ws, o.inv_mass);
    t.excl_ptr = at<int32_t>(ws, o.excl_ptr);
    t.excl_idx = at<int32_t>(ws, o.excl_idx);
    t.bt_ptr = at<int32_t>(ws, o.bt_ptr);
    t.bt = at<int32_t>(ws, o.bt);
    t.bond_ij = at<int32_t>(ws, o.bond_ij);
    t.bond_kr = at<double>(ws, o.bond_kr);
    t.angle_ijk = at<int32_t>(ws, o.angle_ijk);
    t.angle_kt = at<double>(ws, o.angle_kt);
    c->d_reps = at<RepInfo>(ws, o.reps);
    c->d_unit = at<double>(ws, o.unit);
    c->d_Lq = at<uint32_t>(ws, o.Lq);
    c->d_tparams = at<double>(ws, o.tparams);
    c->d_tab_f = at<TypePair<float>>(ws, o.tab_f);
    c->d_tab_d = at<TypePair<double>>(ws, o.tab_d);
    c->d_rep_off = at<int64_t>(ws, o.rep_off);
    c->d_cell_rep = at<int32_t>(ws, o.cell_rep);
    c->d_one_seg = at<int64_t>(ws, o.one_seg);
    c->d_st = at<DevState>(ws, o.st);
    c->d_cnt = at<RepCounters>(ws, o.cnt);
    c->d_wave_cnt = at<unsigned long long>(ws, o.wave_cnt);
    c->d_events = at<Event>(ws, o.events);
    c->d_fpair = at<double>(ws, o.fpair);
    c->d_atom = at<double>(ws, o.atom);
    c->d_seg = at<double>(ws, o.seg);
    c->d_rdf = at<unsigned long long>(ws, o.rdf);
    c->d_grid = at<double2>(ws, o.grid);
    c->d_theta = at<double>(ws, o.theta);
    c->d_grec = at<double>(ws, o.grec);
    c->d_pme_e = at<double>(ws, o.pme_e);
    c->pme_atoms.fl = at<int4>(ws, o.pme_fl);
    c->pme_atoms.f = at<double4>(ws, o.pme_f);
    c->pme_atoms.w = at<double>(ws, o.pme_w);
    c->d_charge = at<double>(ws, o.tparams);     // per-type charges: the first n_types parameters
    if (c->pme) HIPCHK(c, up(sm, ws, o.theta, c->theta));
    HIPCHK(c, hipMemsetAsync(c->d_grec, 0, 24 * (size_t)c->n, sm));
    c->d_ou_c2 = at<double>(ws, o.ou_c2);
    c->d_xcnt = at<int32_t>(ws, o.xcnt);
    c->d_xcol = at<int32_t>(ws, o.xcol);
    for (int k = 0; k < 2; ++k) {
        ListSet &ls = k == 0 ? c->main : c->aux;
        size_t *q = o.ls[k];
        ls.perm = at<int32_t>(ws, q[0]);
        ls.inv_perm = at<int32_t>(ws, q[1]);
        ls.cell_of = at<int32_t>(ws, q[2]);
        ls.slot = at<int32_t>(ws, q[3]);
        ls.cell_count = at<int32_t>(ws, q[4]);
        ls.cell_start = at<int32_t>(ws, q[5]);
        ls.x[0] = at<double4>(ws, q[6]);
        ls.x[1] = at<double4>(ws, q[7]);
        ls.q_build = at<double>(ws, q[8]);
        ls.fcnt = at<int2>(ws, q[9]);
        ls.flist = at<int32_t>(ws, q[10]);
        ls.ccnt = at<int32_t>(ws, q[11]);
        ls.ncls = k == 0 ? c->ncls : 1;
        ls.clist = at<int32_t>(ws, q[11]) + (int64_t)c->n * ls.ncls;
        ls.bslot = k == 0 ? at<int4>(ws, q[12]) : nullptr;
        ls.sinfo = at<int2>(ws, q[13]);
        ls.scan_part = at<int32_t>(ws, q[14]);
        ls.busy = at<int32_t>(ws, q[17]);
        ls.fcap = k == 0 ? c->fcap : c->acap;
        ls.ccap = k == 0 ? c->ccap : 0;
        ls.n_cells = c->n_cells;
        const bool fx = k == 0 && c->fixed;
        ls.xf[0] = fx ? at<int4>(ws, q[15]) : nullptr;
        ls.xf[1] = fx ? at<int4>(ws, q[16]) : nullptr;
        HIPCHK(c, hipMemsetAsync(ls.cell_count, 0, 4 * (size_t)c->n_cells, sm));
    }
    HIPCHK(c, hipStreamSynchronize(sm));
    if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    c->step = 0;
    c->pending = 0;
    c->built_step = -1;
    c->host_steps = 0;
    c->host_rebuilds = 0;
    c->bound = true;
    return BOUNCE_OK;
}

bounce_status bounce_update_params(bounce_ctx *c, const bounce_params *p)
{
    if (!c || !p) return BOUNCE_E_ARG;
    if (!(p->dt > 0) || !(p->gamma >= 0) || !(p->temperature > 0) || !(p->bound_scale > 0))
        return fail(c, BOUNCE_E_ARG, "dt, gamma, temperature, bound_scale");
    c->p.dt = p->dt;
    c->p.gamma = p->gamma;
    c->p.temperature = p->temperature;
    c->p.bound_scale = p->bound_scale;
    if (!c->have_system) return BOUNCE_OK;
    make_ou(c);
    if (c->bound) {
        Layout L;
        Offsets o;
        plan(c, L, o);
        HIPCHK(c, up(c->stream, c->ws, o.ou_c2, c->ou_c2));
        HIPCHK(c, up(c->stream, c->ws, o.unit, bound_units(c)));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
        if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    }
    return BOUNCE_OK;
}

static bounce_status ready(bounce_ctx *c)
{
    if (!c) return BOUNCE_E_ARG;
    if (!c->have_system || !c->bound) return fail(c, BOUNCE_E_STATE, "set_system and bind first");
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[c->static_dev] != c) {
            c->bound = false;
            return fail(c, BOUNCE_E_STATE,
                        "another context was bound to this device's static workspace; bind again");
        }
    }
    return BOUNCE_OK;
}

bounce_status bounce_set_step(bounce_ctx *c, int64_t step)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (step < 0) return BOUNCE_E_ARG;
    DevState st{};
    st.step = step;
    HIPCHK(c, hipMemcpyAsync(c->d_st, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->step = step;
    c->pending = 0;
    c->built_step = -1;
    return BOUNCE_OK;
}

bounce_status bounce_get_step(const bounce_ctx *c, int64_t *step)
{
    if (!c || !step) return BOUNCE_E_ARG;
    *step = c->step;
    return BOUNCE_OK;
}

static PairGlobals pair_globals(const bounce_ctx *c)
{
    PairGlobals g{};
    g.alpha = c->p.ewald_alpha;
    g.r_on = c->p.r_on;
    g.r_off = c->p.r_off;
    g.inv_w = c->p.r_off > c->p.r_on ? 1.0 / (c->p.r_off - c->p.r_on) : 0.0;
    g.split = c->p.jump_split;
    g.r_on_v = c->p.r_on_lj;
    g.inv_w_v = c->p.r_off_lj > c->p.r_on_lj ? 1.0 / (c->p.r_off_lj - c->p.r_on_lj) : 0.0;
    g.r_short = r_short(c->p);
    g.r_cut = c->p.r_cut;
    g.coulomb = c->p.coulomb;
    g.n_types = c->nt;
    return g;
}

static BuildSpec main_spec(const bounce_ctx *c)
{
    BuildSpec b{};
    const bounce_params &p = c->p;
    if (p.integrator == BOUNCE_BJAOAJB) {
        double rf = r_short(p) + p.skin, rn = r_short(p) + 0.5 * p.skin;
        double rmin = r_long(p) - p.skin, rmax = p.r_cut + p.skin;
        b.rf2 = rf * rf;
        b.rfn2 = rn * rn;
        b.rcmin2 = rmin > 0.0 ? rmin * rmin : 0.0;
        b.rcmax2 = rmax * rmax;
        b.rsearch = std::max(rf, rmax);
        b.want_force = 1;
        b.want_cand = 1;
    } else {
        double rf = p.r_cut + p.skin, rn = p.r_cut + 0.5 * p.skin;
        b.rf2 = rf * rf;
        b.rfn2 = rn * rn;
        b.rsearch = rf;
        b.want_force = 1;
        b.want_cand = 0;
    }
    b.mirror_sel = -1;
    return b;
}

static void enqueue_build(bounce_ctx *c, int32_t step_off)
{
    BuildSpec b = main_spec(c);
    b.step_off = step_off;
    launch_build(c->stream, c->n, c->pos, c->d_reps, c->d_cell_rep, c->tp, c->main, b, c->d_st);
    if (c->p.pair_kernel) {
        // the cluster boxes may be apart by up to the force list's radius (plus
        // 1e-3 A for the FP32 rounding of the box test)
        const double rl = (c->p.integrator == BOUNCE_BJAOAJB ? r_short(c->p) : c->p.r_cut) + c->p.skin + 1e-3;
        launch_cluster_build(c->stream, c->cs, c->main, c->d_reps, c->d_st, -1, step_off, (float)rl);
    }
    launch_reset_disp(c->stream, c->d_st);
}

static PairArgs pair_args(bounce_ctx *c, const ListSet &ls, int mirror_sel)
{
    PairArgs a{};
    a.n = c->n;
    a.mirror_sel = mirror_sel;
    a.single_rep = c->R == 1;
    a.reps = c->d_reps;
    a.tp = c->tp;
    a.ls = ls;
    a.st = c->d_st;
    a.type_params = c->d_tparams;
    a.tab_f = c->d_tab_f;
    a.tab_d = c->d_tab_d;
    a.pg = pair_globals(c);
    return a;
}

// the short-range pair force (F_0's pair part, or the outer step's) into out,
// sorted order
static void launch_step_pair(bounce_ctx *c, int32_t step_off, double *out)
{
    PairArgs a = pair_args(c, c->main, -1);
    a.step_off = step_off;
    // far partners (>= lim + s/2 at the build) stay out of range while
    // 2 max|displacement| < s/2; the 1e-3 A margin covers rounding
    a.far_gate = 0.5 * c->p.skin - 1e-3 > 0.0;
    a.out = out;
    a.out_global = 0;
    a.accumulate = 0;
    const int mode = c->p.integrator == BOUNCE_BJAOAJB ? MODE_SHORT : MODE_FULL;
    if (c->p.pair_kernel) launch_pair_cl(c->stream, mode, a, c->cs);
    else launch_pair(c->stream, mode, c->p.pair_precision == BOUNCE_PAIR_FP64, c->p.pair_lanes, a);
}

static void enqueue_force(bounce_ctx *c, int32_t step_off)
{
    if (!c->out_pair) launch_step_pair(c, step_off, c->d_fpair);
}

static PmeArgs pme_args(const bounce_ctx *c, int32_t step_off, int32_t mirror_sel)
{
    PmeArgs pa{};
    const RepInfo &ri = c->reps[0];
    for (int k = 0; k < 3; ++k) {
        pa.K[k] = c->p.pme_grid[k];
        pa.box[k] = ri.box[k];
        pa.inv_box[k] = ri.inv_box[k];
    }
    pa.order = c->p.pme_order;
    pa.alpha = c->p.ewald_alpha;
    pa.st = c->d_st;
    pa.step_off = step_off;
    pa.mirror_sel = mirror_sel;
    pa.qscale = c->pme_qscale;
    pa.inv_qscale = 1.0 / c->pme_qscale;
    for (int k = 0; k < 3; ++k) {
        pa.ncell[k] = ri.ncell[k];
        pa.cw[k] = ri.cw[k];
    }
    // an atom lies within s/2 of the cell it was listed in (the skin guard);
    // the small extra covers rounding at cell edges
    pa.margin = 0.5 * c->p.skin + 1e-9 * std::max(ri.box[0], std::max(ri.box[1], ri.box[2]));
    return pa;
}

// step n is the boundary of a RESPA outer step
static bool outer_at(const bounce_ctx *c, int64_t n)
{
    return c->outer && n % c->p.respa_m == 0;
}

// the forces of step n beyond F_0's own (device offset step_off): the mesh
// force into F_0's pair part every step (respa_m = 0), or, at an outer
// boundary, the outer gradient (mesh force and/or short-range pair force)
static void enqueue_extra(bounce_ctx *c, int64_t n, int32_t step_off)
{
    if (c->pme && c->p.respa_m == 0) {
        launch_pme(c->stream, c->n, c->main, c->pos, c->d_charge, c->tp, pme_args(c, step_off, -1),
                   c->pme_atoms, c->d_grid, c->d_theta, c->d_fpair, 0, 1, nullptr);
        return;
    }
    if (!outer_at(c, n)) return;
    if (c->out_pair) launch_step_pair(c, step_off, c->d_grec);
    if (c->pme)
        launch_pme(c->stream, c->n, c->main, c->pos, c->d_charge, c->tp, pme_args(c, step_off, -1),
                   c->pme_atoms, c->d_grid, c->d_theta, c->d_grec, 0, c->out_pair ? 1 : 0, nullptr);
}

static StepArgs step_args(bounce_ctx *c, int close, int open, int32_t step_off)
{
    StepArgs a{};
    a.n = c->n;
    a.step_off = step_off;
    a.single_rep = c->R == 1;
    a.do_close = close;
    a.do_open = open;
    a.bounce = c->p.integrator == BOUNCE_BJAOAJB;
    a.pair_fp64 = c->p.pair_precision == BOUNCE_PAIR_FP64;
    a.log_events = c->p.log_events;
    a.max_proposals = c->p.max_proposals;
    a.reps = c->d_reps;
    a.tp = c->tp;
    a.ls = c->main;
    a.grec = c->d_grec;
    a.rec_close = a.rec_open = 0.0;
    a.f0_pair = c->out_pair ? 0 : 1;
    a.st = c->d_st;
    a.cnt = c->d_cnt;
    a.wave_cnt = c->d_wave_cnt;
    a.events = c->d_events;
    a.event_cap = c->p.log_events ? c->p.event_capacity : 0;
    a.fpair = c->d_fpair;
    a.pos = c->pos;
    a.vel = c->vel;
    a.ou_c2 = c->d_ou_c2;
    a.Lunit = c->d_unit;
    a.Lq = c->d_Lq;
    a.tab_f = c->d_tab_f;
    a.tab_d = c->d_tab_d;
    a.pg = pair_globals(c);
    a.dt = c->p.dt;
    a.half_dt = 0.5 * c->p.dt;
    a.c1 = std::exp(-c->p.gamma * c->p.dt);
    a.beta = 1.0 / (KB * c->p.temperature);
    a.skin_half2 = 0.25 * c->p.skin * c->p.skin;
    {
        const double g = 0.5 * (0.5 * c->p.skin - 1e-3);
        a.far_gate2 = g > 0.0 ? g * g : 0.0;
    }
    return a;
}

// one launch per step (F_0 pair force + integrator): only where F_0 carries the
// short-range pair force and no mesh force
static bool use_fused(const bounce_ctx *c)
{
    return c->p.persistent && !c->p.pair_kernel && !c->out_pair && !(c->pme && c->p.respa_m == 0) &&
           !c->outer;
}

static void launch_fused_step(bounce_ctx *c, const StepArgs &a, int32_t step_off)
{
    PairArgs p = pair_args(c, c->main, -1);
    p.step_off = step_off;
    p.far_gate = 0.5 * c->p.skin - 1e-3 > 0.0;
    p.out = c->d_fpair;
    p.out_global = 0;
    p.accumulate = 0;
    launch_fused(c->stream, a, p, c->fused, c->fused_grid);
}

// one substep of the fused schedule at the current step index c->step
// (= device counter + c->pending once the launches before it have run)
// (e0, e1: optional events recorded around the integrator kernel alone)
static void enqueue_substep(bounce_ctx *c, int close, int open, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr)
{
    if (c->built_step < 0 || (c->step % c->p.rebuild_interval == 0 && c->built_step != c->step)) {
        enqueue_build(c, c->pending);
        c->built_step = c->step;
        c->host_rebuilds++;
    }
    if (use_fused(c)) {
        if (e0) (void)hipEventRecord(e0, c->stream);
        launch_fused_step(c, step_args(c, close, open, c->pending), c->pending);
        if (e1) (void)hipEventRecord(e1, c->stream);
        if (open) {
            c->step++;
            c->pending++;
        }
        return;
    }
    enqueue_force(c, c->pending);
    enqueue_extra(c, c->step, c->pending);
    StepArgs a = step_args(c, close, open, c->pending);
    if (outer_at(c, c->step)) {
        // step n = c->step ends one RESPA block (close) and starts the next (open)
        const double H = 0.5 * c->p.dt * (double)c->p.respa_m;
        a.rec_close = close ? H : 0.0;
        a.rec_open = open ? H : 0.0;
    }
    if (e0) (void)hipEventRecord(e0, c->stream);
    launch_step(c->stream, a);
    if (e1) (void)hipEventRecord(e1, c->stream);
    if (open) {
        c->step++;
        c->pending++;
    }
}

// bring the device step counter up to c->step
static void flush_pending(bounce_ctx *c)
{
    launch_advance(c->stream, c->d_st, c->pending);
    c->pending = 0;
}

// a graph of K fused steps starting at a multiple of K (rebuild at its head)
static bounce_status make_graph(bounce_ctx *c)
{
    if (c->graph_exec) return BOUNCE_OK;
    hipStream_t cap;
    HIPCHK(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t saved = c->stream;
    c->stream = cap;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        c->stream = saved;
        (void)hipStreamDestroy(cap);
        return fail(c, BOUNCE_E_HIP, std::string("capture: ") + hipGetErrorString(e));
    }
    for (int k = 0; k < c->p.rebuild_interval; ++k) {
        if (k == 0) enqueue_build(c, 0);
        if (use_fused(c)) {
            launch_fused_step(c, step_args(c, 1, 1, k), k);
            continue;
        }
        enqueue_force(c, k);
        // the graph starts at a multiple of K, and K is a multiple of respa_m
        StepArgs a = step_args(c, 1, 1, k);
        enqueue_extra(c, k, k);
        if (outer_at(c, k)) a.rec_close = a.rec_open = 0.5 * c->p.dt * (double)c->p.respa_m;
        launch_step(c->stream, a);
    }
    launch_advance(c->stream, c->d_st, c->p.rebuild_interval);
    e = hipStreamEndCapture(cap, &c->graph);
    c->stream = saved;
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return fail(c, BOUNCE_E_HIP, std::string("end capture: ") + hipGetErrorString(e));
    HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    return BOUNCE_OK;
}

bounce_status bounce_step(bounce_ctx *c, int32_t n_steps)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (n_steps < 0) return BOUNCE_E_ARG;
    if (n_steps == 0) return BOUNCE_OK;
    const int64_t K = c->p.rebuild_interval;
    const int64_t end = c->step + n_steps;
    // open the first step (F_0 at q_n)
    enqueue_substep(c, 0, 1);
    while (c->step < end) {
        if (c->p.use_graph && c->step % K == 0 && c->step + K <= end) {
            s = make_graph(c);
            if (s) return s;
            flush_pending(c);
            HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
            c->step += K;
            c->built_step = c->step - K;
            c->host_rebuilds++;
            continue;
        }
        enqueue_substep(c, 1, 1);
    }
    // close the last step: J(n-1, JB), B(dt/2) with F_0 at q_n
    enqueue_substep(c, 1, 0);
    flush_pending(c);
    c->host_steps += n_steps;
    HIPCHK(c, hipGetLastError());
    return BOUNCE_OK;
}

static bounce_status status_from_bits(bounce_ctx *c, uint32_t bits)
{
    if (!bits) return BOUNCE_OK;
    if (bits & ST_NONFINITE) return fail(c, BOUNCE_E_NONFINITE, bounce_status_string(BOUNCE_E_NONFINITE));
    if (bits & ST_GRID) return fail(c, BOUNCE_E_GRID, bounce_status_string(BOUNCE_E_GRID));
    if (bits & ST_CAPACITY) return fail(c, BOUNCE_E_CAPACITY, bounce_status_string(BOUNCE_E_CAPACITY));
    if (bits & ST_SKIN) return fail(c, BOUNCE_E_SKIN, bounce_status_string(BOUNCE_E_SKIN));
    if (bits & ST_POISSON) return fail(c, BOUNCE_E_POISSON_CAP, bounce_status_string(BOUNCE_E_POISSON_CAP));
    if (bits & ST_BOUND) return fail(c, BOUNCE_E_BOUND, bounce_status_string(BOUNCE_E_BOUND));
    return BOUNCE_OK;
}

bounce_status bounce_sync(bounce_ctx *c)
{
    bounce_status s = ready(c);
    if (s) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    DevState st;
    HIPCHK(c, hipMemcpy(&st, c->d_st, sizeof st, hipMemcpyDeviceToHost));
    if (st.step != c->step)
        return fail(c, BOUNCE_E_STATE, "device step counter out of step with the host");
    return status_from_bits(c, st.status);
}

static BuildSpec aux_spec(const bounce_ctx *c)
{
    BuildSpec b{};
    double r = c->p.r_cut + 0.01;
    b.rf2 = r * r;
    b.rfn2 = b.rf2;       // used at the build positions only: every entry near
    b.rsearch = r;
    b.want_force = 1;
    b.want_cand = 0;
    b.mirror_sel = 0;
    return b;
}

bounce_status bounce_compute_gradient(bounce_ctx *c, int32_t which, double *grad)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!grad || (which & ~63) || !which) return BOUNCE_E_ARG;
    if ((which & BOUNCE_G_RECIP) && !c->pme) return fail(c, BOUNCE_E_ARG, "G_RECIP needs pme_grid");
    hipStream_t sm = c->stream;
    const int pairs[3] = {BOUNCE_G_SHORT, BOUNCE_G_LONG, BOUNCE_G_FULL};
    const int modes[3] = {MODE_SHORT, MODE_LONG, MODE_FULL};
    int first = 1;
    if (which & BOUNCE_G_STEP) {
        // the integrator's own list and pair kernel, into caller order: the
        // lists and position mirrors the steps maintain, rebuilt first only
        // where the next step would rebuild them
        if (c->built_step < 0 ||
            (c->step % c->p.rebuild_interval == 0 && c->built_step != c->step)) {
            enqueue_build(c, 0);
            c->built_step = c->step;
            c->host_rebuilds++;
        }
        PairArgs a = pair_args(c, c->main, -1);
        a.far_gate = 0.5 * c->p.skin - 1e-3 > 0.0;
        a.out = grad;
        a.out_global = 1;
        a.accumulate = 0;
        const int mode = c->p.integrator == BOUNCE_BJAOAJB ? MODE_SHORT : MODE_FULL;
        if (c->p.pair_kernel) launch_pair_cl(sm, mode, a, c->cs);
        else launch_pair(sm, mode, c->p.pair_precision == BOUNCE_PAIR_FP64, c->p.pair_lanes, a);
        first = 0;
    }
    if (which & (BOUNCE_G_SHORT | BOUNCE_G_LONG | BOUNCE_G_FULL))
        launch_build(sm, c->n, c->pos, c->d_reps, c->d_cell_rep, c->tp, c->aux, aux_spec(c), c->d_st);
    for (int k = 0; k < 3; ++k) {
        if (!(which & pairs[k])) continue;
        PairArgs a = pair_args(c, c->aux, 0);
        a.out = grad;
        a.out_global = 1;
        a.accumulate = !first;
        launch_pair(sm, modes[k], c->p.pair_precision == BOUNCE_PAIR_FP64, c->p.pair_lanes, a);
        first = 0;
    }
    if (which & BOUNCE_G_RECIP) {
        if (!(which & (BOUNCE_G_SHORT | BOUNCE_G_LONG | BOUNCE_G_FULL)))
            launch_build(sm, c->n, c->pos, c->d_reps, c->d_cell_rep, c->tp, c->aux, aux_spec(c), c->d_st);
        launch_pme(sm, c->n, c->aux, c->pos, c->d_charge, c->tp, pme_args(c, 0, 0), c->pme_atoms, c->d_grid,
                   c->d_theta,
                   grad, 1, first ? 0 : 1, nullptr);
        first = 0;
    }
    if (which & BOUNCE_G_BONDED) {
        if (first) HIPCHK(c, hipMemsetAsync(grad, 0, 24 * (size_t)c->n, sm));
        launch_bonded_grad(sm, c->n, c->pos, c->d_reps, c->tp, grad);
    }
    return bounce_sync(c);
}

bounce_status bounce_compute_energies(bounce_ctx *c, double *out)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!out) return BOUNCE_E_ARG;
    hipStream_t sm = c->stream;
    launch_build(sm, c->n, c->pos, c->d_reps, c->d_cell_rep, c->tp, c->aux, aux_spec(c), c->d_st);
    PairArgs a = pair_args(c, c->aux, 0);
    a.atom_out = c->d_atom;
    a.energy_total = 0;
    a.atom_stride = 5;
    a.atom_col = 2;
    launch_pair(sm, MODE_ENERGY, c->p.pair_precision == BOUNCE_PAIR_FP64, c->p.pair_lanes, a);
    launch_atom_energy(sm, c->n, c->pos, c->vel, c->d_reps, c->tp, c->d_atom);
    launch_segment_sum(sm, c->R, c->d_rep_off, c->d_atom, 5, 5, 0, c->d_seg);
    std::vector<double> seg(5 * c->R);
    HIPCHK(c, hipMemcpyAsync(seg.data(), c->d_seg, 8 * seg.size(), hipMemcpyDeviceToHost, sm));
    s = bounce_sync(c);
    if (s) return s;
    double emesh[3] = {0.0, 0.0, 0.0};
    if (c->pme) {
        s = bounce_pme_energy(c, emesh);
        if (s) return s;
    }
    for (int32_t r = 0; r < c->R; ++r) {
        const double *v = &seg[5 * r];
        double *o = out + 7 * r;
        int64_t na = c->rep_off[r + 1] - c->rep_off[r];
        const double ec = v[2] + (emesh[0] + emesh[1] + emesh[2]);   // one replica when meshed
        o[0] = v[0]; o[1] = v[1]; o[2] = ec; o[3] = v[3]; o[4] = ec + v[3]; o[5] = v[4];
        o[6] = 2.0 * v[4] / (3.0 * (double)na * KB);
    }
    return BOUNCE_OK;
}

bounce_status bounce_get_counters(bounce_ctx *c, int32_t replica, bounce_counters *out)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!out || replica < 0 || replica >= c->R) return BOUNCE_E_ARG;
    std::vector<RepCounters> rc(CNT_SPREAD);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(rc.data(), c->d_cnt + (int64_t)replica * CNT_SPREAD,
                        sizeof(RepCounters) * CNT_SPREAD, hipMemcpyDeviceToHost));
    out->proposals = out->accepted = out->bound_violations = 0;
    for (const RepCounters &k : rc) {
        out->proposals += (int64_t)k.proposals;
        out->accepted += (int64_t)k.accepted;
        out->bound_violations += (int64_t)k.bound_violations;
    }
    if (c->R == 1) {
        std::vector<unsigned long long> wc(3 * (size_t)wave_slots(c));
        HIPCHK(c, hipMemcpy(wc.data(), c->d_wave_cnt, 8 * wc.size(), hipMemcpyDeviceToHost));
        for (size_t k = 0; k < wc.size(); k += 3) {
            out->proposals += (int64_t)wc[k];
            out->accepted += (int64_t)wc[k + 1];
            out->bound_violations += (int64_t)wc[k + 2];
        }
    }
    out->rebuilds = c->host_rebuilds;
    out->steps = c->host_steps;
    return BOUNCE_OK;
}

bounce_status bounce_get_events(bounce_ctx *c, bounce_event *host, int64_t cap, int64_t *n_total)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!n_total || cap < 0 || (cap > 0 && !host)) return BOUNCE_E_ARG;
    DevState st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&st, c->d_st, sizeof st, hipMemcpyDeviceToHost));
    *n_total = st.n_events;
    int64_t kept = std::min<int64_t>(st.n_events, c->p.log_events ? c->p.event_capacity : 0);
    int64_t k = std::min<int64_t>(kept, cap);
    static_assert(sizeof(Event) == sizeof(bounce_event), "event layout");
    if (k > 0) HIPCHK(c, hipMemcpy(host, c->d_events, sizeof(Event) * k, hipMemcpyDeviceToHost));
    return BOUNCE_OK;
}

bounce_status bounce_get_list(bounce_ctx *c, int32_t which, int64_t *row_ptr, int32_t *col,
                              int64_t cap)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!row_ptr || (which != BOUNCE_LIST_FORCE && which != BOUNCE_LIST_CAND)) return BOUNCE_E_ARG;
    if (which == BOUNCE_LIST_CAND && c->p.integrator != BOUNCE_BJAOAJB) return BOUNCE_E_ARG;
    if (c->built_step < 0) return fail(c, BOUNCE_E_STATE, "no list built yet");
    int32_t rcap = which == 0 ? c->fcap : c->ccap;
    launch_list_to_global(c->stream, c->n, c->main, which, c->d_xcnt, c->d_xcol, rcap);
    s = bounce_sync(c);
    if (s) return s;
    std::vector<int32_t> cnt(c->n);
    std::vector<int32_t> rows((size_t)c->n * rcap);
    HIPCHK(c, hipMemcpy(cnt.data(), c->d_xcnt, 4 * (size_t)c->n, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(rows.data(), c->d_xcol, 4 * rows.size(), hipMemcpyDeviceToHost));
    row_ptr[0] = 0;
    for (int32_t g = 0; g < c->n; ++g) row_ptr[g + 1] = row_ptr[g] + cnt[g];
    if (row_ptr[c->n] > cap) return fail(c, BOUNCE_E_ARG, "col capacity too small");
    for (int32_t g = 0; g < c->n; ++g)
        std::memcpy(col + row_ptr[g], &rows[(size_t)g * rcap], 4 * (size_t)cnt[g]);
    return BOUNCE_OK;
}

bounce_status bounce_rate_bounds(const bounce_ctx *c, double *L_ab, double *L_a)
{
    if (!c || !L_ab || !L_a) return BOUNCE_E_ARG;
    if (!c->have_system) return BOUNCE_E_STATE;
    std::memcpy(L_ab, c->L_ab.data(), 8 * c->L_ab.size());
    std::memcpy(L_a, c->L_a.data(), 8 * c->L_a.size());
    return BOUNCE_OK;
}

bounce_status bounce_pme_energy(bounce_ctx *c, double *e3)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!e3) return BOUNCE_E_ARG;
    if (!c->pme) return fail(c, BOUNCE_E_ARG, "no PME mesh (pme_grid)");
    hipStream_t sm = c->stream;
    launch_build(sm, c->n, c->pos, c->d_reps, c->d_cell_rep, c->tp, c->aux, aux_spec(c), c->d_st);
    const PmeArgs pa = pme_args(c, 0, 0);
    launch_pme(sm, c->n, c->aux, c->pos, c->d_charge, c->tp, pa, c->pme_atoms, c->d_grid, c->d_theta, nullptr,
               0, 0,
               c->d_pme_e);
    launch_pme_excl_energy(sm, c->n, c->pos, c->d_charge, c->tp, pa, c->d_atom);
    launch_segment_sum(sm, 1, c->d_one_seg, c->d_atom, 1, 1, 0, c->d_seg);
    const int64_t nb = pme_energy_parts(pa);
    std::vector<double> part(nb), ex(1);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->d_pme_e, 8 * nb, hipMemcpyDeviceToHost, sm));
    HIPCHK(c, hipMemcpyAsync(ex.data(), c->d_seg, 8, hipMemcpyDeviceToHost, sm));
    s = bounce_sync(c);
    if (s) return s;
    double er = 0.0;
    for (int64_t b = 0; b < nb; ++b) er += part[b];
    double q2 = 0.0;
    for (int32_t g = 0; g < c->n; ++g) q2 += c->tparams[c->type[g]] * c->tparams[c->type[g]];
    e3[0] = er;
    e3[1] = -KE * c->p.ewald_alpha / std::sqrt(M_PI) * q2;
    e3[2] = ex[0];
    return BOUNCE_OK;
}

bounce_status bounce_rdf_counts(bounce_ctx *c, double r_max, int32_t n_bins, uint64_t *counts)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!counts || !(r_max > 0.0) || !(r_max <= c->p.r_cut) || n_bins < 1 ||
        (int64_t)c->nt * c->nt * n_bins > RDF_MAX_BINS)
        return fail(c, BOUNCE_E_ARG, "rdf: 0 < r_max <= r_cut and n_types^2 n_bins <= 8192");
    hipStream_t sm = c->stream;
    const size_t nh = (size_t)c->nt * c->nt * n_bins;
    // the aux list set: every non-excluded pair within r_cut + 0.01 at the current positions
    launch_build(sm, c->n, c->pos, c->d_reps, c->d_cell_rep, c->tp, c->aux, aux_spec(c), c->d_st);
    HIPCHK(c, hipMemsetAsync(c->d_rdf, 0, 8 * nh, sm));
    launch_rdf(sm, c->n, c->d_reps, c->R == 1, c->aux, r_max, n_bins, c->nt, c->d_rdf);
    HIPCHK(c, hipMemcpyAsync(counts, c->d_rdf, 8 * nh, hipMemcpyDeviceToHost, sm));
    return bounce_sync(c);
}

bounce_status bounce_msd(bounce_ctx *c, const double *ref, double *out)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!ref || !out) return BOUNCE_E_ARG;
    hipStream_t sm = c->stream;
    launch_msd_atom(sm, c->n, c->pos, ref, c->tp.type, c->d_atom);
    launch_segment_sum(sm, c->R, c->d_rep_off, c->d_atom, c->nt, MAXT, 0, c->d_seg);
    std::vector<double> seg((size_t)c->R * c->nt);
    HIPCHK(c, hipMemcpyAsync(seg.data(), c->d_seg, 8 * seg.size(), hipMemcpyDeviceToHost, sm));
    s = bounce_sync(c);
    if (s) return s;
    for (int32_t r = 0; r < c->R; ++r) {
        std::vector<int64_t> cnt(c->nt, 0);
        for (int64_t g = c->rep_off[r]; g < c->rep_off[r + 1]; ++g) cnt[c->type[g]]++;
        for (int a = 0; a < c->nt; ++a)
            out[(int64_t)r * c->nt + a] = cnt[a] ? seg[(size_t)r * c->nt + a] / (double)cnt[a] : 0.0;
    }
    return BOUNCE_OK;
}

bounce_status bounce_rate_weights(const bounce_ctx *c, uint32_t *Lq, double *unit)
{
    if (!c || !Lq || !unit) return BOUNCE_E_ARG;
    if (!c->have_system) return BOUNCE_E_STATE;
    const std::vector<double> u = bound_units(c);
    const int w = c->nmech * c->nt;
    for (int a = 0; a < c->nt; ++a) {
        unit[a] = u[a];
        for (int k = 0; k < w; ++k) Lq[a * w + k] = c->Lq[a * LQW + k];
    }
    return BOUNCE_OK;
}

bounce_status bounce_jump_halfstep(bounce_ctx *c, int64_t step, int32_t phase)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (c->p.integrator != BOUNCE_BJAOAJB) return fail(c, BOUNCE_E_ARG, "BAOAB has no J step");
    if (phase != BOUNCE_PH_JA && phase != BOUNCE_PH_JB) return BOUNCE_E_ARG;
    if (c->built_step != c->step) {
        enqueue_build(c, 0);
        c->built_step = c->step;
        c->host_rebuilds++;
    }
    JumpArgs ja{};
    ja.s = step_args(c, 0, 0, 0);
    ja.step = step;
    ja.phase = phase;
    launch_jump(c->stream, ja);
    return bounce_sync(c);
}

bounce_status bounce_direct_energy(bounce_ctx *c, const double *pos, const double *params,
                                   double *energy)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!pos || !params || !energy) return BOUNCE_E_ARG;
    hipStream_t sm = c->stream;
    launch_build(sm, c->n, pos, c->d_reps, c->d_cell_rep, c->tp, c->aux, aux_spec(c), c->d_st);
    PairArgs a = pair_args(c, c->aux, 0);
    a.type_params = params;
    a.tab_f = nullptr;
    a.tab_d = nullptr;
    a.atom_out = c->d_atom;
    a.energy_total = 1;
    launch_pair(sm, MODE_ENERGY, c->p.pair_precision == BOUNCE_PAIR_FP64, c->p.pair_lanes, a);
    launch_segment_sum(sm, 1, c->d_one_seg, c->d_atom, 1, 1, 0, energy);
    HIPCHK(c, hipGetLastError());
    return BOUNCE_OK;
}

bounce_status bounce_direct_energy_bwd(bounce_ctx *c, const double *pos, const double *params,
                                       const double *grad_out, double *grad_pos,
                                       double *grad_params)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!pos || !params || !grad_out || !grad_pos || !grad_params) return BOUNCE_E_ARG;
    hipStream_t sm = c->stream;
    launch_build(sm, c->n, pos, c->d_reps, c->d_cell_rep, c->tp, c->aux, aux_spec(c), c->d_st);
    PairArgs a = pair_args(c, c->aux, 0);
    a.type_params = params;
    a.tab_f = nullptr;
    a.tab_d = nullptr;
    a.out = grad_pos;
    a.out_global = 1;
    a.accumulate = 0;
    a.atom_out = c->d_atom;
    launch_pair(sm, MODE_DBWD, c->p.pair_precision == BOUNCE_PAIR_FP64, c->p.pair_lanes, a);
    launch_dbwd_finish(sm, c->n, c->nt, c->d_atom, c->tp.type, params, grad_out, grad_pos,
                       grad_params, nullptr);
    HIPCHK(c, hipGetLastError());
    return BOUNCE_OK;
}

bounce_status bounce_profile_kernel(bounce_ctx *c, int32_t which, int32_t reps, double *avg_ms)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (!avg_ms || reps < 1 || which < 0 || which > 6) return BOUNCE_E_ARG;
    if (which == 6 && !c->p.persistent) return fail(c, BOUNCE_E_ARG, "the fused launch needs persistent = 1");
    if (which == 4 && !c->pme) return fail(c, BOUNCE_E_ARG, "no PME mesh (pme_grid)");
    if (c->built_step < 0) {
        enqueue_build(c, 0);
        c->built_step = c->step;
        c->host_rebuilds++;
    }
    if (which == 3) {
        // reps real steps; only the integrator kernels are timed
        std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
        for (hipEvent_t &e : ev) HIPCHK(c, hipEventCreate(&e));
        enqueue_substep(c, 0, 1);
        for (int32_t k = 0; k < reps; ++k) enqueue_substep(c, 1, 1, ev[2 * k], ev[2 * k + 1]);
        enqueue_substep(c, 1, 0);
        flush_pending(c);
        c->host_steps += reps + 1;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double tot = 0.0;
        for (int32_t k = 0; k < reps; ++k) {
            float ms = 0.0f;
            HIPCHK(c, hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
            tot += ms;
        }
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        *avg_ms = tot / reps;
        return bounce_sync(c);
    }
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int32_t k = 0; k < reps; ++k) {
        if (which == 0) launch_step_pair(c, 0, c->d_fpair);
        else if (which == 1) enqueue_build(c, 0);
        else if (which == 4)     // into the RESPA buffer, which every outer kick recomputes first
            launch_pme(c->stream, c->n, c->main, c->pos, c->d_charge, c->tp, pme_args(c, 0, -1), c->pme_atoms,
                       c->d_grid, c->d_theta, c->d_grec, 0, 0, nullptr);
        else if (which == 5) {     // a dry step: the pair kernel and the integrator, no kicks, jumps or drifts
            launch_step_pair(c, 0, c->d_fpair);
            launch_step(c->stream, step_args(c, 0, 0, 0));
        } else if (which == 6) {   // the same dry step as one fused launch
            launch_fused_step(c, step_args(c, 0, 0, 0), 0);
        } else launch_step(c->stream, step_args(c, 0, 0, 0));   // no kicks, jumps or drifts
    }
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    return bounce_sync(c);
}

// the autotuner's cache key: the device (name, architecture, compute units)
// and every setting the timed kernels depend on
static std::string tuning_key(const bounce_ctx *c)
{
    int dev = 0;
    hipDeviceProp_t pr{};
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&pr, dev);
    char buf[768];
    std::snprintf(buf, sizeof buf,
                  "%s/%s/%d cu|n=%d R=%d nt=%d int=%d prec=%d coul=%d per=%d rate=%d split=%d "
                  "r_on=%.4g r_off=%.4g lj=%.4g/%.4g rc=%.4g skin=%.4g cell=%.4g K=%d",
                  pr.name, pr.gcnArchName, pr.multiProcessorCount, c->n, c->R, c->nt, c->p.integrator,
                  c->p.pair_precision, c->p.coulomb, c->p.periodic, c->p.rate_mode, c->p.jump_split,
                  c->p.r_on, c->p.r_off, c->p.r_on_lj, c->p.r_off_lj, c->p.r_cut, c->p.skin,
                  c->p.cell_size, c->p.rebuild_interval);
    std::string k(buf);
    for (char &ch : k)
        if (ch == '"' || ch == '\\' || ch == '\n') ch = '_';
    return k;
}

// one cache line: {"key": "...", "pair_lanes": L, "persistent": P, ...}
static bool cache_lookup(const char *path, const std::string &key, int32_t &lanes, int32_t &pers)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    const std::string tag = "{\"key\": \"" + key + "\",";
    char line[2048];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, tag.c_str(), tag.size()) != 0) continue;
        const char *pl = std::strstr(line, "\"pair_lanes\": "), *pp = std::strstr(line, "\"persistent\": ");
        int l = 0, p = 0;
        if (pl && pp && std::sscanf(pl + 14, "%d", &l) == 1 && std::sscanf(pp + 14, "%d", &p) == 1 &&
            (l == 4 || l == 8 || l == 16 || l == 32) && (p == 0 || p == 1)) {
            lanes = l;
            pers = p;
            found = true;      // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

bounce_status bounce_autotune_cached(bounce_ctx *c, int32_t reps, const char *cache_path, bounce_tuning *out)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (reps < 1 || !out) return BOUNCE_E_ARG;
    std::memset(out, 0, sizeof *out);
    for (double &v : out->pair_ms) v = -1.0;
    for (double &v : out->step_ms) v = -1.0;
    const std::string key = tuning_key(c);
    int32_t lanes = 0, pers = 0;
    if (cache_path && cache_lookup(cache_path, key, lanes, pers)) {
        out->from_cache = 1;
    } else {
        s = bounce_autotune(c, reps, &lanes, out->pair_ms);
        if (s) return s;
        pers = 0;
        const int32_t saved = c->p.persistent;
        c->p.persistent = 1;
        const bool can = use_fused(c);
        double sep = 0.0, fus = 0.0;
        if (can) {
            c->p.persistent = 0;
            s = bounce_profile_kernel(c, 5, 2, &sep);
            if (!s) s = bounce_profile_kernel(c, 5, reps, &sep);
            c->p.persistent = 1;
            if (!s) s = bounce_profile_kernel(c, 6, 2, &fus);
            if (!s) s = bounce_profile_kernel(c, 6, reps, &fus);
            if (!s) {
                out->step_ms[0] = sep;
                out->step_ms[1] = fus;
                pers = fus < sep ? 1 : 0;
            }
        }
        c->p.persistent = saved;
        if (s) return s;
        if (cache_path) {
            FILE *f = std::fopen(cache_path, "a");
            if (!f) return fail(c, BOUNCE_E_ARG, std::string("cannot write the tuning cache ") + cache_path);
            std::fprintf(f, "{\"key\": \"%s\", \"pair_lanes\": %d, \"persistent\": %d, "
                            "\"pair_ms\": [%.6g, %.6g, %.6g, %.6g], \"step_ms\": [%.6g, %.6g]}\n",
                         key.c_str(), lanes, pers, out->pair_ms[0], out->pair_ms[1], out->pair_ms[2],
                         out->pair_ms[3], out->step_ms[0], out->step_ms[1]);
            std::fclose(f);
        }
    }
    c->p.pair_lanes = lanes;
    c->p.persistent = pers;
    if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    out->pair_lanes = lanes;
    out->persistent = pers;
    return BOUNCE_OK;
}

bounce_status bounce_autotune(bounce_ctx *c, int32_t reps, int32_t *lanes_out, double *ms_out)
{
    bounce_status s = ready(c);
    if (s) return s;
    if (reps < 1) return BOUNCE_E_ARG;
    const int32_t cand[4] = {4, 8, 16, 32};
    int32_t best = c->p.pair_lanes;
    double best_ms = 1e300;
    for (int k = 0; k < 4; ++k) {
        c->p.pair_lanes = cand[k];
        double ms = 0.0;
        s = bounce_profile_kernel(c, 0, 2, &ms);   // warm the instantiation
        if (s) return s;
        s = bounce_profile_kernel(c, 0, reps, &ms);
        if (s) return s;
        if (ms_out) ms_out[k] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = cand[k];
        }
    }
    c->p.pair_lanes = best;
    if (c->graph_exec) { (void)hipGraphExecDestroy(c->graph_exec); c->graph_exec = nullptr; }
    if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
    if (lanes_out) *lanes_out = best;
    return BOUNCE_OK;
}
