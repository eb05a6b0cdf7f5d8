/*
 * bounce_oracle.c -- plain FP64 CPU oracle of the BOUNCE process.
 *
 * TEST INFRASTRUCTURE ONLY (see bounce_oracle.h).  Built with
 * -ffp-contract=off so every product and sum is rounded exactly where it is
 * written.  Citations name sections / equations of arXiv:2002.07109:
 *   Sec. II.B   jump rate (Eq. Lambda_i) and reflection (Eq. R_i)
 *   Sec. III.C  generator L = L_A + L_B + L_O + L_J and the Strang splitting
 *   Sec. III.D  sampling a jump chain by thinning with constant bounds
 *   Sec. IV.A   force decomposition with a gradient-level switch chi, per-atom
 *               chains, rate bound lambda* = beta |v_i| L
 *   Sec. IV.B   the B J A O A J B algorithm and its J step
 *   Sec. V      final BOUNCE: partners = atoms that interact with i, per-type
 *               bounds, Coulomb handled like van der Waals, Ewald direct part
 */
#include "bounce_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator, from its published definition      */
/* (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",*/
/* SC'11): ten rounds of two 64x64->128 multiplies with a Weyl key schedule. */
/* ------------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in the open interval (0,1): the top 52 bits plus one half, scaled */
double orc_u01(uint64_t w) { return ((double)(w >> 12) + 0.5) * (1.0 / 4503599627370496.0); }

uint64_t orc_umulh(uint64_t a, uint64_t b)
{
    uint64_t hi, lo;
    mulhilo64(a, b, &hi, &lo);
    return hi;
}

static void draw(const orc_params *p, int64_t step, int32_t phase, int32_t atom, uint64_t k,
                 uint64_t out[4])
{
    uint64_t ctr[4] = {(uint64_t)step, ((uint64_t)(uint32_t)phase << 32) | (uint32_t)atom, k, 0};
    uint64_t key[2] = {p->seed, p->replica};
    orc_philox4x64_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Potential (Sec. IV.A Eq. VdW with E0 = 4 eps, r0 = sigma; Sec. V Coulomb  */
/* with the Ewald direct-space erfc split).  Shifted force at the cutoff.    */
/* ------------------------------------------------------------------------ */
static void mix(const orc_params *p, int a, int b, double *qq, double *eps, double *sig)
{
    *qq = ORC_KE * p->charge[a] * p->charge[b];
    *eps = sqrt(p->eps[a] * p->eps[b]);           /* Lorentz-Berthelot */
    *sig = 0.5 * (p->sigma[a] + p->sigma[b]);
}

/* Coulomb kernel g(r) and g'(r): bare 1/r, or erfc(alpha r)/r */
static void coul_g(const orc_params *p, double r, double *g, double *dg)
{
    if (p->coulomb == ORC_COUL_EWALD) {
        double a = p->ewald_alpha;
        double e = erfc(a * r);
        *g = e / r;
        *dg = -e / (r * r) - (2.0 * a / sqrt(M_PI)) * exp(-(a * r) * (a * r)) / r;
    } else {
        *g = 1.0 / r;
        *dg = -1.0 / (r * r);
    }
}

/* 4 eps [(s/r)^12 - (s/r)^6] and its r-derivative */
static void lj(double eps, double sig, double r, double *u, double *du)
{
    if (eps == 0.0) { *u = 0.0; *du = 0.0; return; }
    double sr = sig / r;
    double s6 = sr * sr * sr * sr * sr * sr;
    double s12 = s6 * s6;
    *u = 4.0 * eps * (s12 - s6);
    *du = 4.0 * eps * (-12.0 * s12 + 6.0 * s6) / r;
}

void orc_pair_u(const orc_params *p, int a, int b, double r, double *u, double *du)
{
    double qq, eps, sig, g, dg, ul, dul;
    mix(p, a, b, &qq, &eps, &sig);
    coul_g(p, r, &g, &dg);
    lj(eps, sig, r, &ul, &dul);
    *u = qq * g + ul;
    *du = qq * dg + dul;
}

/* W_sf(r) = u(r) - u(rc) - (r - rc) u'(rc) for r < rc, zero beyond */
void orc_pair_wsf(const orc_params *p, int a, int b, double r, double *w, double *dw)
{
    if (r >= p->r_cut) { *w = 0.0; *dw = 0.0; return; }
    double u, du, uc, duc;
    orc_pair_u(p, a, b, r, &u, &du);
    orc_pair_u(p, a, b, p->r_cut, &uc, &duc);
    *w = u - uc - (r - p->r_cut) * duc;
    *dw = du - duc;
}

/* the two parts of W'_sf(r): Coulomb qq (g'(r) - g'(rc)) and Lennard-Jones
   LJ'(r) - LJ'(rc); zero at and beyond the cutoff */
void orc_pair_dw_parts(const orc_params *p, int a, int b, double r, double *dwc, double *dwv)
{
    *dwc = *dwv = 0.0;
    if (r >= p->r_cut) return;
    double qq, eps, sig, g, dg, gc, dgc, u, du, uc, duc;
    mix(p, a, b, &qq, &eps, &sig);
    coul_g(p, r, &g, &dg);
    coul_g(p, p->r_cut, &gc, &dgc);
    lj(eps, sig, r, &u, &du);
    lj(eps, sig, p->r_cut, &uc, &duc);
    *dwc = qq * (dg - dgc);
    *dwv = du - duc;
}

/* quintic smoothstep switch: 0 below lo, 1 above hi (C^2) */
static double smoothstep(double lo, double hi, double r)
{
    double x = (r - lo) / (hi - lo);
    if (x <= 0.0) return 0.0;
    if (x >= 1.0) return 1.0;
    return x * x * x * (10.0 - 15.0 * x + 6.0 * x * x);
}

/* switch chi: 0 below r', 1 above r'', quintic smoothstep between (C^2) */
double orc_chi(const orc_params *p, double r) { return smoothstep(p->r_on, p->r_off, r); }

int orc_n_mech(const orc_params *p) { return p->jump_split ? 2 : 1; }

/* the switch of jump mechanism m: the Lennard-Jones one has its own window
   when the mechanisms are split */
double orc_chi_mech(const orc_params *p, int m, double r)
{
    return m == 1 ? smoothstep(p->r_on_lj, p->r_off_lj, r) : orc_chi(p, r);
}

static double r_on_mech(const orc_params *p, int m) { return m == 1 ? p->r_on_lj : p->r_on; }

/* the short-range part reaches to r'' (the larger of the two with split
   mechanisms); the jump fields start at r' (the smaller of the two) */
static double r_short(const orc_params *p)
{
    return p->jump_split && p->r_off_lj > p->r_off ? p->r_off_lj : p->r_off;
}

static double r_long(const orc_params *p)
{
    return p->jump_split && p->r_on_lj < p->r_on ? p->r_on_lj : p->r_on;
}

/* the pair field of mechanism m along d/r, as the scalar s with F = s d / r:
   combined chi W'_sf; split: chi_C W'_C or chi_V W'_V (zero outside (r'_m, rc)) */
static double mech_field(const orc_params *p, int m, int a, int b, double r)
{
    if (!(r > r_on_mech(p, m) && r < p->r_cut)) return 0.0;
    if (!p->jump_split) {
        double w, dw;
        orc_pair_wsf(p, a, b, r, &w, &dw);
        return orc_chi(p, r) * dw;
    }
    double dwc, dwv;
    orc_pair_dw_parts(p, a, b, r, &dwc, &dwv);
    return orc_chi_mech(p, m, r) * (m == 1 ? dwv : dwc);
}

/* Sec. IV.A: |F_ij| <= |chi W'|_inf computed numerically once; here the sup
   over a 1e-4 A grid of [r'_m, rc] times (1 + 1e-3) per mechanism and type
   pair. */
void orc_rate_bounds(const orc_params *p, double *L_ab, double *L_a)
{
    const double h = 1e-4;
    const int nt = p->n_types, nm = orc_n_mech(p);
    for (int a = 0; a < nt; ++a) L_a[a] = 0.0;
    for (int m = 0; m < nm; ++m)
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < nt; ++b) {
                double mx = 0.0;
                for (long k = 0;; ++k) {
                    double r = r_on_mech(p, m) + (double)k * h;
                    if (r >= p->r_cut) break;
                    double f = fabs(mech_field(p, m, a, b, r));
                    if (f > mx) mx = f;
                }
                L_ab[(m * nt + a) * nt + b] = mx * (1.0 + 1e-3);
            }
    for (int m = 0; m < nm; ++m)
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < nt; ++b)
                if (L_ab[(m * nt + a) * nt + b] > L_a[a]) L_a[a] = L_ab[(m * nt + a) * nt + b];
}

/* The bounds as integer weights per atom type a: ORC_RATE_ATOM gives every
   partner type the weight 2^20 (bound L_a, Sec. IV.B); ORC_RATE_PAIR rounds
   2^20 L_ab / L_a up to an integer (Sec. V: bounds per pair of types), after
   taking off 1e-4, so that two computations of L_ab that agree to 1e-12 give
   the same weight (the bound then falls short of L_ab by at most 1e-4 of a
   unit, ~1e-10 L_a, far inside the margin L_ab already carries).  The unit
   of row a is bound_scale L_a 2^-20. */
void orc_rate_weights(const orc_params *p, uint32_t *Lq, double *unit)
{
    double L_ab[2 * ORC_MAXT * ORC_MAXT], L_a[ORC_MAXT];
    const int nt = p->n_types, nm = orc_n_mech(p);
    const double one = (double)(1u << ORC_WEIGHT_BITS);
    const int per_class = p->rate_mode == ORC_RATE_PAIR || p->jump_split;
    orc_rate_bounds(p, L_ab, L_a);
    for (int a = 0; a < nt; ++a) {
        unit[a] = p->bound_scale * L_a[a] / one;
        for (int m = 0; m < nm; ++m)
            for (int b = 0; b < nt; ++b) {
                uint32_t w = 1u << ORC_WEIGHT_BITS;
                if (per_class && L_a[a] > 0.0)
                    w = (uint32_t)ceil(L_ab[(m * nt + a) * nt + b] / L_a[a] * one - ORC_WEIGHT_SLACK);
                Lq[a * nm * nt + m * nt + b] = w;
            }
    }
}

/* Eq. R_i with a scalar mass: v - 2 (v.F)/|F|^2 F */
void orc_reflect(const double v[3], const double F[3], double out[3])
{
    double s = v[0] * F[0] + v[1] * F[1] + v[2] * F[2];
    double f2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    double c = 2.0 * s / f2;
    for (int d = 0; d < 3; ++d) out[d] = v[d] - c * F[d];
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                 */
/* ------------------------------------------------------------------------ */
static void min_image(const orc_params *p, const double *qi, const double *qj, double d[3])
{
    for (int k = 0; k < 3; ++k) {
        d[k] = qi[k] - qj[k];
        if (p->periodic) {
            double inv = 1.0 / p->box[k];
            d[k] = d[k] - p->box[k] * rint(d[k] * inv);
        }
    }
}

static double norm2(const double d[3]) { return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]; }

/* cell of a position on the canonical-order grid; -1 if outside a droplet grid */
static int64_t cell_index(const orc_params *p, const double *x)
{
    int64_t c[3], dims[3];
    for (int k = 0; k < 3; ++k) {
        if (p->periodic) {
            double inv = 1.0 / p->box[k];
            int64_t n = (int64_t)floor(p->box[k] / p->cell_size);
            if (n < 1) n = 1;
            double xw = x[k] - p->box[k] * floor(x[k] * inv);
            double cinv = (double)n * inv;
            int64_t ck = (int64_t)floor(xw * cinv);
            if (ck < 0) ck = 0;
            if (ck > n - 1) ck = n - 1;
            c[k] = ck; dims[k] = n;
        } else {
            double inv = 1.0 / p->cell_size;
            double f = floor((x[k] - p->grid_origin[k]) * inv);
            if (!(f >= 0.0) || f >= (double)p->grid_dims[k]) return -1;
            c[k] = (int64_t)f; dims[k] = p->grid_dims[k];
        }
    }
    return (c[0] * dims[1] + c[1]) * dims[2] + c[2];
}

static const int64_t *g_sort_cell;   /* comparator context (single-threaded use) */
static int cmp_cell_id(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    if (g_sort_cell[i] != g_sort_cell[j]) return g_sort_cell[i] < g_sort_cell[j] ? -1 : 1;
    return (i > j) - (i < j);
}

int orc_sort_order(const orc_params *p, int32_t n, const double *q, int32_t *order, int64_t *cell)
{
    for (int32_t i = 0; i < n; ++i) {
        cell[i] = cell_index(p, q + 3 * i);
        if (cell[i] < 0) return ORC_E_GRID;
        order[i] = i;
    }
    g_sort_cell = cell;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_cell_id);
    return ORC_OK;
}

/* exclusion lookup: a plain scan of the exclusion pairs touching atom i */
typedef struct { int64_t *ptr; int32_t *idx; } excl_table;

static excl_table make_excl(const orc_topology *t)
{
    excl_table e;
    e.ptr = calloc((size_t)t->n_atoms + 1, sizeof(int64_t));
    e.idx = malloc(sizeof(int32_t) * (size_t)(2 * t->n_excl + 1));
    for (int32_t k = 0; k < t->n_excl; ++k) {
        e.ptr[t->excl[2 * k] + 1]++;
        e.ptr[t->excl[2 * k + 1] + 1]++;
    }
    for (int32_t i = 0; i < t->n_atoms; ++i) e.ptr[i + 1] += e.ptr[i];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(t->n_atoms + 1));
    memcpy(fill, e.ptr, sizeof(int64_t) * (size_t)(t->n_atoms + 1));
    for (int32_t k = 0; k < t->n_excl; ++k) {
        int32_t a = t->excl[2 * k], b = t->excl[2 * k + 1];
        e.idx[fill[a]++] = b;
        e.idx[fill[b]++] = a;
    }
    free(fill);
    return e;
}

static void free_excl(excl_table *e) { free(e->ptr); free(e->idx); }

static int excluded(const excl_table *e, int32_t i, int32_t j)
{
    for (int64_t k = e->ptr[i]; k < e->ptr[i + 1]; ++k)
        if (e->idx[k] == j) return 1;
    return 0;
}

static int in_shell(const orc_params *p, const double *q, int32_t i, int32_t j, double rmin,
                    double rmax)
{
    double d[3];
    min_image(p, q + 3 * i, q + 3 * j, d);
    double r2 = norm2(d);
    if (rmin > 0.0 && r2 < rmin * rmin) return 0;
    return r2 < rmax * rmax;
}

static int32_t list_row(const orc_params *p, const excl_table *ex, int32_t n, const double *q,
                        double rmin, double rmax, const int32_t *order, int32_t i, int32_t *col,
                        int32_t cap)
{
    int32_t m = 0;
    for (int32_t k = 0; k < n; ++k) {
        int32_t j = order[k];
        if (j == i || excluded(ex, i, j)) continue;
        if (!in_shell(p, q, i, j, rmin, rmax)) continue;
        if (col && m < cap) col[m] = j;
        ++m;
    }
    return m;
}

int32_t orc_list_row(const orc_params *p, const orc_topology *t, const double *q, double rmin,
                     double rmax, const int32_t *order, int32_t i, int32_t *col, int32_t cap)
{
    excl_table ex = make_excl(t);
    int32_t m = list_row(p, &ex, t->n_atoms, q, rmin, rmax, order, i, col, cap);
    free_excl(&ex);
    return m;
}

int64_t orc_build_list(const orc_params *p, const orc_topology *t, const double *q, double rmin,
                       double rmax, const int32_t *order, int64_t *row_ptr, int32_t *col,
                       int64_t cap)
{
    int32_t n = t->n_atoms;
    excl_table ex = make_excl(t);
    int32_t *cnt = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < n; ++i)
        cnt[i] = list_row(p, &ex, n, q, rmin, rmax, order, i, NULL, 0);
    row_ptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    int64_t total = row_ptr[n];
    if (total <= cap && col) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int32_t i = 0; i < n; ++i)
            list_row(p, &ex, n, q, rmin, rmax, order, i, col + row_ptr[i], cnt[i]);
    }
    free(cnt);
    free_excl(&ex);
    return total <= cap ? total : -1;
}

/* ------------------------------------------------------------------------ */
/* Gradients and energies                                                   */
/* ------------------------------------------------------------------------ */

/* contribution of pair (i,j) to the gradient on i for the selected parts:
   SHORT (1-chi) W'_sf d/r for r < r'', LONG chi W'_sf d/r for r' < r < rc
   (Sec. IV.A F_shortVdW and F_ij, Sec. V F_shortdir), FULL W'_sf d/r. */
static void pair_grad(const orc_params *p, int which, int ti, int tj, const double d[3],
                      double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    double r = sqrt(norm2(d));
    if (r >= p->r_cut) return;
    double w, dw;
    orc_pair_wsf(p, ti, tj, r, &w, &dw);
    double s = 0.0;
    if (!p->jump_split) {
        double chi = orc_chi(p, r);
        if ((which & ORC_G_SHORT) && r < p->r_off) s += (1.0 - chi) * dw;
        if ((which & ORC_G_LONG) && r > p->r_on) s += chi * dw;
    } else {
        /* each part with its own switch: (1 - chi_C) W'_C + (1 - chi_V) W'_V,
           and the long-range fields of the two jump mechanisms */
        double dwc, dwv;
        orc_pair_dw_parts(p, ti, tj, r, &dwc, &dwv);
        double chc = orc_chi_mech(p, 0, r), chv = orc_chi_mech(p, 1, r);
        if (which & ORC_G_SHORT) {
            if (r < p->r_off) s += (1.0 - chc) * dwc;
            if (r < p->r_off_lj) s += (1.0 - chv) * dwv;
        }
        if (which & ORC_G_LONG) {
            if (r > p->r_on) s += chc * dwc;
            if (r > p->r_on_lj) s += chv * dwv;
        }
    }
    if (which & ORC_G_FULL) s += dw;
    for (int k = 0; k < 3; ++k) g[k] = s * d[k] / r;
}

/* bonded gradient of E = k (r - r0)^2 and E = k (theta - theta0)^2 on one atom */
static void bonded_atom(const orc_params *p, const orc_topology *t, const double *q, int32_t i,
                        double g[3])
{
    for (int32_t b = 0; b < t->n_bonds; ++b) {
        int32_t a0 = t->bonds[2 * b], a1 = t->bonds[2 * b + 1];
        if (a0 != i && a1 != i) continue;
        double d[3];
        min_image(p, q + 3 * a0, q + 3 * a1, d);
        double r = sqrt(norm2(d));
        double c = 2.0 * t->bond_k[b] * (r - t->bond_r0[b]) / r;
        double sgn = (a0 == i) ? 1.0 : -1.0;
        for (int k = 0; k < 3; ++k) g[k] += sgn * c * d[k];
    }
    for (int32_t a = 0; a < t->n_angles; ++a) {
        int32_t x = t->angles[3 * a], v = t->angles[3 * a + 1], y = t->angles[3 * a + 2];
        if (x != i && v != i && y != i) continue;
        double e1[3], e2[3];
        min_image(p, q + 3 * x, q + 3 * v, e1);
        min_image(p, q + 3 * y, q + 3 * v, e2);
        double l1 = sqrt(norm2(e1)), l2 = sqrt(norm2(e2));
        double cs = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) / (l1 * l2);
        if (cs > 1.0) cs = 1.0;
        if (cs < -1.0) cs = -1.0;
        double th = acos(cs);
        double sn = sqrt(1.0 - cs * cs);
        double dEdth = 2.0 * t->angle_k[a] * (th - t->angle_t0[a]);
        /* d theta / d e = -(1/sin) d cos / d e */
        double gx[3], gy[3];
        for (int k = 0; k < 3; ++k) {
            gx[k] = -(e2[k] / (l1 * l2) - cs * e1[k] / (l1 * l1)) / sn * dEdth;
            gy[k] = -(e1[k] / (l1 * l2) - cs * e2[k] / (l2 * l2)) / sn * dEdth;
        }
        for (int k = 0; k < 3; ++k) {
            if (i == x) g[k] += gx[k];
            if (i == y) g[k] += gy[k];
            if (i == v) g[k] -= gx[k] + gy[k];
        }
    }
}

static void gradient_atom(const orc_params *p, const orc_topology *t, const excl_table *ex,
                          const double *q, int which, int32_t i, double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    if (which & (ORC_G_SHORT | ORC_G_LONG | ORC_G_FULL)) {
        for (int32_t j = 0; j < t->n_atoms; ++j) {
            if (j == i || excluded(ex, i, j)) continue;
            double d[3], gp[3];
            min_image(p, q + 3 * i, q + 3 * j, d);
            pair_grad(p, which, t->type[i], t->type[j], d, gp);
            for (int k = 0; k < 3; ++k) g[k] += gp[k];
        }
    }
    if (which & ORC_G_BONDED) bonded_atom(p, t, q, i, g);
}

void orc_gradient_atom(const orc_params *p, const orc_topology *t, const double *q, int which,
                       int32_t i, double g[3])
{
    excl_table ex = make_excl(t);
    gradient_atom(p, t, &ex, q, which, i, g);
    free_excl(&ex);
}

void orc_gradient(const orc_params *p, const orc_topology *t, const double *q, int which, double *g)
{
    excl_table ex = make_excl(t);
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < t->n_atoms; ++i) gradient_atom(p, t, &ex, q, which, i, g + 3 * i);
    free_excl(&ex);
    if ((which & ORC_G_RECIP) && p->periodic && p->pme_grid[0] > 0) {
        double *gr = malloc(sizeof(double) * 3 * (size_t)t->n_atoms), e[3];
        orc_pme(p, t, q, gr, e);
        for (int64_t k = 0; k < 3 * (int64_t)t->n_atoms; ++k) g[k] += gr[k];
        free(gr);
    }
}

/* shifted-force Coulomb and LJ parts of one pair */
static void pair_energy_parts(const orc_params *p, int a, int b, double r, double *ec, double *el)
{
    *ec = *el = 0.0;
    if (r >= p->r_cut) return;
    double qq, eps, sig, g, dg, gc, dgc, u, du, uc, duc;
    double rc = p->r_cut;
    mix(p, a, b, &qq, &eps, &sig);
    coul_g(p, r, &g, &dg);
    coul_g(p, rc, &gc, &dgc);
    *ec = qq * (g - gc - (r - rc) * dgc);
    lj(eps, sig, r, &u, &du);
    lj(eps, sig, rc, &uc, &duc);
    *el = u - uc - (r - rc) * duc;
}

void orc_energies(const orc_params *p, const orc_topology *t, const double *q, const double *v,
                  double out[7])
{
    excl_table ex = make_excl(t);
    double eb = 0.0, ea = 0.0, ec = 0.0, el = 0.0, ek = 0.0;
    for (int32_t b = 0; b < t->n_bonds; ++b) {
        double d[3];
        min_image(p, q + 3 * t->bonds[2 * b], q + 3 * t->bonds[2 * b + 1], d);
        double x = sqrt(norm2(d)) - t->bond_r0[b];
        eb += t->bond_k[b] * x * x;
    }
    for (int32_t a = 0; a < t->n_angles; ++a) {
        double e1[3], e2[3];
        min_image(p, q + 3 * t->angles[3 * a], q + 3 * t->angles[3 * a + 1], e1);
        min_image(p, q + 3 * t->angles[3 * a + 2], q + 3 * t->angles[3 * a + 1], e2);
        double cs = (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]) / sqrt(norm2(e1) * norm2(e2));
        if (cs > 1.0) cs = 1.0;
        if (cs < -1.0) cs = -1.0;
        double x = acos(cs) - t->angle_t0[a];
        ea += t->angle_k[a] * x * x;
    }
#pragma omp parallel for reduction(+ : ec, el) schedule(dynamic, 16)
    for (int32_t i = 0; i < t->n_atoms; ++i) {
        for (int32_t j = i + 1; j < t->n_atoms; ++j) {
            if (excluded(&ex, i, j)) continue;
            double d[3], c, l;
            min_image(p, q + 3 * i, q + 3 * j, d);
            pair_energy_parts(p, t->type[i], t->type[j], sqrt(norm2(d)), &c, &l);
            ec += c;
            el += l;
        }
    }
    for (int32_t i = 0; i < t->n_atoms; ++i) {
        const double *vi = v + 3 * i;
        ek += 0.5 * t->mass[i] * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]) / ORC_ACC;
    }
    free_excl(&ex);
    if (p->periodic && p->pme_grid[0] > 0) {   /* mesh, self and exclusion terms */
        double e[3];
        orc_pme(p, t, q, NULL, e);
        ec += e[0] + e[1] + e[2];
    }
    out[0] = eb; out[1] = ea; out[2] = ec; out[3] = el; out[4] = ec + el; out[5] = ek;
    out[6] = t->n_atoms > 0 ? 2.0 * ek / (3.0 * t->n_atoms * ORC_KB) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* J step (Sec. IV.B, with Sec. V partners and Sec. III.D thinning)          */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t Lq[2 * ORC_MAXT * ORC_MAXT];
    double unit[ORC_MAXT];
    double beta;
} jump_consts;

static jump_consts make_jump_consts(const orc_params *p)
{
    jump_consts jc;
    orc_rate_weights(p, jc.Lq, jc.unit);
    jc.beta = 1.0 / (ORC_KB * p->temperature);
    return jc;
}

/* the velocity chain of atom i over a time dt/2 at fixed q */
static int jump_atom(const orc_params *p, const orc_topology *t, const jump_consts *jc,
                     const double *q, double *vi, int32_t i, const int32_t *cand, int32_t nc,
                     int64_t step, int32_t phase, orc_event *ev, int64_t ev_cap, int64_t *n_ev,
                     orc_counters *cnt)
{
    int status = ORC_OK;
    const int nt = p->n_types, a = t->type[i];
    double v0 = sqrt(vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
    /* the candidates grouped by the partner's type under ORC_RATE_PAIR or
       jump_split (a single group under ORC_RATE_ATOM), each group in canonical
       order; a proposal class k is a (mechanism m, group b) pair, k = m ncls + b,
       and a partner of class k has the bound Lq[a][k] * unit[a] */
    const int nm = orc_n_mech(p);
    const int ncls = (p->rate_mode == ORC_RATE_PAIR || p->jump_split) ? nt : 1;
    const int nw = nm * ncls;
    const uint32_t *Lqa = jc->Lq + a * nm * nt;
    int32_t ncl[ORC_MAXT] = {0};
    int32_t *grp = (int32_t *)malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
    int32_t *cls_start[ORC_MAXT];
    {
        int32_t k = 0;
        for (int b = 0; b < ncls; ++b) {
            cls_start[b] = grp + k;
            for (int32_t m = 0; m < nc; ++m)
                if (ncls == 1 || t->type[cand[m]] == b) grp[k++] = cand[m];
            ncl[b] = (int32_t)(grp + k - cls_start[b]);
        }
    }
    uint64_t W = 0;     /* sum over candidates and mechanisms of their integer weights */
    for (int k = 0; k < nw; ++k) W += (uint64_t)ncl[k % ncls] * Lqa[k];
    const double unit = jc->unit[a];
    if (nc == 0 || v0 == 0.0 || W == 0 || unit == 0.0) {
        free(grp);
        return status;
    }
    /* superposed Poisson clocks: one count with mean beta |v_i| dt/2 sum_j L_ij */
    double mu = (double)W * jc->beta * v0 * unit * (0.5 * p->dt);
    uint64_t w[4];
    draw(p, step, phase, i, 0, w);
    double U = orc_u01(w[0]);
    int64_t M = 0;
    double term = exp(-mu), cdf = term;
    while (U > cdf) {
        ++M;
        if (M > p->max_proposals) {
            free(grp);
            return ORC_E_POISSON_CAP;
        }
        term *= mu / (double)M;
        cdf += term;
    }
    for (int64_t k = 1; k <= M; ++k) {
        draw(p, step, phase, i, (uint64_t)k, w);
        /* (mechanism, partner) with probability weight / W: X uniform on
           [0, W), then the class whose weight range holds X and the member
           within it */
        uint64_t X = orc_umulh(w[0], W), lo = 0;
        int cls = 0;
        while (X >= lo + (uint64_t)ncl[cls % ncls] * Lqa[cls]) {
            lo += (uint64_t)ncl[cls % ncls] * Lqa[cls];
            ++cls;
        }
        const int mech = cls / ncls;
        int32_t j = cls_start[cls % ncls][(X - lo) / Lqa[cls]];
        const double L = (double)Lqa[cls] * unit;   /* this proposal's bound */
        double u = orc_u01(w[1]);
        double d[3], F[3];
        min_image(p, q + 3 * i, q + 3 * j, d);
        double r = sqrt(norm2(d));
        /* the mechanism's long-range field chi W' d / r (zero outside (r'_m, rc)) */
        const double fs = mech_field(p, mech, t->type[i], t->type[j], r);
        for (int c = 0; c < 3; ++c) F[c] = fs * d[c] / r;
        double s = vi[0] * F[0] + vi[1] * F[1] + vi[2] * F[2];
        /* U < lambda / lambda* with lambda = beta max(0, v.F), lambda* = beta |v| L */
        int acc = (u * v0 * L) < s;
        if (s > v0 * L * (1.0 + 1e-9)) {
            cnt->bound_violations++;
            status = ORC_E_BOUND;
        }
        if (acc) {
            double out[3];
            orc_reflect(vi, F, out);
            vi[0] = out[0]; vi[1] = out[1]; vi[2] = out[2];
            cnt->accepted++;
        }
        cnt->proposals++;
        if (ev && *n_ev < ev_cap) {
            orc_event *e = &ev[*n_ev];
            e->step = step; e->phase = phase; e->atom = i; e->k = (int32_t)k;
            e->partner = j; e->accepted = acc; e->mech = mech;
            e->margin = u * v0 * L - s;
            e->scale = v0 * sqrt(norm2(F));
        }
        if (ev) ++*n_ev;
    }
    free(grp);
    return status;
}

int orc_jump_halfstep(const orc_params *p, const orc_topology *t, const double *q, double *v,
                      const int64_t *row_ptr, const int32_t *col, int64_t step, int32_t phase,
                      orc_event *ev, int64_t ev_cap, int64_t *n_ev, orc_counters *cnt)
{
    jump_consts jc = make_jump_consts(p);
    int status = ORC_OK;
    for (int32_t i = 0; i < t->n_atoms; ++i) {
        int s = jump_atom(p, t, &jc, q, v + 3 * i, i, col + row_ptr[i],
                          (int32_t)(row_ptr[i + 1] - row_ptr[i]), step, phase, ev, ev_cap, n_ev,
                          cnt);
        if (s == ORC_E_POISSON_CAP) return s;
        if (s != ORC_OK) status = s;
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* Integrator (Sec. III.C splitting, Sec. IV.B steps B, J, A, O)             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t *order;
    int64_t *cell;
    int64_t *s_ptr, *c_ptr;   /* force list and candidate list (CSR) */
    int32_t *s_col, *c_col;
    double *q_build;
} run_lists;

static double wall_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int build_run_lists_raw(const orc_params *p, const orc_topology *t, const double *q,
                               run_lists *L);

/* the lists, with the wall time they take added to the counters */
static int build_run_lists(const orc_params *p, const orc_topology *t, const double *q,
                           run_lists *L, orc_counters *cnt)
{
    const double t0 = wall_seconds();
    const int s = build_run_lists_raw(p, t, q, L);
    cnt->list_seconds += wall_seconds() - t0;
    return s;
}

static int build_run_lists_raw(const orc_params *p, const orc_topology *t, const double *q,
                               run_lists *L)
{
    int32_t n = t->n_atoms;
    int s = orc_sort_order(p, n, q, L->order, L->cell);
    if (s != ORC_OK) return s;
    double rf = (p->integrator == ORC_BOUNCE ? r_short(p) : p->r_cut) + p->skin;
    free(L->s_col); free(L->c_col);
    L->s_col = NULL; L->c_col = NULL;
    int64_t ns = orc_build_list(p, t, q, 0.0, rf, L->order, L->s_ptr, NULL, 0);
    (void)ns;
    L->s_col = malloc(sizeof(int32_t) * (size_t)(L->s_ptr[n] + 1));
    orc_build_list(p, t, q, 0.0, rf, L->order, L->s_ptr, L->s_col, L->s_ptr[n]);
    if (p->integrator == ORC_BOUNCE) {
        double rmin = r_long(p) - p->skin, rmax = p->r_cut + p->skin;
        orc_build_list(p, t, q, rmin, rmax, L->order, L->c_ptr, NULL, 0);
        L->c_col = malloc(sizeof(int32_t) * (size_t)(L->c_ptr[n] + 1));
        orc_build_list(p, t, q, rmin, rmax, L->order, L->c_ptr, L->c_col, L->c_ptr[n]);
    }
    memcpy(L->q_build, q, sizeof(double) * 3 * (size_t)n);
    return ORC_OK;
}

/* F_0 (Sec. IV.A / V): bonded + short pair part ((1-chi) W'_sf, r < r'') for
   BOUNCE, bonded + full W'_sf (r < rc) for BAOAB; pairs from the force list in
   canonical order. */
/* F_0: bonded terms plus (pair != 0) the short-range pair part; with
   bonded = 0 only the pair part (the outer force of BOUNCE-RESPA) */
static void grad_parts(const orc_params *p, const orc_topology *t, const double *q,
                       const run_lists *L, double *g, orc_counters *cnt, int pair, int bonded)
{
    int which = p->integrator == ORC_BOUNCE ? ORC_G_SHORT : ORC_G_FULL;
    double rlim = p->integrator == ORC_BOUNCE ? r_short(p) : p->r_cut;
    int64_t evals = 0;
#pragma omp parallel for reduction(+ : evals) schedule(dynamic, 16)
    for (int32_t i = 0; i < t->n_atoms; ++i) {
        double gi[3] = {0.0, 0.0, 0.0};
        for (int64_t k = L->s_ptr[i]; k < L->s_ptr[i + 1] && pair; ++k) {
            int32_t j = L->s_col[k];
            double d[3], gp[3];
            min_image(p, q + 3 * i, q + 3 * j, d);
            if (norm2(d) >= rlim * rlim) continue;
            pair_grad(p, which, t->type[i], t->type[j], d, gp);
            for (int c = 0; c < 3; ++c) gi[c] += gp[c];
            ++evals;
        }
        if (bonded) bonded_atom(p, t, q, i, gi);
        for (int c = 0; c < 3; ++c) g[3 * i + c] = gi[c];
    }
    cnt->pair_evals += evals / 2;
}

static void kick(const orc_topology *t, double *v, const double *g, double h)
{
    for (int32_t i = 0; i < t->n_atoms; ++i) {
        double s = ORC_ACC / t->mass[i];
        for (int c = 0; c < 3; ++c) v[3 * i + c] = v[3 * i + c] - h * (g[3 * i + c] * s);
    }
}

static void drift(const orc_topology *t, double *q, const double *v, double h)
{
    for (int64_t k = 0; k < 3 * (int64_t)t->n_atoms; ++k) q[k] = q[k] + h * v[k];
}

/* O step: v <- e^{-gamma dt} v + sqrt(kT (1 - e^{-2 gamma dt}) / m) G, with G
   from Box-Muller on the four words of the atom's O-phase block */
static void ou(const orc_params *p, const orc_topology *t, double *v, int64_t step)
{
    double c1 = exp(-p->gamma * p->dt);
    double kt = ORC_KB * p->temperature;
    for (int32_t i = 0; i < t->n_atoms; ++i) {
        uint64_t w[4];
        draw(p, step, ORC_PH_O, i, 0, w);
        double u1 = orc_u01(w[0]), u2 = orc_u01(w[1]), u3 = orc_u01(w[2]), u4 = orc_u01(w[3]);
        double ra = sqrt(-2.0 * log(u1)), rb = sqrt(-2.0 * log(u3));
        double G[3] = {ra * cos(2.0 * M_PI * u2), ra * sin(2.0 * M_PI * u2), rb * cos(2.0 * M_PI * u4)};
        double c2 = sqrt(kt * (1.0 - c1 * c1) * ORC_ACC / t->mass[i]);
        for (int c = 0; c < 3; ++c) v[3 * i + c] = c1 * v[3 * i + c] + c2 * G[c];
    }
}

static int finite_state(const orc_topology *t, const double *q, const double *v)
{
    for (int64_t k = 0; k < 3 * (int64_t)t->n_atoms; ++k)
        if (!isfinite(q[k]) || !isfinite(v[k])) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Reciprocal-space Ewald: smooth PME (Sec. V; Essmann et al. 1995)          */
/* ------------------------------------------------------------------------ */
/* cardinal B-spline of order n, by its recursion (Essmann et al., Eq. 4.1) */
static double bspline(int n, double u)
{
    if (n == 2) return (u < 0.0 || u > 2.0) ? 0.0 : 1.0 - fabs(u - 1.0);
    return (u * bspline(n - 1, u) + ((double)n - u) * bspline(n - 1, u - 1.0)) / (double)(n - 1);
}

/* its derivative, M_n'(u) = M_{n-1}(u) - M_{n-1}(u - 1) */
static double bspline_d(int n, double u) { return bspline(n - 1, u) - bspline(n - 1, u - 1.0); }

/* |b(k)|^2 of one axis (Essmann et al., Eq. 4.7); where the sum vanishes (odd
   order at k = K/2) the mean of the two neighbouring values is used */
static void bspline_moduli(int n, int K, double *bsq)
{
    for (int k = 0; k < K; ++k) {
        double complex s = 0.0;
        for (int j = 0; j <= n - 2; ++j) s += bspline(n, (double)(j + 1)) * cexp(2.0 * M_PI * I * k * j / K);
        const double d = creal(s * conj(s));
        bsq[k] = d > 1e-30 ? 1.0 / d : -1.0;
    }
    for (int k = 0; k < K; ++k)
        if (bsq[k] < 0.0) bsq[k] = 0.5 * (bsq[(k + K - 1) % K] + bsq[(k + 1) % K]);
}

/* one-dimensional DFT along axis `ax` of a K0 x K1 x K2 complex grid, written
   as the plain sum (sign -1 or +1 in the exponent) */
static void dft_axis(double complex *a, const int K[3], int ax, int sign)
{
    const int n = K[ax];
    const int64_t stride = ax == 2 ? 1 : (ax == 1 ? K[2] : (int64_t)K[1] * K[2]);
    double complex *line = malloc(sizeof(double complex) * n), *out = malloc(sizeof(double complex) * n);
    double complex *tw = malloc(sizeof(double complex) * n);     /* exp(sign 2 pi i j / n) */
    for (int j = 0; j < n; ++j) tw[j] = cexp(sign * 2.0 * M_PI * I * (double)j / n);
    const int64_t total = (int64_t)K[0] * K[1] * K[2];
    for (int64_t base = 0; base < total; ++base) {
        /* visit each line once: its first element has index 0 along ax */
        if ((base / stride) % n != 0) continue;
        for (int l = 0; l < n; ++l) line[l] = a[base + l * stride];
        for (int k = 0; k < n; ++k) {
            double complex acc = 0.0;
            for (int l = 0; l < n; ++l) acc += line[l] * tw[(int64_t)k * l % n];
            out[k] = acc;
        }
        for (int k = 0; k < n; ++k) a[base + k * stride] = out[k];
    }
    free(line);
    free(out);
    free(tw);
}

/* the B-spline weights of one atom along one axis: grid points
   l_j = (floor(u) - j) mod K and M_n(u - floor(u) + j), M_n' likewise */
static void atom_weights(int n, int K, double u, int *l, double *w, double *dw)
{
    const double fl = floor(u);
    for (int j = 0; j < n; ++j) {
        int g = ((int)fl - j) % K;
        if (g < 0) g += K;
        l[j] = g;
        w[j] = bspline(n, u - fl + j);
        dw[j] = bspline_d(n, u - fl + j);
    }
}

void orc_pme(const orc_params *p, const orc_topology *t, const double *q, double *grad, double e[3])
{
    const int n = p->pme_order;
    const int K[3] = {p->pme_grid[0], p->pme_grid[1], p->pme_grid[2]};
    const int64_t KK = (int64_t)K[0] * K[1] * K[2];
    const double a = p->ewald_alpha;
    const double V = p->box[0] * p->box[1] * p->box[2];
    const int32_t N = t->n_atoms;
    e[0] = e[1] = e[2] = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * 3 * (size_t)N);
    /* fractional grid coordinates u = K x / L with x wrapped into [0, L) */
    double *u = malloc(sizeof(double) * 3 * (size_t)N);
    for (int32_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) {
            double x = q[3 * i + c] - p->box[c] * floor(q[3 * i + c] / p->box[c]);
            u[3 * i + c] = (double)K[c] * x / p->box[c];
        }
    /* charge grid Q(l) = sum_i q_i prod_c M_n(u_ic - l_c), periodic images */
    double complex *Q = calloc((size_t)KK, sizeof(double complex));
    for (int32_t i = 0; i < N; ++i) {
        int l[3][ORC_MAX_PME_ORDER];
        double w[3][ORC_MAX_PME_ORDER], dw[3][ORC_MAX_PME_ORDER];
        for (int c = 0; c < 3; ++c) atom_weights(n, K[c], u[3 * i + c], l[c], w[c], dw[c]);
        const double qi = p->charge[t->type[i]];
        for (int j0 = 0; j0 < n; ++j0)
            for (int j1 = 0; j1 < n; ++j1)
                for (int j2 = 0; j2 < n; ++j2)
                    Q[((int64_t)l[0][j0] * K[1] + l[1][j1]) * K[2] + l[2][j2]] += qi * w[0][j0] * w[1][j1] * w[2][j2];
    }
    /* F(Q)(k) = sum_l Q(l) exp(2 pi i k.l / K) */
    double complex *FQ = malloc(sizeof(double complex) * (size_t)KK);
    memcpy(FQ, Q, sizeof(double complex) * (size_t)KK);
    for (int ax = 0; ax < 3; ++ax) dft_axis(FQ, K, ax, +1);
    /* theta(k) = k_e / (pi V) exp(-pi^2 m^2 / alpha^2) / m^2 B(k), theta(0) = 0 */
    double *bsq[3];
    for (int c = 0; c < 3; ++c) {
        bsq[c] = malloc(sizeof(double) * K[c]);
        bspline_moduli(n, K[c], bsq[c]);
    }
    double Erec = 0.0;
    for (int k0 = 0; k0 < K[0]; ++k0)
        for (int k1 = 0; k1 < K[1]; ++k1)
            for (int k2 = 0; k2 < K[2]; ++k2) {
                const int64_t idx = ((int64_t)k0 * K[1] + k1) * K[2] + k2;
                const int kk[3] = {k0, k1, k2};
                double m2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double mc = (double)(kk[c] <= K[c] / 2 ? kk[c] : kk[c] - K[c]) / p->box[c];
                    m2 += mc * mc;
                }
                double th = 0.0;
                if (idx != 0)
                    th = ORC_KE / (M_PI * V) * exp(-M_PI * M_PI * m2 / (a * a)) / m2 * bsq[0][k0] *
                         bsq[1][k1] * bsq[2][k2];
                Erec += 0.5 * th * creal(FQ[idx] * conj(FQ[idx]));
                FQ[idx] *= th;
            }
    e[0] = Erec;
    if (grad) {
        /* phi(l) = Re sum_k theta(k) F(Q)(k) exp(-2 pi i k.l / K); dE/dx_ic =
           q_i sum_l phi(l) dQ_i(l)/dx_ic */
        for (int ax = 0; ax < 3; ++ax) dft_axis(FQ, K, ax, -1);
        for (int32_t i = 0; i < N; ++i) {
            int l[3][ORC_MAX_PME_ORDER];
            double w[3][ORC_MAX_PME_ORDER], dw[3][ORC_MAX_PME_ORDER];
            for (int c = 0; c < 3; ++c) atom_weights(n, K[c], u[3 * i + c], l[c], w[c], dw[c]);
            const double qi = p->charge[t->type[i]];
            double gi[3] = {0.0, 0.0, 0.0};
            for (int j0 = 0; j0 < n; ++j0)
                for (int j1 = 0; j1 < n; ++j1)
                    for (int j2 = 0; j2 < n; ++j2) {
                        const double phi = creal(FQ[((int64_t)l[0][j0] * K[1] + l[1][j1]) * K[2] + l[2][j2]]);
                        gi[0] += phi * dw[0][j0] * w[1][j1] * w[2][j2];
                        gi[1] += phi * w[0][j0] * dw[1][j1] * w[2][j2];
                        gi[2] += phi * w[0][j0] * w[1][j1] * dw[2][j2];
                    }
            for (int c = 0; c < 3; ++c) grad[3 * i + c] = qi * gi[c] * (double)K[c] / p->box[c];
        }
    }
    /* self term and the excluded pairs' share of the mesh sum */
    double esf = 0.0;
    for (int32_t i = 0; i < N; ++i) esf += p->charge[t->type[i]] * p->charge[t->type[i]];
    e[1] = -ORC_KE * a / sqrt(M_PI) * esf;
    for (int32_t k = 0; k < t->n_excl; ++k) {
        const int32_t i = t->excl[2 * k], j = t->excl[2 * k + 1];
        double d[3];
        min_image(p, q + 3 * i, q + 3 * j, d);
        const double r = sqrt(norm2(d));
        const double qq = ORC_KE * p->charge[t->type[i]] * p->charge[t->type[j]];
        e[2] -= qq * erf(a * r) / r;
        if (grad) {
            /* d/dr [erf(a r)/r] = (2a/sqrt(pi) exp(-a^2 r^2) r - erf(a r)) / r^2 */
            const double dfdr = (2.0 * a / sqrt(M_PI) * exp(-a * a * r * r) * r - erf(a * r)) / (r * r);
            for (int c = 0; c < 3; ++c) {
                grad[3 * i + c] -= qq * dfdr * d[c] / r;
                grad[3 * j + c] += qq * dfdr * d[c] / r;
            }
        }
    }
    for (int c = 0; c < 3; ++c) free(bsq[c]);
    free(u); free(Q); free(FQ);
}

double orc_ewald_recip(const orc_params *p, const orc_topology *t, const double *q, int32_t kmax,
                       double *grad)
{
    const double a = p->ewald_alpha, V = p->box[0] * p->box[1] * p->box[2];
    const int32_t N = t->n_atoms;
    double E = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * 3 * (size_t)N);
    for (int k0 = -kmax; k0 <= kmax; ++k0)
        for (int k1 = -kmax; k1 <= kmax; ++k1)
            for (int k2 = -kmax; k2 <= kmax; ++k2) {
                if (!k0 && !k1 && !k2) continue;
                const double m[3] = {k0 / p->box[0], k1 / p->box[1], k2 / p->box[2]};
                const double m2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
                const double f = ORC_KE / (2.0 * M_PI * V) * exp(-M_PI * M_PI * m2 / (a * a)) / m2;
                double complex S = 0.0;
                for (int32_t j = 0; j < N; ++j)
                    S += p->charge[t->type[j]] *
                         cexp(2.0 * M_PI * I * (m[0] * q[3 * j] + m[1] * q[3 * j + 1] + m[2] * q[3 * j + 2]));
                E += f * creal(S * conj(S));
                if (grad)
                    for (int32_t i = 0; i < N; ++i) {
                        /* d|S|^2/dx_i = 2 Re(conj(S) q_i 2 pi i m exp(2 pi i m.x_i)) */
                        const double complex ei = cexp(2.0 * M_PI * I * (m[0] * q[3 * i] + m[1] * q[3 * i + 1] + m[2] * q[3 * i + 2]));
                        const double s = 2.0 * creal(conj(S) * p->charge[t->type[i]] * 2.0 * M_PI * I * ei);
                        for (int c = 0; c < 3; ++c) grad[3 * i + c] += f * s * m[c];
                    }
            }
    return E;
}

/* the gradients of one step at q: g = F_0 (bonded terms, the short-range
   pair part unless it is on the outer step, the mesh part unless it is on
   the outer step) and gout = the outer-step gradient (mesh part and, with
   out_pair, the short-range pair part) */
static void forces(const orc_params *p, const orc_topology *t, const double *q, const run_lists *L,
                   double *g, double *gout, orc_counters *cnt, int pme, int respa, int out_pair,
                   double erec[3])
{
    const int64_t n3 = 3 * (int64_t)t->n_atoms;
    grad_parts(p, t, q, L, g, cnt, !out_pair, 1);
    if (out_pair) grad_parts(p, t, q, L, gout, cnt, 1, 0);
    else
        for (int64_t k = 0; k < n3; ++k) gout[k] = 0.0;
    if (pme) {
        double *gr = malloc(sizeof(double) * (size_t)(n3 + 1));
        orc_pme(p, t, q, gr, erec);
        double *dst = respa ? gout : g;
        for (int64_t k = 0; k < n3; ++k) dst[k] += gr[k];
        free(gr);
    }
}

int orc_run(const orc_params *p, const orc_topology *t, double *q, double *v, int64_t step0,
            int32_t nsteps, orc_event *ev, int64_t ev_cap, int64_t *n_ev, orc_counters *cnt)
{
    int32_t n = t->n_atoms;
    int status = ORC_OK;
    int64_t nev_local = 0;
    if (!n_ev) n_ev = &nev_local;
    run_lists L;
    memset(&L, 0, sizeof L);
    L.order = malloc(sizeof(int32_t) * (size_t)(n + 1));
    L.cell = malloc(sizeof(int64_t) * (size_t)(n + 1));
    L.s_ptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    L.c_ptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    L.q_build = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *g = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *grec = malloc(sizeof(double) * 3 * (size_t)(n + 1));
    jump_consts jc = make_jump_consts(p);
    int bounce = p->integrator == ORC_BOUNCE;
    double h = 0.5 * p->dt;
    /* reciprocal-space force: in F_0 (respa_m = 0) or as RESPA outer half kicks;
       with respa_outer = NONBONDED the short-range pair force moves to the
       outer step as well (F_0 keeps the bonded terms) */
    const int pme = p->periodic && p->pme_grid[0] > 0;
    const int out_pair = p->respa_m >= 1 && p->respa_outer == ORC_OUTER_NONBONDED;
    const int respa = p->respa_m >= 1 && (pme || out_pair);
    const double H = 0.5 * p->dt * (double)p->respa_m;
    double erec[3];

#define JUMP(STEP, PHASE)                                                                        \
    do {                                                                                         \
        for (int32_t i = 0; i < n && bounce; ++i) {                                              \
            int s_ = jump_atom(p, t, &jc, q, v + 3 * i, i, L.c_col + L.c_ptr[i],                 \
                               (int32_t)(L.c_ptr[i + 1] - L.c_ptr[i]), (STEP), (PHASE), ev,      \
                               ev_cap, n_ev, cnt);                                               \
            if (s_ == ORC_E_POISSON_CAP) { status = s_; goto done; }                             \
            if (s_ != ORC_OK) status = s_;                                                       \
        }                                                                                        \
    } while (0)

    status = build_run_lists(p, t, q, &L, cnt);
    if (status != ORC_OK) goto done;
    cnt->rebuilds++;
    forces(p, t, q, &L, g, grec, cnt, pme, respa, out_pair, erec);
    for (int64_t n_step = step0; n_step < step0 + nsteps; ++n_step) {
        if (respa && n_step % p->respa_m == 0) kick(t, v, grec, H);   /* outer half kick */
        kick(t, v, g, h);                          /* B */
        JUMP(n_step, ORC_PH_JA);                   /* J */
        drift(t, q, v, h);                         /* A */
        ou(p, t, v, n_step);                       /* O */
        drift(t, q, v, h);                         /* A */
        /* skin guard: every atom within s/2 of where the lists were built */
        for (int32_t i = 0; i < n; ++i) {
            double d[3];
            for (int c = 0; c < 3; ++c) d[c] = q[3 * i + c] - L.q_build[3 * i + c];
            if (norm2(d) >= 0.25 * p->skin * p->skin) { status = ORC_E_SKIN; goto done; }
        }
        if ((n_step + 1) % p->rebuild_interval == 0) {
            int s = build_run_lists(p, t, q, &L, cnt);
            if (s != ORC_OK) { status = s; goto done; }
            cnt->rebuilds++;
        }
        forces(p, t, q, &L, g, grec, cnt, pme, respa, out_pair, erec);
        JUMP(n_step, ORC_PH_JB);                   /* J */
        kick(t, v, g, h);                          /* B */
        if (respa && (n_step + 1) % p->respa_m == 0) kick(t, v, grec, H);   /* outer half kick */
        cnt->steps++;
        if (!finite_state(t, q, v)) { status = ORC_E_NONFINITE; goto done; }
    }
#undef JUMP
done:
    free(L.order); free(L.cell); free(L.s_ptr); free(L.c_ptr); free(L.s_col); free(L.c_col);
    free(L.q_build); free(g); free(grec);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Differentiable direct-space energy (Sec. V E_direct + E_VdW, full cutoff) */
/* ------------------------------------------------------------------------ */
/* Structure diagnostic (the paper compares pair structure of BOUNCE and
   reference runs, Sec. VI): ordered non-excluded pairs (i != j) with
   r^2 < r_max^2 counted per type pair in bins of width dr = r_max / nbins,
   pair (i, j) in bin k when (k dr)^2 <= r^2 < ((k + 1) dr)^2.  Brute force. */
void orc_rdf_counts(const orc_params *p, const orc_topology *t, const double *q, double r_max,
                    int32_t nbins, int64_t *counts)
{
    const int nt = p->n_types;
    const double dr = r_max / (double)nbins, rmax2 = r_max * r_max;
    excl_table ex = make_excl(t);
    memset(counts, 0, sizeof(int64_t) * (size_t)nt * nt * nbins);
    for (int32_t i = 0; i < t->n_atoms; ++i)
        for (int32_t j = 0; j < t->n_atoms; ++j) {
            if (j == i || excluded(&ex, i, j)) continue;
            double d[3];
            min_image(p, q + 3 * i, q + 3 * j, d);
            const double r2 = norm2(d);
            if (!(r2 < rmax2)) continue;
            int32_t k = 0;
            while (k + 1 < nbins && ((double)(k + 1) * dr) * ((double)(k + 1) * dr) <= r2) ++k;
            counts[((int64_t)t->type[i] * nt + t->type[j]) * nbins + k]++;
        }
    free_excl(&ex);
}

double orc_direct_energy(const orc_params *p, const orc_topology *t, const double *q,
                         double *grad_q, double *grad_charge, double *grad_eps, double *grad_sigma)
{
    excl_table ex = make_excl(t);
    int nt = p->n_types;
    double rc = p->r_cut;
    double E = 0.0;
    double gq[ORC_MAXT] = {0}, ge[ORC_MAXT] = {0}, gs[ORC_MAXT] = {0};
    /* per-type-pair sums of the shifted basis functions */
    double Sg[ORC_MAXT * ORC_MAXT] = {0}, Se[ORC_MAXT * ORC_MAXT] = {0},
           Ss[ORC_MAXT * ORC_MAXT] = {0};
    double gc, dgc;
    coul_g(p, rc, &gc, &dgc);
    for (int32_t i = 0; i < t->n_atoms; ++i) {
        for (int32_t j = i + 1; j < t->n_atoms; ++j) {
            if (excluded(&ex, i, j)) continue;
            double d[3];
            min_image(p, q + 3 * i, q + 3 * j, d);
            double r = sqrt(norm2(d));
            if (r >= rc) continue;
            int a = t->type[i], b = t->type[j];
            double w, dw;
            orc_pair_wsf(p, a, b, r, &w, &dw);
            E += w;
            double g, dg;
            coul_g(p, r, &g, &dg);
            double qq, eps, sig;
            mix(p, a, b, &qq, &eps, &sig);
            Sg[a * nt + b] += g - gc - (r - rc) * dgc;
            /* d u_LJ / d eps_ab and d u_LJ / d sigma_ab, then the sf transform in r */
            double sr = sig / r, src = sig / rc;
            double s6 = pow(sr, 6), s12 = s6 * s6, c6 = pow(src, 6), c12 = c6 * c6;
            double fe = 4.0 * (s12 - s6), fe_c = 4.0 * (c12 - c6);
            double dfe_c = 4.0 * (-12.0 * c12 + 6.0 * c6) / rc;
            Se[a * nt + b] += fe - fe_c - (r - rc) * dfe_c;
            if (sig > 0.0) {
                double fs = 4.0 * eps * (12.0 * s12 - 6.0 * s6) / sig;
                double fs_c = 4.0 * eps * (12.0 * c12 - 6.0 * c6) / sig;
                double dfs_c = 4.0 * eps * (-144.0 * c12 + 36.0 * c6) / (sig * rc);
                Ss[a * nt + b] += fs - fs_c - (r - rc) * dfs_c;
            }
        }
    }
    for (int a = 0; a < nt; ++a) {
        for (int b = 0; b < nt; ++b) {
            double sg = Sg[a * nt + b], se = Se[a * nt + b], ss = Ss[a * nt + b];
            /* E_C = KE q_a q_b Sg : derivative on each endpoint type */
            gq[a] += ORC_KE * p->charge[b] * sg;
            gq[b] += ORC_KE * p->charge[a] * sg;
            /* eps_ab = sqrt(eps_a eps_b); sigma_ab = (sigma_a + sigma_b)/2 */
            if (a == b) {
                ge[a] += se;
                gs[a] += ss;
            } else {
                /* d sqrt(eps_a eps_b) / d eps_a = sqrt(eps_b / eps_a) / 2: infinite
                   where eps_a = 0 < eps_b (undefined there) */
                ge[a] += se * 0.5 * sqrt(p->eps[b] / p->eps[a]);
                ge[b] += se * 0.5 * sqrt(p->eps[a] / p->eps[b]);
                gs[a] += 0.5 * ss;
                gs[b] += 0.5 * ss;
            }
        }
    }
    if (grad_charge) memcpy(grad_charge, gq, sizeof(double) * (size_t)nt);
    if (grad_eps) memcpy(grad_eps, ge, sizeof(double) * (size_t)nt);
    if (grad_sigma) memcpy(grad_sigma, gs, sizeof(double) * (size_t)nt);
    if (grad_q) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int32_t i = 0; i < t->n_atoms; ++i)
            gradient_atom(p, t, &ex, q, ORC_G_FULL, i, grad_q + 3 * i);
    }
    free_excl(&ex);
    return E;
}
