/*
 * oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Written for readability, not speed: global lists, adjacency rebuilt from the
 * bond list whenever the bond list changes, straightforward loops.  Built with
 * -ffp-contract=off so that every cutoff decision is made with plain IEEE
 * double multiplies and adds in the order written.
 */
#include "oracle.h"

#define _GNU_SOURCE
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXT 32          /* bond/angle/dihedral types 1..31 */
#define MAXRULES 64
#define KIND_LANGEVIN 0u
#define KIND_CREATE 1u
#define KIND_BREAK 2u
#define KIND_DPD 3u

enum { R_CREATE = 1, R_CREATEDIR, R_BREAK, R_KILL, R_CONVERT };

typedef struct {
    int kind;
    int bt1, bt2;   /* create: bt1=bt2; createdir: bt1 (stored by the bead1-type bead), bt2; break/kill: bt1; convert: bt1->bt2 */
    int b1, b2;     /* bead types (0 = any) */
    double r2;      /* squared distance threshold */
    double p;
} rule_t;

typedef struct { int bt, bead, max; } maxrule_t;
typedef struct { int type; int b[3]; uint32_t m[2]; } angrule_t;
typedef struct { int type; int b[4]; uint32_t m[3]; } dihrule_t;

typedef struct { int i, j, tij, tji; } bond_t;          /* i < j */
typedef struct { int type, a, b, c; } ang_t;            /* a < c */
typedef struct { int type, a, b, c, d; } dih_t;         /* a < d */

struct or_sys {
    int n;
    double L, hL;
    uint64_t seed;
    double *x, *v;      /* n*3 */
    double *fext;       /* n*3 constant external force per bead, or NULL */
    int *type;
    uint8_t *reactive;

    bond_t *bond; int64_t nb, cap_b;
    ang_t *ang; int64_t na, cap_a;
    dih_t *dih; int64_t nd, cap_d;

    /* adjacency (CSR) derived from the bond list */
    int *aoff, *anbr, *atype, *abond;
    int adj_valid;

    /* force field */
    double eps, sig, rc; int excl_depth; int have_pair;
    int pair_style;                 /* 0: WCA, 1: DPD */
    double dpd_a, dpd_gamma;
    double bK[MAXT], bR0[MAXT]; int bset[MAXT];
    int bstyle[MAXT];                              /* 0: harmonic, 1: well */
    double bUmin[MAXT], bRw[MAXT], bRz[MAXT], bRcut[MAXT];
    double aK[MAXT], aT0[MAXT]; int aset[MAXT];
    double dK[MAXT], dP0[MAXT]; int dset[MAXT];
    double T0, T1, gamma, dt; int64_t ramp;

    /* rules */
    int every, pc13, pc14;
    rule_t rule[MAXRULES]; int nrule;
    maxrule_t maxr[MAXRULES]; int nmax;
    angrule_t arule[MAXRULES]; int narule;
    dihrule_t drule[MAXRULES]; int ndrule;

    int accept_average;             /* 1: the appendix's averaged per-bead uniforms */
    int64_t step, swept_step;
    int64_t stat_last[8], stat_cum[8], sweeps;
    int *nomC, *nomK;
    int64_t degenerate_dihedrals;
};

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the Philox
 * S-box on a 128-bit counter with a 64-bit key bumped by the Weyl constants. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(const or_sys* s, uint32_t a, uint32_t b, int64_t step, uint32_t kind, uint32_t out[4]) {
    uint64_t st = (uint64_t)step;
    uint32_t ctr[4] = {a, b, (uint32_t)st, ((uint32_t)(st >> 32) & 0x0FFFFFFFu) | (kind << 28)};
    uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

/* standard normal for the unordered pair {i, j}: Box-Muller (Box and Muller, 1958)
 * on the first two 32-bit words, each mapped to (0,1) as (w + 1/2) / 2^32 */
static double pair_gaussian(const or_sys* s, int i, int j, int64_t step) {
    uint32_t lo = (uint32_t)(i < j ? i : j), hi = (uint32_t)(i < j ? j : i);
    uint32_t w[4];
    draw(s, lo, hi, step, KIND_DPD, w);
    double u1 = ((double)w[0] + 0.5) * (1.0 / 4294967296.0);
    double u2 = ((double)w[1] + 0.5) * (1.0 / 4294967296.0);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* uniform on [0,1) with 53 random bits, for the acceptance test u < p */
static double pair_uniform(const or_sys* s, int i, int j, int64_t step, uint32_t kind) {
    uint32_t lo = (uint32_t)(i < j ? i : j), hi = (uint32_t)(i < j ? j : i);
    uint32_t w[4];
    draw(s, lo, hi, step, kind, w);
    uint64_t bits = (((uint64_t)w[0] << 32) | (uint64_t)w[1]) >> 11;
    return (double)bits * (1.0 / 9007199254740992.0);
}

/* uniform on [0,1) with 53 random bits drawn by bead i alone (its counter names
 * the bead twice, which no pair draw does) */
static double bead_uniform(const or_sys* s, int i, int64_t step, uint32_t kind) {
    uint32_t w[4];
    draw(s, (uint32_t)i, (uint32_t)i, step, kind, w);
    uint64_t bits = (((uint64_t)w[0] << 32) | (uint64_t)w[1]) >> 11;
    return (double)bits * (1.0 / 9007199254740992.0);
}

/* The number a mutual pair's acceptance compares with p (appendix, steps 5 and 7).
 * Default: one uniform for the pair.  Literal form: every bead draws its own
 * uniform, the pair takes the mean of the two and accepts when it is below p, so
 * that both beads reach the same decision; the acceptance probability is then
 * 2p^2 for p <= 1/2 and 1 - 2(1 - p)^2 above. */
static double accept_number(const or_sys* s, int i, int j, int64_t step, uint32_t kind) {
    if (!s->accept_average) return pair_uniform(s, i, j, step, kind);
    int lo = i < j ? i : j, hi = i < j ? j : i;
    return (bead_uniform(s, lo, step, kind) + bead_uniform(s, hi, step, kind)) * 0.5;
}

/* ------------------------------------------------------------------------- */
static double min_image(double d, double L, double hL) {
    if (d > hL) return d - L;
    if (d < -hL) return d + L;
    return d;
}

/* separation vector x_j - x_i (minimum image) and its squared length */
static double sep(const or_sys* s, int i, int j, double d[3]) {
    for (int k = 0; k < 3; ++k) d[k] = min_image(s->x[3 * j + k] - s->x[3 * i + k], s->L, s->hL);
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

static int type_ok(int rule_bead, int bead_type) { return rule_bead == 0 || rule_bead == bead_type; }
static int in_mask(uint32_t m, int t) { return t >= 0 && t < 32 && ((m >> t) & 1u); }

/* ------------------------------------------------------------------------- */
or_sys* or_create(int32_t n, double L, uint64_t seed) {
    if (n < 0 || !(L > 0)) return NULL;
    or_sys* s = (or_sys*)calloc(1, sizeof(or_sys));
    s->n = n; s->L = L; s->hL = 0.5 * L; s->seed = seed;
    size_t nn = n > 0 ? (size_t)n : 1;
    s->x = (double*)calloc(3 * nn, sizeof(double));
    s->v = (double*)calloc(3 * nn, sizeof(double));
    s->type = (int*)calloc(nn, sizeof(int));
    s->reactive = (uint8_t*)calloc(nn, 1);
    for (int i = 0; i < n; ++i) s->reactive[i] = 1;
    s->aoff = (int*)calloc(nn + 1, sizeof(int));
    s->nomC = (int*)malloc(nn * sizeof(int));
    s->nomK = (int*)malloc(nn * sizeof(int));
    for (int i = 0; i < n; ++i) { s->nomC[i] = -1; s->nomK[i] = -1; }
    s->eps = 1.0; s->sig = 1.0; s->rc = pow(2.0, 1.0 / 6.0); s->excl_depth = 1;
    s->T0 = s->T1 = 1.0; s->gamma = 0.0; s->dt = 0.005;
    s->every = 0;
    s->swept_step = -1;
    return s;
}

void or_destroy(or_sys* s) {
    if (!s) return;
    free(s->x); free(s->v); free(s->fext); free(s->type); free(s->reactive);
    free(s->bond); free(s->ang); free(s->dih);
    free(s->aoff); free(s->anbr); free(s->atype); free(s->abond);
    free(s->nomC); free(s->nomK);
    free(s);
}

int or_set_state(or_sys* s, const double* x, const double* v, const int32_t* type) {
    for (int i = 0; i < 3 * s->n; ++i) {
        if (!isfinite(x[i]) || x[i] < 0 || x[i] >= s->L) return -1;
        s->x[i] = x[i];
        s->v[i] = v ? v[i] : 0.0;
    }
    if (type)
        for (int i = 0; i < s->n; ++i) s->type[i] = type[i];
    return 0;
}

int or_set_reactive(or_sys* s, const uint8_t* f) {
    for (int i = 0; i < s->n; ++i) s->reactive[i] = f[i] ? 1 : 0;
    return 0;
}

static void push_bond(or_sys* s, int i, int j, int tij, int tji) {
    if (s->nb == s->cap_b) {
        s->cap_b = s->cap_b ? 2 * s->cap_b : 1024;
        s->bond = (bond_t*)realloc(s->bond, (size_t)s->cap_b * sizeof(bond_t));
    }
    if (i > j) { int t = i; i = j; j = t; t = tij; tij = tji; tji = t; }
    s->bond[s->nb].i = i; s->bond[s->nb].j = j;
    s->bond[s->nb].tij = tij; s->bond[s->nb].tji = tji;
    s->nb++;
    s->adj_valid = 0;
}

static void push_ang(or_sys* s, int type, int a, int b, int c) {
    if (s->na == s->cap_a) {
        s->cap_a = s->cap_a ? 2 * s->cap_a : 1024;
        s->ang = (ang_t*)realloc(s->ang, (size_t)s->cap_a * sizeof(ang_t));
    }
    if (a > c) { int t = a; a = c; c = t; }
    ang_t e = {type, a, b, c};
    s->ang[s->na++] = e;
}

static void push_dih(or_sys* s, int type, int a, int b, int c, int d) {
    if (s->nd == s->cap_d) {
        s->cap_d = s->cap_d ? 2 * s->cap_d : 1024;
        s->dih = (dih_t*)realloc(s->dih, (size_t)s->cap_d * sizeof(dih_t));
    }
    if (a > d) { int t = a; a = d; d = t; t = b; b = c; c = t; }
    dih_t e = {type, a, b, c, d};
    s->dih[s->nd++] = e;
}

int or_set_bonds(or_sys* s, int64_t nb, const int32_t* ij, const int32_t* tij, const int32_t* tji) {
    s->nb = 0;
    for (int64_t k = 0; k < nb; ++k) {
        int i = ij[2 * k], j = ij[2 * k + 1];
        if (i < 0 || j < 0 || i >= s->n || j >= s->n || i == j) return -1;
        if (tij[k] < 1 || tij[k] >= MAXT || tji[k] < 1 || tji[k] >= MAXT) return -1;
        push_bond(s, i, j, tij[k], tji[k]);
    }
    s->adj_valid = 0;
    return 0;
}

int or_set_angles(or_sys* s, int64_t na, const int32_t* abc, const int32_t* type) {
    s->na = 0;
    for (int64_t k = 0; k < na; ++k) push_ang(s, type[k], abc[3 * k], abc[3 * k + 1], abc[3 * k + 2]);
    return 0;
}

int or_set_dihedrals(or_sys* s, int64_t nd, const int32_t* abcd, const int32_t* type) {
    s->nd = 0;
    for (int64_t k = 0; k < nd; ++k)
        push_dih(s, type[k], abcd[4 * k], abcd[4 * k + 1], abcd[4 * k + 2], abcd[4 * k + 3]);
    return 0;
}

/* adjacency: for bead u, entries (neighbour, type stored by u, bond index) */
static void build_adj(or_sys* s) {
    if (s->adj_valid) return;
    int n = s->n;
    memset(s->aoff, 0, (size_t)(n + 1) * sizeof(int));
    for (int64_t k = 0; k < s->nb; ++k) { s->aoff[s->bond[k].i + 1]++; s->aoff[s->bond[k].j + 1]++; }
    for (int i = 0; i < n; ++i) s->aoff[i + 1] += s->aoff[i];
    size_t m = (size_t)(2 * s->nb) + 1;
    s->anbr = (int*)realloc(s->anbr, m * sizeof(int));
    s->atype = (int*)realloc(s->atype, m * sizeof(int));
    s->abond = (int*)realloc(s->abond, m * sizeof(int));
    int* fill = (int*)calloc((size_t)n + 1, sizeof(int));
    for (int64_t k = 0; k < s->nb; ++k) {
        const bond_t* b = &s->bond[k];
        int p = s->aoff[b->i] + fill[b->i]++;
        s->anbr[p] = b->j; s->atype[p] = b->tij; s->abond[p] = (int)k;
        p = s->aoff[b->j] + fill[b->j]++;
        s->anbr[p] = b->i; s->atype[p] = b->tji; s->abond[p] = (int)k;
    }
    free(fill);
    s->adj_valid = 1;
}

/* bond index between u and v, or -1 */
static int bond_between(const or_sys* s, int u, int v) {
    for (int p = s->aoff[u]; p < s->aoff[u + 1]; ++p)
        if (s->anbr[p] == v) return s->abond[p];
    return -1;
}

/* type stored by u for its bond to v, or -1 */
static int stored_type(const or_sys* s, int u, int v) {
    for (int p = s->aoff[u]; p < s->aoff[u + 1]; ++p)
        if (s->anbr[p] == v) return s->atype[p];
    return -1;
}

int or_graph_distance(or_sys* s, int32_t i, int32_t j) {
    build_adj(s);
    if (i == j) return 0;
    /* breadth-first search to depth 3 */
    int frontier[4096], next[4096], seen[8192];
    int nf = 1, nseen = 1;
    frontier[0] = i; seen[0] = i;
    for (int depth = 1; depth <= 3; ++depth) {
        int nn = 0;
        for (int f = 0; f < nf; ++f) {
            int u = frontier[f];
            for (int p = s->aoff[u]; p < s->aoff[u + 1]; ++p) {
                int w = s->anbr[p];
                int dup = 0;
                for (int q = 0; q < nseen; ++q) if (seen[q] == w) { dup = 1; break; }
                if (dup) continue;
                if (w == j) return depth;
                if (nseen < 8192) seen[nseen++] = w;
                if (nn < 4096) next[nn++] = w;
            }
        }
        memcpy(frontier, next, (size_t)nn * sizeof(int));
        nf = nn;
    }
    return 4;
}

/* ------------------------------------------------------------------------- */
/* parameters and rules */
int or_pair_wca(or_sys* s, double eps, double sigma, double rc, int depth) {
    if (!(rc > 0) || depth < 0 || depth > 2) return -1;
    s->eps = eps; s->sig = sigma; s->rc = rc; s->excl_depth = depth; s->have_pair = 1; s->pair_style = 0;
    return 0;
}
/* DPD pair force of section 3: conservative a w(r), dissipative and random parts
 * with friction gamma and sigma = sqrt(2 T gamma) (T from the thermostat settings) */
int or_pair_dpd(or_sys* s, double a, double gamma, double rc, int depth) {
    if (!(rc > 0) || depth < 0 || depth > 2 || gamma < 0) return -1;
    s->dpd_a = a; s->dpd_gamma = gamma; s->rc = rc; s->excl_depth = depth; s->have_pair = 1; s->pair_style = 1;
    return 0;
}
int or_bond_harmonic(or_sys* s, int32_t t, double K, double r0) {
    if (t < 1 || t >= MAXT) return -1;
    s->bK[t] = K; s->bR0[t] = r0; s->bset[t] = 1; s->bstyle[t] = 0; return 0;
}
/* bond well of the 1-bead DNA model, section 3, in the reading that makes the
 * printed backbone and hybridization forms consistent: U = U_min [(r - r_w)^2 /
 * (r_z - r_w)^2 - 1] for r < r_cut, 0 beyond; minimum -U_min at the well r_w,
 * zero at r_z (r_cut = +inf: no cutoff) */
int or_bond_well(or_sys* s, int32_t t, double umin, double rw, double rz, double rcut) {
    if (t < 1 || t >= MAXT || !isfinite(umin) || !isfinite(rw) || !isfinite(rz) || rz == rw || !(rcut > 0))
        return -1;
    s->bUmin[t] = umin; s->bRw[t] = rw; s->bRz[t] = rz; s->bRcut[t] = rcut;
    s->bset[t] = 1; s->bstyle[t] = 1;
    return 0;
}
int or_angle_harmonic(or_sys* s, int32_t t, double K, double th0) {
    if (t < 1 || t >= MAXT) return -1;
    s->aK[t] = K; s->aT0[t] = th0; s->aset[t] = 1; return 0;
}
int or_dihedral_cosine(or_sys* s, int32_t t, double K, double p0) {
    if (t < 1 || t >= MAXT) return -1;
    s->dK[t] = K; s->dP0[t] = p0; s->dset[t] = 1; return 0;
}
int or_langevin(or_sys* s, double T, double gamma, double dt) {
    if (!(dt > 0) || gamma < 0 || T < 0) return -1;
    s->T0 = s->T1 = T; s->gamma = gamma; s->dt = dt; s->ramp = 0; return 0;
}
int or_temperature_ramp(or_sys* s, double T0, double T1, int64_t n) {
    if (n < 0) return -1;
    s->T0 = T0; s->T1 = T1; s->ramp = n; return 0;
}
int or_acceptance(or_sys* s, int mode) {
    if (mode != 0 && mode != 1) return -1;
    s->accept_average = mode;
    return 0;
}
int or_sweep_every(or_sys* s, int32_t every, int pc13, int pc14) {
    if (every < 0) return -1;
    s->every = every; s->pc13 = pc13 ? 1 : 0; s->pc14 = pc14 ? 1 : 0; return 0;
}
static int add_rule(or_sys* s, rule_t r) {
    if (s->nrule >= MAXRULES) return -2;
    s->rule[s->nrule++] = r; return 0;
}
int or_bond_create(or_sys* s, int32_t bt, int32_t b1, int32_t b2, double rmax, double p) {
    if (bt < 1 || bt >= MAXT || !(rmax > 0) || p < 0 || p > 1) return -1;
    rule_t r = {R_CREATE, bt, bt, b1, b2, rmax * rmax, p};
    return add_rule(s, r);
}
int or_bond_create_dir(or_sys* s, int32_t bt1, int32_t bt2, int32_t b1, int32_t b2, double rmax, double p) {
    if (bt1 < 1 || bt1 >= MAXT || bt2 < 1 || bt2 >= MAXT || !(rmax > 0) || p < 0 || p > 1) return -1;
    rule_t r = {R_CREATEDIR, bt1, bt2, b1, b2, rmax * rmax, p};
    return add_rule(s, r);
}
int or_bond_break(or_sys* s, int32_t bt, double rmin, double p) {
    if (bt < 1 || bt >= MAXT || rmin < 0 || p < 0 || p > 1) return -1;
    rule_t r = {R_BREAK, bt, bt, 0, 0, rmin * rmin, p};
    return add_rule(s, r);
}
int or_bond_kill(or_sys* s, int32_t bt, double rmin) {
    if (bt < 1 || bt >= MAXT || rmin < 0) return -1;
    rule_t r = {R_KILL, bt, bt, 0, 0, rmin * rmin, 1.0};
    return add_rule(s, r);
}
int or_bond_convert(or_sys* s, int32_t bf, int32_t bto, double rmin, double p) {
    if (bf < 1 || bf >= MAXT || bto < 1 || bto >= MAXT || rmin < 0 || p < 0 || p > 1) return -1;
    rule_t r = {R_CONVERT, bf, bto, 0, 0, rmin * rmin, p};
    return add_rule(s, r);
}
int or_max_bonds(or_sys* s, int32_t bt, int32_t bead, int32_t max) {
    if (bt < 1 || bt >= MAXT || max < 0 || s->nmax >= MAXRULES) return -1;
    maxrule_t m = {bt, bead, max};
    s->maxr[s->nmax++] = m; return 0;
}
int or_angle_pattern(or_sys* s, int32_t t, const int32_t b[3], const uint32_t m[2]) {
    if (t < 1 || t >= MAXT || s->narule >= MAXRULES) return -1;
    angrule_t r; r.type = t;
    for (int k = 0; k < 3; ++k) r.b[k] = b[k];
    r.m[0] = m[0]; r.m[1] = m[1];
    s->arule[s->narule++] = r; return 0;
}
int or_dihedral_pattern(or_sys* s, int32_t t, const int32_t b[4], const uint32_t m[3]) {
    if (t < 1 || t >= MAXT || s->ndrule >= MAXRULES) return -1;
    dihrule_t r; r.type = t;
    for (int k = 0; k < 4; ++k) r.b[k] = b[k];
    for (int k = 0; k < 3; ++k) r.m[k] = m[k];
    s->drule[s->ndrule++] = r; return 0;
}
int or_set_step(or_sys* s, int64_t st) { s->step = st; s->swept_step = -1; return 0; }

/* ------------------------------------------------------------------------- */
/* pattern matching (section 2).  Notation: t(u->v) = type stored by u for its
 * bond to v.  Angle ABC: bead types match and t(B->A) in S1, t(B->C) in S2;
 * else the same test on CBA.  Dihedral ABCD: bead types match, t(B->A) in S1,
 * t(C->B) or t(B->C) in S2, t(C->D) in S3; else the same test on DCBA. */
static int angle_rule_matches(const or_sys* s, const angrule_t* r, int a, int b, int c) {
    int tba = stored_type(s, b, a), tbc = stored_type(s, b, c);
    if (type_ok(r->b[0], s->type[a]) && type_ok(r->b[1], s->type[b]) && type_ok(r->b[2], s->type[c]) &&
        in_mask(r->m[0], tba) && in_mask(r->m[1], tbc))
        return 1;
    if (type_ok(r->b[0], s->type[c]) && type_ok(r->b[1], s->type[b]) && type_ok(r->b[2], s->type[a]) &&
        in_mask(r->m[0], tbc) && in_mask(r->m[1], tba))
        return 1;
    return 0;
}

static int dihedral_rule_matches(const or_sys* s, const dihrule_t* r, int a, int b, int c, int d) {
    int tba = stored_type(s, b, a), tbc = stored_type(s, b, c);
    int tcb = stored_type(s, c, b), tcd = stored_type(s, c, d);
    if (type_ok(r->b[0], s->type[a]) && type_ok(r->b[1], s->type[b]) && type_ok(r->b[2], s->type[c]) &&
        type_ok(r->b[3], s->type[d]) && in_mask(r->m[0], tba) &&
        (in_mask(r->m[1], tcb) || in_mask(r->m[1], tbc)) && in_mask(r->m[2], tcd))
        return 1;
    if (type_ok(r->b[0], s->type[d]) && type_ok(r->b[1], s->type[c]) && type_ok(r->b[2], s->type[b]) &&
        type_ok(r->b[3], s->type[a]) && in_mask(r->m[0], tcd) &&
        (in_mask(r->m[1], tbc) || in_mask(r->m[1], tcb)) && in_mask(r->m[2], tba))
        return 1;
    return 0;
}

/* first matching rule in table order, or 0 */
static int match_angle(const or_sys* s, int a, int b, int c) {
    for (int q = 0; q < s->narule; ++q)
        if (angle_rule_matches(s, &s->arule[q], a, b, c)) return s->arule[q].type;
    return 0;
}
static int match_dihedral(const or_sys* s, int a, int b, int c, int d) {
    for (int q = 0; q < s->ndrule; ++q)
        if (dihedral_rule_matches(s, &s->drule[q], a, b, c, d)) return s->drule[q].type;
    return 0;
}

/* Enumerate every non-cyclic 3-path (a,b,c) and 4-path (a,b,c,d) of the current
 * bond graph.  If is_new is NULL every path qualifies; otherwise a path
 * qualifies when at least one of its bonds is flagged new.  Qualifying paths
 * that match a pattern rule are appended to the angle/dihedral lists. */
static void generate(or_sys* s, const uint8_t* is_new, int64_t* n_ang, int64_t* n_dih) {
    build_adj(s);
    int64_t ca = 0, cd = 0;
    for (int b = 0; b < s->n; ++b) {
        for (int p = s->aoff[b]; p < s->aoff[b + 1]; ++p) {
            for (int q = p + 1; q < s->aoff[b + 1]; ++q) {
                int a = s->anbr[p], c = s->anbr[q];
                if (a == c) continue;
                if (is_new && !is_new[s->abond[p]] && !is_new[s->abond[q]]) continue;
                int t = match_angle(s, a, b, c);
                if (t) { push_ang(s, t, a, b, c); ++ca; }
            }
        }
    }
    for (int64_t k = 0; k < s->nb; ++k) {
        int b = s->bond[k].i, c = s->bond[k].j;
        for (int p = s->aoff[b]; p < s->aoff[b + 1]; ++p) {
            int a = s->anbr[p];
            if (a == c) continue;
            for (int q = s->aoff[c]; q < s->aoff[c + 1]; ++q) {
                int d = s->anbr[q];
                if (d == b || d == a) continue;
                if (is_new && !is_new[s->abond[p]] && !is_new[k] && !is_new[s->abond[q]]) continue;
                int t = match_dihedral(s, a, b, c, d);
                if (t) { push_dih(s, t, a, b, c, d); ++cd; }
            }
        }
    }
    if (n_ang) *n_ang = ca;
    if (n_dih) *n_dih = cd;
}

int or_generate_angles_dihedrals(or_sys* s) {
    s->na = 0; s->nd = 0;
    generate(s, NULL, NULL, NULL);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* neighbour search: visit every unordered pair (i<j) with r^2 < rcut^2 */
typedef void (*pair_fn)(or_sys* s, int i, int j, const double d[3], double r2, void* ctx);

static void for_pairs(or_sys* s, double rcut, int brute, pair_fn fn, void* ctx) {
    double rc2 = rcut * rcut;
    /* cells no narrower than rcut, and no more of them than about two per bead
     * (a large sparse box would otherwise ask for more cells than memory holds) */
    double ncd = floor(s->L / (rcut * (1.0 + 1e-9)));
    double ncap = floor(cbrt(2.0 * (double)s->n + 64.0));
    int nc = (int)(ncd < ncap ? ncd : ncap);
    if (brute || nc < 3) {
        double d[3];
        for (int i = 0; i < s->n; ++i)
            for (int j = i + 1; j < s->n; ++j) {
                double r2 = sep(s, i, j, d);
                if (r2 < rc2) fn(s, i, j, d, r2, ctx);
            }
        return;
    }
    int ncell = nc * nc * nc;
    int* head = (int*)malloc((size_t)ncell * sizeof(int));
    int* next = (int*)malloc((size_t)(s->n > 0 ? s->n : 1) * sizeof(int));
    for (int c = 0; c < ncell; ++c) head[c] = -1;
    int* cell = (int*)malloc((size_t)(s->n > 0 ? s->n : 1) * sizeof(int));
    for (int i = s->n - 1; i >= 0; --i) {
        int ix[3];
        for (int k = 0; k < 3; ++k) {
            ix[k] = (int)(s->x[3 * i + k] / s->L * nc);
            if (ix[k] >= nc) ix[k] = nc - 1;
            if (ix[k] < 0) ix[k] = 0;
        }
        int c = (ix[2] * nc + ix[1]) * nc + ix[0];
        cell[i] = c;
        next[i] = head[c];
        head[c] = i;
    }
    double d[3];
    for (int i = 0; i < s->n; ++i) {
        int c = cell[i];
        int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int nx = (cx + dx + nc) % nc, ny = (cy + dy + nc) % nc, nz = (cz + dz + nc) % nc;
                    int c2 = (nz * nc + ny) * nc + nx;
                    for (int j = head[c2]; j >= 0; j = next[j]) {
                        if (j <= i) continue;
                        double r2 = sep(s, i, j, d);
                        if (r2 < rc2) fn(s, i, j, d, r2, ctx);
                    }
                }
    }
    free(head); free(next); free(cell);
}

typedef struct { int32_t* out; int64_t cap, n; } pairlist_ctx;
static void collect_pair(or_sys* s, int i, int j, const double d[3], double r2, void* vctx) {
    (void)s; (void)d; (void)r2;
    pairlist_ctx* c = (pairlist_ctx*)vctx;
    if (c->n < c->cap) { c->out[2 * c->n] = i; c->out[2 * c->n + 1] = j; }
    c->n++;
}
int64_t or_pairs_within(or_sys* s, double rcut, int brute, int32_t* out, int64_t cap) {
    pairlist_ctx c = {out, cap, 0};
    for_pairs(s, rcut, brute, collect_pair, &c);
    return c.n;
}

/* ------------------------------------------------------------------------- */
/* conservative forces and energies */
typedef struct { double* f; double upair, ubond, uang, udih, vir; } force_ctx;

static int excluded_pair(const or_sys* s, int i, int j) {
    if (s->excl_depth >= 1 && bond_between(s, i, j) >= 0) return 1;
    if (s->excl_depth >= 2) {
        for (int p = s->aoff[i]; p < s->aoff[i + 1]; ++p)
            if (bond_between(s, s->anbr[p], j) >= 0) return 1;
    }
    return 0;
}

/* WCA: U = 4 eps [(sig/r)^12 - (sig/r)^6] + eps for r < rc */
static void wca_pair(or_sys* s, int i, int j, const double d[3], double r2, void* vctx) {
    force_ctx* c = (force_ctx*)vctx;
    if (excluded_pair(s, i, j)) return;
    double sr2 = s->sig * s->sig / r2;
    double sr6 = sr2 * sr2 * sr2;
    c->upair += 4.0 * s->eps * (sr6 * sr6 - sr6) + s->eps;
    double fr = 24.0 * s->eps * (2.0 * sr6 * sr6 - sr6) / r2;   /* -dU/dr / r */
    for (int k = 0; k < 3; ++k) {
        c->f[3 * i + k] -= fr * d[k];
        c->f[3 * j + k] += fr * d[k];
    }
    c->vir += fr * r2;
}

/* DPD, section 3.  With r_ij = x_i - x_j, r = |r_ij|, e = r_ij / r and
 * w = 1 - r / rc: F_i = -F_j = (F^C + F^D + F^R) e with F^C = a w,
 * F^D = -gamma w^2 (e . v_ij), F^R = sigma w xi / sqrt(dt).  U = a rc w^2 / 2. */
static void dpd_conservative_pair(or_sys* s, int i, int j, const double d[3], double r2, void* vctx) {
    force_ctx* c = (force_ctx*)vctx;
    if (excluded_pair(s, i, j)) return;
    double r = sqrt(r2);
    if (!(r > 0)) return;
    double w = 1.0 - r / s->rc;
    double fc = s->dpd_a * w;
    c->upair += 0.5 * s->dpd_a * s->rc * w * w;
    for (int k = 0; k < 3; ++k) {
        double e = -d[k] / r;   /* d = x_j - x_i */
        c->f[3 * i + k] += fc * e;
        c->f[3 * j + k] -= fc * e;
    }
    c->vir += fc * r;
}

typedef struct { double* f; double sigma_over_sqrt_dt; int64_t step; } dpd_thermo_ctx;

static void dpd_thermostat_pair(or_sys* s, int i, int j, const double d[3], double r2, void* vctx) {
    dpd_thermo_ctx* c = (dpd_thermo_ctx*)vctx;
    if (excluded_pair(s, i, j)) return;
    double r = sqrt(r2);
    if (!(r > 0)) return;
    double w = 1.0 - r / s->rc;
    double e[3], ev = 0.0;
    for (int k = 0; k < 3; ++k) {
        e[k] = -d[k] / r;
        ev += e[k] * (s->v[3 * i + k] - s->v[3 * j + k]);
    }
    double fd = -s->dpd_gamma * w * w * ev;
    double fr = c->sigma_over_sqrt_dt * w * pair_gaussian(s, i, j, c->step);
    for (int k = 0; k < 3; ++k) {
        c->f[3 * i + k] += (fd + fr) * e[k];
        c->f[3 * j + k] -= (fd + fr) * e[k];
    }
}

/* energy u and dU/dr of bond type t at length r, as the bead storing t feels it */
static void bond_potential(const or_sys* s, int t, double r, double* u, double* du) {
    if (s->bstyle[t] == 1) {
        if (r < s->bRcut[t]) {
            double w = s->bRz[t] - s->bRw[t];
            *u = s->bUmin[t] * ((r - s->bRw[t]) * (r - s->bRw[t]) / (w * w) - 1.0);
            *du = 2.0 * s->bUmin[t] * (r - s->bRw[t]) / (w * w);
        } else {
            *u = 0.0;
            *du = 0.0;
        }
        return;
    }
    *u = s->bK[t] * (r - s->bR0[t]) * (r - s->bR0[t]);
    *du = 2.0 * s->bK[t] * (r - s->bR0[t]);
}

static void bonded_forces(or_sys* s, force_ctx* c) {
    double* f = c->f;
    /* bonds: bead i feels the potential of the type it stores (t_ij), bead j that of t_ji */
    for (int64_t k = 0; k < s->nb; ++k) {
        const bond_t* b = &s->bond[k];
        double d[3];
        double r = sqrt(sep(s, b->i, b->j, d));
        if (!(r > 0)) continue;
        double ui, dui, uj, duj;
        bond_potential(s, b->tij, r, &ui, &dui);
        bond_potential(s, b->tji, r, &uj, &duj);
        c->ubond += 0.5 * (ui + uj);
        double gi = dui / r;   /* F_i = gi * d (d points from i to j) */
        double gj = duj / r;   /* F_j = -gj * d */
        for (int q = 0; q < 3; ++q) {
            f[3 * b->i + q] += gi * d[q];
            f[3 * b->j + q] -= gj * d[q];
        }
        c->vir -= 0.5 * (gi + gj) * r * r;
    }
    /* angles: U = K (theta - theta0)^2 */
    for (int64_t k = 0; k < s->na; ++k) {
        const ang_t* e = &s->ang[k];
        double K = s->aK[e->type], th0 = s->aT0[e->type];
        double u[3], w[3];
        double ru2 = sep(s, e->b, e->a, u);
        double rw2 = sep(s, e->b, e->c, w);
        double ru = sqrt(ru2), rw = sqrt(rw2);
        if (!(ru > 0) || !(rw > 0)) continue;
        double cu[3], cw[3];
        for (int q = 0; q < 3; ++q) { cu[q] = u[q] / ru; cw[q] = w[q] / rw; }
        double cs = cu[0] * cw[0] + cu[1] * cw[1] + cu[2] * cw[2];
        double cr[3] = {cu[1] * cw[2] - cu[2] * cw[1], cu[2] * cw[0] - cu[0] * cw[2], cu[0] * cw[1] - cu[1] * cw[0]};
        double sn = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        double th = atan2(sn, cs);
        c->uang += K * (th - th0) * (th - th0);
        /* A = dU/dtheta / sin(theta), split so that theta0 = pi has a finite limit:
         * theta - theta0 = -(pi - theta) + (pi - theta0); (pi-theta)/sin(theta) -> 1 */
        double del = atan2(sn, -cs);          /* pi - theta */
        double ratio = del < 1e-6 ? 1.0 + del * del / 6.0 : del / (sn > 1e-8 ? sn : 1e-8);
        double pth = 3.14159265358979323846 - th0;
        double A = 2.0 * K * (-ratio + (pth != 0.0 ? pth / (sn > 1e-8 ? sn : 1e-8) : 0.0));
        double fa[3], fc[3];
        for (int q = 0; q < 3; ++q) {
            fa[q] = -A * (cs * cu[q] - cw[q]) / ru;
            fc[q] = -A * (cs * cw[q] - cu[q]) / rw;
            f[3 * e->a + q] += fa[q];
            f[3 * e->c + q] += fc[q];
            f[3 * e->b + q] -= fa[q] + fc[q];
        }
        c->vir += (u[0] * fa[0] + u[1] * fa[1] + u[2] * fa[2]) + (w[0] * fc[0] + w[1] * fc[1] + w[2] * fc[2]);
    }
    /* dihedrals: U = K [1 - cos(phi - phi0)], phi the IUPAC signed dihedral (cis = 0) */
    for (int64_t k = 0; k < s->nd; ++k) {
        const dih_t* e = &s->dih[k];
        double K = s->dK[e->type], p0 = s->dP0[e->type];
        double b1[3], b2[3], b3[3];
        sep(s, e->a, e->b, b1);
        sep(s, e->b, e->c, b2);
        sep(s, e->c, e->d, b3);
        double m[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2], b1[0] * b2[1] - b1[1] * b2[0]};
        double nn[3] = {b2[1] * b3[2] - b2[2] * b3[1], b2[2] * b3[0] - b2[0] * b3[2], b2[0] * b3[1] - b2[1] * b3[0]};
        double m2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
        double n2 = nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2];
        double b22 = b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2];
        if (m2 < 1e-24 || n2 < 1e-24 || b22 < 1e-24) { s->degenerate_dihedrals++; continue; }
        double nb2 = sqrt(b22);
        double inv = 1.0 / sqrt(m2 * n2);
        double cphi = (m[0] * nn[0] + m[1] * nn[1] + m[2] * nn[2]) * inv;
        double sphi = nb2 * (b1[0] * nn[0] + b1[1] * nn[1] + b1[2] * nn[2]) * inv;
        double c0 = cos(p0), s0 = sin(p0);
        c->udih += K * (1.0 - (cphi * c0 + sphi * s0));
        double dU = K * (sphi * c0 - cphi * s0);      /* dU/dphi = K sin(phi - phi0) */
        double ga[3], gd[3];
        for (int q = 0; q < 3; ++q) {
            ga[q] = -nb2 / m2 * m[q];   /* dphi/dx_a */
            gd[q] = nb2 / n2 * nn[q];   /* dphi/dx_d */
        }
        double p = (b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2]) / b22;
        double r = (b3[0] * b2[0] + b3[1] * b2[1] + b3[2] * b2[2]) / b22;
        double fa[3], fb[3], fc[3], fd[3];
        for (int q = 0; q < 3; ++q) {
            double gb = r * gd[q] - (p + 1.0) * ga[q];
            double gc = p * ga[q] - (r + 1.0) * gd[q];
            fa[q] = -dU * ga[q]; fb[q] = -dU * gb; fc[q] = -dU * gc; fd[q] = -dU * gd[q];
            f[3 * e->a + q] += fa[q];
            f[3 * e->b + q] += fb[q];
            f[3 * e->c + q] += fc[q];
            f[3 * e->d + q] += fd[q];
        }
        /* reference bead b: x_a - x_b = -b1, x_c - x_b = b2, x_d - x_b = b2 + b3 */
        for (int q = 0; q < 3; ++q) c->vir += -b1[q] * fa[q] + b2[q] * fc[q] + (b2[q] + b3[q]) * fd[q];
    }
}

static void conservative(or_sys* s, force_ctx* c) {
    build_adj(s);
    memset(c->f, 0, (size_t)s->n * 3 * sizeof(double));
    c->upair = c->ubond = c->uang = c->udih = c->vir = 0.0;
    if (s->have_pair) for_pairs(s, s->rc, 0, s->pair_style == 1 ? dpd_conservative_pair : wca_pair, c);
    bonded_forces(s, c);
    if (s->fext)
        for (int i = 0; i < 3 * s->n; ++i) c->f[i] += s->fext[i];
}

/* constant external forces (the unzipping experiments of section 3): bead ids[k]
 * feels f[3k..3k+2] in every force evaluation; count = 0 removes them all; a
 * bead listed twice keeps the sum */
int or_external_force(or_sys* s, int64_t count, const int32_t* ids, const double* f) {
    if (count < 0) return -1;
    for (int64_t k = 0; k < count; ++k)
        if (ids[k] < 0 || ids[k] >= s->n || !isfinite(f[3 * k]) || !isfinite(f[3 * k + 1]) || !isfinite(f[3 * k + 2]))
            return -1;
    free(s->fext);
    s->fext = NULL;
    if (count == 0) return 0;
    s->fext = (double*)calloc(3 * (size_t)s->n, sizeof(double));
    for (int64_t k = 0; k < count; ++k)
        for (int q = 0; q < 3; ++q) s->fext[3 * (size_t)ids[k] + q] += f[3 * k + q];
    return 0;
}

int or_forces(or_sys* s, double* f) {
    force_ctx c = {f, 0, 0, 0, 0, 0};
    conservative(s, &c);
    return 0;
}

static double temperature(const or_sys* s, int64_t step) {
    if (s->ramp <= 0) return s->T0;
    int64_t k = step < s->ramp ? step : s->ramp;
    return s->T0 + (s->T1 - s->T0) * (double)k / (double)s->ramp;
}

/* total force = conservative - gamma v + sqrt(24 gamma T / dt) (u - 1/2) per
 * component, u uniform from Philox keyed by (bead id, step) */
static void add_langevin(or_sys* s, double* f, int64_t step) {
    if (s->gamma == 0.0) return;
    double pref = sqrt(24.0 * s->gamma * temperature(s, step) / s->dt);
    for (int i = 0; i < s->n; ++i) {
        uint32_t w[4];
        draw(s, (uint32_t)i, 0u, step, KIND_LANGEVIN, w);
        for (int k = 0; k < 3; ++k) {
            double u = ((double)w[k] + 0.5) * (1.0 / 4294967296.0);
            f[3 * i + k] = f[3 * i + k] - s->gamma * s->v[3 * i + k] + pref * (u - 0.5);
        }
    }
}

/* the dissipative and random DPD forces of a step, added to f */
static void add_dpd(or_sys* s, double* f, int64_t step) {
    if (!s->have_pair || s->pair_style != 1 || s->dpd_gamma == 0.0) return;
    dpd_thermo_ctx c = {f, sqrt(2.0 * temperature(s, step) * s->dpd_gamma) / sqrt(s->dt), step};
    for_pairs(s, s->rc, 0, dpd_thermostat_pair, &c);
}

int or_energy(or_sys* s, double out[6]) {
    double* f = (double*)malloc((size_t)(s->n > 0 ? s->n : 1) * 3 * sizeof(double));
    force_ctx c = {f, 0, 0, 0, 0, 0};
    conservative(s, &c);
    add_dpd(s, f, s->step);
    add_langevin(s, f, s->step);
    double ke = 0.0, hdt = 0.5 * s->dt;
    for (int i = 0; i < 3 * s->n; ++i) {
        double vf = s->v[i] + hdt * f[i];   /* full-step velocity */
        ke += 0.5 * vf * vf;
    }
    free(f);
    out[0] = ke; out[1] = c.upair; out[2] = c.ubond; out[3] = c.uang; out[4] = c.udih; out[5] = c.vir;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* the dynamic-bonding sweep (appendix, steps 2-9) */

static int count_type(const or_sys* s, int k, int t) {
    int c = 0;
    for (int p = s->aoff[k]; p < s->aoff[k + 1]; ++p) c += (s->atype[p] == t);
    return c;
}

/* maxbond: bead k may take one more bond that it would store as type t */
static int max_ok(const or_sys* s, int k, int t) {
    for (int q = 0; q < s->nmax; ++q)
        if (s->maxr[q].bt == t && type_ok(s->maxr[q].bead, s->type[k]) && count_type(s, k, t) >= s->maxr[q].max)
            return 0;
    return 1;
}

/* The last creation rule applicable to the pair (i,j) at squared distance r2,
 * with the bond types i and j would store.  Returns rule index or -1. */
static int create_rule_for(const or_sys* s, int i, int j, double r2, int* bti, int* btj) {
    int found = -1;
    for (int q = 0; q < s->nrule; ++q) {
        const rule_t* r = &s->rule[q];
        if (r->kind != R_CREATE && r->kind != R_CREATEDIR) continue;
        int o1 = type_ok(r->b1, s->type[i]) && type_ok(r->b2, s->type[j]);   /* i plays bead1 */
        int o2 = type_ok(r->b1, s->type[j]) && type_ok(r->b2, s->type[i]);   /* j plays bead1 */
        if (!o1 && !o2) continue;
        if (o1 && o2) { o1 = i < j; o2 = !o1; }   /* both orientations: lower id plays bead1 */
        int ti = o1 ? r->bt1 : r->bt2;
        int tj = o1 ? r->bt2 : r->bt1;
        if (!(r2 < r->r2)) continue;
        if (!max_ok(s, i, ti) || !max_ok(s, j, tj)) continue;
        found = q; *bti = ti; *btj = tj;
    }
    return found;
}

/* The last break-class rule (breakbond / convertbond) applicable to the
 * symmetric bond (i,j) of type t at squared length r2, or -1. */
static int break_rule_for(const or_sys* s, int i, int j, int t, double r2) {
    int found = -1;
    for (int q = 0; q < s->nrule; ++q) {
        const rule_t* r = &s->rule[q];
        if (r->kind == R_BREAK) {
            if (r->bt1 == t && r2 > r->r2) found = q;
        } else if (r->kind == R_CONVERT) {
            if (r->bt1 == t && r2 > r->r2 && max_ok(s, i, r->bt2) && max_ok(s, j, r->bt2)) found = q;
        }
    }
    return found;
}

typedef struct { int* best; double* bestr2; int* rule; int* bt; } nomc_ctx;

/* candidate (i,j) for creation: both reactive, not 1-2 neighbours, not 1-3 or
 * 1-4 unless the paircheck switch admits them, and some creation rule applies */
static void consider_create(or_sys* s, int i, int j, double r2, nomc_ctx* c) {
    if (!s->reactive[i] || !s->reactive[j]) return;
    int bti, btj;
    int q = create_rule_for(s, i, j, r2, &bti, &btj);
    if (q < 0) return;
    int g = or_graph_distance(s, i, j);
    if (g == 1) return;
    if (g == 2 && !s->pc13) return;
    if (g == 3 && !s->pc14) return;
    /* closest partner; exact ties go to the lower id */
    if (c->best[i] < 0 || r2 < c->bestr2[i] || (r2 == c->bestr2[i] && j < c->best[i])) {
        c->best[i] = j; c->bestr2[i] = r2; c->rule[i] = q; c->bt[i] = bti;
    }
    if (c->best[j] < 0 || r2 < c->bestr2[j] || (r2 == c->bestr2[j] && i < c->best[j])) {
        c->best[j] = i; c->bestr2[j] = r2; c->rule[j] = q; c->bt[j] = btj;
    }
}

static void create_pair_cb(or_sys* s, int i, int j, const double d[3], double r2, void* vctx) {
    (void)d;
    consider_create(s, i, j, r2, (nomc_ctx*)vctx);
}

static int sweep(or_sys* s, int64_t step) {
    int n = s->n;
    build_adj(s);
    int64_t st[8] = {0, 0, 0, 0, 0, 0, 0, 0};

    /* step 2: creation nomination (closest eligible partner) */
    int* bestC = s->nomC;
    double* bestr2 = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int* ruleC = (int*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int* btC = (int*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    for (int i = 0; i < n; ++i) { bestC[i] = -1; ruleC[i] = -1; btC[i] = 0; bestr2[i] = 0; }
    double rmax2 = 0.0;
    for (int q = 0; q < s->nrule; ++q)
        if ((s->rule[q].kind == R_CREATE || s->rule[q].kind == R_CREATEDIR) && s->rule[q].r2 > rmax2)
            rmax2 = s->rule[q].r2;
    if (rmax2 > 0) {
        nomc_ctx c = {bestC, bestr2, ruleC, btC};
        for_pairs(s, sqrt(rmax2) * (1.0 + 1e-12), 0, create_pair_cb, &c);
    }

    /* step 3: breakage nomination (most distant eligible bonded partner) */
    int* bestK = s->nomK;
    int* ruleK = (int*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    for (int i = 0; i < n; ++i) {
        bestK[i] = -1; ruleK[i] = -1;
        if (!s->reactive[i]) continue;
        double br2 = 0.0;
        for (int p = s->aoff[i]; p < s->aoff[i + 1]; ++p) {
            int j = s->anbr[p];
            if (!s->reactive[j]) continue;
            int tij = s->atype[p], tji = stored_type(s, j, i);
            if (tij != tji) continue;   /* only symmetric bonds break */
            double d[3];
            double r2 = sep(s, i, j, d);
            int q = break_rule_for(s, i, j, tij, r2);
            if (q < 0) continue;
            if (bestK[i] < 0 || r2 > br2 || (r2 == br2 && j < bestK[i])) { bestK[i] = j; br2 = r2; ruleK[i] = q; }
        }
    }

    /* step 5: killbond marks, then mutual break nominations accepted with
     * probability p (one uniform per pair, keyed by the pair and the step) */
    int64_t nb = s->nb;
    uint8_t* killed = (uint8_t*)calloc((size_t)nb + 1, 1);
    uint8_t* removed = (uint8_t*)calloc((size_t)nb + 1, 1);   /* killed, broken or converted */
    int* conv_to = (int*)calloc((size_t)nb + 1, sizeof(int));
    uint8_t* conv_bead = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t k = 0; k < nb; ++k) {
        const bond_t* b = &s->bond[k];
        if (!s->reactive[b->i] || !s->reactive[b->j] || b->tij != b->tji) continue;
        double d[3];
        double r2 = sep(s, b->i, b->j, d);
        for (int q = 0; q < s->nrule; ++q)
            if (s->rule[q].kind == R_KILL && s->rule[q].bt1 == b->tij && r2 > s->rule[q].r2) killed[k] = 1;
        if (killed[k]) { removed[k] = 1; st[2]++; }
    }
    for (int i = 0; i < n; ++i) {
        int j = bestK[i];
        if (j < 0 || j < i || bestK[j] != i) continue;   /* each mutual pair once, from its lower id */
        int k = bond_between(s, i, j);
        if (killed[k]) continue;
        const rule_t* r = &s->rule[ruleK[i]];
        if (accept_number(s, i, j, step, KIND_BREAK) < r->p) {
            removed[k] = 1;
            if (r->kind == R_CONVERT) { conv_to[k] = r->bt2; conv_bead[i] = conv_bead[j] = 1; st[3]++; }
            else st[1]++;
        }
    }

    /* step 6: remove every angle / dihedral crossing a removed bond, judged on
     * the outdated bond graph (which still holds the removed bonds) */
    {
        int64_t w = 0;
        for (int64_t k = 0; k < s->na; ++k) {
            const ang_t* e = &s->ang[k];
            int b1 = bond_between(s, e->a, e->b), b2 = bond_between(s, e->b, e->c);
            if ((b1 >= 0 && removed[b1]) || (b2 >= 0 && removed[b2])) { st[5]++; continue; }
            s->ang[w++] = *e;
        }
        s->na = w;
        w = 0;
        for (int64_t k = 0; k < s->nd; ++k) {
            const dih_t* e = &s->dih[k];
            int b1 = bond_between(s, e->a, e->b), b2 = bond_between(s, e->b, e->c), b3 = bond_between(s, e->c, e->d);
            if ((b1 >= 0 && removed[b1]) || (b2 >= 0 && removed[b2]) || (b3 >= 0 && removed[b3])) { st[7]++; continue; }
            s->dih[w++] = *e;
        }
        s->nd = w;
    }

    /* step 7: drop killed/broken bonds; converted bonds change type */
    {
        int64_t w = 0;
        for (int64_t k = 0; k < nb; ++k) {
            bond_t b = s->bond[k];
            if (removed[k] && !conv_to[k]) continue;
            if (conv_to[k]) { b.tij = b.tji = conv_to[k]; }
            s->bond[w] = b;
            /* carry the conversion mark to the compacted index */
            conv_to[w] = conv_to[k];
            ++w;
        }
        s->nb = w;
        s->adj_valid = 0;
    }
    int64_t nb_kept = s->nb;

    /* step 8: mutual creation nominations, accepted with probability p; a bead
     * taking part in an accepted conversion creates nothing this sweep */
    for (int i = 0; i < n; ++i) {
        int j = bestC[i];
        if (j < 0 || j < i || bestC[j] != i) continue;
        if (conv_bead[i] || conv_bead[j]) continue;
        const rule_t* r = &s->rule[ruleC[i]];
        if (accept_number(s, i, j, step, KIND_CREATE) < r->p) {
            push_bond(s, i, j, btC[i], btC[j]);
            st[0]++;
        }
    }

    /* step 9: new angles / dihedrals on paths holding at least one new bond
     * (created or converted) of the updated graph */
    uint8_t* is_new = (uint8_t*)calloc((size_t)s->nb + 1, 1);
    int any_new = 0;
    for (int64_t k = 0; k < s->nb; ++k) {
        is_new[k] = (k >= nb_kept) || (conv_to[k] != 0);
        any_new |= is_new[k];
    }
    s->adj_valid = 0;
    build_adj(s);
    if (any_new) generate(s, is_new, &st[4], &st[6]);

    for (int q = 0; q < 8; ++q) { s->stat_last[q] = st[q]; s->stat_cum[q] += st[q]; }
    s->sweeps++;
    free(bestr2); free(ruleC); free(btC); free(ruleK);
    free(killed); free(removed); free(conv_to); free(conv_bead); free(is_new);
    return 0;
}

int or_sweep_now(or_sys* s) {
    if (s->swept_step == s->step) return -5;
    int rc = sweep(s, s->step);
    s->swept_step = s->step;
    return rc;
}

/* ------------------------------------------------------------------------- */
/* time stepping: velocity Verlet (section 3) with the Langevin force.  The
 * stored velocity is the one entering the force evaluation of the current
 * step (after the first half-kick and the drift).  One step:
 *   sweep if due;  F = F_c(x) - gamma v + noise;  v_full = v + dt/2 F;
 *   v = v_full + dt/2 F;  x = wrap(x + dt v). */
static double wrap1(double x, double L) {
    if (x >= L) return x - L;
    if (x < 0.0) {
        double y = x + L;
        return y >= L ? 0.0 : y;
    }
    return x;
}

int or_step(or_sys* s, int64_t nsteps) {
    double* f = (double*)malloc((size_t)(s->n > 0 ? s->n : 1) * 3 * sizeof(double));
    double hdt = 0.5 * s->dt;
    for (int64_t it = 0; it < nsteps; ++it) {
        if (s->every > 0 && s->step % s->every == 0 && s->swept_step != s->step) {
            sweep(s, s->step);
            s->swept_step = s->step;
        }
        force_ctx c = {f, 0, 0, 0, 0, 0};
        conservative(s, &c);
        add_dpd(s, f, s->step);
        add_langevin(s, f, s->step);
        for (int i = 0; i < 3 * s->n; ++i) {
            double vh = s->v[i] + hdt * f[i];
            s->v[i] = vh + hdt * f[i];
            double xn = s->x[i] + s->dt * s->v[i];
            if (!isfinite(xn)) { free(f); return -3; }
            s->x[i] = wrap1(xn, s->L);
            if (s->x[i] < 0.0 || s->x[i] >= s->L) { free(f); return -3; }
        }
        s->step++;
    }
    free(f);
    return 0;
}

int or_get_state(or_sys* s, double* x, double* v) {
    if (x) memcpy(x, s->x, (size_t)s->n * 3 * sizeof(double));
    if (v) memcpy(v, s->v, (size_t)s->n * 3 * sizeof(double));
    return 0;
}

int or_topology_counts(or_sys* s, int64_t* nb, int64_t* na, int64_t* nd) {
    if (nb) *nb = s->nb;
    if (na) *na = s->na;
    if (nd) *nd = s->nd;
    return 0;
}

static int cmp_bond(const void* p, const void* q) {
    const bond_t *a = (const bond_t*)p, *b = (const bond_t*)q;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}
static int cmp_ang(const void* p, const void* q) {
    const ang_t *a = (const ang_t*)p, *b = (const ang_t*)q;
    if (a->a != b->a) return a->a < b->a ? -1 : 1;
    if (a->b != b->b) return a->b < b->b ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    return a->type < b->type ? -1 : (a->type > b->type);
}
static int cmp_dih(const void* p, const void* q) {
    const dih_t *a = (const dih_t*)p, *b = (const dih_t*)q;
    if (a->a != b->a) return a->a < b->a ? -1 : 1;
    if (a->b != b->b) return a->b < b->b ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    if (a->d != b->d) return a->d < b->d ? -1 : 1;
    return a->type < b->type ? -1 : (a->type > b->type);
}

int or_get_bonds(or_sys* s, int32_t* ij, int32_t* tij, int32_t* tji) {
    bond_t* tmp = (bond_t*)malloc((size_t)(s->nb + 1) * sizeof(bond_t));
    memcpy(tmp, s->bond, (size_t)s->nb * sizeof(bond_t));
    qsort(tmp, (size_t)s->nb, sizeof(bond_t), cmp_bond);
    for (int64_t k = 0; k < s->nb; ++k) {
        ij[2 * k] = tmp[k].i; ij[2 * k + 1] = tmp[k].j; tij[k] = tmp[k].tij; tji[k] = tmp[k].tji;
    }
    free(tmp);
    return 0;
}

int or_get_angles(or_sys* s, int32_t* abc, int32_t* type) {
    ang_t* tmp = (ang_t*)malloc((size_t)(s->na + 1) * sizeof(ang_t));
    memcpy(tmp, s->ang, (size_t)s->na * sizeof(ang_t));
    qsort(tmp, (size_t)s->na, sizeof(ang_t), cmp_ang);
    for (int64_t k = 0; k < s->na; ++k) {
        abc[3 * k] = tmp[k].a; abc[3 * k + 1] = tmp[k].b; abc[3 * k + 2] = tmp[k].c; type[k] = tmp[k].type;
    }
    free(tmp);
    return 0;
}

int or_get_dihedrals(or_sys* s, int32_t* abcd, int32_t* type) {
    dih_t* tmp = (dih_t*)malloc((size_t)(s->nd + 1) * sizeof(dih_t));
    memcpy(tmp, s->dih, (size_t)s->nd * sizeof(dih_t));
    qsort(tmp, (size_t)s->nd, sizeof(dih_t), cmp_dih);
    for (int64_t k = 0; k < s->nd; ++k) {
        abcd[4 * k] = tmp[k].a; abcd[4 * k + 1] = tmp[k].b; abcd[4 * k + 2] = tmp[k].c; abcd[4 * k + 3] = tmp[k].d;
        type[k] = tmp[k].type;
    }
    free(tmp);
    return 0;
}

int or_get_stats(or_sys* s, int64_t out[17]) {
    for (int q = 0; q < 8; ++q) { out[q] = s->stat_last[q]; out[8 + q] = s->stat_cum[q]; }
    out[16] = s->sweeps;
    return 0;
}

int or_last_nominations(or_sys* s, int32_t* nc, int32_t* nk) {
    for (int i = 0; i < s->n; ++i) { nc[i] = s->nomC[i]; nk[i] = s->nomK[i]; }
    return 0;
}
