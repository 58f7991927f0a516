// Per-step force pass: one thread per bead gathers its own force (Newton's third
// law is not used for bonded terms: every bead evaluates each bond, angle and
// dihedral it takes part in, as in the paper's directional-bond storage, section 2
// and appendix), so nothing is accumulated across threads.  Pair forces: WCA, or
// the DPD conservative, dissipative and random forces (section 3), from the
// Verlet list.  Bonded: harmonic
// bonds with the type the bead stores, harmonic angles, cosine dihedrals
// (section 3 potentials).  Then the Langevin force and the velocity-Verlet
// update of the bead, written to a second position buffer.
//
// R is the force arithmetic type: double (DB_FP64) or float (DB_MIXED).  In
// both, coordinate differences with the minimum image, force accumulation,
// energies, the thermostat and the integration are double.
#include "cell_scan.h"

namespace db {

enum { MODE_STEP = 0, MODE_FORCES = 1, MODE_ENERGY = 2 };

template <typename R>
struct Acc {
    double fx = 0, fy = 0, fz = 0;
    double e_pair = 0, e_bond = 0, e_ang = 0, e_dih = 0, vir = 0;
};

// Per-type bonded coefficients in the force arithmetic type, staged in LDS by
// every workgroup: the type of an entry is known only once the entry is read,
// and an LDS lookup costs far less than a second dependent global load.
template <typename R>
struct Coef {
    double bRc2[DB_MAXT];                         // squared bond cutoff (+inf: none), tested in double
    R bK[DB_MAXT], bR0[DB_MAXT];
    R aK[DB_MAXT], aT0[DB_MAXT], aPm[DB_MAXT];   // aPm = pi - theta0
    R dK[DB_MAXT], dC0[DB_MAXT], dS0[DB_MAXT];
};

// fill C from P with the first DB_MAXT threads; the caller synchronises
template <typename R>
__device__ __forceinline__ void load_coef(const Params& P, Coef<R>& C) {
    const int t = threadIdx.x;
    if (t < DB_MAXT) {
        C.bK[t] = (R)P.bK[t];
        C.bR0[t] = (R)P.bR0[t];
        C.bRc2[t] = P.bRc2[t];
        C.aK[t] = (R)P.aK[t];
        C.aT0[t] = (R)P.aT0[t];
        C.aPm[t] = (R)P.aPiMinusT0[t];
        C.dK[t] = (R)P.dK[t];
        C.dC0[t] = (R)P.dC0[t];
        C.dS0[t] = (R)P.dS0[t];
    }
}

// Minimum image for separations that are short next to half a box (interacting
// pairs, members of a bond, angle or dihedral): the nearest multiple of L, which
// is -L, 0 or L, is removed by one fused multiply-add.  L times that multiple is
// exact, so the result equals d - L, d or d + L rounded once, as in the
// comparison form; the two forms can pick different images only for d within a
// rounding error of L/2, where both images are equally near.
__device__ __forceinline__ double near_image(double d, const Box& X) {
    return fma(-rint(d * X.invL), X.L, d);
}

template <typename R>
__device__ __forceinline__ R r_sqrt(R v);
template <>
__device__ __forceinline__ double r_sqrt<double>(double v) { return sqrt(v); }
template <>
__device__ __forceinline__ float r_sqrt<float>(float v) { return sqrtf(v); }
// reciprocal and reciprocal square root: IEEE in double; in float the native
// single-instruction approximations (about 1 ulp), far inside the float path's
// error budget
template <typename R>
__device__ __forceinline__ R r_rcp(R v);
template <>
__device__ __forceinline__ double r_rcp<double>(double v) { return 1.0 / v; }
template <>
__device__ __forceinline__ float r_rcp<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <typename R>
__device__ __forceinline__ R r_rsqrt(R v);
template <>
__device__ __forceinline__ double r_rsqrt<double>(double v) { return 1.0 / sqrt(v); }
template <>
__device__ __forceinline__ float r_rsqrt<float>(float v) { return __builtin_amdgcn_rsqf(v); }
template <typename R>
__device__ __forceinline__ R r_atan2(R y, R x);
template <>
__device__ __forceinline__ double r_atan2<double>(double y, double x) { return atan2(y, x); }
// Single-precision arctangent for y >= 0 (every call here passes a sine): the
// octant reduction z = min(|x|, y) / max(|x|, y) <= 1 and the odd polynomial of
// Abramowitz and Stegun 4.4.49 (|error| <= 2e-8 on [0, 1]; about 1e-7 in float
// arithmetic), then pi/2 - a above the diagonal and pi - a for x < 0.
template <>
__device__ __forceinline__ float r_atan2<float>(float y, float x) {
    const float ax = fabsf(x);
    const float mx = fmaxf(ax, y), mn = fminf(ax, y);
    const float z = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float t = z * z;
    float p = 0.0028662257f;
    p = p * t - 0.0161657367f;
    p = p * t + 0.0429096138f;
    p = p * t - 0.0752896400f;
    p = p * t + 0.1065626393f;
    p = p * t - 0.1420889944f;
    p = p * t + 0.1999355085f;
    p = p * t - 0.3333314528f;
    p = p * t + 1.0f;
    float a = z * p;
    a = y > ax ? 1.5707963267948966f - a : a;
    return x < 0.0f ? 3.1415926535897932f - a : a;
}

// bead i is bonded to j (one of its own table entries)
__device__ __forceinline__ bool in_list4(int j, int nb, int p0, int p1, int p2, int p3) {
    return (nb > 0 && j == p0) || (nb > 1 && j == p1) || (nb > 2 && j == p2) || (nb > 3 && j == p3);
}

// j is one bond from any partner of i
__device__ bool two_bonds_apart(const Bank& B, int n, int j, int nb, int p0, int p1, int p2, int p3) {
    int ps[4] = {p0, p1, p2, p3};
    for (int k = 0; k < nb; ++k) {
        int q = ps[k];
        int nq = B.nb[q];
        for (int m = 0; m < nq; ++m)
            if (B.bp[m * n + q] == j) return true;
    }
    return false;
}

template <typename R, int MODE>
__device__ __forceinline__ void pair_term(const Params& P, const Box& X, const double4& xi, const double4& xj, Acc<R>& a) {
    double dx, dy, dz;
    dx = near_image(xj.x - xi.x, X);
    dy = near_image(xj.y - xi.y, X);
    dz = near_image(xj.z - xi.z, X);
    R rx = (R)dx, ry = (R)dy, rz = (R)dz;
    R r2 = (rx * rx + ry * ry) + rz * rz;
    R ir2 = r_rcp<R>(r2);
    R sr2 = (R)P.sig2 * ir2;
    R sr6 = sr2 * sr2 * sr2;
    R fr = (R)24.0 * (R)P.eps * ((R)2.0 * sr6 * sr6 - sr6) * ir2;   // -dU/dr / r
    a.fx -= (double)(fr * rx);
    a.fy -= (double)(fr * ry);
    a.fz -= (double)(fr * rz);
    if (MODE == MODE_ENERGY) {
        a.e_pair += 0.5 * (double)((R)4.0 * (R)P.eps * (sr6 * sr6 - sr6) + (R)P.eps);
        a.vir += 0.5 * (double)(fr * r2);
    }
}

// DPD pair (i, j) as seen by bead i (section 3).  With d = x_j - x_i (minimum
// image), r = |d|, e = -d / r (from j to i) and w = 1 - r / rc, bead i receives
// (F^C + F^D + F^R) e with F^C = a w, F^D = -gamma w^2 (e . v_ij) and
// F^R = sigma w xi / sqrt(dt); dsig = sigma / sqrt(dt).  Bead j forms the same
// three terms from -d and -v_ij and the pair's single Gaussian, so the two forces
// cancel exactly.  Without THERMO only the conservative part is formed.
template <typename R, bool THERMO, bool ENERGY>
__device__ __forceinline__ void dpd_pair(const Params& P, const Box& X, const double4& xi, const double4& xj,
                                         R rx, R ry, R rz, R r2, double dvx, double dvy, double dvz, int64_t step,
                                         double dsig, Acc<R>& a) {
    const R r = r_sqrt<R>(r2);
    const R ir = r_rcp<R>(r);
    const R w = (R)1.0 - r * (R)P.inv_rc;
    R f = (R)P.dpd_a * w;
    if (ENERGY) {
        a.e_pair += 0.25 * (double)((R)P.dpd_a * (R)P.rc * w * w);   // half of a rc w^2 / 2
        a.vir += 0.5 * (double)(f * r);
    }
    if (THERMO) {
        const R ev = -(((R)dvx * rx + (R)dvy * ry) + (R)dvz * rz) * ir;   // e . v_ij
        R xg;
        if constexpr (sizeof(R) == 4) xg = pair_gaussian_f(X, meta_gid(xi), meta_gid(xj), step);
        else xg = pair_gaussian(X, meta_gid(xi), meta_gid(xj), step);
        f += -(R)P.dpd_gamma * w * w * ev + (R)dsig * w * xg;
    }
    const R fi = f * ir;
    a.fx -= (double)(fi * rx);
    a.fy -= (double)(fi * ry);
    a.fz -= (double)(fi * rz);
}

// pair forces over the 27 cells (energy evaluation); vi and dsig feed the DPD
// thermostat terms when the DPD friction is not zero
template <typename R, int MODE>
__device__ void pair_forces(const Params& P, const Box& X, const Bank& B, const int* __restrict__ cstart,
                            const int* __restrict__ clist, int i, const double4& xi, int nb, int p0, int p1, int p2,
                            int p3, double vix, double viy, double viz, int64_t step, double dsig, Acc<R>& a) {
    const int nc = X.nc;
    int cx = cell_coord(xi.x, X.cell_scale, nc);
    int cy = cell_coord(xi.y, X.cell_scale, nc);
    int cz = cell_coord(xi.z, X.cell_scale, nc);
    const R rc2 = (R)P.rc2;
    const bool rowmerge = (X.noff == 3) && cx >= 1 && cx <= nc - 2;
    cstart += X.cell_off;
    for (int oz = 0; oz < X.noff; ++oz) {
        int zz = wrap_cell(cz + box_off(X, oz), nc);
        for (int oy = 0; oy < X.noff; ++oy) {
            int yy = wrap_cell(cy + box_off(X, oy), nc);
            int row = (zz * nc + yy) * nc;
            // the three cells of one x-row are contiguous in the list unless the row wraps
            int nseg = rowmerge ? 1 : X.noff;
            for (int ox = 0; ox < nseg; ++ox) {
                int s0, s1;
                if (rowmerge) {
                    s0 = cstart[row + cx - 1];
                    s1 = cstart[row + cx + 2];
                } else {
                    int c = row + wrap_cell(cx + box_off(X, ox), nc);
                    s0 = cstart[c];
                    s1 = cstart[c + 1];
                }
                for (int p = s0; p < s1; ++p) {
                    int j = clist[p];
                    if (j == i) continue;
                    double4 xj = B.x[j];
                    double dx = near_image(xj.x - xi.x, X);
                    double dy = near_image(xj.y - xi.y, X);
                    double dz = near_image(xj.z - xi.z, X);
                    R rx = (R)dx, ry = (R)dy, rz = (R)dz;
                    R r2 = (rx * rx + ry * ry) + rz * rz;
                    if (!(r2 < rc2)) continue;
                    if (P.excl_depth >= 1 && in_list4(j, nb, p0, p1, p2, p3)) continue;
                    if (P.excl_depth >= 2 && two_bonds_apart(B, P.n, j, nb, p0, p1, p2, p3)) continue;
                    if (P.pair_style == PAIR_DPD) {
                        const int n = P.n;
                        if (P.dpd_gamma != 0.0)
                            dpd_pair<R, true, MODE == MODE_ENERGY>(P, X, xi, xj, rx, ry, rz, r2, vix - B.v[j],
                                                                   viy - B.v[n + j], viz - B.v[2 * n + j], step,
                                                                   dsig, a);
                        else
                            dpd_pair<R, false, MODE == MODE_ENERGY>(P, X, xi, xj, rx, ry, rz, r2, 0, 0, 0, 0, 0,
                                                                    a);
                    } else {
                        pair_term<R, MODE>(P, X, xi, xj, a);
                    }
                }
            }
        }
    }
}

// The beads a list of bead i leaves out: its bond partners (exclusion depth 1)
// and their partners (depth 2), -1 for an empty entry, so that testing a
// candidate compares registers instead of re-reading the partners' tables.  The
// bond rows exist for every bead: all are requested at once with the count and
// the unused ones ignored, and likewise for the partners' rows, so that gathering
// the set costs two memory latencies.
struct ExclSet {
    int nb, p0, p1, p2, p3;
    bool d1, d2;
    int two[DB_MAXB * DB_MAXB];
    __device__ __forceinline__ bool has(int j) const {
        if (d1 && in_list4(j, nb, p0, p1, p2, p3)) return true;
        bool ex = false;
        if (d2 && nb > 0) {
#pragma unroll
            for (int k = 0; k < DB_MAXB * DB_MAXB; ++k) ex |= two[k] == j;
        }
        return ex;
    }
};

__device__ __forceinline__ void gather_excl(const Params& P, const Bank& B, int n, int i, ExclSet& E) {
    static_assert(DB_MAXB == 4, "the exclusion test holds four partners");
    E.d1 = P.excl_depth >= 1;
    E.d2 = P.excl_depth >= 2;
    E.nb = B.nb[i];
    int pr[DB_MAXB];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) pr[k] = B.bp[k * n + i];
    E.p0 = E.nb > 0 ? pr[0] : -1;
    E.p1 = E.nb > 1 ? pr[1] : -1;
    E.p2 = E.nb > 2 ? pr[2] : -1;
    E.p3 = E.nb > 3 ? pr[3] : -1;
    const int pp[DB_MAXB] = {E.p0, E.p1, E.p2, E.p3};
#pragma unroll
    for (int k = 0; k < DB_MAXB * DB_MAXB; ++k) E.two[k] = -1;
    if (E.d2) {
        int nq[DB_MAXB];
#pragma unroll
        for (int k = 0; k < DB_MAXB; ++k) {
            const int q = k < E.nb ? pp[k] : i;
            nq[k] = k < E.nb ? B.nb[q] : 0;
#pragma unroll
            for (int m = 0; m < DB_MAXB; ++m) E.two[k * DB_MAXB + m] = B.bp[m * n + q];
        }
#pragma unroll
        for (int k = 0; k < DB_MAXB; ++k)
#pragma unroll
            for (int m = 0; m < DB_MAXB; ++m)
                if (m >= nq[k]) E.two[k * DB_MAXB + m] = -1;
    }
}

// Verlet list of bead i: every bead within the list cutoff (pair cutoff plus a
// skin) that is not excluded, from the 27 cells of the current cell list.  The
// float prefilter's cutoff is widened by the box's bound on float rounding
// (Box::pf_slack), so the list is a superset of the pairs within the cutoff in
// double.  The full build of every bead; with DPD the bead's position is kept in
// xref, from which the step kernels measure displacements.
template <bool BATCH>
__global__ __launch_bounds__(DB_BLOCK) void k_build_nlist(const Params* __restrict__ Pp, Bank B,
                                                          const int* __restrict__ cstart,
                                                          const float4* __restrict__ xs, NList NL,
                                                          int* __restrict__ err, double4* __restrict__ xref) {
    const Params& P = *Pp;
    const int n = P.n;
    // list rows staged in LDS, plus one row that takes the writes of the
    // candidates that are not kept
    constexpr int NL_STAGE = 24;
    __shared__ int stage[NL_STAGE + 1][DB_BLOCK];
    const int i = xcd_tile(blockIdx.x, gridDim.x) * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    const double4 xi = B.x[i];
    if (xref) xref[i] = xi;
    ExclSet E;
    gather_excl(P, B, n, i, E);
    // The first NL_STAGE entries go to the thread's own LDS column and are written
    // out afterwards one row at a time, so that a store covers consecutive beads of
    // one row; entries beyond go straight to memory.  (Written as they are found,
    // the lanes of a wave store into rows that differ by their counts, and each
    // store scatters over as many rows.)
    const int tid = threadIdx.x;
    auto put = [&](int k, int j) {
        if (k < NL_STAGE) stage[k][tid] = j;
        else if (k < DB_NLCAP) NL.nl[k * n + i] = j;
    };
    int cnt = 0;
    const Box& X = box_of<BATCH>(P, meta_word(xi));
    // Every candidate within the cutoff is kept first, in the LDS rows, and the
    // exclusions are applied afterwards, compacting in place in scan order.  The
    // scan writes every candidate into the row of the next kept entry (a candidate
    // not kept is overwritten by the next one kept; past the LDS rows the extra row
    // takes them all) and advances the count by the test, with no branch per
    // candidate; tested inside the scan, the exclusion test and the store ran for
    // every candidate some lane of the wave kept, which is nearly every candidate.
    // A bead with more kept candidates than the LDS rows hold, or a grid of fewer
    // than three cells per edge, is scanned with the test inside.
    int raw = 0;
    if (X.noff == 3) {
        scan_cells_all(X, cstart, xs, i, xi, X.pf_list2, [&](int w, bool hit) {
            stage[min(raw, NL_STAGE)][tid] = w;   // the word; its slot is taken below
            raw += hit ? 1 : 0;
        });
    } else {
        raw = NL_STAGE + 1;
    }
    if (raw <= NL_STAGE) {
        for (int k = 0; k < raw; ++k) {
            const int j = xs_slot(stage[k][tid]);
            if (E.has(j)) continue;
            stage[cnt][tid] = j;
            ++cnt;
        }
    } else {
        scan_cells(X, cstart, xs, i, xi, X.pf_list2, [&](int j, int) {
            if (E.has(j)) return;
            put(cnt, j);
            ++cnt;
        });
    }
    const int ns = min(cnt, NL_STAGE);
    for (int k = 0; k < ns; ++k) NL.nl[k * n + i] = stage[k][tid];
    if (cnt > DB_NLCAP) {
        atomicOr(err, ERR_NLIST);
        cnt = DB_NLCAP;
    }
    NL.cnt[i] = (uint8_t)cnt;
}

// The list of one bead whose exclusions a sweep changed, redone with cutoff cut
// (beyond the list cutoff by the displacement margin; the 5 x 5 x 5 stencil
// reaches it) by LANES threads that share its rows (row r to thread r mod LANES).
// A first pass counts each thread's kept candidates, a shuffle within the group
// gives each thread its offset, and a second pass writes the entries: thread by
// thread in lane order, each in its rows' scan order.
template <bool BATCH, int LANES>
__device__ __forceinline__ void patch_one(const Params& P, const Bank& B, const int* __restrict__ cstart,
                                          const float4* __restrict__ xs, const NList& NL, int* __restrict__ err,
                                          int i, int lane, double cut) {
    const int n = P.n;
    const double4 xi = B.x[i];
    ExclSet E;
    gather_excl(P, B, n, i, E);
    const Box& X = box_of<BATCH>(P, meta_word(xi));
    const float cut2 = (float)((cut + X.pf_slack) * (cut + X.pf_slack) * 1.0001);
    int c = 0;
    scan_cells_wide<LANES>(X, cstart, xs, i, xi, cut2, [&](int j, int) { c += E.has(j) ? 0 : 1; }, lane);
    int incl = c;
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
        const int t = __shfl_up(incl, o, LANES);
        if (lane >= o) incl += t;
    }
    int tot = __shfl(incl, LANES - 1, LANES);
    int k = incl - c;
    scan_cells_wide<LANES>(X, cstart, xs, i, xi, cut2, [&](int j, int) {
        if (E.has(j)) return;
        if (k < DB_NLCAP) NL.nl[k * n + i] = j;
        ++k;
    }, lane);
    if (lane == 0) {
        if (tot > DB_NLCAP) {
            atomicOr(err, ERR_NLIST);
            tot = DB_NLCAP;
        }
        NL.cnt[i] = (uint8_t)tot;
    }
}

template <bool BATCH, int LANES>
__device__ __forceinline__ void patch_all(const Params& P, const Bank& B, const int* __restrict__ cstart,
                                          const float4* __restrict__ xs, const NList& NL, int* __restrict__ err,
                                          const int* __restrict__ list, int nl, double cut) {
    static_assert(64 % LANES == 0 && DB_BLOCK % 64 == 0, "groups lie within a wavefront");
    const int ntile = (int)(((long long)nl * LANES + DB_BLOCK - 1) / DB_BLOCK);
    for (int tb = blockIdx.x; tb < ntile; tb += gridDim.x) {
        const long long pos = (long long)xcd_tile(tb, ntile) * DB_BLOCK + threadIdx.x;
        const int t = (int)(pos / LANES);
        const int lane = (int)(pos % LANES);
        // the lanes of a group share t: they take this branch together
        if (t < nl) patch_one<BATCH, LANES>(P, B, cstart, xs, NL, err, list[t], lane, cut);
    }
}

// The beads listed in list (count at list_n).  After a sweep few beads are
// listed; with one thread each the pass would last as long as the slowest bead's
// chain of memory latencies, so a short list takes eight threads per bead, and a
// list of 2^16 beads or more, which fills the GPU, one.  Both passes of a thread
// run the same scan on the same data, so they keep the same candidates.
template <bool BATCH>
__global__ __launch_bounds__(DB_BLOCK) void k_patch_nlist(const Params* __restrict__ Pp, Bank B,
                                                          const int* __restrict__ cstart,
                                                          const float4* __restrict__ xs, NList NL,
                                                          int* __restrict__ err, const int* __restrict__ list,
                                                          const int* __restrict__ list_n, double cut) {
    const Params& P = *Pp;
    const int nl = *list_n;
    if (nl >= (1 << 16)) patch_all<BATCH, 1>(P, B, cstart, xs, NL, err, list, nl, cut);
    else patch_all<BATCH, 8>(P, B, cstart, xs, NL, err, list, nl, cut);
}

// pair forces from the Verlet list (exclusions were applied when it was built).
// Entries are taken four at a time: the four indices, then the four positions are
// requested before any of them is used, so one bead keeps several loads in flight.
template <typename R>
__device__ __forceinline__ void pair_one(const Params& P, const Box& X, const double4& xi, const double4& xj, R rc2, Acc<R>& a) {
    R rx = (R)near_image(xj.x - xi.x, X);
    R ry = (R)near_image(xj.y - xi.y, X);
    R rz = (R)near_image(xj.z - xi.z, X);
    R r2 = (rx * rx + ry * ry) + rz * rz;
    if (r2 < rc2) {
        R ir2 = r_rcp<R>(r2);
        R sr2 = (R)P.sig2 * ir2;
        R sr6 = sr2 * sr2 * sr2;
        R fr = (R)24.0 * (R)P.eps * ((R)2.0 * sr6 * sr6 - sr6) * ir2;
        a.fx -= (double)(fr * rx);
        a.fy -= (double)(fr * ry);
        a.fz -= (double)(fr * rz);
    }
}

// entries of the Verlet list requested together: eight in the FP64 WCA kernel
// (its occupancy is set by its LDS, so registers are free), four in the FP32
// kernel and with DPD (which also requests the partners' velocities)
template <typename R, int PAIR>
constexpr int pair_batch() { return (sizeof(R) == 8 && PAIR != PAIR_DPD) ? 8 : 4; }

// m and jpre (the first batch of entries, read whether occupied or not) are
// loaded by the caller ahead of the bonded terms, so that their latency overlaps
// them; each later batch of entries is requested before the previous batch's
// pairs are evaluated.
template <typename R>
__device__ __forceinline__ void list_pair_forces(const Params& P, const Box& X, const Bank& B, const NList& NL, int i,
                                                 const double4& xi, int m, const int (&jpre)[pair_batch<R, PAIR_WCA>()],
                                                 Acc<R>& a) {
    constexpr int Q = pair_batch<R, PAIR_WCA>();
    const int n = P.n;
    const R rc2 = (R)P.rc2;
    int j[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) j[q] = q < m ? jpre[q] : i;
    for (int k0 = 0; k0 < m; k0 += Q) {
        double4 xj[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) xj[q] = B.x[j[q]];
        // the next batch's entries are requested before this batch is evaluated
        const int k1 = k0 + Q;
#pragma unroll
        for (int q = 0; q < Q; ++q) j[q] = k1 + q < m ? NL.nl[(k1 + q) * n + i] : i;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (k0 + q < m) pair_one<R>(P, X, xi, xj[q], rc2, a);
    }
}

// DPD pair forces from the Verlet list; THERMO adds the dissipative and random
// parts, which read the neighbours' velocities (from the step's input buffer).
// The FP64 kernel requests the velocities of a batch with its positions, whether
// or not the pair turns out to lie within the cutoff; the FP32 kernel reads them
// per interacting pair, which keeps its registers within five waves per SIMD.
// m and jpre as for the WCA list.
template <typename R, bool THERMO>
__device__ __forceinline__ void list_pair_dpd(const Params& P, const Box& X, const Bank& B, const NList& NL, int i,
                                              const double4& xi, double vix, double viy, double viz, int64_t step,
                                              double dsig, int m, const int (&jpre)[pair_batch<R, PAIR_DPD>()],
                                              Acc<R>& a) {
    constexpr int Q = pair_batch<R, PAIR_DPD>();
    const int n = P.n;
    const R rc2 = (R)P.rc2;
    for (int k0 = 0; k0 < m; k0 += Q) {
        int j[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q)
            j[q] = (k0 + q < m) ? (k0 == 0 ? jpre[q] : NL.nl[(k0 + q) * n + i]) : i;
        double4 xj[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) xj[q] = B.x[j[q]];
        constexpr bool vbatch = THERMO && sizeof(R) == 8;
        double vjx[Q], vjy[Q], vjz[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            vjx[q] = vbatch ? B.v[j[q]] : 0.0;
            vjy[q] = vbatch ? B.v[n + j[q]] : 0.0;
            vjz[q] = vbatch ? B.v[2 * n + j[q]] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const R rx = (R)near_image(xj[q].x - xi.x, X);
            const R ry = (R)near_image(xj[q].y - xi.y, X);
            const R rz = (R)near_image(xj[q].z - xi.z, X);
            const R r2 = (rx * rx + ry * ry) + rz * rz;
            if ((k0 + q < m) & (r2 < rc2)) {
                if (THERMO) {
                    if (!vbatch) {
                        const int jq = j[q];
                        vjx[q] = B.v[jq];
                        vjy[q] = B.v[n + jq];
                        vjz[q] = B.v[2 * n + jq];
                    }
                    dpd_pair<R, true, false>(P, X, xi, xj[q], rx, ry, rz, r2, vix - vjx[q], viy - vjy[q],
                                             viz - vjz[q], step, dsig, a);
                } else {
                    dpd_pair<R, false, false>(P, X, xi, xj[q], rx, ry, rz, r2, 0, 0, 0, 0, 0, a);
                }
            }
        }
    }
}

// harmonic bond U = K (r - r0)^2 with the type bead i stores (all partners requested at once)
template <typename R, int MODE>
__device__ __forceinline__ void bond_terms(const Params& P, const Box& X, const Coef<R>& C, const Bank& B, int i, const double4& xi, int nb,
                                           Acc<R>& a) {
    const int n = P.n;
    int jj[DB_MAXB], tt[DB_MAXB];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) {
        jj[k] = k < nb ? B.bp[k * n + i] : i;
        tt[k] = k < nb ? (int)B.bt[k * n + i] & (DB_MAXT - 1) : 0;
    }
    double4 xs[DB_MAXB];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) xs[k] = B.x[jj[k]];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) {
        if (k >= nb) continue;
        const double4& xj = xs[k];
        const int t = tt[k];
        double dx = near_image(xj.x - xi.x, X);
        double dy = near_image(xj.y - xi.y, X);
        double dz = near_image(xj.z - xi.z, X);
        // the cutoff decision in double, whatever the force type
        const double rd2 = (dx * dx + dy * dy) + dz * dz;
        if (!(rd2 > 0.0) || !(rd2 < C.bRc2[t])) continue;
        R rx = (R)dx, ry = (R)dy, rz = (R)dz;
        R rr2 = (rx * rx + ry * ry) + rz * rz;
        R ir = r_rsqrt<R>(rr2);
        R r = rr2 * ir;
        R K = C.bK[t], r0 = C.bR0[t];
        R g = (R)2.0 * K * (r - r0) * ir;   // F_i = g * (x_j - x_i)
        a.fx += (double)(g * rx);
        a.fy += (double)(g * ry);
        a.fz += (double)(g * rz);
        if (MODE == MODE_ENERGY) {
            a.e_bond += 0.5 * ((double)(K * (r - r0) * (r - r0)) + P.bE0[t]);
            a.vir -= 0.5 * (double)(g * r * r);
        }
    }
}

// harmonic angle U = K (theta - theta0)^2 on u = x_a - x_b, w = x_c - x_b; the
// bead takes the force of its role (0: end a, 1: centre b, 2: end c)
template <typename R, int MODE>
__device__ __forceinline__ void angle_core(const Coef<R>& C, int role, int t, R ux, R uy, R uz, R wx, R wy, R wz,
                                           Acc<R>& a) {
    R ru2 = (ux * ux + uy * uy) + uz * uz;
    R rw2 = (wx * wx + wy * wy) + wz * wz;
    if (!(ru2 > (R)0) || !(rw2 > (R)0)) return;
    R iru = r_rsqrt<R>(ru2), irw = r_rsqrt<R>(rw2);
    R cux = ux * iru, cuy = uy * iru, cuz = uz * iru;
    R cwx = wx * irw, cwy = wy * irw, cwz = wz * irw;
    R cs = (cux * cwx + cuy * cwy) + cuz * cwz;
    R crx = cuy * cwz - cuz * cwy, cry = cuz * cwx - cux * cwz, crz = cux * cwy - cuy * cwx;
    R sn = r_sqrt<R>((crx * crx + cry * cry) + crz * crz);
    R K = C.aK[t];
    // dU/dtheta / sin(theta), finite at theta = pi when theta0 = pi
    R del = r_atan2<R>(sn, -cs);   // pi - theta
    R isn = r_rcp<R>(sn > (R)1e-8 ? sn : (R)1e-8);
    R ratio = del < (R)1e-6 ? (R)1.0 + del * del * (R)(1.0 / 6.0) : del * isn;
    R pth = C.aPm[t];
    R A = (R)2.0 * K * (-ratio + (pth != (R)0 ? pth * isn : (R)0));
    R Au = -A * iru, Aw = -A * irw;
    R fax = Au * (cs * cux - cwx), fay = Au * (cs * cuy - cwy), faz = Au * (cs * cuz - cwz);
    R fcx = Aw * (cs * cwx - cux), fcy = Aw * (cs * cwy - cuy), fcz = Aw * (cs * cwz - cuz);
    if (role == 0) {
        a.fx += (double)fax; a.fy += (double)fay; a.fz += (double)faz;
    } else if (role == 2) {
        a.fx += (double)fcx; a.fy += (double)fcy; a.fz += (double)fcz;
    } else {
        a.fx -= (double)(fax + fcx); a.fy -= (double)(fay + fcy); a.fz -= (double)(faz + fcz);
    }
    if (MODE == MODE_ENERGY) {
        R th = r_atan2<R>(sn, cs);
        R th0 = C.aT0[t];
        a.e_ang += (double)(K * (th - th0) * (th - th0)) / 3.0;
        a.vir += (double)((ux * fax + uy * fay + uz * faz) + (wx * fcx + wy * fcy + wz * fcz)) / 3.0;
    }
}

// angle entry e = (a, b, c, type) of bead i from the members' positions
template <typename R, int MODE>
__device__ __forceinline__ void angle_one(const Params& P, const Box& X, const Coef<R>& C, int i, const int4& e,
                                          const double4& xa, const double4& xb, const double4& xc, Acc<R>& a) {
    R ux = (R)near_image(xa.x - xb.x, X), uy = (R)near_image(xa.y - xb.y, X), uz = (R)near_image(xa.z - xb.z, X);
    R wx = (R)near_image(xc.x - xb.x, X), wy = (R)near_image(xc.y - xb.y, X), wz = (R)near_image(xc.z - xb.z, X);
    const int role = e.x == i ? 0 : (e.z == i ? 2 : 1);
    angle_core<R, MODE>(C, role, e.w & (DB_MAXT - 1), ux, uy, uz, wx, wy, wz, a);
}

template <typename R, int MODE>
__device__ __forceinline__ void angle_terms(const Params& P, const Box& X, const Coef<R>& C, const Bank& B, int i, int na,
                                            Acc<R>& a) {
    const int n = P.n;
    for (int k = 0; k < na; ++k) {
        int4 e = B.ang[k * n + i];
        angle_one<R, MODE>(P, X, C, i, e, B.x[e.x], B.x[e.y], B.x[e.z], a);
    }
}

// cosine dihedral U = K [1 - cos(phi - phi0)], phi = atan2(|b2| b1.(b2 x b3), (b1 x b2).(b2 x b3))
// on the bond vectors b1 = x_b - x_a, b2 = x_c - x_b, b3 = x_d - x_c; role 0..3 = a..d
template <typename R, int MODE>
__device__ __forceinline__ void dihedral_core(const Coef<R>& C, int role, int t, R b1x, R b1y, R b1z, R b2x, R b2y,
                                              R b2z, R b3x, R b3y, R b3z, Acc<R>& a) {
    R mx = b1y * b2z - b1z * b2y, my = b1z * b2x - b1x * b2z, mz = b1x * b2y - b1y * b2x;
    R nx = b2y * b3z - b2z * b3y, ny = b2z * b3x - b2x * b3z, nz = b2x * b3y - b2y * b3x;
    R m2 = (mx * mx + my * my) + mz * mz;
    R n2 = (nx * nx + ny * ny) + nz * nz;
    R b22 = (b2x * b2x + b2y * b2y) + b2z * b2z;
    if (m2 < (R)1e-24 || n2 < (R)1e-24 || b22 < (R)1e-24) return;   // collinear: no defined plane
    R nb2 = r_sqrt<R>(b22);
    R inv = r_rsqrt<R>(m2 * n2);
    R cphi = ((mx * nx + my * ny) + mz * nz) * inv;
    R sphi = nb2 * ((b1x * nx + b1y * ny) + b1z * nz) * inv;
    R K = C.dK[t], c0 = C.dC0[t], s0 = C.dS0[t];
    R dU = K * (sphi * c0 - cphi * s0);   // dU/dphi
    R sa = -nb2 * r_rcp<R>(m2), sd = nb2 * r_rcp<R>(n2), ib22 = r_rcp<R>(b22);
    R gax = sa * mx, gay = sa * my, gaz = sa * mz;
    R gdx = sd * nx, gdy = sd * ny, gdz = sd * nz;
    R pp = ((b1x * b2x + b1y * b2y) + b1z * b2z) * ib22;
    R qq = ((b3x * b2x + b3y * b2y) + b3z * b2z) * ib22;
    R fx, fy, fz;
    if (role == 0) {
        fx = -dU * gax; fy = -dU * gay; fz = -dU * gaz;
    } else if (role == 3) {
        fx = -dU * gdx; fy = -dU * gdy; fz = -dU * gdz;
    } else if (role == 1) {
        fx = -dU * (qq * gdx - (pp + (R)1) * gax);
        fy = -dU * (qq * gdy - (pp + (R)1) * gay);
        fz = -dU * (qq * gdz - (pp + (R)1) * gaz);
    } else {
        fx = -dU * (pp * gax - (qq + (R)1) * gdx);
        fy = -dU * (pp * gay - (qq + (R)1) * gdy);
        fz = -dU * (pp * gaz - (qq + (R)1) * gdz);
    }
    a.fx += (double)fx; a.fy += (double)fy; a.fz += (double)fz;
    if (MODE == MODE_ENERGY) {
        a.e_dih += (double)(K * ((R)1 - (cphi * c0 + sphi * s0))) / 4.0;
        // virial about bead b: (x_a - x_b).F_a + (x_c - x_b).F_c + (x_d - x_b).F_d
        R fa_x = -dU * gax, fa_y = -dU * gay, fa_z = -dU * gaz;
        R fd_x = -dU * gdx, fd_y = -dU * gdy, fd_z = -dU * gdz;
        R fc_x = -dU * (pp * gax - (qq + (R)1) * gdx), fc_y = -dU * (pp * gay - (qq + (R)1) * gdy),
          fc_z = -dU * (pp * gaz - (qq + (R)1) * gdz);
        R w = -(b1x * fa_x + b1y * fa_y + b1z * fa_z) + (b2x * fc_x + b2y * fc_y + b2z * fc_z) +
              ((b2x + b3x) * fd_x + (b2y + b3y) * fd_y + (b2z + b3z) * fd_z);
        a.vir += (double)w / 4.0;
    }
}

// The forces on all three members of an angle (a, b, c), u = x_a - x_b, w = x_c - x_b:
// the arithmetic of angle_core, every role at once (f[role][component])
template <typename R>
__device__ __forceinline__ void angle_all(const Coef<R>& C, int t, R ux, R uy, R uz, R wx, R wy, R wz,
                                          R (&f)[3][3]) {
#pragma unroll
    for (int r = 0; r < 3; ++r) f[r][0] = f[r][1] = f[r][2] = (R)0;
    R ru2 = (ux * ux + uy * uy) + uz * uz;
    R rw2 = (wx * wx + wy * wy) + wz * wz;
    if (!(ru2 > (R)0) || !(rw2 > (R)0)) return;
    R iru = r_rsqrt<R>(ru2), irw = r_rsqrt<R>(rw2);
    R cux = ux * iru, cuy = uy * iru, cuz = uz * iru;
    R cwx = wx * irw, cwy = wy * irw, cwz = wz * irw;
    R cs = (cux * cwx + cuy * cwy) + cuz * cwz;
    R crx = cuy * cwz - cuz * cwy, cry = cuz * cwx - cux * cwz, crz = cux * cwy - cuy * cwx;
    R sn = r_sqrt<R>((crx * crx + cry * cry) + crz * crz);
    R K = C.aK[t];
    R del = r_atan2<R>(sn, -cs);   // pi - theta
    R isn = r_rcp<R>(sn > (R)1e-8 ? sn : (R)1e-8);
    R ratio = del < (R)1e-6 ? (R)1.0 + del * del * (R)(1.0 / 6.0) : del * isn;
    R pth = C.aPm[t];
    R A = (R)2.0 * K * (-ratio + (pth != (R)0 ? pth * isn : (R)0));
    R Au = -A * iru, Aw = -A * irw;
    f[0][0] = Au * (cs * cux - cwx);
    f[0][1] = Au * (cs * cuy - cwy);
    f[0][2] = Au * (cs * cuz - cwz);
    f[2][0] = Aw * (cs * cwx - cux);
    f[2][1] = Aw * (cs * cwy - cuy);
    f[2][2] = Aw * (cs * cwz - cuz);
    f[1][0] = -(f[0][0] + f[2][0]);
    f[1][1] = -(f[0][1] + f[2][1]);
    f[1][2] = -(f[0][2] + f[2][2]);
}

// The forces on the end members (a, d) of a dihedral (a, b, c, d) from its bond
// vectors, and the projections pp = b1.b2 / |b2|^2, qq = b3.b2 / |b2|^2 that give
// those on the inner ones: f_b = qq f_d - (pp + 1) f_a, f_c = pp f_a - (qq + 1) f_d.
// The arithmetic of dihedral_core.
template <typename R>
__device__ __forceinline__ void dihedral_ends(const Coef<R>& C, int t, R b1x, R b1y, R b1z, R b2x, R b2y, R b2z,
                                              R b3x, R b3y, R b3z, R (&fa)[3], R (&fd)[3], R& pp, R& qq) {
    fa[0] = fa[1] = fa[2] = (R)0;
    fd[0] = fd[1] = fd[2] = (R)0;
    pp = qq = (R)0;
    R mx = b1y * b2z - b1z * b2y, my = b1z * b2x - b1x * b2z, mz = b1x * b2y - b1y * b2x;
    R nx = b2y * b3z - b2z * b3y, ny = b2z * b3x - b2x * b3z, nz = b2x * b3y - b2y * b3x;
    R m2 = (mx * mx + my * my) + mz * mz;
    R n2 = (nx * nx + ny * ny) + nz * nz;
    R b22 = (b2x * b2x + b2y * b2y) + b2z * b2z;
    if (m2 < (R)1e-24 || n2 < (R)1e-24 || b22 < (R)1e-24) return;   // collinear: no defined plane
    R nb2 = r_sqrt<R>(b22);
    R inv = r_rsqrt<R>(m2 * n2);
    R cphi = ((mx * nx + my * ny) + mz * nz) * inv;
    R sphi = nb2 * ((b1x * nx + b1y * ny) + b1z * nz) * inv;
    R K = C.dK[t], c0 = C.dC0[t], s0 = C.dS0[t];
    R dU = K * (sphi * c0 - cphi * s0);   // dU/dphi
    R sa = -nb2 * r_rcp<R>(m2), sd = nb2 * r_rcp<R>(n2), ib22 = r_rcp<R>(b22);
    pp = ((b1x * b2x + b1y * b2y) + b1z * b2z) * ib22;
    qq = ((b3x * b2x + b3y * b2y) + b3z * b2z) * ib22;
    fa[0] = -dU * (sa * mx);
    fa[1] = -dU * (sa * my);
    fa[2] = -dU * (sa * mz);
    fd[0] = -dU * (sd * nx);
    fd[1] = -dU * (sd * ny);
    fd[2] = -dU * (sd * nz);
}

template <typename R, int MODE>
__device__ __forceinline__ void dihedral_one(const Params& P, const Box& X, const Coef<R>& C, int i, const int4& e, int t,
                                             const double4& xa, const double4& xb, const double4& xc,
                                             const double4& xd, Acc<R>& a) {
    R b1x = (R)near_image(xb.x - xa.x, X), b1y = (R)near_image(xb.y - xa.y, X), b1z = (R)near_image(xb.z - xa.z, X);
    R b2x = (R)near_image(xc.x - xb.x, X), b2y = (R)near_image(xc.y - xb.y, X), b2z = (R)near_image(xc.z - xb.z, X);
    R b3x = (R)near_image(xd.x - xc.x, X), b3y = (R)near_image(xd.y - xc.y, X), b3z = (R)near_image(xd.z - xc.z, X);
    const int role = e.x == i ? 0 : (e.w == i ? 3 : (e.y == i ? 1 : 2));
    dihedral_core<R, MODE>(C, role, t, b1x, b1y, b1z, b2x, b2y, b2z, b3x, b3y, b3z, a);
}

template <typename R, int MODE>
__device__ __forceinline__ void dihedral_terms(const Params& P, const Box& X, const Coef<R>& C, const Bank& B, int i, int nd,
                                               Acc<R>& a) {
    const int n = P.n;
    for (int k = 0; k < nd; ++k) {
        int4 e = B.dih[k * n + i];
        int t = B.dt[k * n + i] & (DB_MAXT - 1);
        dihedral_one<R, MODE>(P, X, C, i, e, t, B.x[e.x], B.x[e.y], B.x[e.z], B.x[e.w], a);
    }
}

// ---- bonded terms through the bead's halo ----------------------------------
// The halo of bead i lists, once per topology and slot order, the distinct beads
// its bonded terms reach (its bond partners first, in table order, then the
// other members of its angles and dihedrals), and re-expresses every angle and
// dihedral entry as the bead's role plus halo indices of the other members.
// The step kernel then reads each of those positions once, as a separation from
// bead i, instead of once per entry that names it.
//   acode: role (2 bits) | other member 1 << 2 | other member 2 << 5 | type << 8
//   dcode: role (2 bits) | others 1..3 << 2, 5, 8 (3 bits each) | type << 11
// only == nullptr: every bead; else only the beads flagged there (those whose own
// tables the last sweep changed: a bead's halo depends on its own tables alone)
__global__ __launch_bounds__(DB_BLOCK) void k_halo(const Params* __restrict__ Pp, Bank B, Halo H,
                                                   const uint8_t* __restrict__ only) {
    const Params& P = *Pp;
    const int n = P.n;
    const int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i >= n || (only && !only[i])) return;
    int u[DB_MAXU];
    const int nb = B.nb[i];
#pragma unroll
    for (int q = 0; q < DB_MAXU; ++q) u[q] = (q < DB_MAXB && q < nb) ? B.bp[q * n + i] : -1;
    int nu = nb;
    bool ovf = false;
    // halo index of slot m, appended when new
    auto code_of = [&](int m) -> int {
        int idx = -1;
#pragma unroll
        for (int q = 0; q < DB_MAXU; ++q)
            if (idx < 0 && q < nu && u[q] == m) idx = q;
        if (idx >= 0) return idx;
        if (nu >= DB_MAXU) {
            ovf = true;
            return 0;
        }
#pragma unroll
        for (int q = 0; q < DB_MAXU; ++q)
            if (q == nu) u[q] = m;
        return nu++;
    };
    // entries are read four at a time (an entry past the count re-reads the
    // batch's first), so that the loads of a batch are in flight together; they
    // are then coded in table order
    const int na = B.na[i];
    for (int k0 = 0; k0 < na; k0 += 4) {
        int4 e4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e4[q] = B.ang[(k0 + q < na ? k0 + q : k0) * n + i];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (k0 + q >= na) continue;
            const int4 e = e4[q];
            const int role = e.x == i ? 0 : (e.z == i ? 2 : 1);
            const int m1 = role == 0 ? e.y : e.x;
            const int m2 = role == 2 ? e.y : e.z;
            const int c1 = code_of(m1);
            const int c2 = code_of(m2);
            H.acode[(k0 + q) * n + i] = (uint32_t)(role | c1 << 2 | c2 << 5 | (e.w & (DB_MAXT - 1)) << 8);
        }
    }
    const int nd = B.nd[i];
    for (int k0 = 0; k0 < nd; k0 += 4) {
        int4 e4[4];
        int t4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + q < nd ? k0 + q : k0;
            e4[q] = B.dih[k * n + i];
            t4[q] = B.dt[k * n + i] & (DB_MAXT - 1);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (k0 + q >= nd) continue;
            const int4 e = e4[q];
            const int t = t4[q];
            const int role = e.x == i ? 0 : (e.w == i ? 3 : (e.y == i ? 1 : 2));
            const int o1 = role == 0 ? e.y : e.x;
            const int o2 = role <= 1 ? e.z : e.y;
            const int o3 = role <= 2 ? e.w : e.z;
            const int c1 = code_of(o1);
            const int c2 = code_of(o2);
            const int c3 = code_of(o3);
            H.dcode[(k0 + q) * n + i] = (uint32_t)(role | c1 << 2 | c2 << 5 | c3 << 8 | t << 11);
        }
    }
#pragma unroll
    for (int q = 0; q < DB_MAXU; ++q)
        if (q < nu) H.u[q * n + i] = u[q];
    H.nu[i] = ovf ? (uint8_t)DB_HALO_OVF : (uint8_t)nu;
}

// all bonded forces on bead i from its halo (nu <= DB_MAXU entries).  The
// separations are parked in LDS, one column per thread, so that angle and
// dihedral entries can index them at run time without holding 24 registers.
template <typename R>
__device__ __forceinline__ void halo_bonded(const Params& P, const Box& X, const Coef<R>& C, const Bank& B, const Halo& H, int i,
                                            const double4& xi, int nu, Acc<R>& a) {
    const int n = P.n;
    const int tid = threadIdx.x;
    __shared__ R hs[3][DB_MAXU][DB_BLOCK];
    R hx[DB_MAXU], hy[DB_MAXU], hz[DB_MAXU];
    // Every per-bead word used below is requested before the first of them is
    // waited for, so that they share one memory latency instead of one each.
    // Rows exist for every bead: unused rows are read and then ignored.  The FP64
    // kernel, whose occupancy its LDS already limits, also gathers all halo
    // positions at once; the FP32 kernel takes them four at a time.
    constexpr bool wide = sizeof(R) == 8;
    constexpr int G = wide ? DB_MAXU : 4;
    int su[DB_MAXU];
#pragma unroll
    for (int q = 0; q < DB_MAXU; ++q) su[q] = H.u[q * n + i];
    int btk[DB_MAXB];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) btk[k] = B.bt[k * n + i];
    const int nb = B.nb[i];
    const int na = B.na[i];
    const int nd = B.nd[i];
    const uint32_t acode0 = H.acode[i];
    const uint32_t dcode0 = H.dcode[i];
    // separations x_k - x_i, G at a time; for the bond partners (the first nb
    // entries) the cutoff decision is taken here, in double, whatever the force type
    unsigned inb = 0;
#pragma unroll
    for (int k0 = 0; k0 < DB_MAXU; k0 += G) {
        int s[G];
#pragma unroll
        for (int q = 0; q < G; ++q) s[q] = k0 + q < nu ? su[k0 + q] : i;
        double4 xk[G];
#pragma unroll
        for (int q = 0; q < G; ++q) xk[q] = B.x[s[q]];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const double dx = near_image(xk[q].x - xi.x, X);
            const double dy = near_image(xk[q].y - xi.y, X);
            const double dz = near_image(xk[q].z - xi.z, X);
            if (k0 + q < DB_MAXB) {
                const double rd2 = (dx * dx + dy * dy) + dz * dz;
                const int t = btk[k0 + q] & (DB_MAXT - 1);
                inb |= (k0 + q < nb && rd2 > 0.0 && rd2 < C.bRc2[t]) ? 1u << (k0 + q) : 0u;
            }
            hx[k0 + q] = (R)dx;
            hy[k0 + q] = (R)dy;
            hz[k0 + q] = (R)dz;
            hs[0][k0 + q][tid] = hx[k0 + q];
            hs[1][k0 + q][tid] = hy[k0 + q];
            hs[2][k0 + q][tid] = hz[k0 + q];
        }
    }
    // bonds: the first nb halo entries are the partners in table order
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) {
        if (!((inb >> k) & 1u)) continue;
        const int t = btk[k] & (DB_MAXT - 1);
        const R rx = hx[k], ry = hy[k], rz = hz[k];
        R rr2 = (rx * rx + ry * ry) + rz * rz;
        R ir = r_rsqrt<R>(rr2);
        R r = rr2 * ir;
        R g = (R)2.0 * C.bK[t] * (r - C.bR0[t]) * ir;   // F_i = g * (x_j - x_i)
        a.fx += (double)(g * rx);
        a.fy += (double)(g * ry);
        a.fz += (double)(g * rz);
    }
    for (int k = 0; k < na; ++k) {
        const uint32_t code = k == 0 ? acode0 : H.acode[k * n + i];
        const int role = code & 3, k1 = (code >> 2) & 7, k2 = (code >> 5) & 7, t = (code >> 8) & (DB_MAXT - 1);
        const R s1x = hs[0][k1][tid], s1y = hs[1][k1][tid], s1z = hs[2][k1][tid];
        const R s2x = hs[0][k2][tid], s2y = hs[1][k2][tid], s2z = hs[2][k2][tid];
        // member positions relative to bead i (which sits at the origin)
        const R z = (R)0;
        const R pax = role == 0 ? z : s1x, pay = role == 0 ? z : s1y, paz = role == 0 ? z : s1z;
        const R pbx = role == 0 ? s1x : (role == 1 ? z : s2x), pby = role == 0 ? s1y : (role == 1 ? z : s2y),
                pbz = role == 0 ? s1z : (role == 1 ? z : s2z);
        const R pcx = role == 2 ? z : s2x, pcy = role == 2 ? z : s2y, pcz = role == 2 ? z : s2z;
        angle_core<R, MODE_STEP>(C, role, t, pax - pbx, pay - pby, paz - pbz, pcx - pbx, pcy - pby, pcz - pbz, a);
    }
    for (int k = 0; k < nd; ++k) {
        const uint32_t code = k == 0 ? dcode0 : H.dcode[k * n + i];
        const int role = code & 3, k1 = (code >> 2) & 7, k2 = (code >> 5) & 7, k3 = (code >> 8) & 7;
        const int t = (code >> 11) & (DB_MAXT - 1);
        const R s1x = hs[0][k1][tid], s1y = hs[1][k1][tid], s1z = hs[2][k1][tid];
        const R s2x = hs[0][k2][tid], s2y = hs[1][k2][tid], s2z = hs[2][k2][tid];
        const R s3x = hs[0][k3][tid], s3y = hs[1][k3][tid], s3z = hs[2][k3][tid];
        const R z = (R)0;
        const R pax = role == 0 ? z : s1x, pay = role == 0 ? z : s1y, paz = role == 0 ? z : s1z;
        const R pbx = role == 0 ? s1x : (role == 1 ? z : s2x), pby = role == 0 ? s1y : (role == 1 ? z : s2y),
                pbz = role == 0 ? s1z : (role == 1 ? z : s2z);
        const R pcx = role <= 1 ? s2x : (role == 2 ? z : s3x), pcy = role <= 1 ? s2y : (role == 2 ? z : s3y),
                pcz = role <= 1 ? s2z : (role == 2 ? z : s3z);
        const R pdx = role == 3 ? z : s3x, pdy = role == 3 ? z : s3y, pdz = role == 3 ? z : s3z;
        dihedral_core<R, MODE_STEP>(C, role, t, pbx - pax, pby - pay, pbz - paz, pcx - pbx, pcy - pby, pcz - pbz,
                                    pdx - pcx, pdy - pcy, pdz - pcz, a);
    }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Replayed from a HIP graph, a step kernel's arguments are those of its capture:
// the block's first step is then read from the device word step_base (step is the
// offset within the block) and the single system's thermostat amplitudes are
// formed here from the temperature schedule, with the host's arithmetic.
__device__ __forceinline__ void step_amplitudes(const Params& P, const int64_t* step_base, int64_t& step,
                                                double& pref, double& dsig) {
    step += *step_base;
    const double T = box_temperature(P.box, step);
    pref = P.gamma != 0.0 ? sqrt(24.0 * P.gamma * T / P.dt) : 0.0;
    dsig = (P.pair_style == PAIR_DPD && P.dpd_gamma != 0.0) ? sqrt(2.0 * T * P.dpd_gamma) / sqrt(P.dt) : 0.0;
}

// pref: sqrt(24 gamma T / dt) of a single system (from the host), dsig: the DPD
// sigma / sqrt(dt) = sqrt(2 T gamma_DPD) / sqrt(dt); a batch forms both per bead
// from the replica's temperature.  PAIR selects the pair style at compile time.
// The new velocities go to vout, which is B.v itself unless the DPD thermostat
// reads the neighbours' input velocities.  Each step reports the workgroup maxima
// of |v|^2 (WCA) or, with DPD, of the squared displacement of the new position
// from xref, the position at the last full Verlet-list build.
// The FP32 WCA step is held to the registers of six waves per SIMD (its LDS
// allows six), which the compiler otherwise gives up for a few registers (the
// batched form took 94 and ran at five).
template <typename R, int MODE, bool BATCH, int PAIR>
__global__ __launch_bounds__(DB_BLOCK, (sizeof(R) == 4 && PAIR == PAIR_WCA && MODE == MODE_STEP) ? 6 : 1)
void k_step(const Params* __restrict__ Pp, Bank B, NList NL, Halo H, double4* __restrict__ xout, double* vout,
            int64_t step, double pref, double dsig, unsigned int* __restrict__ vmax2_slot, double* __restrict__ fout,
            int* __restrict__ err, double4* __restrict__ xsave, double* __restrict__ vsave,
            const double4* __restrict__ xref, const int64_t* __restrict__ step_base) {
    static_assert(MODE == MODE_STEP || MODE == MODE_FORCES, "energies use k_energy");
    const Params& P = *Pp;
    const int n = P.n;
    if (step_base) step_amplitudes(P, step_base, step, pref, dsig);
    __shared__ Coef<R> C;
    load_coef<R>(P, C);
    __syncthreads();
    int tile = xcd_tile(blockIdx.x, gridDim.x);
    int i = tile * DB_BLOCK + threadIdx.x;
    bool active = i < n;
    Acc<R> a;
    double4 xi = make_double4(0, 0, 0, 0);
    double vx = 0, vy = 0, vz = 0;
    double m2 = 0.0;   // |v|^2, or the squared displacement from the reference
    if (active) {
        xi = B.x[i];
        with_box<BATCH>(P, meta_word(xi), [&](const Box& X) __attribute__((always_inline)) {
            const int nu = H.nu[i];
            // the list's count and first entries are requested ahead of the bonded terms
            constexpr int PQ = pair_batch<R, PAIR>();
            int m_pair = 0;
            int jpre[PQ];
#pragma unroll
            for (int q = 0; q < PQ; ++q) jpre[q] = i;
            if (P.have_pair) {
                m_pair = NL.cnt[i];
#pragma unroll
                for (int q = 0; q < PQ; ++q) jpre[q] = NL.nl[q * n + i];
            }
            if (nu <= DB_MAXU) {
                halo_bonded<R>(P, X, C, B, H, i, xi, nu, a);
            } else {
                // more distinct bonded partners than the halo holds: read them per entry
                bond_terms<R, MODE_STEP>(P, X, C, B, i, xi, B.nb[i], a);
                angle_terms<R, MODE_STEP>(P, X, C, B, i, B.na[i], a);
                dihedral_terms<R, MODE_STEP>(P, X, C, B, i, B.nd[i], a);
            }
            if constexpr (PAIR == PAIR_DPD) {
                if (MODE == MODE_STEP && P.dpd_gamma != 0.0) {
                    if (BATCH) dsig = sqrt(2.0 * box_temperature(X, step) * P.dpd_gamma) / sqrt(P.dt);
                    list_pair_dpd<R, true>(P, X, B, NL, i, xi, B.v[i], B.v[n + i], B.v[2 * n + i], step, dsig, m_pair,
                                           jpre, a);
                } else {
                    list_pair_dpd<R, false>(P, X, B, NL, i, xi, 0, 0, 0, 0, 0, m_pair, jpre, a);
                }
            } else {
                if (P.have_pair) list_pair_forces<R>(P, X, B, NL, i, xi, m_pair, jpre, a);
            }
            if (P.has_ext) {
                const size_t g = (size_t)meta_gid(xi);
                a.fx += P.fext[3 * g];
                a.fy += P.fext[3 * g + 1];
                a.fz += P.fext[3 * g + 2];
            }
            if (MODE == MODE_FORCES) {
                int g = meta_gid(xi);
                fout[3 * (size_t)g] = a.fx;
                fout[3 * (size_t)g + 1] = a.fy;
                fout[3 * (size_t)g + 2] = a.fz;
                return;
            }
            vx = B.v[i];
            vy = B.v[n + i];
            vz = B.v[2 * n + i];
            if (xsave) {   // first step of a block: keep its input state for a re-run
                xsave[i] = xi;
                vsave[i] = vx;
                vsave[n + i] = vy;
                vsave[2 * n + i] = vz;
            }
            double Fx = a.fx, Fy = a.fy, Fz = a.fz;
            if (P.gamma != 0.0) {
                if (BATCH) pref = sqrt(24.0 * P.gamma * box_temperature(X, step) / P.dt);
                uint4 w = rng_draw(X, (uint32_t)(meta_gid(xi) - X.gid_off), 0u, step, RNG_LANGEVIN);
                const double s32 = 1.0 / 4294967296.0;
                double ux = ((double)w.x + 0.5) * s32, uy = ((double)w.y + 0.5) * s32, uz = ((double)w.z + 0.5) * s32;
                Fx = (Fx - P.gamma * vx) + pref * (ux - 0.5);
                Fy = (Fy - P.gamma * vy) + pref * (uy - 0.5);
                Fz = (Fz - P.gamma * vz) + pref * (uz - 0.5);
            }
            const double hdt = 0.5 * P.dt;
            {
                double hx = vx + hdt * Fx, hy = vy + hdt * Fy, hz = vz + hdt * Fz;
                vx = hx + hdt * Fx;
                vy = hy + hdt * Fy;
                vz = hz + hdt * Fz;
                double nxp = xi.x + P.dt * vx, nyp = xi.y + P.dt * vy, nzp = xi.z + P.dt * vz;
                double4 xo;
                xo.x = wrap1(nxp, X.L);
                xo.y = wrap1(nyp, X.L);
                xo.z = wrap1(nzp, X.L);
                xo.w = xi.w;
                bool bad = !(xo.x >= 0.0 && xo.x < X.L && xo.y >= 0.0 && xo.y < X.L && xo.z >= 0.0 && xo.z < X.L);
                if (bad) atomicOr(err, ERR_NONFINITE);
                if (PAIR == PAIR_DPD) {
                    const double4 r = xref[i];
                    const double ex = near_image(xo.x - r.x, X), ey = near_image(xo.y - r.y, X),
                                 ez = near_image(xo.z - r.z, X);
                    m2 = (ex * ex + ey * ey) + ez * ez;
                } else {
                    m2 = (vx * vx + vy * vy) + vz * vz;
                }
                xout[i] = xo;
                vout[i] = vx;
                vout[n + i] = vy;
                vout[2 * n + i] = vz;
            }
        });
    }
    if (MODE == MODE_STEP) {
        // largest speed of the workgroup; one atomic per workgroup, spread over
        // 64 words so that the workgroups of one step do not serialise on one address
        __shared__ float wmax[DB_BLOCK / 64];
        double v2 = wave_max(m2);
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = (float)v2 * 1.0001f;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = wmax[0];
            for (int w = 1; w < DB_BLOCK / 64; ++w) m = fmaxf(m, wmax[w]);
            atomicMax(vmax2_slot + (blockIdx.x & (DB_VMAX_SPREAD - 1)), __float_as_uint(m));
        }
    }
}

// ---- brick tiles: regions staged in LDS -------------------------------------------
// The distinct beads a tile's list and halo entries name are collected in an LDS
// hash table (open addressing on the slot), sorted by slot with a bitonic network,
// written out as the tile's region, and every entry is re-coded as its index in
// the region.  Slots sorted within a region come in runs of neighbouring cells, so
// the step kernel's loads of the region positions are mostly contiguous.
#define DB_RHASH 2048   // hash slots per tile; at most DB_RCAP + DB_BLOCK keys are ever inserted
#define DB_NLHEAD 16    // list entries kept bead-major (one 32-byte row per bead)

// place of list entry k of bead i in the 16-bit table: the first DB_NLHEAD entries
// of a bead are one contiguous row, so one bead reads them with two 16-byte loads;
// later entries follow column-major
__device__ __forceinline__ size_t nl16_index(int n, int i, int k) {
    return k < DB_NLHEAD ? (size_t)i * DB_NLHEAD + k : (size_t)DB_NLHEAD * n + (size_t)(k - DB_NLHEAD) * n + i;
}

__device__ __forceinline__ unsigned region_hash(int key) { return ((unsigned)key * 2654435761u) >> (32 - 11); }

__device__ __forceinline__ void region_insert(int* ht, int* nuniq, int key) {
    unsigned h = region_hash(key);
    for (int probe = 0; probe < DB_RHASH; ++probe) {
        const int old = atomicCAS(&ht[h], -1, key);
        if (old == -1) {
            atomicAdd(nuniq, 1);
            return;
        }
        if (old == key) return;
        h = (h + 1) & (DB_RHASH - 1);
    }
}

// table slot of a key that is present
__device__ __forceinline__ int region_find(const int* ht, int key) {
    unsigned h = region_hash(key);
    for (int probe = 0; probe < DB_RHASH && ht[h] != key; ++probe) h = (h + 1) & (DB_RHASH - 1);
    return (int)h;
}

__global__ __launch_bounds__(DB_BLOCK) void k_region(const Params* __restrict__ Pp, Bank B, NList NL, Halo H,
                                                     Tiles T, int ntile) {
    __shared__ int ht[DB_RHASH];
    __shared__ uint16_t hv[DB_RHASH];
    __shared__ int reg[DB_RCAP];
    __shared__ int nuniq;
    __shared__ int wsum[DB_BLOCK / 64];
    const int n = Pp->n;
    const int tile = blockIdx.x;
    const int tid = threadIdx.x;
    if (tile >= ntile) return;
    const int i = tile * DB_BLOCK + tid;
    const bool active = i < n;
    // every word of the bead is requested before any is used: the list's first
    // DB_NLHEAD entries and the halo (rows exist for every bead; unused ones are
    // ignored), the counts, the types, the meta word and the first codes
    int m = 0, nu = 0, nb = 0, na = 0, nd = 0;
    int e[DB_NLHEAD], u[DB_MAXU];
    uint32_t bt4 = 0, cw[8];
    double4 xi = make_double4(0, 0, 0, 0);
    if (active) {
        m = NL.cnt[i];
        nu = H.nu[i];
        nb = B.nb[i];
        na = B.na[i];
        nd = B.nd[i];
#pragma unroll
        for (int k = 0; k < DB_NLHEAD; ++k) e[k] = NL.nl[k * n + i];
#pragma unroll
        for (int q = 0; q < DB_MAXU; ++q) u[q] = H.u[q * n + i];
#pragma unroll
        for (int k = 0; k < DB_MAXB; ++k) bt4 |= (uint32_t)(uint8_t)B.bt[k * n + i] << (8 * k);
        xi = B.x[i];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cw[k] = H.acode[k * n + i];
            cw[4 + k] = H.dcode[k * n + i];
        }
    }
    for (int k = tid; k < DB_RHASH; k += DB_BLOCK) ht[k] = -1;
    if (tid == 0) nuniq = 0;
    __syncthreads();
    // every thread checks the count before each insertion, so that at most
    // DB_RCAP + DB_BLOCK keys enter the table (a free slot always remains)
    if (active) {
        region_insert(ht, &nuniq, i);   // the bead itself: the step reads its position from the region too
#pragma unroll
        for (int k = 0; k < DB_NLHEAD; ++k)
            if (k < m && *(volatile int*)&nuniq <= DB_RCAP) region_insert(ht, &nuniq, e[k]);
        for (int k = DB_NLHEAD; k < m && *(volatile int*)&nuniq <= DB_RCAP; ++k)
            region_insert(ht, &nuniq, NL.nl[k * n + i]);
        if (nu <= DB_MAXU) {
#pragma unroll
            for (int q = 0; q < DB_MAXU; ++q)
                if (q < nu && *(volatile int*)&nuniq <= DB_RCAP) region_insert(ht, &nuniq, u[q]);
        }
    }
    __syncthreads();
    const int R = nuniq;
    if (R > DB_RCAP) {   // too many to stage: the tile reads its partners from memory
        if (tid == 0) T.rcount[tile] = R;
        return;
    }
    // compact the keys (eight table slots per thread), then sort them
    constexpr int PER = DB_RHASH / DB_BLOCK;
    int mine = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) mine += ht[tid * PER + k] != -1;
    int incl = mine;
    const int lane = tid & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[tid >> 6] = incl;
    __syncthreads();
    int off = incl - mine;
    for (int w = 0; w < (tid >> 6); ++w) off += wsum[w];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int key = ht[tid * PER + k];
        if (key != -1) reg[off++] = key;
    }
    int P2 = 1;
    while (P2 < R) P2 <<= 1;
    for (int k = R + tid; k < P2; k += DB_BLOCK) reg[k] = 0x7FFFFFFF;
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < P2 / 2; t += DB_BLOCK) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const int a = reg[lo], b = reg[hi];
                if ((a > b) == ((lo & size) == 0)) {
                    reg[lo] = b;
                    reg[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int r = tid; r < R; r += DB_BLOCK) {
        const int key = reg[r];
        T.rslot[(size_t)tile * DB_RCAP + r] = key;
        hv[region_find(ht, key)] = (uint16_t)r;
    }
    if (tid == 0) T.rcount[tile] = R;
    __syncthreads();
    if (active) {
        // the entries as region indices: the first DB_NLHEAD of the list in one row
        uint32_t w16[DB_NLHEAD / 2];
#pragma unroll
        for (int k = 0; k < DB_NLHEAD / 2; ++k) {
            const uint32_t lo = 2 * k < m ? hv[region_find(ht, e[2 * k])] : 0u;
            const uint32_t hi = 2 * k + 1 < m ? hv[region_find(ht, e[2 * k + 1])] : 0u;
            w16[k] = lo | hi << 16;
        }
        uint4* row = reinterpret_cast<uint4*>(T.nl16 + (size_t)i * DB_NLHEAD);
        row[0] = make_uint4(w16[0], w16[1], w16[2], w16[3]);
        row[1] = make_uint4(w16[4], w16[5], w16[6], w16[7]);
        for (int k = DB_NLHEAD; k < m; ++k) T.nl16[nl16_index(n, i, k)] = hv[region_find(ht, NL.nl[k * n + i])];
        uint32_t h16[DB_MAXU / 2];
#pragma unroll
        for (int q = 0; q < DB_MAXU / 2; ++q) {
            const uint32_t lo = (nu <= DB_MAXU && 2 * q < nu) ? hv[region_find(ht, u[2 * q])] : 0u;
            const uint32_t hi = (nu <= DB_MAXU && 2 * q + 1 < nu) ? hv[region_find(ht, u[2 * q + 1])] : 0u;
            h16[q] = lo | hi << 16;
        }
        *reinterpret_cast<uint4*>(T.hu16 + (size_t)i * DB_MAXU) = make_uint4(h16[0], h16[1], h16[2], h16[3]);
        const uint32_t mhi = (uint32_t)meta_word(xi) & 0xFFFFu;   // type | reactive << 8 (one box: replica 0)
        T.rec[i] = make_uint4(bt4, (uint32_t)nu | (uint32_t)m << 8 | (uint32_t)nb << 16 | (uint32_t)na << 20 |
                                       (uint32_t)nd << 24,
                              (uint32_t)hv[region_find(ht, i)] | mhi << 16, (uint32_t)meta_gid(xi));
    }
    // Work items.  Every angle (dihedral) with a member in the tile is emitted once,
    // by its centre (its second bead) when that is in the tile, else by its lowest
    // member in the tile; each member then finds the item through the emitter's
    // table and records it with its own role.  A tile whose beads hold more than four
    // angles or dihedrals, or whose halo overflows, keeps per-bead terms.
    __shared__ uint16_t emitA[DB_BLOCK][4], emitD[DB_BLOCK][4];
    __shared__ int nA, nD, bad;
    if (tid == 0) {
        nA = 0;
        nD = 0;
        bad = 0;
    }
    const int t0 = tile * DB_BLOCK, t1 = min(t0 + DB_BLOCK, n);
    auto in_tile = [&](int x) { return x >= t0 && x < t1; };
    int4 ang[4], dih[4];
    int dt4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ang[k] = make_int4(0, 0, 0, 0);
        dih[k] = make_int4(0, 0, 0, 0);
        dt4[k] = 0;
        if (active && k < na) ang[k] = B.ang[k * n + i];
        if (active && k < nd) {
            dih[k] = B.dih[k * n + i];
            dt4[k] = B.dt[k * n + i] & (DB_MAXT - 1);
        }
    }
    __syncthreads();
    if (active && (na > 4 || nd > 4 || nu > DB_MAXU)) bad = 1;
    auto emitter3 = [&](int4 q) {   // centre if in the tile, else the lowest member in the tile
        if (in_tile(q.y)) return q.y;
        int em = 0x7FFFFFFF;
        if (in_tile(q.x)) em = min(em, q.x);
        if (in_tile(q.z)) em = min(em, q.z);
        return em;
    };
    auto emitter4 = [&](int4 q) {
        if (in_tile(q.y)) return q.y;
        int em = 0x7FFFFFFF;
        if (in_tile(q.x)) em = min(em, q.x);
        if (in_tile(q.z)) em = min(em, q.z);
        if (in_tile(q.w)) em = min(em, q.w);
        return em;
    };
    auto rix = [&](int slot) { return (uint32_t)hv[region_find(ht, slot)]; };
    if (active && na <= 4 && nd <= 4 && nu <= DB_MAXU) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            emitA[tid][k] = 0xFFFF;
            emitD[tid][k] = 0xFFFF;
            if (k < na && emitter3(ang[k]) == i) {
                const int idx = atomicAdd(&nA, 1);
                if (idx < DB_CAPA) {
                    T.itemA[(size_t)tile * DB_CAPA + idx] =
                        make_uint2(rix(ang[k].x) | rix(ang[k].y) << 10 | rix(ang[k].z) << 20,
                                   (uint32_t)(ang[k].w & (DB_MAXT - 1)));
                    emitA[tid][k] = (uint16_t)idx;
                }
            }
            if (k < nd && emitter4(dih[k]) == i) {
                const int idx = atomicAdd(&nD, 1);
                if (idx < DB_CAPD) {
                    T.itemD[(size_t)tile * DB_CAPD + idx] =
                        make_uint2(rix(dih[k].x) | rix(dih[k].y) << 10 | rix(dih[k].z) << 20,
                                   rix(dih[k].w) | (uint32_t)dt4[k] << 10);
                    emitD[tid][k] = (uint16_t)idx;
                }
            }
        }
    }
    __syncthreads();
    const bool items = !bad && nA <= DB_CAPA && nD <= DB_CAPD;
    if (tid == 0) T.nitems[tile] = items ? ((uint32_t)nA | (uint32_t)nD << 16) : 0xFFFFFFFFu;
    if (!active) return;
    if (items) {
        // code of entry k: item | role << 16 | 1 << 31, found through the emitter's table
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t ca = 0u, cd = 0u;
            if (k < na) {
                const int4 q = ang[k];
                const int em = emitter3(q);
                int idx = 0xFFFF;
                if (em == i) {
                    idx = emitA[tid][k];
                } else {
                    const int ne = B.na[em];
                    for (int kk = 0; kk < ne && kk < 4; ++kk) {
                        const int4 r = B.ang[kk * n + em];
                        if (r.x == q.x && r.y == q.y && r.z == q.z && r.w == q.w) idx = emitA[em - t0][kk];
                    }
                }
                const int role = q.x == i ? 0 : (q.y == i ? 1 : 2);
                ca = (uint32_t)idx | (uint32_t)role << 16 | 1u << 31;
            }
            if (k < nd) {
                const int4 q = dih[k];
                const int em = emitter4(q);
                int idx = 0xFFFF;
                if (em == i) {
                    idx = emitD[tid][k];
                } else {
                    const int ne = B.nd[em];
                    for (int kk = 0; kk < ne && kk < 4; ++kk) {
                        const int4 r = B.dih[kk * n + em];
                        const int rt = B.dt[kk * n + em] & (DB_MAXT - 1);
                        if (r.x == q.x && r.y == q.y && r.z == q.z && r.w == q.w && rt == dt4[k])
                            idx = emitD[em - t0][kk];
                    }
                }
                const int role = q.x == i ? 0 : (q.y == i ? 1 : (q.z == i ? 2 : 3));
                cd = (uint32_t)idx | (uint32_t)role << 16 | 1u << 31;
            }
            cw[k] = ca;
            cw[4 + k] = cd;
        }
    } else {
        // per-bead terms: the first angle and dihedral codes of the halo
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k >= na) cw[k] = 0u;
            if (k >= nd) cw[4 + k] = 0u;
        }
    }
    T.code8[2 * (size_t)i] = make_uint4(cw[0], cw[1], cw[2], cw[3]);
    T.code8[2 * (size_t)i + 1] = make_uint4(cw[4], cw[5], cw[6], cw[7]);
}

// Separation of a partner from the bead.  STAGED: region entry r from LDS, where
// the region's positions are stored as images next to the tile (unwrapped about
// one reference point when staged), and xs is the bead's own entry there, so the
// separation is a plain difference.  Otherwise slot r from memory, with the
// minimum image.
// A region spread over more than half a box edge (small boxes) keeps the minimum
// image on the differences (IMAGE).
template <bool STAGED, bool IMAGE = false>
struct TilePos {
    const double *rx, *ry, *rz;
    const double4* x;
    __device__ __forceinline__ void sep(int r, const double4& xs, const Box& X, double& dx, double& dy,
                                        double& dz) const {
        if constexpr (STAGED) {
            dx = rx[r] - xs.x;
            dy = ry[r] - xs.y;
            dz = rz[r] - xs.z;
            if constexpr (IMAGE) {
                dx = near_image(dx, X);
                dy = near_image(dy, X);
                dz = near_image(dz, X);
            }
        } else {
            const double4 q = x[r];
            dx = near_image(q.x - xs.x, X);
            dy = near_image(q.y - xs.y, X);
            dz = near_image(q.z - xs.z, X);
        }
    }
};

// The words of bead i that the tile step needs before any partner position, all
// requested at the start of the kernel so that their latency overlaps the loads
// of the region: the halo members and the first DB_NLHEAD list entries as 16-bit
// region indices (packed two to a word), the bond types, the counts, and the
// first four angle and dihedral codes.
struct TileBead {
    uint32_t hu[DB_MAXU / 2];      // halo members, two 16-bit region indices a word
    uint32_t nl[DB_NLHEAD / 2];    // list entries 0..15, two a word
    int btk[DB_MAXB];
    int nb, na, nd, nu, m;
    uint32_t ac[4], dc[4];
};

__device__ __forceinline__ int half16(const uint32_t* w, int k) { return (int)((w[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu); }

// element k < 4 of a register array by selects (an indexed access would go
// through scratch memory)
__device__ __forceinline__ uint32_t pick4(const uint32_t* a, int k) {
    return k == 0 ? a[0] : (k == 1 ? a[1] : (k == 2 ? a[2] : a[3]));
}

// the bead's words of a staged tile: its record, halo row, first list entries and
// first angle and dihedral codes, five 16-byte loads in all; returns the record
__device__ __forceinline__ uint4 tile_bead_load(const Tiles& T, int i, TileBead& tb) {
    const uint4 rc = T.rec[i];
    const uint4 h = *reinterpret_cast<const uint4*>(T.hu16 + (size_t)i * DB_MAXU);
    const uint4* row = reinterpret_cast<const uint4*>(T.nl16 + (size_t)i * DB_NLHEAD);
    const uint4 l0 = row[0], l1 = row[1];
    const uint4 a4 = T.code8[2 * (size_t)i], d4 = T.code8[2 * (size_t)i + 1];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) tb.btk[k] = (int)((rc.x >> (8 * k)) & 0xFFu);
    tb.nu = (int)(rc.y & 0xFFu);
    tb.m = (int)((rc.y >> 8) & 0xFFu);
    tb.nb = (int)((rc.y >> 16) & 0xFu);
    tb.na = (int)((rc.y >> 20) & 0xFu);
    tb.nd = (int)((rc.y >> 24) & 0x1Fu);
    tb.hu[0] = h.x;
    tb.hu[1] = h.y;
    tb.hu[2] = h.z;
    tb.hu[3] = h.w;
    tb.nl[0] = l0.x;
    tb.nl[1] = l0.y;
    tb.nl[2] = l0.z;
    tb.nl[3] = l0.w;
    tb.nl[4] = l1.x;
    tb.nl[5] = l1.y;
    tb.nl[6] = l1.z;
    tb.nl[7] = l1.w;
    tb.ac[0] = a4.x;
    tb.ac[1] = a4.y;
    tb.ac[2] = a4.z;
    tb.ac[3] = a4.w;
    tb.dc[0] = d4.x;
    tb.dc[1] = d4.y;
    tb.dc[2] = d4.z;
    tb.dc[3] = d4.w;
    return rc;
}

// The bond forces on bead i (its halo's first nb members), as in tile_bonded
template <typename R, bool STAGED, bool IMAGE>
__device__ __forceinline__ void tile_bonds(const Params& P, const Box& X, const Coef<R>& C,
                                           const TilePos<STAGED, IMAGE>& tp, const double4& xi, const TileBead& tb,
                                           Acc<R>& a) {
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) {
        if (k >= tb.nb) continue;
        double dx, dy, dz;
        tp.sep(half16(tb.hu, k), xi, X, dx, dy, dz);
        const int t = tb.btk[k] & (DB_MAXT - 1);
        const double rd2 = (dx * dx + dy * dy) + dz * dz;
        if (!(rd2 > 0.0) || !(rd2 < C.bRc2[t])) continue;
        const R ex = (R)dx, ey = (R)dy, ez = (R)dz;
        R rr2 = (ex * ex + ey * ey) + ez * ez;
        R ir = r_rsqrt<R>(rr2);
        R r = rr2 * ir;
        R g = (R)2.0 * C.bK[t] * (r - C.bR0[t]) * ir;
        a.fx += (double)(g * ex);
        a.fy += (double)(g * ey);
        a.fz += (double)(g * ez);
    }
}

// All bonded forces on bead i through its halo, with the same arithmetic in the
// same order as halo_bonded, members read from the staged region (STAGED) or from
// memory by slot.  hidx holds the thread's member references for the angle and
// dihedral entries.
template <typename R, bool STAGED, bool IMAGE>
__device__ __forceinline__ void tile_bonded(const Params& P, const Box& X, const Coef<R>& C, const Halo& H,
                                            const TilePos<STAGED, IMAGE>& tp, uint16_t (*hidx)[DB_BLOCK], int i,
                                            const double4& xi, const TileBead& tb, Acc<R>& a) {
    const int n = P.n;
    const int tid = threadIdx.x;
    // halo member q: a region index parked in LDS (staged), else its slot from memory
    auto member = [&](int q) -> int { return STAGED ? (int)hidx[q][tid] : H.u[q * n + i]; };
    if (STAGED) {
#pragma unroll
        for (int q = 0; q < DB_MAXU; ++q)
            if (q < tb.nu) hidx[q][tid] = (uint16_t)half16(tb.hu, q);
    }
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) {
        if (k >= tb.nb) continue;
        double dx, dy, dz;
        tp.sep(STAGED ? half16(tb.hu, k) : member(k), xi, X, dx, dy, dz);
        const int t = tb.btk[k] & (DB_MAXT - 1);
        const double rd2 = (dx * dx + dy * dy) + dz * dz;
        if (!(rd2 > 0.0) || !(rd2 < C.bRc2[t])) continue;
        const R ex = (R)dx, ey = (R)dy, ez = (R)dz;
        R rr2 = (ex * ex + ey * ey) + ez * ez;
        R ir = r_rsqrt<R>(rr2);
        R r = rr2 * ir;
        R g = (R)2.0 * C.bK[t] * (r - C.bR0[t]) * ir;
        a.fx += (double)(g * ex);
        a.fy += (double)(g * ey);
        a.fz += (double)(g * ez);
    }
    // the first four entries unrolled (codes in registers, so every member's loads
    // can be issued together), then any further ones
#pragma unroll
    for (int k = 0; k < DB_MAXA; ++k) {
        if (k >= tb.na) continue;
        const uint32_t code = k < 4 ? tb.ac[k < 4 ? k : 0] : H.acode[k * n + i];
        const int role = code & 3, k1 = (code >> 2) & 7, k2 = (code >> 5) & 7, t = (code >> 8) & (DB_MAXT - 1);
        double d1x, d1y, d1z, d2x, d2y, d2z;
        tp.sep(member(k1), xi, X, d1x, d1y, d1z);
        tp.sep(member(k2), xi, X, d2x, d2y, d2z);
        const R s1x = (R)d1x, s1y = (R)d1y, s1z = (R)d1z, s2x = (R)d2x, s2y = (R)d2y, s2z = (R)d2z;
        const R z = (R)0;
        const R pax = role == 0 ? z : s1x, pay = role == 0 ? z : s1y, paz = role == 0 ? z : s1z;
        const R pbx = role == 0 ? s1x : (role == 1 ? z : s2x), pby = role == 0 ? s1y : (role == 1 ? z : s2y),
                pbz = role == 0 ? s1z : (role == 1 ? z : s2z);
        const R pcx = role == 2 ? z : s2x, pcy = role == 2 ? z : s2y, pcz = role == 2 ? z : s2z;
        angle_core<R, MODE_STEP>(C, role, t, pax - pbx, pay - pby, paz - pbz, pcx - pbx, pcy - pby, pcz - pbz, a);
    }
#pragma unroll
    for (int k = 0; k < DB_MAXD; ++k) {
        if (k >= tb.nd) continue;
        const uint32_t code = k < 4 ? tb.dc[k < 4 ? k : 0] : H.dcode[k * n + i];
        const int role = code & 3, k1 = (code >> 2) & 7, k2 = (code >> 5) & 7, k3 = (code >> 8) & 7;
        const int t = (code >> 11) & (DB_MAXT - 1);
        double d1x, d1y, d1z, d2x, d2y, d2z, d3x, d3y, d3z;
        tp.sep(member(k1), xi, X, d1x, d1y, d1z);
        tp.sep(member(k2), xi, X, d2x, d2y, d2z);
        tp.sep(member(k3), xi, X, d3x, d3y, d3z);
        const R s1x = (R)d1x, s1y = (R)d1y, s1z = (R)d1z, s2x = (R)d2x, s2y = (R)d2y, s2z = (R)d2z;
        const R s3x = (R)d3x, s3y = (R)d3y, s3z = (R)d3z;
        const R z = (R)0;
        const R pax = role == 0 ? z : s1x, pay = role == 0 ? z : s1y, paz = role == 0 ? z : s1z;
        const R pbx = role == 0 ? s1x : (role == 1 ? z : s2x), pby = role == 0 ? s1y : (role == 1 ? z : s2y),
                pbz = role == 0 ? s1z : (role == 1 ? z : s2z);
        const R pcx = role <= 1 ? s2x : (role == 2 ? z : s3x), pcy = role <= 1 ? s2y : (role == 2 ? z : s3y),
                pcz = role <= 1 ? s2z : (role == 2 ? z : s3z);
        const R pdx = role == 3 ? z : s3x, pdy = role == 3 ? z : s3y, pdz = role == 3 ? z : s3z;
        dihedral_core<R, MODE_STEP>(C, role, t, pbx - pax, pby - pay, pbz - paz, pcx - pbx, pcy - pby, pcz - pbz,
                                    pdx - pcx, pdy - pcy, pdz - pcz, a);
    }
}

// WCA force of one list partner (the arithmetic of pair_one)
template <typename R, bool STAGED, bool IMAGE>
__device__ __forceinline__ void tile_pair(const Params& P, const Box& X, const TilePos<STAGED, IMAGE>& tp, int r,
                                          const double4& xi, R rc2, Acc<R>& a) {
    double dx, dy, dz;
    tp.sep(r, xi, X, dx, dy, dz);
    const R ex = (R)dx, ey = (R)dy, ez = (R)dz;
    const R r2 = (ex * ex + ey * ey) + ez * ez;
    if (r2 < rc2) {
        R ir2 = r_rcp<R>(r2);
        R sr2 = (R)P.sig2 * ir2;
        R sr6 = sr2 * sr2 * sr2;
        R fr = (R)24.0 * (R)P.eps * ((R)2.0 * sr6 * sr6 - sr6) * ir2;
        a.fx -= (double)(fr * ex);
        a.fy -= (double)(fr * ey);
        a.fz -= (double)(fr * ez);
    }
}

// Bonded forces of a bead with more distinct bonded partners than the halo holds:
// every entry reads its members from memory, one member at a time (the arithmetic
// of bond_terms, angle_one and dihedral_one).
template <typename R>
__device__ __forceinline__ void wide_bonded(const Params& P, const Box& X, const Coef<R>& C, const Bank& B, int i,
                                         const double4& xi, Acc<R>& a) {
    const int n = P.n;
    const int nb = B.nb[i];
    for (int k = 0; k < nb; ++k) {
        const int j = B.bp[k * n + i];
        const int t = (int)B.bt[k * n + i] & (DB_MAXT - 1);
        const double4 xj = B.x[j];
        const double dx = near_image(xj.x - xi.x, X), dy = near_image(xj.y - xi.y, X), dz = near_image(xj.z - xi.z, X);
        const double rd2 = (dx * dx + dy * dy) + dz * dz;
        if (!(rd2 > 0.0) || !(rd2 < C.bRc2[t])) continue;
        R rx = (R)dx, ry = (R)dy, rz = (R)dz;
        R rr2 = (rx * rx + ry * ry) + rz * rz;
        R ir = r_rsqrt<R>(rr2);
        R r = rr2 * ir;
        R g = (R)2.0 * C.bK[t] * (r - C.bR0[t]) * ir;
        a.fx += (double)(g * rx);
        a.fy += (double)(g * ry);
        a.fz += (double)(g * rz);
    }
    const int na = B.na[i];
    for (int k = 0; k < na; ++k) {
        const int4 e = B.ang[k * n + i];
        angle_one<R, MODE_STEP>(P, X, C, i, e, B.x[e.x], B.x[e.y], B.x[e.z], a);
    }
    const int nd = B.nd[i];
    for (int k = 0; k < nd; ++k) {
        const int4 e = B.dih[k * n + i];
        const int t = B.dt[k * n + i] & (DB_MAXT - 1);
        dihedral_one<R, MODE_STEP>(P, X, C, i, e, t, B.x[e.x], B.x[e.y], B.x[e.z], B.x[e.w], a);
    }
}

// Forces on one bead of a tile (the first part of k_step_tile's work): partners
// from the staged region (STAGED) or from memory by slot.  Bonds and pairs always;
// angles and dihedrals here only without ITEMS (with ITEMS the tile's work items
// form them and tile_collect adds them afterwards).
template <typename R, bool STAGED, bool IMAGE, bool ITEMS>
__device__ __forceinline__ void tile_bead_forces(const Params& P, const Box& X, const Coef<R>& C, const Bank& B,
                                                 const NList& NL, const Halo& H, const Tiles& T, const double* rx,
                                                 const double* ry, const double* rz, uint16_t (*hidx)[DB_BLOCK], int i,
                                                 const double4& xi, const double4& xs, const TileBead& tb, Acc<R>& a) {
    const int n = P.n;
    const TilePos<STAGED, IMAGE> tp{rx, ry, rz, B.x};
    const R rc2 = (R)P.rc2;
    if constexpr (ITEMS) {
        tile_bonds<R, STAGED, IMAGE>(P, X, C, tp, xs, tb, a);
    } else {
        if (tb.nu <= DB_MAXU) tile_bonded<R, STAGED, IMAGE>(P, X, C, H, tp, hidx, i, xs, tb, a);
        else wide_bonded<R>(P, X, C, B, i, xi, a);
    }
    const int m = tb.m;
    if constexpr (STAGED) {
        // the first DB_NLHEAD entries from registers, in list order, then the rest
#pragma unroll
        for (int k = 0; k < DB_NLHEAD; ++k)
            if (k < m) tile_pair<R, true, IMAGE>(P, X, tp, half16(tb.nl, k), xs, rc2, a);
        for (int k = DB_NLHEAD; k < m; ++k)
            tile_pair<R, true, IMAGE>(P, X, tp, T.nl16[nl16_index(n, i, k)], xs, rc2, a);
    } else {
        for (int k = 0; k < m; ++k) tile_pair<R, false, IMAGE>(P, X, tp, NL.nl[k * n + i], xs, rc2, a);
    }
}

// Work-item force tables of a tile in LDS.  An angle item keeps the forces on its
// two outer members (the centre's is minus their sum); a dihedral item keeps the
// forces on its end members and the two projections pp, qq from which those on
// the inner members follow.
template <typename R>
struct ItemForces {
    R a[6][DB_CAPA];   // angle: role 0 then role 2, x y z
    R d[8][DB_CAPD];   // dihedral: role 0, role 3 (x y z), pp, qq
};

// The angle and dihedral forces of a bead from its tile's work items, in its table
// order (codes: item | role << 16)
template <typename R>
__device__ __forceinline__ void tile_collect(const ItemForces<R>& F, const TileBead& tb, int nAi, int nDi, Acc<R>& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k >= tb.na) continue;
        const uint32_t code = tb.ac[k];
        const int it = (int)(code & 0xFFFFu), role = (int)((code >> 16) & 3u);
        if (it >= nAi) continue;
        R f[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R f0 = F.a[c][it], f2 = F.a[3 + c][it];
            f[c] = role == 0 ? f0 : (role == 2 ? f2 : -(f0 + f2));
        }
        a.fx += (double)f[0];
        a.fy += (double)f[1];
        a.fz += (double)f[2];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k >= tb.nd) continue;
        const uint32_t code = tb.dc[k];
        const int it = (int)(code & 0xFFFFu), role = (int)((code >> 16) & 3u);
        if (it >= nDi) continue;
        const R pp = F.d[6][it], qq = F.d[7][it];
        R f[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R f0 = F.d[c][it], f3 = F.d[3 + c][it];
            const R f1 = qq * f3 - (pp + (R)1) * f0, f2 = pp * f0 - (qq + (R)1) * f3;
            f[c] = role == 0 ? f0 : (role == 3 ? f3 : (role == 1 ? f1 : f2));
        }
        a.fx += (double)f[0];
        a.fy += (double)f[1];
        a.fz += (double)f[2];
    }
}

// The rest of one bead's step once its force is complete: the external force, the
// Langevin force and the velocity-Verlet update.  Returns |v|^2 after the step.
template <typename R>
__device__ __forceinline__ double tile_bead_finish(const Params& P, const Box& X, Bank& B, int i, const double4& xi,
                                                   double vx, double vy, double vz, const Acc<R>& a,
                                                   double4* __restrict__ xout, int64_t step, double pref,
                                                   int* __restrict__ err, double4* __restrict__ xsave,
                                                   double* __restrict__ vsave) {
    const int n = P.n;
    double Fx = a.fx, Fy = a.fy, Fz = a.fz;
    if (P.has_ext) {
        const size_t g = (size_t)meta_gid(xi);
        Fx += P.fext[3 * g];
        Fy += P.fext[3 * g + 1];
        Fz += P.fext[3 * g + 2];
    }
    if (xsave) {   // first step of a block: keep its input state for a re-run
        xsave[i] = xi;
        vsave[i] = vx;
        vsave[n + i] = vy;
        vsave[2 * n + i] = vz;
    }
    if (P.gamma != 0.0) {
        uint4 w = rng_draw(X, (uint32_t)(meta_gid(xi) - X.gid_off), 0u, step, RNG_LANGEVIN);
        const double s32 = 1.0 / 4294967296.0;
        double ux = ((double)w.x + 0.5) * s32, uy = ((double)w.y + 0.5) * s32, uz = ((double)w.z + 0.5) * s32;
        Fx = (Fx - P.gamma * vx) + pref * (ux - 0.5);
        Fy = (Fy - P.gamma * vy) + pref * (uy - 0.5);
        Fz = (Fz - P.gamma * vz) + pref * (uz - 0.5);
    }
    const double hdt = 0.5 * P.dt;
    double hx = vx + hdt * Fx, hy = vy + hdt * Fy, hz = vz + hdt * Fz;
    vx = hx + hdt * Fx;
    vy = hy + hdt * Fy;
    vz = hz + hdt * Fz;
    double4 xo;
    xo.x = wrap1(xi.x + P.dt * vx, X.L);
    xo.y = wrap1(xi.y + P.dt * vy, X.L);
    xo.z = wrap1(xi.z + P.dt * vz, X.L);
    xo.w = xi.w;
    const bool bad = !(xo.x >= 0.0 && xo.x < X.L && xo.y >= 0.0 && xo.y < X.L && xo.z >= 0.0 && xo.z < X.L);
    if (bad) atomicOr(err, ERR_NONFINITE);
    xout[i] = xo;
    B.v[i] = vx;
    B.v[n + i] = vy;
    B.v[2 * n + i] = vz;
    return (vx * vx + vy * vy) + vz * vz;
}

// The fused step (WCA pairs, bonded terms, Langevin force, velocity Verlet) of one
// tile of DB_BLOCK consecutive slots per workgroup, one bead per thread.  Slots
// are in brick order, so a tile is a compact piece of space.  Each bead's own
// words are requested first, then the positions of the tile's region are loaded
// into LDS, and after one barrier every partner position comes from there.  A
// tile whose region could not be staged reads partners from memory by slot, and a
// bead whose halo overflows reads its table entries.  In a staged tile whose beads
// hold at most four angles and four dihedrals each (and whose counts fit
// DB_CAPA / DB_CAPD), every angle and dihedral is evaluated once, by one thread,
// after the bead's bonds and pairs, and its members add their shares after a
// second barrier; otherwise each bead evaluates its own terms as k_step does.  The
// terms are those of k_step; the order in which a bead's force is summed differs
// (bonds, pairs, then angles and dihedrals), so the trajectories agree to rounding.
template <typename R>
__global__ __launch_bounds__(DB_BLOCK) void k_step_tile(const Params* __restrict__ Pp, Bank B, NList NL, Halo H,
                                                        Tiles T, double4* __restrict__ xout, int64_t step,
                                                        double pref, unsigned int* __restrict__ vmax2_slot,
                                                        int* __restrict__ err, double4* __restrict__ xsave,
                                                        double* __restrict__ vsave,
                                                        const int64_t* __restrict__ step_base) {
    const Params& P = *Pp;
    const int n = P.n;
    if (step_base) {
        double dsig = 0.0;
        step_amplitudes(P, step_base, step, pref, dsig);
    }
    const Box& X = P.box;
    __shared__ Coef<R> C;
    __shared__ double rx[DB_RCAP], ry[DB_RCAP], rz[DB_RCAP];
    // per-thread halo indices (per-bead bonded terms) or the work items' forces:
    // a tile uses one or the other
    __shared__ union {
        uint16_t hidx[DB_MAXU][DB_BLOCK];
        ItemForces<R> f;
    } lu;
    auto& hidx = lu.hidx;
    load_coef<R>(P, C);
    const int tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int i = tile * DB_BLOCK + tid;
    const bool active = i < n;
    const int nreg = T.rcount[tile];
    const bool staged = nreg <= DB_RCAP;
    // work items of the tile (a staged tile whose beads hold at most four angles and
    // dihedrals each): requested with the bead's own words
    const uint32_t ni = staged ? T.nitems[tile] : 0xFFFFFFFFu;
    const bool items = ni != 0xFFFFFFFFu;
    const int nAi = items ? (int)(ni & 0xFFFFu) : 0, nDi = items ? (int)(ni >> 16) : 0;
    constexpr int APT = (DB_CAPA + DB_BLOCK - 1) / DB_BLOCK;
    uint2 ia[APT], idh = make_uint2(0, 0);
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        ia[q] = make_uint2(0, 0);
        if (q * DB_BLOCK + tid < nAi) ia[q] = T.itemA[(size_t)tile * DB_CAPA + q * DB_BLOCK + tid];
    }
    static_assert(DB_CAPD <= DB_BLOCK, "one dihedral item per thread");
    if (tid < nDi) idh = T.itemD[(size_t)tile * DB_CAPD + tid];
    TileBead tb;
    double4 xi = make_double4(0, 0, 0, 0);
    double vx = 0, vy = 0, vz = 0;
    uint4 rc = make_uint4(0, 0, 0, 0);
    if (active) {
        xi = B.x[i];
        vx = B.v[i];
        vy = B.v[n + i];
        vz = B.v[2 * n + i];
        if (staged) {
            rc = tile_bead_load(T, i, tb);
        } else {   // partners by slot: only the counts and types here
            tb.nu = H.nu[i];
            tb.m = P.have_pair ? (int)NL.cnt[i] : 0;
            tb.nb = B.nb[i];
            tb.na = B.na[i];
            tb.nd = B.nd[i];
#pragma unroll
            for (int k = 0; k < DB_MAXB; ++k) tb.btk[k] = B.bt[k * n + i];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                tb.ac[k] = H.acode[k * n + i];
                tb.dc[k] = H.dcode[k * n + i];
            }
        }
    }
    int far = 0;   // some stored image lies L/4 or more from the reference (small boxes)
    if (staged) {
        // the region's slots, then their positions: all of a thread's loads of one
        // kind are in flight together.  Each position is stored as its image nearest
        // to one reference point of the tile (its first bead): when every member of
        // the region lies within L/4 of it, differences of stored positions are the
        // minimum-image separations and the pair loop needs no image arithmetic
        constexpr int RPT = DB_RCAP / DB_BLOCK;
        const int* rs = T.rslot + (size_t)tile * DB_RCAP;
        const double4 ref = B.x[tile * DB_BLOCK];
        const double wmax_img = 0.25 * X.L;   // stored images within L/4 of ref: differences are minimum images
        int sl[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q) sl[q] = q * DB_BLOCK + tid < nreg ? rs[q * DB_BLOCK + tid] : -1;
        double4 xq[RPT];
#pragma unroll
        for (int q = 0; q < RPT; ++q)
            if (sl[q] >= 0) xq[q] = B.x[sl[q]];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            if (sl[q] < 0) continue;
            const double ox = near_image(xq[q].x - ref.x, X), oy = near_image(xq[q].y - ref.y, X),
                         oz = near_image(xq[q].z - ref.z, X);
            far |= !(fabs(ox) < wmax_img && fabs(oy) < wmax_img && fabs(oz) < wmax_img);
            rx[q * DB_BLOCK + tid] = ref.x + ox;
            ry[q * DB_BLOCK + tid] = ref.y + oy;
            rz[q * DB_BLOCK + tid] = ref.z + oz;
        }
    }
    const bool image = __syncthreads_or(far) != 0;
    // origin of the separations: the bead's own region entry (staged), else itself
    double4 xs = xi;
    if (active && staged) {
        const int self = (int)(rc.z & 0xFFFFu);
        xs = make_double4(rx[self], ry[self], rz[self], 0.0);
    }
    Acc<R> a;
    if (active) {
        if (items && !image)
            tile_bead_forces<R, true, false, true>(P, X, C, B, NL, H, T, rx, ry, rz, hidx, i, xi, xs, tb, a);
        else if (items)
            tile_bead_forces<R, true, true, true>(P, X, C, B, NL, H, T, rx, ry, rz, hidx, i, xi, xs, tb, a);
        else if (staged && !image)
            tile_bead_forces<R, true, false, false>(P, X, C, B, NL, H, T, rx, ry, rz, hidx, i, xi, xs, tb, a);
        else if (staged)
            tile_bead_forces<R, true, true, false>(P, X, C, B, NL, H, T, rx, ry, rz, hidx, i, xi, xs, tb, a);
        else
            tile_bead_forces<R, false, true, false>(P, X, C, B, NL, H, T, rx, ry, rz, hidx, i, xi, xs, tb, a);
    }
    if (items) {
        // every angle and dihedral of the tile once, from the stored positions
        // (differences of images, or with the minimum image in a small box); after
        // the barrier each member adds its share
        auto dif = [&](const double* r, int p, int q) {
            const double d = r[p] - r[q];
            return image ? near_image(d, X) : d;
        };
#pragma unroll
        for (int q = 0; q < APT; ++q) {
            const int it = q * DB_BLOCK + tid;
            if (it >= nAi) continue;
            const int ra = (int)(ia[q].x & 0x3FFu), rb = (int)((ia[q].x >> 10) & 0x3FFu),
                      rcn = (int)((ia[q].x >> 20) & 0x3FFu), t = (int)(ia[q].y & (DB_MAXT - 1));
            R f[3][3];
            angle_all<R>(C, t, (R)dif(rx, ra, rb), (R)dif(ry, ra, rb), (R)dif(rz, ra, rb), (R)dif(rx, rcn, rb),
                         (R)dif(ry, rcn, rb), (R)dif(rz, rcn, rb), f);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lu.f.a[c][it] = f[0][c];
                lu.f.a[3 + c][it] = f[2][c];
            }
        }
        if (tid < nDi) {
            const int ra = (int)(idh.x & 0x3FFu), rb = (int)((idh.x >> 10) & 0x3FFu),
                      rcn = (int)((idh.x >> 20) & 0x3FFu), rd = (int)(idh.y & 0x3FFu),
                      t = (int)((idh.y >> 10) & (DB_MAXT - 1));
            R f0[3], f3[3], pp, qq;
            dihedral_ends<R>(C, t, (R)dif(rx, rb, ra), (R)dif(ry, rb, ra), (R)dif(rz, rb, ra), (R)dif(rx, rcn, rb),
                             (R)dif(ry, rcn, rb), (R)dif(rz, rcn, rb), (R)dif(rx, rd, rcn), (R)dif(ry, rd, rcn),
                             (R)dif(rz, rd, rcn), f0, f3, pp, qq);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lu.f.d[c][tid] = f0[c];
                lu.f.d[3 + c][tid] = f3[c];
            }
            lu.f.d[6][tid] = pp;
            lu.f.d[7][tid] = qq;
        }
        __syncthreads();
        if (active) tile_collect<R>(lu.f, tb, nAi, nDi, a);
    }
    const double m2 = active ? tile_bead_finish<R>(P, X, B, i, xi, vx, vy, vz, a, xout, step, pref, err, xsave, vsave)
                             : 0.0;
    // largest speed of the tile: one atomic per workgroup, spread over 64 words
    __shared__ float wmax[DB_BLOCK / 64];
    const double v2 = wave_max(m2);
    if ((tid & 63) == 0) wmax[tid >> 6] = (float)v2 * 1.0001f;
    __syncthreads();
    if (tid == 0) {
        float mm = wmax[0];
        for (int w = 1; w < DB_BLOCK / 64; ++w) mm = fmaxf(mm, wmax[w]);
        atomicMax(vmax2_slot + (blockIdx.x & (DB_VMAX_SPREAD - 1)), __float_as_uint(mm));
    }
}

// energy reduction: a separate, simpler kernel keeps the step kernel lean
template <typename R, bool BATCH>
__global__ __launch_bounds__(DB_BLOCK) void k_energy(const Params* __restrict__ Pp, Bank B,
                                                      const int* __restrict__ cstart, const int* __restrict__ clist,
                                                      int64_t step, double* __restrict__ epart) {
    const Params& P = *Pp;
    const int n = P.n;
    __shared__ Coef<R> C;
    load_coef<R>(P, C);
    __syncthreads();
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    double vals[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        Acc<R> a;
        double4 xi = B.x[i];
        const Box& X = box_of<BATCH>(P, meta_word(xi));
        int nb = B.nb[i];
        int p0 = nb > 0 ? B.bp[i] : -1;
        int p1 = nb > 1 ? B.bp[n + i] : -1;
        int p2 = nb > 2 ? B.bp[2 * n + i] : -1;
        int p3 = nb > 3 ? B.bp[3 * n + i] : -1;
        double vx = B.v[i], vy = B.v[n + i], vz = B.v[2 * n + i];
        const double dsig = P.pair_style == PAIR_DPD && P.dpd_gamma != 0.0
                                ? sqrt(2.0 * box_temperature(X, step) * P.dpd_gamma) / sqrt(P.dt)
                                : 0.0;
        if (P.have_pair)
            pair_forces<R, MODE_ENERGY>(P, X, B, cstart, clist, i, xi, nb, p0, p1, p2, p3, vx, vy, vz, step, dsig,
                                        a);
        bond_terms<R, MODE_ENERGY>(P, X, C, B, i, xi, nb, a);
        angle_terms<R, MODE_ENERGY>(P, X, C, B, i, B.na[i], a);
        dihedral_terms<R, MODE_ENERGY>(P, X, C, B, i, B.nd[i], a);
        if (P.has_ext) {
            const size_t g = (size_t)meta_gid(xi);
            a.fx += P.fext[3 * g];
            a.fy += P.fext[3 * g + 1];
            a.fz += P.fext[3 * g + 2];
        }
        double Fx = a.fx, Fy = a.fy, Fz = a.fz;
        if (P.gamma != 0.0) {
            double pref = sqrt(24.0 * P.gamma * box_temperature(X, step) / P.dt);
            uint4 w = rng_draw(X, (uint32_t)(meta_gid(xi) - X.gid_off), 0u, step, RNG_LANGEVIN);
            const double s32 = 1.0 / 4294967296.0;
            double ux = ((double)w.x + 0.5) * s32, uy = ((double)w.y + 0.5) * s32, uz = ((double)w.z + 0.5) * s32;
            Fx = (Fx - P.gamma * vx) + pref * (ux - 0.5);
            Fy = (Fy - P.gamma * vy) + pref * (uy - 0.5);
            Fz = (Fz - P.gamma * vz) + pref * (uz - 0.5);
        }
        const double hdt = 0.5 * P.dt;
        double fvx = vx + hdt * Fx, fvy = vy + hdt * Fy, fvz = vz + hdt * Fz;
        vals[0] = 0.5 * (fvx * fvx + fvy * fvy + fvz * fvz);
        vals[1] = a.e_pair;
        vals[2] = a.e_bond;
        vals[3] = a.e_ang;
        vals[4] = a.e_dih;
        vals[5] = a.vir;
    }
    __shared__ double red[6][DB_BLOCK / 64];
    for (int q = 0; q < 6; ++q) {
        double v = vals[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0;
        for (int w = 0; w < DB_BLOCK / 64; ++w) s += red[threadIdx.x][w];
        epart[(size_t)blockIdx.x * 6 + threadIdx.x] = s;
    }
}

// fixed-order sum of the per-workgroup partials
__global__ void k_energy_final(const double* __restrict__ epart, int nblocks, double* __restrict__ out) {
    int q = threadIdx.x;
    if (q >= 6) return;
    double s = 0;
    for (int b = 0; b < nblocks; ++b) s += epart[(size_t)b * 6 + q];
    out[q] = s;
}

static unsigned grid_for(int n) { return (unsigned)((n + DB_BLOCK - 1) / DB_BLOCK); }

// the halo of every bead after slots or tables changed wholesale; after a sweep only
// of the beads whose own tables it changed
void launch_halo(db_ctx* c) {
    if (c->n == 0) return;
    if (c->halo_force || c->halo_sweep)
        hipLaunchKernelGGL(k_halo, dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream, c->dp, c->bank[c->cur],
                           c->halo, c->halo_force ? (const uint8_t*)nullptr : c->sw.tchg);
    c->halo_force = false;
    c->halo_sweep = false;
}

void launch_regions(db_ctx* c) {
    c->regions_valid = false;
    if (c->n == 0 || !tiles_enabled(c) || !c->tiles_valid) return;
    hipLaunchKernelGGL(k_region, dim3(c->ntile), dim3(DB_BLOCK), 0, c->stream, c->dp, c->bank[c->cur], c->nlist,
                       c->halo, c->tiles, c->ntile);
    c->regions_valid = true;
}

void launch_build_nlist(db_ctx* c) {
    if (c->n == 0) return;
    launch_halo(c);
    double4* xref = c->hp.have_pair && c->hp.pair_style == PAIR_DPD ? c->xref : nullptr;
    if (c->nrep > 0)
        hipLaunchKernelGGL((k_build_nlist<true>), dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream, c->dp,
                           c->bank[c->cur], c->cells.start, c->cells.xs, c->nlist, c->err_d, xref);
    else
        hipLaunchKernelGGL((k_build_nlist<false>), dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream, c->dp,
                           c->bank[c->cur], c->cells.start, c->cells.xs, c->nlist, c->err_d, xref);
    launch_regions(c);
}

// beads whose exclusions the sweep changed: a changed bond table, or (exclusion
// depth 2) a partner whose table changed
__global__ __launch_bounds__(DB_BLOCK) void k_patch_flags(const Params* __restrict__ Pp, Bank B, SweepBuf S) {
    const Params& P = *Pp;
    const int n = P.n;
    const int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    bool d = S.chg[i] != 0;
    if (!d && P.excl_depth >= 2) {
        const int nb = B.nb[i];
        for (int k = 0; k < nb; ++k) d |= S.chg[B.bp[k * n + i]] != 0;
    }
    S.act[i] = d ? 1 : 0;
}

void launch_patch_nlist(db_ctx* c, double cut) {
    if (c->n == 0) return;
    launch_halo(c);
    hipStream_t s = c->stream;
    const unsigned g = grid_for(c->n);
    Bank& B = c->bank[c->cur];
    hipLaunchKernelGGL(k_patch_flags, dim3(g), dim3(DB_BLOCK), 0, s, c->dp, B, c->sw);
    launch_compact(c->sw.act, c->n, c->sw.aoff, c->sw.aoff + c->n, c->cells.blocksum, s);
    // the workgroups step over the tiles of the list (its length is on the device)
    const unsigned gp = std::min(g, 2048u);
    if (c->nrep > 0)
        hipLaunchKernelGGL((k_patch_nlist<true>), dim3(gp), dim3(DB_BLOCK), 0, s, c->dp, B, c->cells.start,
                           c->cells.xs, c->nlist, c->err_d, c->sw.aoff, c->sw.aoff + c->n, cut);
    else
        hipLaunchKernelGGL((k_patch_nlist<false>), dim3(gp), dim3(DB_BLOCK), 0, s, c->dp, B, c->cells.start,
                           c->cells.xs, c->nlist, c->err_d, c->sw.aoff, c->sw.aoff + c->n, cut);
    launch_regions(c);
}

// temperature of the single system's box at a step
static double host_temperature(const Params& P, int64_t step) {
    const Box& X = P.box;
    if (X.ramp <= 0) return X.T0;
    int64_t k = step < X.ramp ? step : X.ramp;
    return X.T0 + (X.T1 - X.T0) * (double)k / (double)X.ramp;
}

// sqrt(24 gamma T / dt), the amplitude of the uniform Langevin noise of a single system
static double langevin_prefactor(const Params& P, int64_t step) {
    if (P.gamma == 0.0) return 0.0;
    return sqrt(24.0 * P.gamma * host_temperature(P, step) / P.dt);
}

// sigma / sqrt(dt) = sqrt(2 T gamma_DPD) / sqrt(dt) of a single system
static double dpd_sigma(const Params& P, int64_t step) {
    if (P.pair_style != PAIR_DPD || P.dpd_gamma == 0.0) return 0.0;
    return sqrt(2.0 * host_temperature(P, step) * P.dpd_gamma) / sqrt(P.dt);
}

// the DPD thermostat reads the neighbours' velocities: the step writes the new
// ones to the second buffer
static bool velocity_double_buffer(const db_ctx* c) {
    return c->hp.have_pair && c->hp.pair_style == PAIR_DPD && c->hp.dpd_gamma != 0.0;
}

template <typename R, int MODE, bool BATCH, int PAIR>
static void launch_step_kernel(db_ctx* c, const Bank& B, double4* xout, double* vout, int64_t step, double pref,
                               double dsig, unsigned* vm, double* f, bool save) {
    hipLaunchKernelGGL((k_step<R, MODE, BATCH, PAIR>), dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream, c->dp,
                       B, c->nlist, c->halo, xout, vout, step, pref, dsig, vm, f, c->err_d,
                       save ? c->xsave : nullptr, save ? c->vsave : nullptr, c->xref,
                       MODE == MODE_STEP ? (const int64_t*)c->step_base_d : nullptr);
}

template <int MODE, int PAIR>
static void launch_step_pair(db_ctx* c, const Bank& B, double4* xout, double* vout, int64_t step, double pref,
                             double dsig, unsigned* vm, double* f, bool save) {
    const bool batch = c->nrep > 0;
    if (c->precision == DB_MIXED) {
        if (batch) launch_step_kernel<float, MODE, true, PAIR>(c, B, xout, vout, step, pref, dsig, vm, f, save);
        else launch_step_kernel<float, MODE, false, PAIR>(c, B, xout, vout, step, pref, dsig, vm, f, save);
    } else {
        if (batch)
            launch_step_kernel<double, MODE, true, PAIR>(c, B, xout, vout, step, pref, dsig, vm, f, save);
        else
            launch_step_kernel<double, MODE, false, PAIR>(c, B, xout, vout, step, pref, dsig, vm, f, save);
    }
}

template <int MODE>
static void launch_step_any(db_ctx* c, const Bank& B, double4* xout, double* vout, int64_t step, double pref,
                            double dsig, unsigned* vm, double* f, bool save = false) {
    if (c->hp.have_pair && c->hp.pair_style == PAIR_DPD)
        launch_step_pair<MODE, PAIR_DPD>(c, B, xout, vout, step, pref, dsig, vm, f, save);
    else
        launch_step_pair<MODE, PAIR_WCA>(c, B, xout, vout, step, pref, dsig, vm, f, save);
}

// c->step_base_d set (the launch is captured into a graph): step is the offset within
// the block and the kernel reads the block's first step from the device
void launch_step(db_ctx* c, int64_t step, int slot_in_block, bool save) {
    if (c->n == 0) return;
    const double pref = c->step_base_d ? 0.0 : langevin_prefactor(c->hp, step);
    const double dsig = c->step_base_d ? 0.0 : dpd_sigma(c->hp, step);
    Bank& B = c->bank[c->cur];
    unsigned* vm = (unsigned*)(c->vmax2 + (size_t)slot_in_block * DB_VMAX_SPREAD);
    const bool vbuf = velocity_double_buffer(c);
    if (tiles_enabled(c) && c->tiles_valid && c->regions_valid) {
        double4* xs = save ? c->xsave : nullptr;
        double* vs = save ? c->vsave : nullptr;
        if (c->precision == DB_MIXED)
            hipLaunchKernelGGL(k_step_tile<float>, dim3(c->ntile), dim3(DB_BLOCK), 0, c->stream, c->dp, B, c->nlist,
                               c->halo, c->tiles, c->xnext, step, pref, vm, c->err_d, xs, vs,
                               (const int64_t*)c->step_base_d);
        else
            hipLaunchKernelGGL(k_step_tile<double>, dim3(c->ntile), dim3(DB_BLOCK), 0, c->stream, c->dp, B,
                               c->nlist, c->halo, c->tiles, c->xnext, step, pref, vm, c->err_d, xs, vs,
                               (const int64_t*)c->step_base_d);
    } else {
        launch_step_any<MODE_STEP>(c, B, c->xnext, vbuf ? c->vnext : B.v, step, pref, dsig, vm, nullptr, save);
    }
    double4* t = B.x;
    B.x = c->xnext;
    c->xnext = t;
    if (vbuf) {
        double* u = B.v;
        B.v = c->vnext;
        c->vnext = u;
    }
}

void launch_forces(db_ctx* c, double* f) {
    if (c->n == 0) return;
    launch_step_any<MODE_FORCES>(c, c->bank[c->cur], nullptr, nullptr, 0, 0.0, 0.0, nullptr, f);
}

template <typename R, bool BATCH>
static void launch_energy_kernel(db_ctx* c, unsigned nb, double* part) {
    hipLaunchKernelGGL((k_energy<R, BATCH>), dim3(nb), dim3(DB_BLOCK), 0, c->stream, c->dp, c->bank[c->cur],
                       c->cells.start, c->cells.list, c->step, part);
}

void launch_energy(db_ctx* c, double* out6, double* partials) {
    unsigned nb = grid_for(c->n);
    double* part = partials ? partials : c->red;
    if (c->n > 0) {
        const bool batch = c->nrep > 0;
        if (c->precision == DB_MIXED) {
            if (batch) launch_energy_kernel<float, true>(c, nb, part);
            else launch_energy_kernel<float, false>(c, nb, part);
        } else {
            if (batch) launch_energy_kernel<double, true>(c, nb, part);
            else launch_energy_kernel<double, false>(c, nb, part);
        }
    }
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, c->stream, part, (int)(c->n > 0 ? nb : 0), out6);
}

}  // namespace db
