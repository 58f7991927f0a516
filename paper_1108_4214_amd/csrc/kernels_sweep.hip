// The dynamic-bonding sweep (section 2 and the appendix "Implementation
// details", steps 2-9) as per-bead kernels.  Every bead owns its bond, angle and
// dihedral table (the paper's Newton-off storage), so each kernel writes only
// the entries of its own bead and reads other beads' tables; no atomics touch
// the topology.  Both beads of a pair evaluate the same pair-keyed decisions
// (distance, rule, random number), so their tables stay consistent without any
// exchange.
//
//   nominate_create   closest eligible creation partner per bead (step 2)
//   nominate_break    most distant eligible bonded partner; killbond marks (step 3, 5)
//   resolve           mutual breakage nominations accepted with probability p (step 5)
//   apply             drop angles/dihedrals crossing removed bonds (step 6),
//                     remove / convert bonds (step 7), accept mutual creation
//                     nominations with probability p (step 8)
//   generate          new angles/dihedrals on paths through new bonds (step 9)
#include "cell_scan.h"

namespace db {


// A bead's bond table held in registers.  Entries are read through selects, so
// loops over a run-time count never index a private array (which would spill it
// to scratch memory).
struct Tab {
    static_assert(DB_MAXB == 4, "Tab holds four entries");
    int n;
    int p0, p1, p2, p3;
    int t0, t1, t2, t3;
    __device__ int p(int k) const { return k == 0 ? p0 : (k == 1 ? p1 : (k == 2 ? p2 : p3)); }
    __device__ int t(int k) const { return k == 0 ? t0 : (k == 1 ? t1 : (k == 2 ? t2 : t3)); }
};

__device__ __forceinline__ Tab load_tab(const Bank& B, int n, int s) {
    Tab T;
    T.n = B.nb[s];
    T.p0 = T.n > 0 ? B.bp[s] : -1;
    T.p1 = T.n > 1 ? B.bp[n + s] : -1;
    T.p2 = T.n > 2 ? B.bp[2 * n + s] : -1;
    T.p3 = T.n > 3 ? B.bp[3 * n + s] : -1;
    T.t0 = T.n > 0 ? (int)B.bt[s] : 0;
    T.t1 = T.n > 1 ? (int)B.bt[n + s] : 0;
    T.t2 = T.n > 2 ? (int)B.bt[2 * n + s] : 0;
    T.t3 = T.n > 3 ? (int)B.bt[3 * n + s] : 0;
    return T;
}

// the same with every row requested together with the count (rows exist for
// every bead): one memory latency instead of two, for the latency-bound paths
// that read few tables; streaming passes over all beads keep load_tab, which
// reads only the occupied rows
__device__ __forceinline__ Tab load_tab_all(const Bank& B, int n, int s) {
    Tab T;
    T.n = B.nb[s];
    const int p0 = B.bp[s], p1 = B.bp[n + s], p2 = B.bp[2 * n + s], p3 = B.bp[3 * n + s];
    const int t0 = B.bt[s], t1 = B.bt[n + s], t2 = B.bt[2 * n + s], t3 = B.bt[3 * n + s];
    T.p0 = T.n > 0 ? p0 : -1;
    T.p1 = T.n > 1 ? p1 : -1;
    T.p2 = T.n > 2 ? p2 : -1;
    T.p3 = T.n > 3 ? p3 : -1;
    T.t0 = T.n > 0 ? t0 : 0;
    T.t1 = T.n > 1 ? t1 : 0;
    T.t2 = T.n > 2 ? t2 : 0;
    T.t3 = T.n > 3 ? t3 : 0;
    return T;
}

// the tables of a bead's four partners, selected by a run-time index field by
// field (a select of whole tables would go through scratch memory)
__device__ __forceinline__ int sel4(int k, int x0, int x1, int x2, int x3) {
    return k == 0 ? x0 : (k == 1 ? x1 : (k == 2 ? x2 : x3));
}
struct Tab4 {
    Tab a, b, c, d;
    __device__ Tab get(int k) const {
        Tab T;
        T.n = sel4(k, a.n, b.n, c.n, d.n);
        T.p0 = sel4(k, a.p0, b.p0, c.p0, d.p0);
        T.p1 = sel4(k, a.p1, b.p1, c.p1, d.p1);
        T.p2 = sel4(k, a.p2, b.p2, c.p2, d.p2);
        T.p3 = sel4(k, a.p3, b.p3, c.p3, d.p3);
        T.t0 = sel4(k, a.t0, b.t0, c.t0, d.t0);
        T.t1 = sel4(k, a.t1, b.t1, c.t1, d.t1);
        T.t2 = sel4(k, a.t2, b.t2, c.t2, d.t2);
        T.t3 = sel4(k, a.t3, b.t3, c.t3, d.t3);
        return T;
    }
};

__device__ __forceinline__ int tab_type_of(const Tab& T, int v) {
    for (int k = 0; k < T.n; ++k)
        if (T.p(k) == v) return T.t(k);
    return -1;
}
__device__ __forceinline__ bool tab_has(const Tab& T, int v) {
    for (int k = 0; k < T.n; ++k)
        if (T.p(k) == v) return true;
    return false;
}
__device__ __forceinline__ int tab_count(const Tab& T, int t) {
    int c = 0;
    for (int k = 0; k < T.n; ++k) c += (T.t(k) == t);
    return c;
}
__device__ __forceinline__ bool type_ok(int rule_bead, int bead_type) { return rule_bead == 0 || rule_bead == bead_type; }
__device__ __forceinline__ bool in_mask(uint32_t m, int t) { return t >= 0 && t < 32 && ((m >> t) & 1u); }

// maxbond: a bead of type bead_type holding table T may store one more bond of type t
__device__ __forceinline__ bool max_ok(const Params& P, int bead_type, const Tab& T, int t) {
    for (int q = 0; q < P.nmax; ++q) {
        const MaxRule& m = P.maxr[q];
        if (m.bt == t && type_ok(m.bead, bead_type) && tab_count(T, t) >= m.max) return false;
    }
    return true;
}

__device__ __forceinline__ void stat_add(unsigned long long* st, int k, unsigned long long v) {
    if (v) atomicAdd(&st[k], v);
}

// ---- step 2: creation nomination -------------------------------------------------
// Every candidate that passes the float prefilter of the neighbour scan is
// re-tested with the exact double arithmetic of the method (minimum-image
// separation summed as (dx^2 + dy^2) + dz^2, strict comparison), then against the
// rules in call order (the last applicable one wins), maxbond on both beads and
// the graph distance; the closest survivor (ties: lower id) is nominated.

// bead types that some creation rule pairs with type ti (a superset of the
// partners that can pass every test: distance and maxbond are not looked at)
__device__ __forceinline__ uint32_t create_partner_types(const Params& P, int ti) {
    uint32_t m = 0;
    for (int q = 0; q < P.nrule; ++q) {
        const Rule& r = P.rule[q];
        if (r.kind != RK_CREATE && r.kind != RK_CREATEDIR) continue;
        if (type_ok(r.b1, ti)) m |= r.b2 == 0 ? 0xFFFFFFFFu : 1u << r.b2;
        if (type_ok(r.b2, ti)) m |= r.b1 == 0 ? 0xFFFFFFFFu : 1u << r.b1;
    }
    return m;
}

// some creation rule admits a bead of type ti holding table Ti in one of its two
// roles (type and maxbond)
__device__ __forceinline__ bool create_admits(const Params& P, int ti, const Tab& Ti) {
    for (int q = 0; q < P.nrule; ++q) {
        const Rule& r = P.rule[q];
        if (r.kind != RK_CREATE && r.kind != RK_CREATEDIR) continue;
        if ((type_ok(r.b1, ti) && max_ok(P, ti, Ti, r.bt1)) || (type_ok(r.b2, ti) && max_ok(P, ti, Ti, r.bt2)))
            return true;
    }
    return false;
}

// The beads that may nominate a creation partner (reactive, of a type some
// creation rule names, with room for one of its bond types under maxbond) are
// flagged by the breakage nomination (in S.act), which reads every bead's table
// anyway; the flagged beads are listed in slot order in S.aoff (their count at
// S.aoff[n]) by a stream compaction, so that the creation scan runs on full
// wavefronts.

// LANES threads per listed bead, each scanning a share of every cell run; the
// group's nominee is the least (r^2, id) of its members' nominees, which is what
// one thread scanning every run in any order would find.  The listed range is
// split per XCD; the workgroups step over the tiles of the list, so that a list
// longer than the grid's share is covered too.  The kernel picks LANES from the
// list's length: a list of half a million beads or more (the bases of a melted
// system) fills the GPU with one thread per bead (on the 4M-bead stress case 239
// against 300 us with two, 377 with four), a short one (a few melted bases among
// hybridized duplexes) needs sixteen to fill it at all.
__device__ __forceinline__ int create_lanes_for(int nl) {
    return nl >= (1 << 19) ? 1 : (nl >= (1 << 18) ? 2 : (nl >= (1 << 17) ? 4 : (nl >= (1 << 16) ? 8 : 16)));
}

// candidates a thread queues before examining them (more are examined at once)
constexpr int CREATE_QUEUE = 8;

template <bool BATCH, int LANES>
__device__ __forceinline__ void nominate_create_one(const Params& P, const int n, const Bank& B,
                                                    const int* __restrict__ cstart, const float4* __restrict__ xs,
                                                    const SweepBuf& S, const int i, const int lane,
                                                    int (*queue)[DB_BLOCK]) {
    const double4 xi = B.x[i];
    const int mi = meta_word(xi);
    const Box& X = box_of<BATCH>(P, mi);
    const int ti = meta_type(mi);
    const int gi = meta_gid(xi);
    int best = -1, best_rule = -1, best_bt = 0, best_g = 0;
    double best_r2 = 0.0;
    const Tab Ti = load_tab_all(B, n, i);
    {
        const float cut2 = X.pf_create2;
        // types and reactivity ride in the scan's words: most candidates are
        // rejected before anything else of them is read
        const uint32_t partner_types = create_partner_types(P, ti);
        // the beads two bonds away, gathered once for the distance-3 test
        int two[DB_MAXB * DB_MAXB];
#pragma unroll
        for (int a = 0; a < DB_MAXB; ++a) {
            const int q = Ti.p(a);
            const int nq = (!P.pc14 && a < Ti.n) ? B.nb[q] : 0;
#pragma unroll
            for (int b = 0; b < DB_MAXB; ++b) two[a * DB_MAXB + b] = b < nq ? B.bp[b * n + q] : -1;
        }
        // A candidate of a wanted type is queued and examined after the scan: taken
        // as found, the examination ran for every candidate any lane of the wave
        // kept, with the other lanes idle.  The nominee, the least (r^2, id), does
        // not depend on the order of the examinations.
        auto examine = [&](int j) {
            // the candidate's table is requested with its position (nearly every
            // examined candidate passes the distance and rule tests that need it)
            const double4 xj = B.x[j];
            const Tab Tj = load_tab_all(B, n, j);
            const int mj = meta_word(xj);
            double dx, dy, dz;
            const double r2 = separation(X, xi, xj, dx, dy, dz);
            if (!(r2 < P.rmax2_create)) return;
            const int tj = meta_type(mj);
            const int gj = meta_gid(xj);
            // last creation rule that applies to the pair
            int rule = -1, bti = 0;
            for (int q = 0; q < P.nrule; ++q) {
                const Rule& r = P.rule[q];
                if (r.kind != RK_CREATE && r.kind != RK_CREATEDIR) continue;
                bool o1 = type_ok(r.b1, ti) && type_ok(r.b2, tj);
                const bool o2 = type_ok(r.b1, tj) && type_ok(r.b2, ti);
                if (!o1 && !o2) continue;
                if (o1 && o2) o1 = gi < gj;   // both orientations: the lower id plays bead1
                const int si = o1 ? r.bt1 : r.bt2;
                const int sj = o1 ? r.bt2 : r.bt1;
                if (!(r2 < r.r2)) continue;
                if (!max_ok(P, ti, Ti, si)) continue;
                if (!max_ok(P, tj, Tj, sj)) continue;
                rule = q;
                bti = si;
            }
            if (rule < 0) return;
            // graph distance 1, 2 or 3 on the bond graph before the sweep
            if (tab_has(Ti, j)) return;
            bool d2 = false;
            for (int a = 0; a < Ti.n && !d2; ++a)
                if (tab_has(Tj, Ti.p(a))) d2 = true;
            if (d2 && !P.pc13) return;
            if (!d2 && !P.pc14) {
                // distance 3: a partner of j is a partner of a partner of i
                bool d3 = false;
#pragma unroll
                for (int b = 0; b < DB_MAXB; ++b) {
                    const int pj = Tj.p(b);
                    if (b < Tj.n) {
#pragma unroll
                        for (int k = 0; k < DB_MAXB * DB_MAXB; ++k) d3 |= two[k] == pj;
                    }
                }
                if (d3) return;
            }
            if (best < 0 || r2 < best_r2 || (r2 == best_r2 && gj < best_g)) {
                best = j;
                best_r2 = r2;
                best_g = gj;
                best_rule = rule;
                best_bt = bti;
            }
        };
        const int tid = threadIdx.x;
        int nq = 0;
        auto visit = [&](int j, int w) {
            if (!xs_reactive(w) || !((partner_types >> xs_type(w)) & 1u)) return;
            if (nq == CREATE_QUEUE) {   // full: examine the queue
                for (int k = 0; k < CREATE_QUEUE; ++k) examine(queue[k][tid]);
                nq = 0;
            }
            queue[nq][tid] = j;
            ++nq;
        };
        if (X.wide_create) scan_cells_wide<LANES, 1>(X, cstart, xs, i, xi, cut2, visit, lane);
        else scan_cells<LANES>(X, cstart, xs, i, xi, cut2, visit, lane);
        for (int k = 0; k < nq; ++k) examine(queue[k][tid]);
    }
    // the group's least (r^2, id), exchanged within the aligned group of lanes
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
        const double r2o = __shfl_xor(best_r2, o, 64);
        const int go = __shfl_xor(best_g, o, 64);
        const int jo = __shfl_xor(best, o, 64);
        const int ro = __shfl_xor(best_rule, o, 64);
        const int bo = __shfl_xor(best_bt, o, 64);
        if (jo >= 0 && (best < 0 || r2o < best_r2 || (r2o == best_r2 && go < best_g))) {
            best = jo;
            best_r2 = r2o;
            best_g = go;
            best_rule = ro;
            best_bt = bo;
        }
    }
    if (lane == 0) {
        S.nomC[i] = best;
        S.ruleC[i] = (int8_t)best_rule;
        S.btC[i] = (int8_t)best_bt;
    }
}

template <bool BATCH, int LANES>
__device__ __forceinline__ void nominate_create_all(const Params& P, const Bank& B, const int* __restrict__ cstart,
                                                    const float4* __restrict__ xs, const SweepBuf& S, int nl,
                                                    int (*queue)[DB_BLOCK]) {
    static_assert(64 % LANES == 0 && DB_BLOCK % 64 == 0, "groups lie within a wavefront");
    const int ntile = (int)(((long long)nl * LANES + DB_BLOCK - 1) / DB_BLOCK);
    for (int tb = blockIdx.x; tb < ntile; tb += gridDim.x) {
        const long long pos = (long long)xcd_tile(tb, ntile) * DB_BLOCK + threadIdx.x;
        const int t = (int)(pos / LANES);
        const int lane = (int)(pos % LANES);
        // the lanes of a group share t: they take this branch together
        if (t < nl) nominate_create_one<BATCH, LANES>(P, P.n, B, cstart, xs, S, S.aoff[t], lane, queue);
    }
}

template <bool BATCH>
__global__ __launch_bounds__(DB_BLOCK) void k_nominate_create(const Params* __restrict__ Pp, Bank B,
                                                              const int* __restrict__ cstart,
                                                              const float4* __restrict__ xs, SweepBuf S) {
    const Params& P = *Pp;
    const int nl = S.aoff[P.n];
    __shared__ int queue[CREATE_QUEUE][DB_BLOCK];   // a column per thread
    switch (create_lanes_for(nl)) {   // uniform over the grid
        case 1: nominate_create_all<BATCH, 1>(P, B, cstart, xs, S, nl, queue); break;
        case 2: nominate_create_all<BATCH, 2>(P, B, cstart, xs, S, nl, queue); break;
        case 4: nominate_create_all<BATCH, 4>(P, B, cstart, xs, S, nl, queue); break;
        case 8: nominate_create_all<BATCH, 8>(P, B, cstart, xs, S, nl, queue); break;
        default: nominate_create_all<BATCH, 16>(P, B, cstart, xs, S, nl, queue); break;
    }
}

// ---- steps 3 and 5: breakage nomination and killbond marks ----------------------
template <bool BATCH>
__global__ __launch_bounds__(DB_BLOCK) void k_nominate_break(const Params* __restrict__ Pp, Bank B, SweepBuf S) {
    const Params& P = *Pp;
    const int n = P.n;
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    double4 xi = B.x[i];
    int mi = meta_word(xi);
    const Box& X = box_of<BATCH>(P, mi);
    int gi = meta_gid(xi);
    int best = -1, best_rule = -1, best_g = 0;
    double best_r2 = 0.0;
    int rm = 0;
    unsigned long long killed_here = 0;
    // the bead's table with all rows requested at once, then the positions of the
    // partners whose bond type some breaking rule acts on, all in flight together
    const Tab Ti = load_tab_all(B, n, i);
    const bool scan_bonds = meta_reactive(mi) && (P.has_kill || P.has_break_class);
    double4 xp[DB_MAXB];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k)
        if (scan_bonds && k < Ti.n && ((P.break_types >> Ti.t(k)) & 1u)) xp[k] = B.x[Ti.p(k)];
    {
        // creation: flag the bead for the creation scan's list; its nomination starts empty
        const int ti = meta_type(mi);
        bool can = meta_reactive(mi) && ((P.create_types >> ti) & 1u) && P.rmax2_create > 0.0;
        if (can) can = create_admits(P, ti, Ti);
        S.act[i] = can ? 1 : 0;
        S.chg[i] = 0;
        S.tchg[i] = 0;
        S.npurge[i] = 0;
        S.ngen[i] = 0;
        S.nomC[i] = -1;
        S.ruleC[i] = -1;
        S.btC[i] = 0;
    }
    if (scan_bonds) {
        int ti = meta_type(mi);
#pragma unroll
        for (int k = 0; k < DB_MAXB; ++k) {
            if (k >= Ti.n || !((P.break_types >> Ti.t(k)) & 1u)) continue;
            int j = Ti.p(k), t = Ti.t(k);
            const double4 xj = xp[k];
            int mj = meta_word(xj);
            if (!meta_reactive(mj)) continue;
            double dx, dy, dz;
            double r2 = separation(X, xi, xj, dx, dy, dz);
            int gj = meta_gid(xj);
            bool killed = false;
            int rule = -1;
            // the partner's table is read only for a bond some rule could act on
            bool have_tj = false;
            Tab Tj{0, -1, -1, -1, -1, 0, 0, 0, 0};
            for (int q = 0; q < P.nrule; ++q) {
                const Rule& r = P.rule[q];
                if (r.bt1 != t || !(r2 > r.r2)) continue;
                if (r.kind == RK_KILL) {
                    killed = true;
                } else if (r.kind == RK_BREAK) {
                    rule = q;
                } else if (r.kind == RK_CONVERT) {
                    if (!have_tj) {
                        Tj = load_tab(B, n, j);
                        have_tj = true;
                    }
                    if (max_ok(P, ti, Ti, r.bt2) && max_ok(P, meta_type(mj), Tj, r.bt2)) rule = q;
                }
            }
            if (!killed && rule < 0) continue;
            if (!have_tj) Tj = load_tab(B, n, j);
            if (tab_type_of(Tj, i) != t) continue;   // only symmetric bonds break
            if (killed) {
                S.rmlist[rm * n + i] = j;
                ++rm;
                if (gi < gj) ++killed_here;
            }
            if (rule < 0) continue;
            if (best < 0 || r2 > best_r2 || (r2 == best_r2 && gj < best_g)) {
                best = j;
                best_r2 = r2;
                best_g = gj;
                best_rule = rule;
            }
        }
    }
    S.nomK[i] = best;
    S.ruleK[i] = (int8_t)best_rule;
    S.rmcnt[i] = (uint8_t)rm;
    stat_add(S.stats, ST_KILLED, killed_here);
}

// flag bead s, its bond partners and theirs (in the current tables); several
// beads may flag one bead, all with the same value
__device__ __forceinline__ void mark_two_bonds(const Bank& B, int n, int s, uint8_t* __restrict__ f) {
    f[s] = 1;
    const int nb = B.nb[s];
    for (int k = 0; k < nb; ++k) {
        const int q = B.bp[k * n + s];
        f[q] = 1;
        const int nq = B.nb[q];
        for (int m = 0; m < nq; ++m) f[B.bp[m * n + q]] = 1;
    }
}

// ---- step 5: mutual breakage nominations ----------------------------------------
template <bool BATCH>
__global__ __launch_bounds__(DB_BLOCK) void k_resolve(const Params* __restrict__ Pp, Bank B, SweepBuf S,
                                                      int64_t step) {
    const Params& P = *Pp;
    const int n = P.n;
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    int j = S.nomK[i];
    int conv = 0, newp = -1;
    if (j >= 0 && S.nomK[j] == i) {
        int rm = S.rmcnt[i];
        bool killed = false;
        for (int k = 0; k < rm; ++k)
            if (S.rmlist[k * n + i] == j) killed = true;   // killbond wins over the nomination
        if (!killed) {
            const double4 xi = B.x[i];
            int gi = meta_gid(xi), gj = meta_gid(B.x[j]);
            const Rule& r = P.rule[S.ruleK[i]];
            if (accept_number(P, box_of<BATCH>(P, meta_word(xi)), gi, gj, step, RNG_BREAK) < r.p) {
                S.rmlist[rm * n + i] = j;
                S.rmcnt[i] = (uint8_t)(rm + 1);
                if (r.kind == RK_CONVERT) {
                    conv = 1;
                    newp = j;
                    if (gi < gj) stat_add(S.stats, ST_CONVERTED, 1);
                } else if (gi < gj) {
                    stat_add(S.stats, ST_BROKEN, 1);
                }
            }
        }
    }
    S.conv[i] = (uint8_t)conv;
    S.newp[i] = newp;
    // every member of an angle or dihedral through a removed bond lies within two
    // bonds of one of that bond's ends, and both ends list the removal: they flag
    // those beads (the tables still hold the old graph), the only ones whose
    // tables the purge must read
    if (S.rmcnt[i] > 0) mark_two_bonds(B, n, i, S.npurge);
}

__device__ __forceinline__ bool bond_removed(const SweepBuf& S, int n, int u, int v) {
    int rm = S.rmcnt[u];
    for (int k = 0; k < rm; ++k)
        if (S.rmlist[k * n + u] == v) return true;
    return false;
}

// the same with u's removal count already read
__device__ __forceinline__ bool listed_removed(const SweepBuf& S, int n, int u, int rm, int v) {
    for (int k = 0; k < rm; ++k)
        if (S.rmlist[k * n + u] == v) return true;
    return false;
}

// ---- steps 6-8: purge, remove / convert, create ---------------------------------
template <bool BATCH>
__global__ __launch_bounds__(DB_BLOCK) void k_apply(const Params* __restrict__ Pp, Bank B, SweepBuf S, int64_t step,
                                                    int* __restrict__ err) {
    const Params& P = *Pp;
    const int n = P.n;
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    unsigned long long ang_del = 0, dih_del = 0;
    // removals of this sweep were all counted by the kernels before this one; with
    // none (the common case at low reaction density) no table needs editing
    const bool any_removed = (S.stats[ST_BROKEN] | S.stats[ST_KILLED] | S.stats[ST_CONVERTED]) != 0;
    int w = 0;
    bool purged = false;
    // step 6: angles and dihedrals crossing a removed bond (judged on the old graph)
    if (any_removed && S.npurge[i]) {
        // first which entries cross a removed bond: four entries and the removal
        // counts of their members are read together, before any row is moved
        static_assert(DB_MAXA <= 32 && DB_MAXD <= 32, "one bit per entry");
        const int na = B.na[i];
        uint32_t drop = 0;
        for (int k0 = 0; k0 < na; k0 += 4) {
            int4 e4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) e4[q] = B.ang[(k0 + q < na ? k0 + q : k0) * n + i];
            int rx[4], ry[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                rx[q] = S.rmcnt[e4[q].x];
                ry[q] = S.rmcnt[e4[q].y];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int4 e = e4[q];
                if (k0 + q < na && (listed_removed(S, n, e.x, rx[q], e.y) || listed_removed(S, n, e.y, ry[q], e.z))) {
                    drop |= 1u << (k0 + q);
                    if (e.y == i) ++ang_del;
                }
            }
        }
        // then the kept entries close up in order
        for (int k = 0; k < na; ++k) {
            if ((drop >> k) & 1u) continue;
            if (w != k) B.ang[w * n + i] = B.ang[k * n + i];
            ++w;
        }
        purged |= w != na;
        B.na[i] = (uint8_t)w;
        const int nd = B.nd[i];
        drop = 0;
        for (int k0 = 0; k0 < nd; k0 += 4) {
            int4 e4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) e4[q] = B.dih[(k0 + q < nd ? k0 + q : k0) * n + i];
            int rx[4], ry[4], rz[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                rx[q] = S.rmcnt[e4[q].x];
                ry[q] = S.rmcnt[e4[q].y];
                rz[q] = S.rmcnt[e4[q].z];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int4 e = e4[q];
                if (k0 + q < nd && (listed_removed(S, n, e.x, rx[q], e.y) || listed_removed(S, n, e.y, ry[q], e.z) ||
                                    listed_removed(S, n, e.z, rz[q], e.w))) {
                    drop |= 1u << (k0 + q);
                    if (e.y == i) ++dih_del;
                }
            }
        }
        w = 0;
        for (int k = 0; k < nd; ++k) {
            if ((drop >> k) & 1u) continue;
            if (w != k) {
                B.dih[w * n + i] = B.dih[k * n + i];
                B.dt[w * n + i] = B.dt[k * n + i];
            }
            ++w;
        }
        purged |= w != nd;
        B.nd[i] = (uint8_t)w;
    }
    // step 7: own bond entries (a conversion is listed among the removed entries)
    const int rm = S.rmcnt[i];
    const int conv = S.conv[i];
    const int nb = B.nb[i];
    w = nb;
    bool changed = false;   // the bead's bond graph changed (a conversion keeps it)
    if (rm > 0) {
        const int convp = conv ? S.newp[i] : -1;
        w = 0;
        for (int k = 0; k < nb; ++k) {
            int j = B.bp[k * n + i];
            int t = B.bt[k * n + i];
            if (bond_removed(S, n, i, j)) {
                changed |= j != convp;
                if (j != convp) continue;
                t = P.rule[S.ruleK[i]].bt2;   // converted: same partner, new type
            }
            B.bp[w * n + i] = j;
            B.bt[w * n + i] = (int8_t)t;
            ++w;
        }
    }
    // step 8: mutual creation nominations, no creation for converting beads
    int j = S.nomC[i];
    if (j >= 0 && !conv && S.nomC[j] == i && !S.conv[j]) {
        const double4 xi = B.x[i];
        int gi = meta_gid(xi), gj = meta_gid(B.x[j]);
        const Rule& r = P.rule[S.ruleC[i]];
        if (accept_number(P, box_of<BATCH>(P, meta_word(xi)), gi, gj, step, RNG_CREATE) < r.p) {
            if (w >= DB_MAXB) {
                atomicOr(err, ERR_BOND_CAP);
            } else {
                B.bp[w * n + i] = j;
                B.bt[w * n + i] = S.btC[i];
                ++w;
            }
            S.newp[i] = j;
            changed = true;
            if (gi < gj) stat_add(S.stats, ST_CREATED, 1);
        }
    }
    if (changed) S.chg[i] = 1;
    if (changed || purged) S.tchg[i] = 1;
    if (w != nb) B.nb[i] = (uint8_t)w;
    stat_add(S.stats, ST_ANG_DEL, ang_del);
    stat_add(S.stats, ST_DIH_DEL, dih_del);
}

// ---- step 9: angles / dihedrals on paths holding a new bond -----------------------
// Pattern match of section 2.  t(u->v) is the type u stores for its bond to v.
// Angle ABC: bead types match and t(B->A) in S1, t(B->C) in S2; else CBA.
// Dihedral ABCD: bead types match, t(B->A) in S1, t(C->B) or t(B->C) in S2,
// t(C->D) in S3; else DCBA.  The first rule in table order that matches wins.
// (nrule rules of the table at rules, which the generation pass keeps in LDS)
__device__ int match_angle(int nrule, const AngRule* rules, int ta, int tb, int tc, int t_ba, int t_bc) {
    for (int q = 0; q < nrule; ++q) {
        const AngRule& r = rules[q];
        if (type_ok(r.b[0], ta) && type_ok(r.b[1], tb) && type_ok(r.b[2], tc) && in_mask(r.m[0], t_ba) &&
            in_mask(r.m[1], t_bc))
            return r.type;
        if (type_ok(r.b[0], tc) && type_ok(r.b[1], tb) && type_ok(r.b[2], ta) && in_mask(r.m[0], t_bc) &&
            in_mask(r.m[1], t_ba))
            return r.type;
    }
    return 0;
}

__device__ int match_dihedral(int nrule, const DihRule* rules, int ta, int tb, int tc, int td, int t_ba, int t_bc,
                              int t_cb, int t_cd) {
    for (int q = 0; q < nrule; ++q) {
        const DihRule& r = rules[q];
        if (type_ok(r.b[0], ta) && type_ok(r.b[1], tb) && type_ok(r.b[2], tc) && type_ok(r.b[3], td) &&
            in_mask(r.m[0], t_ba) && (in_mask(r.m[1], t_cb) || in_mask(r.m[1], t_bc)) && in_mask(r.m[2], t_cd))
            return r.type;
        if (type_ok(r.b[0], td) && type_ok(r.b[1], tc) && type_ok(r.b[2], tb) && type_ok(r.b[3], ta) &&
            in_mask(r.m[0], t_cd) && (in_mask(r.m[1], t_bc) || in_mask(r.m[1], t_cb)) && in_mask(r.m[2], t_ba))
            return r.type;
    }
    return 0;
}

struct Gen {
    const Params& P;
    const Bank B;   // by value: a reference to the kernel argument would force a private copy
    const SweepBuf& S;
    int n;
    bool all;
    __device__ bool is_new(int u, int v) const { return all || S.newp[u] == v; }
    __device__ int type_of(int s) const { return meta_type(meta_word(B.x[s])); }
    __device__ int gid_of(int s) const { return meta_gid(B.x[s]); }
};

template <bool ALL>
__global__ __launch_bounds__(DB_BLOCK) void k_generate(const Params* __restrict__ Pp, Bank B, SweepBuf S,
                                                       int* __restrict__ err) {
    const Params& P = *Pp;
    const int n = P.n;
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (P.narule == 0 && P.ndrule == 0) return;
    // no bond was created or converted in this sweep: nothing to generate
    if (!ALL && (S.stats[ST_CREATED] | S.stats[ST_CONVERTED]) == 0) return;
    // only beads within two bonds of a new bond can lie on a qualifying path
    // (flagged by k_mark_new)
    const bool mine = i < n && (ALL || S.ngen[i]);
    // The pattern rules are matched from LDS: a workgroup holding a bead to work
    // on copies them once.  After a sweep few wavefronts run this pass, and read
    // from memory one rule at a time the rules cost a cache miss each.
    __shared__ AngRule sar[DB_MAXRULES];
    __shared__ DihRule sdr[DB_MAXRULES];
    if (!__syncthreads_or(mine)) return;
    for (int t = threadIdx.x; t < P.narule; t += DB_BLOCK) sar[t] = P.arule[t];
    for (int t = threadIdx.x; t < P.ndrule; t += DB_BLOCK) sdr[t] = P.drule[t];
    __syncthreads();
    if (!mine) return;
    const int nar = P.narule, ndr = P.ndrule;
    const Tab Ti = load_tab_all(B, n, i);
    Gen g{P, B, S, n, ALL};
    const int gi = g.gid_of(i), ti = g.type_of(i);
    // the partners' tables and types, requested together once (a missing
    // partner reads bead i's own, unused)
    Tab4 Tp;
    Tp.a = load_tab_all(B, n, Ti.n > 0 ? Ti.p0 : i);
    Tp.b = load_tab_all(B, n, Ti.n > 1 ? Ti.p1 : i);
    Tp.c = load_tab_all(B, n, Ti.n > 2 ? Ti.p2 : i);
    Tp.d = load_tab_all(B, n, Ti.n > 3 ? Ti.p3 : i);
    const int ty0 = g.type_of(Ti.n > 0 ? Ti.p0 : i), ty1 = g.type_of(Ti.n > 1 ? Ti.p1 : i);
    const int ty2 = g.type_of(Ti.n > 2 ? Ti.p2 : i), ty3 = g.type_of(Ti.n > 3 ? Ti.p3 : i);
    auto ptype = [&](int k) { return k == 0 ? ty0 : (k == 1 ? ty1 : (k == 2 ? ty2 : ty3)); };
    int na = B.na[i], nd = B.nd[i];
    const int na0 = na, nd0 = nd;
    unsigned long long ang_new = 0, dih_new = 0;
    bool overflow_a = false, overflow_d = false;
    auto push_angle = [&](int a, int b, int c, int type) {
        if (g.gid_of(a) > g.gid_of(c)) {
            int t = a;
            a = c;
            c = t;
        }
        if (na >= DB_MAXA) {
            overflow_a = true;
            return;
        }
        B.ang[na * n + i] = make_int4(a, b, c, type);
        ++na;
    };
    auto push_dih = [&](int a, int b, int c, int d, int type) -> bool {
        bool rev = g.gid_of(a) > g.gid_of(d);
        if (rev) {
            int t = a; a = d; d = t;
            t = b; b = c; c = t;
        }
        if (nd >= DB_MAXD) {
            overflow_d = true;
            return false;
        }
        B.dih[nd * n + i] = make_int4(a, b, c, d);
        B.dt[nd * n + i] = (uint8_t)type;
        ++nd;
        return b == i;
    };
    // angles with i in the centre
    if (P.narule) {
        for (int k1 = 0; k1 < Ti.n; ++k1)
            for (int k2 = k1 + 1; k2 < Ti.n; ++k2) {
                int a = Ti.p(k1), c = Ti.p(k2);
                if (a == c) continue;
                if (!(g.is_new(i, a) || g.is_new(i, c))) continue;
                int t = match_angle(nar, sar, ptype(k1), ti, ptype(k2), Ti.t(k1), Ti.t(k2));
                if (t) {
                    push_angle(a, i, c, t);
                    ++ang_new;
                }
            }
        // angles with i at an end: i - b - c
        for (int k = 0; k < Ti.n; ++k) {
            int b = Ti.p(k);
            const Tab Tb = Tp.get(k);
            int t_bi = tab_type_of(Tb, i);
            int tb = ptype(k);
            for (int m = 0; m < Tb.n; ++m) {
                int c = Tb.p(m);
                if (c == i) continue;
                if (!(g.is_new(i, b) || g.is_new(b, c))) continue;
                int t = match_angle(nar, sar, ti, tb, g.type_of(c), t_bi, Tb.t(m));
                if (t) push_angle(i, b, c, t);
            }
        }
    }
    if (P.ndrule) {
        // dihedrals with i at an end: i - b - c - d
        for (int k = 0; k < Ti.n; ++k) {
            int b = Ti.p(k);
            const Tab Tb = Tp.get(k);
            int t_bi = tab_type_of(Tb, i);
            int tb = ptype(k);
            for (int m = 0; m < Tb.n; ++m) {
                int c = Tb.p(m);
                if (c == i) continue;
                const Tab Tc = load_tab_all(B, n, c);
                int t_cb = tab_type_of(Tc, b);
                int tc = g.type_of(c);
                for (int q = 0; q < Tc.n; ++q) {
                    int d = Tc.p(q);
                    if (d == b || d == i) continue;
                    if (!(g.is_new(i, b) || g.is_new(b, c) || g.is_new(c, d))) continue;
                    int t = match_dihedral(ndr, sdr, ti, tb, tc, g.type_of(d), t_bi, Tb.t(m), t_cb, Tc.t(q));
                    if (t) push_dih(i, b, c, d, t);
                }
            }
        }
        // dihedrals with i second: a - i - c - d
        for (int k1 = 0; k1 < Ti.n; ++k1) {
            int a = Ti.p(k1);
            int ta = ptype(k1);
            for (int k2 = 0; k2 < Ti.n; ++k2) {
                if (k2 == k1) continue;
                int c = Ti.p(k2);
                if (c == a) continue;
                const Tab Tc = Tp.get(k2);
                int t_ci = tab_type_of(Tc, i);
                int tc = ptype(k2);
                for (int q = 0; q < Tc.n; ++q) {
                    int d = Tc.p(q);
                    if (d == i || d == a) continue;
                    if (!(g.is_new(a, i) || g.is_new(i, c) || g.is_new(c, d))) continue;
                    int t = match_dihedral(ndr, sdr, ta, ti, tc, g.type_of(d), Ti.t(k1), Ti.t(k2), t_ci, Tc.t(q));
                    if (t && push_dih(a, i, c, d, t)) ++dih_new;
                }
            }
        }
    }
    // the counters above count an entry at its centre only; the halo follows any
    // entry appended to this bead's tables, whatever its role
    if (!ALL && (na != na0 || nd != nd0)) S.tchg[i] = 1;
    B.na[i] = (uint8_t)na;
    B.nd[i] = (uint8_t)nd;
    if (overflow_a) atomicOr(err, ERR_ANGLE_CAP);
    if (overflow_d) atomicOr(err, ERR_DIH_CAP);
    if (!ALL) {
        stat_add(S.stats, ST_ANG_NEW, ang_new);
        stat_add(S.stats, ST_DIH_NEW, dih_new);
    }
    (void)gi;
}

// the beads within two bonds of a bond this sweep created or converted, from the
// new tables (both ends hold it); nothing when the sweep made no bond
__global__ __launch_bounds__(DB_BLOCK) void k_mark_new(int n, Bank B, SweepBuf S) {
    const int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    if ((S.stats[ST_CREATED] | S.stats[ST_CONVERTED]) == 0) return;
    if (S.newp[i] >= 0) mark_two_bonds(B, n, i, S.ngen);
}

__global__ void k_clear_angles(int n, uint8_t* na, uint8_t* nd) {
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i < n) {
        na[i] = 0;
        nd[i] = 0;
    }
}

static unsigned grid_for(int n) { return (unsigned)((n + DB_BLOCK - 1) / DB_BLOCK); }

template <bool BATCH>
static void sweep_kernels(db_ctx* c, const Bank& B, unsigned g, int64_t step) {
    hipStream_t s = c->stream;
    hipLaunchKernelGGL(k_nominate_break<BATCH>, dim3(g), dim3(DB_BLOCK), 0, s, c->dp, B, c->sw);
    launch_compact(c->sw.act, c->n, c->sw.aoff, c->sw.aoff + c->n, c->cells.blocksum, s);
    hipLaunchKernelGGL(k_nominate_create<BATCH>, dim3(g), dim3(DB_BLOCK), 0, s, c->dp, B, c->cells.start,
                       c->cells.xs, c->sw);
    hipLaunchKernelGGL(k_resolve<BATCH>, dim3(g), dim3(DB_BLOCK), 0, s, c->dp, B, c->sw, step);
    hipLaunchKernelGGL(k_apply<BATCH>, dim3(g), dim3(DB_BLOCK), 0, s, c->dp, B, c->sw, step, c->err_d);
}

void launch_sweep(db_ctx* c, int64_t step) {
    if (c->n == 0) return;
    // the halo follows any topology event of this sweep; a second sweep before the
    // next build would reset the counters of the first, so then rebuild regardless
    if (c->halo_sweep) c->halo_force = true;
    c->halo_sweep = true;
    hipStream_t s = c->stream;
    Bank& B = c->bank[c->cur];
    unsigned g = grid_for(c->n);
    if (c->nrep > 0) sweep_kernels<true>(c, B, g, step);
    else sweep_kernels<false>(c, B, g, step);
    if (c->hp.narule || c->hp.ndrule) {
        hipLaunchKernelGGL(k_mark_new, dim3(g), dim3(DB_BLOCK), 0, s, c->n, B, c->sw);
        hipLaunchKernelGGL(k_generate<false>, dim3(g), dim3(DB_BLOCK), 0, s, c->dp, B, c->sw, c->err_d);
    }
}

void launch_generate_all(db_ctx* c) {
    if (c->n == 0) return;
    hipStream_t s = c->stream;
    Bank& B = c->bank[c->cur];
    unsigned g = grid_for(c->n);
    hipLaunchKernelGGL(k_clear_angles, dim3(g), dim3(DB_BLOCK), 0, s, c->n, B.na, B.nd);
    hipLaunchKernelGGL(k_generate<true>, dim3(g), dim3(DB_BLOCK), 0, s, c->dp, B, c->sw, c->err_d);
    c->halo_force = true;
}

// ---- canonical output lists: each bond / angle / dihedral is emitted once -------
// owner: bonds by the bead with the lower id, angles by the centre, dihedrals by
// the second bead of the canonical (a < d) orientation.  Per-bead counts, an
// exclusive scan, then every owner writes its entries at its offset.
__global__ __launch_bounds__(DB_BLOCK) void k_count_owned(int n, int kind, Bank B, int* __restrict__ cnt) {
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    if (kind == 0) {
        int gi = meta_gid(B.x[i]);
        int nb = B.nb[i];
        for (int k = 0; k < nb; ++k) c += gi < meta_gid(B.x[B.bp[k * n + i]]);
    } else if (kind == 1) {
        int na = B.na[i];
        for (int k = 0; k < na; ++k) c += B.ang[k * n + i].y == i;
    } else {
        int nd = B.nd[i];
        for (int k = 0; k < nd; ++k) c += B.dih[k * n + i].y == i;
    }
    cnt[i] = c;
}

__global__ __launch_bounds__(DB_BLOCK) void k_write_owned(int n, int kind, Bank B, const int* __restrict__ off,
                                                          int32_t* __restrict__ tup, int32_t* __restrict__ typ) {
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    int o = off[i];
    int gi = meta_gid(B.x[i]);
    if (kind == 0) {
        int nb = B.nb[i];
        for (int k = 0; k < nb; ++k) {
            int j = B.bp[k * n + i];
            int gj = meta_gid(B.x[j]);
            if (!(gi < gj)) continue;
            int tji = -1;
            int nbj = B.nb[j];
            for (int m = 0; m < nbj; ++m)
                if (B.bp[m * n + j] == i) tji = B.bt[m * n + j];
            tup[2 * o] = gi;
            tup[2 * o + 1] = gj;
            typ[2 * o] = B.bt[k * n + i];
            typ[2 * o + 1] = tji;
            ++o;
        }
    } else if (kind == 1) {
        int na = B.na[i];
        for (int k = 0; k < na; ++k) {
            int4 e = B.ang[k * n + i];
            if (e.y != i) continue;
            tup[3 * o] = meta_gid(B.x[e.x]);
            tup[3 * o + 1] = gi;
            tup[3 * o + 2] = meta_gid(B.x[e.z]);
            typ[o] = e.w;
            ++o;
        }
    } else {
        int nd = B.nd[i];
        for (int k = 0; k < nd; ++k) {
            int4 e = B.dih[k * n + i];
            if (e.y != i) continue;
            tup[4 * o] = meta_gid(B.x[e.x]);
            tup[4 * o + 1] = gi;
            tup[4 * o + 2] = meta_gid(B.x[e.z]);
            tup[4 * o + 3] = meta_gid(B.x[e.w]);
            typ[o] = B.dt[k * n + i];
            ++o;
        }
    }
}

// counts of owned entries -> offsets in c->scan_buf (n + 1 ints; [n] = total)
void launch_owned_offsets(db_ctx* c, int kind, int* buf) {
    if (c->n == 0) return;
    unsigned g = grid_for(c->n);
    hipLaunchKernelGGL(k_count_owned, dim3(g), dim3(DB_BLOCK), 0, c->stream, c->n, kind, c->bank[c->cur], buf);
    launch_exclusive_scan(buf, c->n, nullptr, c->cells.blocksum, c->stream);
}

void launch_write_owned(db_ctx* c, int kind, const int* off, int32_t* tup, int32_t* typ) {
    if (c->n == 0) return;
    unsigned g = grid_for(c->n);
    hipLaunchKernelGGL(k_write_owned, dim3(g), dim3(DB_BLOCK), 0, c->stream, c->n, kind, c->bank[c->cur], off, tup,
                       typ);
}

}  // namespace db
