// Device-side helpers of libdynbond: counter-based random numbers, minimum
// image, bead metadata packing, workgroup-to-XCD mapping.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "db_internal.h"

namespace db {

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two 32x32->64
// multiplies with the published multipliers, key schedule bumped by the Weyl
// constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// counter layout: (a, b, step low word, step high bits | stream tag << 28)
// a and b are bead ids within the box; the key is the box's seed
__device__ __forceinline__ uint4 rng_draw(const Box& X, uint32_t a, uint32_t b, int64_t step, uint32_t kind) {
    uint64_t st = (uint64_t)step;
    uint4 c = make_uint4(a, b, (uint32_t)st, ((uint32_t)(st >> 32) & 0x0FFFFFFFu) | (kind << 28));
    return philox4x32_10(c, X.seed_lo, X.seed_hi);
}

// uniform in [0,1) with 53 random bits, drawn for the unordered pair {ga, gb}
// of global ids, both in box X
__device__ __forceinline__ double pair_uniform(const Box& X, int ga, int gb, int64_t step, uint32_t kind) {
    ga -= X.gid_off;
    gb -= X.gid_off;
    uint32_t lo = (uint32_t)(ga < gb ? ga : gb), hi = (uint32_t)(ga < gb ? gb : ga);
    uint4 w = rng_draw(X, lo, hi, step, kind);
    uint64_t bits = ((((uint64_t)w.x) << 32) | (uint64_t)w.y) >> 11;
    return (double)bits * (1.0 / 9007199254740992.0);
}

// uniform in [0,1) with 53 random bits drawn by one bead (global id g) alone: its
// counter names the bead twice, which no pair draw does
__device__ __forceinline__ double bead_uniform(const Box& X, int g, int64_t step, uint32_t kind) {
    g -= X.gid_off;
    uint4 w = rng_draw(X, (uint32_t)g, (uint32_t)g, step, kind);
    uint64_t bits = ((((uint64_t)w.x) << 32) | (uint64_t)w.y) >> 11;
    return (double)bits * (1.0 / 9007199254740992.0);
}

// The number a mutual pair compares with its rule's probability (appendix steps
// 5 and 7): one uniform for the pair, or in the literal form of the appendix the
// mean of one uniform per bead.  Both beads form the same value (the sum is taken
// lower id first, though IEEE addition does not depend on the order).
__device__ __forceinline__ double accept_number(const Params& P, const Box& X, int ga, int gb, int64_t step,
                                                uint32_t kind) {
    if (!P.accept_average) return pair_uniform(X, ga, gb, step, kind);
    const int lo = ga < gb ? ga : gb, hi = ga < gb ? gb : ga;
    return (bead_uniform(X, lo, step, kind) + bead_uniform(X, hi, step, kind)) * 0.5;
}

// Standard normal for the unordered pair {ga, gb} of global ids in box X at a
// step (DPD random force): the Box-Muller transform (Box and Muller, 1958) of the
// first two words, each taken to (0, 1) as (w + 1/2) / 2^32.  Both beads of the
// pair draw the same value.
__device__ __forceinline__ uint4 pair_draw(const Box& X, int ga, int gb, int64_t step, uint32_t kind) {
    ga -= X.gid_off;
    gb -= X.gid_off;
    return rng_draw(X, (uint32_t)(ga < gb ? ga : gb), (uint32_t)(ga < gb ? gb : ga), step, kind);
}
__device__ __forceinline__ double pair_gaussian(const Box& X, int ga, int gb, int64_t step) {
    const uint4 w = pair_draw(X, ga, gb, step, RNG_DPD);
    const double s32 = 1.0 / 4294967296.0;
    const double u1 = ((double)w.x + 0.5) * s32, u2 = ((double)w.y + 0.5) * s32;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
// single-precision form for the mixed path: the hardware base-2 logarithm and the
// hardware cosine, whose argument is in turns (cos 2 pi u)
__device__ __forceinline__ float pair_gaussian_f(const Box& X, int ga, int gb, int64_t step) {
    const uint4 w = pair_draw(X, ga, gb, step, RNG_DPD);
    const float s32 = 1.0f / 4294967296.0f;
    const float u1 = ((float)w.x + 0.5f) * s32, u2 = ((float)w.y + 0.5f) * s32;
    return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1)) * __builtin_amdgcn_cosf(u2);
}

// both shifted values are formed and one is selected, so the compiler emits
// selects rather than divergent branches; the result is bit-identical to the
// branching form
__device__ __forceinline__ double min_image(double d, double L, double hL) {
    const double lo = d - L, hi = d + L;
    double r = d > hL ? lo : d;
    return d < -hL ? hi : r;
}

// x_j - x_i with the minimum-image convention, and its squared length summed
// as (dx^2 + dy^2) + dz^2 (the order the cutoff decisions are defined in)
__device__ __forceinline__ double separation(const Box& X, const double4& xi, const double4& xj, double& dx,
                                             double& dy, double& dz) {
    dx = min_image(xj.x - xi.x, X.L, X.hL);
    dy = min_image(xj.y - xi.y, X.L, X.hL);
    dz = min_image(xj.z - xi.z, X.L, X.hL);
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ int meta_gid(const double4& x) {
    return (int)(uint32_t)((unsigned long long)__double_as_longlong(x.w));
}
__device__ __forceinline__ int meta_word(const double4& x) {
    return (int)(uint32_t)(((unsigned long long)__double_as_longlong(x.w)) >> 32);
}
__device__ __forceinline__ int meta_type(int m) { return m & 0xFF; }
__device__ __forceinline__ int meta_reactive(int m) { return (m >> 8) & 1; }
__device__ __forceinline__ int meta_rep(int m) { return (int)((uint32_t)m >> 16); }

// low word: global bead id; high word: type | reactive << 8 | replica << 16
__host__ __device__ inline double pack_meta(int gid, int type, int reactive, int rep = 0) {
    unsigned long long bits = (unsigned long long)(uint32_t)gid |
                              ((unsigned long long)(uint32_t)(type | (reactive << 8) | (rep << 16)) << 32);
    double d;
    __builtin_memcpy(&d, &bits, sizeof(d));
    return d;
}

// The word stored with each entry of the cell-ordered float position copy: the
// slot, the bead type and the reactive flag, so that scans can reject candidates
// by type before reading anything else of them.
__device__ __forceinline__ float xs_word(int slot, int meta) {
    return __int_as_float((int)((uint32_t)slot | ((uint32_t)meta_type(meta) << DB_SLOT_BITS) |
                                ((uint32_t)meta_reactive(meta) << 31)));
}
__device__ __forceinline__ int xs_slot(int w) { return w & DB_MAX_BEADS; }
__device__ __forceinline__ int xs_type(int w) { return (int)(((uint32_t)w >> DB_SLOT_BITS) & 31u); }
__device__ __forceinline__ bool xs_reactive(int w) { return ((uint32_t)w >> 31) != 0u; }

// The box of a bead: the system's own, or in a batch the replica's (BATCH is a
// template flag of the kernels, so the single-system path reads uniform values).
template <bool BATCH>
__device__ __forceinline__ const Box& box_of(const Params& P, int meta) {
    if (BATCH) return P.rep[meta_rep(meta)];
    return P.box;
}

// f(X) with the box of the lane's bead.  In a batch, a wave whose beads all lie in
// one replica (every wave but those that straddle a boundary between replicas)
// reads the replica's box with scalar loads into scalar registers, as the
// single-system path does; the others read it per lane.
template <bool BATCH, class F>
__device__ __forceinline__ void with_box(const Params& P, int meta, F&& f) {
    if constexpr (!BATCH) {
        f(P.box);
    } else {
        const int rep = meta_rep(meta);
        const int ru = __builtin_amdgcn_readfirstlane(rep);
        if (__builtin_amdgcn_ballot_w64(rep != ru) == 0) {
            // word by word through the constant address space: the table is never
            // written by a kernel, and a uniform load from there is a scalar load
            using CWord = __attribute__((address_space(4))) const uint32_t;
            static_assert(sizeof(Box) % 4 == 0, "box of whole words");
            constexpr int NW = (int)(sizeof(Box) / 4);
            const CWord* src = (const CWord*)(P.rep) + (size_t)ru * NW;
            uint32_t w[NW];
#pragma unroll
            for (int k = 0; k < NW; ++k) w[k] = src[k];
            Box X;
            __builtin_memcpy(&X, w, sizeof(Box));
            f(X);
        } else {
            f(P.rep[rep]);
        }
    }
}

// temperature of box X at a step: T0 + (T1 - T0) min(step, ramp) / ramp
__device__ __forceinline__ double box_temperature(const Box& X, int64_t step) {
    if (X.ramp <= 0) return X.T0;
    int64_t k = step < X.ramp ? step : X.ramp;
    return X.T0 + (X.T1 - X.T0) * (double)k / (double)X.ramp;
}

// Workgroups are dealt round-robin to the 8 XCDs.  Map them so that each XCD
// processes one contiguous range of tiles and neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    int per = nblocks >> 3;
    int full = per << 3;
    if (bid >= full) return bid;           // the tail keeps its own index
    return (bid & 7) * per + (bid >> 3);   // XCD (bid % 8) owns tiles [x*per, (x+1)*per)
}

// cell coordinate of x in [0, nc): every input, NaN and infinities included, lands
// in range without an out-of-range conversion (a non-finite position is reported
// by the step kernel after its block; the cell build of the next block may read it
// before the host stops)
__device__ __forceinline__ int cell_coord(double x, double scale, int nc) {
    const double t = x * scale;
    return t >= 0.0 ? (t < (double)nc ? (int)t : nc - 1) : 0;
}

// neighbour offset k < 3 of box X by selects (an indexed read would place a box
// held in registers in scratch memory)
__device__ __forceinline__ int box_off(const Box& X, int k) { return k == 0 ? X.off[0] : (k == 1 ? X.off[1] : X.off[2]); }

__device__ __forceinline__ int wrap_cell(int c, int nc) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); }

// position update with the periodic wrap into [0, L)
__device__ __forceinline__ double wrap1(double x, double L) {
    const double lo = x - L;
    double y = x + L;
    y = y >= L ? 0.0 : y;
    double r = x < 0.0 ? y : x;
    return x >= L ? lo : r;
}

}  // namespace db
