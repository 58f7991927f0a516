// Cell list (counting sort of beads by cell) and spatial reordering of the
// per-bead state.  The cell edge is at least the longest reaction distance and
// at least the pair cutoff plus a skin, so a bead's partners within reach lie in
// its own or the adjacent cells (the neighbour structure needs a communication
// distance at least as long as the longest reaction distance, appendix).
#include "db_device.h"

namespace db {

__global__ void k_fill_int(int* __restrict__ p, int value, size_t count) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

void launch_fill_int(int* p, int value, size_t count, hipStream_t s) {
    if (count == 0) return;
    unsigned blocks = (unsigned)((count + DB_BLOCK - 1) / DB_BLOCK);
    hipLaunchKernelGGL(k_fill_int, dim3(blocks), dim3(DB_BLOCK), 0, s, p, value, count);
}

// ---- binning -----------------------------------------------------------------
// The run of equal keys around this lane within its wavefront: [start, end) lanes.
__device__ __forceinline__ void wave_run(int key, int lane, int& start, int& end) {
    const int prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || prev != key;
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    start = 63 - __clzll(heads & upto);
    const unsigned long long after = start == 63 ? 0ull : (heads & ~((2ull << start) - 1ull));
    end = after ? __ffsll((long long)after) - 1 : 64;
}

// Cell of every bead and its rank among the beads of that cell.  Beads in slot
// order are mostly sorted by cell, so neighbouring lanes of a wavefront usually
// share a cell: each run of equal cells takes one atomic for the whole run and
// hands out consecutive ranks.  (Counting the beads per scan tile of cells here as
// well costs far more than a pass of its own: thousands of waves then add into
// each of a few words, and atomics on one word from all XCDs are serialised.)
template <bool BATCH>
__global__ __launch_bounds__(DB_BLOCK) void k_bin(const Params* __restrict__ Pp, const double4* __restrict__ x,
                                                   int* __restrict__ cellid, int* __restrict__ rank,
                                                   int* __restrict__ cnt) {
    const Params& P = *Pp;
    const int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int c = -1;
    if (i < P.n) {
        const double4 xi = x[i];
        const Box& X = box_of<BATCH>(P, meta_word(xi));
        const int cx = cell_coord(xi.x, X.cell_scale, X.nc);
        const int cy = cell_coord(xi.y, X.cell_scale, X.nc);
        const int cz = cell_coord(xi.z, X.cell_scale, X.nc);
        c = X.cell_off + (cz * X.nc + cy) * X.nc + cx;
    }
    int start, end;
    wave_run(c, lane, start, end);
    int base = 0;
    if (lane == start && c >= 0) base = atomicAdd(&cnt[c], end - start);
    base = __shfl(base, start, 64);
    if (i < P.n) {
        cellid[i] = c;
        rank[i] = base + (lane - start);
    }
}

// ---- exclusive scan in two launches -------------------------------------------
// Tiles of 4096 items: 256 threads of 16 consecutive items each.  The first launch
// sums every tile; in the second every tile adds up the sums of the tiles before
// it (from L2: at most one int per thread up to a million items, 128 for the
// largest cell grid) and scans its own items on top.
#define SCAN2_ITEMS 16
#define SCAN2_TILE 4096
static_assert(SCAN2_TILE == DB_BLOCK * SCAN2_ITEMS, "a scan tile is one workgroup's items");

__device__ __forceinline__ int wave_inclusive_scan(int v) {
    // Hillis-Steele over the 64 lanes of a wavefront
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// The 16 items of one thread; a thread reads and writes only its own items, so
// that a scan may run in place.
__device__ __forceinline__ void load_items(const int* in, int base, int count, int (&v)[SCAN2_ITEMS]) {
    if (base + SCAN2_ITEMS <= count && (reinterpret_cast<uintptr_t>(in) & 15) == 0) {
        const int4* p = reinterpret_cast<const int4*>(in + base);
#pragma unroll
        for (int q = 0; q < SCAN2_ITEMS / 4; ++q) {
            const int4 a = p[q];
            v[4 * q] = a.x;
            v[4 * q + 1] = a.y;
            v[4 * q + 2] = a.z;
            v[4 * q + 3] = a.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < SCAN2_ITEMS; ++k) v[k] = base + k < count ? in[base + k] : 0;
    }
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// this thread's share of the sum of the tile sums tsum[0..b): the threads of a
// workgroup take every DB_BLOCK-th one, four at a time
__device__ __forceinline__ int thread_share_before(const int* __restrict__ tsum, int b, int tid) {
    int p0 = 0, p1 = 0, p2 = 0, p3 = 0;
    int k = tid;
    for (; k + 3 * DB_BLOCK < b; k += 4 * DB_BLOCK) {
        p0 += tsum[k];
        p1 += tsum[k + DB_BLOCK];
        p2 += tsum[k + 2 * DB_BLOCK];
        p3 += tsum[k + 3 * DB_BLOCK];
    }
    for (; k < b; k += DB_BLOCK) p0 += tsum[k];
    return p0 + ((p1 + p2) + p3);
}

// tsum[b] = sum of tile b's items
__global__ __launch_bounds__(DB_BLOCK) void k_scan_tile_sums(const int* __restrict__ in, int count,
                                                             int* __restrict__ tsum) {
    __shared__ int wsum[DB_BLOCK / 64];
    int v[SCAN2_ITEMS];
    load_items(in, blockIdx.x * SCAN2_TILE + threadIdx.x * SCAN2_ITEMS, count, v);
    int local = 0;
#pragma unroll
    for (int k = 0; k < SCAN2_ITEMS; ++k) local += v[k];
    local = wave_sum(local);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
#pragma unroll
        for (int w = 0; w < DB_BLOCK / 64; ++w) t += wsum[w];
        tsum[blockIdx.x] = t;
    }
}

// Tile b: the sum of the totals of tiles 0..b-1 (every tile adds them up itself),
// then the tile's own exclusive scan on top.  The last tile writes the total of
// all items to total (when not null).  in == out is allowed.
__global__ __launch_bounds__(DB_BLOCK) void k_scan_apply(const int* in, int* out, int count,
                                                         const int* __restrict__ tsum, int* __restrict__ total) {
    __shared__ int wpre[DB_BLOCK / 64], wtot[DB_BLOCK / 64];
    const int b = blockIdx.x, tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    int pre = thread_share_before(tsum, b, tid);
    const int base = b * SCAN2_TILE + tid * SCAN2_ITEMS;
    int v[SCAN2_ITEMS];
    load_items(in, base, count, v);
    int local = 0;
#pragma unroll
    for (int k = 0; k < SCAN2_ITEMS; ++k) local += v[k];
    pre = wave_sum(pre);
    const int incl = wave_inclusive_scan(local);
    if (lane == 0) wpre[wid] = pre;
    if (lane == 63) wtot[wid] = incl;
    __syncthreads();
    int run = incl - local;
#pragma unroll
    for (int w = 0; w < DB_BLOCK / 64; ++w) run += wpre[w] + (w < wid ? wtot[w] : 0);
    int o[SCAN2_ITEMS];
#pragma unroll
    for (int k = 0; k < SCAN2_ITEMS; ++k) {
        o[k] = run;
        run += v[k];
    }
    if (base + SCAN2_ITEMS <= count && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
        int4* p = reinterpret_cast<int4*>(out + base);
#pragma unroll
        for (int q = 0; q < SCAN2_ITEMS / 4; ++q) p[q] = make_int4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < SCAN2_ITEMS; ++k)
            if (base + k < count) out[base + k] = o[k];
    }
    // items past count are zero, so the last thread's running sum is the total
    if (total && b == (int)gridDim.x - 1 && tid == DB_BLOCK - 1) *total = run;
}

// The same pass for a stream compaction: flags in[0..count) (0 or 1) give each
// flagged item its place, and the item's index is written there; the last tile
// writes the number of flagged items to total.  list must not overlap in.
__global__ __launch_bounds__(DB_BLOCK) void k_compact_apply(const int* __restrict__ in, int* __restrict__ list,
                                                            int count, const int* __restrict__ tsum,
                                                            int* __restrict__ total) {
    __shared__ int wpre[DB_BLOCK / 64], wtot[DB_BLOCK / 64];
    const int b = blockIdx.x, tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    int pre = thread_share_before(tsum, b, tid);
    const int base = b * SCAN2_TILE + tid * SCAN2_ITEMS;
    int v[SCAN2_ITEMS];
    load_items(in, base, count, v);
    int local = 0;
#pragma unroll
    for (int k = 0; k < SCAN2_ITEMS; ++k) local += v[k];
    pre = wave_sum(pre);
    const int incl = wave_inclusive_scan(local);
    if (lane == 0) wpre[wid] = pre;
    if (lane == 63) wtot[wid] = incl;
    __syncthreads();
    int run = incl - local;
#pragma unroll
    for (int w = 0; w < DB_BLOCK / 64; ++w) run += wpre[w] + (w < wid ? wtot[w] : 0);
#pragma unroll
    for (int k = 0; k < SCAN2_ITEMS; ++k) {
        if (v[k]) list[run] = base + k;   // items past count are zero
        run += v[k];
    }
    if (b == (int)gridDim.x - 1 && tid == DB_BLOCK - 1) *total = run;
}

static int scan2_tiles(int count) { return (count + SCAN2_TILE - 1) / SCAN2_TILE; }

// two-launch scan; tsum holds scan2_tiles(count) ints
static void scan2(const int* in, int* out, int count, int* tsum, hipStream_t s, int* total) {
    const int tiles = scan2_tiles(count);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(tiles), dim3(DB_BLOCK), 0, s, in, count, tsum);
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(DB_BLOCK), 0, s, in, out, count, tsum, total);
}

// out[0..count) = exclusive prefix sums of in[0..count), out[count] = their total;
// blocksum holds at least ceil(count / 4096) ints
void launch_scan_total(const int* in, int* out, int count, int* blocksum, hipStream_t s) {
    if (count <= 0) {
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, out, 0, (size_t)1);
        return;
    }
    scan2(in, out, count, blocksum, s, out + count);
}

// list[0..m) = the indices k < count with flags[k] = 1, ascending, and *total = m
// (two launches; blocksum holds at least ceil(count / 4096) ints)
void launch_compact(const int* flags, int count, int* list, int* total, int* blocksum, hipStream_t s) {
    if (count <= 0) {
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(1), 0, s, total, 0, (size_t)1);
        return;
    }
    const int tiles = scan2_tiles(count);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(tiles), dim3(DB_BLOCK), 0, s, flags, count, blocksum);
    hipLaunchKernelGGL(k_compact_apply, dim3(tiles), dim3(DB_BLOCK), 0, s, flags, list, count, blocksum, total);
}

// data[0..count) -> exclusive prefix sums in place, and the total in data[count]
void launch_exclusive_scan(int* data, int count, int* total_out, int* blocksum, hipStream_t s) {
    (void)total_out;
    if (count <= 0) return;
    scan2(data, data, count, blocksum, s, data + count);
}

// ---- scatter and in-cell ordering --------------------------------------------
// the bead's place in the unsorted list from its cell start and rank; the first
// bead of every cell clears the count for the next build (the scan has consumed it)
__global__ __launch_bounds__(DB_BLOCK) void k_scatter(int n, const int* __restrict__ cellid,
                                                       const int* __restrict__ rank, const int* __restrict__ start,
                                                       int* __restrict__ cnt, int* __restrict__ unsorted,
                                                       unsigned long long* __restrict__ stats) {
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (i < 8) stats[i] = 0ull;   // the counters of the sweep that follows this build
    if (i >= n) return;
    const int c = cellid[i], k = rank[i];
    unsorted[start[c] + k] = i;
    if (k == 0) cnt[c] = 0;
}

// Ascending slot order inside each cell makes the list independent of the
// arrival order of the atomics above.  One thread per entry of the unsorted
// list: the entry's place in its cell is the number of the cell's entries with a
// smaller slot.  The float copy of the positions is written in list order, so a
// scan over neighbouring cells reads contiguous runs.
__global__ __launch_bounds__(DB_BLOCK) void k_cellsort(int n, const int* __restrict__ start,
                                                        const int* __restrict__ cellid,
                                                        const int* __restrict__ unsorted, int* __restrict__ list,
                                                        const double4* __restrict__ x, float4* __restrict__ xs) {
    const int t = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (t >= n) return;
    const int j = unsorted[t];
    const double4 xj = x[j];
    const int c = cellid[j];
    const int s0 = start[c], s1 = start[c + 1];
    int r = 0;
    for (int k = s0; k < s1; ++k) r += unsorted[k] < j ? 1 : 0;
    list[s0 + r] = j;
    xs[s0 + r] = make_float4((float)xj.x, (float)xj.y, (float)xj.z, xs_word(j, meta_word(xj)));
}

void launch_build_cells(db_ctx* c) {
    const int n = c->n;
    const int ncell = c->hp.ncell;
    hipStream_t s = c->stream;
    db::Bank& B = c->bank[c->cur];
    unsigned nb = (unsigned)((n + DB_BLOCK - 1) / DB_BLOCK);
    if (n > 0) {
        if (c->nrep > 0)
            hipLaunchKernelGGL(k_bin<true>, dim3(nb), dim3(DB_BLOCK), 0, s, c->dp, B.x, c->cells.cellid,
                               c->cells.rank, c->cells.cnt);
        else
            hipLaunchKernelGGL(k_bin<false>, dim3(nb), dim3(DB_BLOCK), 0, s, c->dp, B.x, c->cells.cellid,
                               c->cells.rank, c->cells.cnt);
    }
    // start = exclusive scan of cnt; start[ncell] = their total, n
    launch_scan_total(c->cells.cnt, c->cells.start, ncell, c->cells.blocksum, s);
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(DB_BLOCK), 0, s, n, c->cells.cellid, c->cells.rank,
                           c->cells.start, c->cells.cnt, c->cells.unsorted, c->sw.stats);
        hipLaunchKernelGGL(k_cellsort, dim3(nb), dim3(DB_BLOCK), 0, s, n, c->cells.start, c->cells.cellid,
                           c->cells.unsorted, c->cells.list, B.x, c->cells.xs);
    }
}

// ---- permutation of the whole per-bead state into the new slot order ----------
__global__ __launch_bounds__(DB_BLOCK) void k_newslot(int n, const int* __restrict__ list, int* __restrict__ newslot) {
    int s = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (s < n) newslot[list[s]] = s;
}

// 1 for the beads (in cell order) that hold a bond, which are the ones with bonded terms
__global__ __launch_bounds__(DB_BLOCK) void k_bonded_flags(int n, const int* __restrict__ list,
                                                           const uint8_t* __restrict__ nb, int* __restrict__ flag) {
    int s = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (s < n) flag[s] = nb[list[s]] > 0 ? 1 : 0;
}

// Slots in cell order, except that within each XCD's share of the slots (the
// contiguous tile range xcd_tile gives it; the tail is a share of its own) the
// bonded beads come first.  A wavefront then holds bonded beads only or none, so
// that solvent waves skip the bonded terms instead of waiting on the one bonded
// bead among them, and each XCD keeps its share of both kinds.  off: exclusive
// prefix sums of the flags in cell order, off[n] their total.
__global__ __launch_bounds__(DB_BLOCK) void k_newslot_bonded_first(int n, const int* __restrict__ list,
                                                                   const int* __restrict__ off,
                                                                   int* __restrict__ newslot) {
    int s = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (s >= n) return;
    const int per = ((n + DB_BLOCK - 1) / DB_BLOCK) >> 3;
    const int share = per * DB_BLOCK;
    int st, en;
    if (share > 0 && s < 8 * share) {
        st = (s / share) * share;
        en = min(st + share, n);   // the last tile may be partial: the eighth share can end short
    } else {
        st = 8 * share;
        en = n;
    }
    const int before = off[s] - off[st];   // bonded beads of the share ahead of s
    const int bonded = off[en] - off[st];
    newslot[list[s]] = off[s + 1] > off[s] ? st + before : st + bonded + (s - st - before);
}

// Brick order of the cells: bricks of bB^3 cells (the last brick of each dimension
// takes the remaining nc - (nbk - 1) bB cells) in z, y, x order, the cells of a
// brick in z, y, x order.  Position of cell (cx, cy, cz) in that order.
__device__ __forceinline__ int brick_pos(int cx, int cy, int cz, int nc, int bB) {
    const int nbk = (nc + bB - 1) / bB;
    const int last = nc - (nbk - 1) * bB;
    const int bx = cx / bB, by = cy / bB, bz = cz / bB;
    const int lx = cx - bx * bB, ly = cy - by * bB, lz = cz - bz * bB;
    const int dx = bx == nbk - 1 ? last : bB, dy = by == nbk - 1 ? last : bB, dz = bz == nbk - 1 ? last : bB;
    return (bz * bB) * nc * nc + dz * (by * bB) * nc + dz * dy * (bx * bB) + (lz * dy + ly) * dx + lx;
}

// bead counts of the cells, written at the cells' brick-order positions
__global__ __launch_bounds__(DB_BLOCK) void k_brick_counts(int nc, int bB, const int* __restrict__ start,
                                                           int* __restrict__ out) {
    const int ncell = nc * nc * nc;
    const int c = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (c >= ncell) return;
    const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    out[brick_pos(cx, cy, cz, nc, bB)] = start[c + 1] - start[c];
}

// the new slot of every bead: its cell's start in brick order plus its place in
// the (ascending) cell list; bscan holds the exclusive prefix sums of the counts
// in brick order
__global__ __launch_bounds__(DB_BLOCK) void k_newslot_brick(int n, int nc, int bB, const int* __restrict__ list,
                                                            const int* __restrict__ cellid,
                                                            const int* __restrict__ start,
                                                            const int* __restrict__ bscan,
                                                            int* __restrict__ newslot) {
    const int s = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (s >= n) return;
    const int o = list[s];
    const int c = cellid[o];
    const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    newslot[o] = bscan[brick_pos(cx, cy, cz, nc, bB)] + (s - start[c]);
}

// first slot of every brick (tile), and n after the last
__global__ __launch_bounds__(DB_BLOCK) void k_tile_starts(int n, int nc, int bB, const int* __restrict__ bscan,
                                                          int* __restrict__ tstart) {
    const int nbk = (nc + bB - 1) / bB;
    const int ntile = nbk * nbk * nbk;
    const int b = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (b > ntile) return;
    if (b == ntile) {
        tstart[b] = n;
        return;
    }
    const int bx = b % nbk, by = (b / nbk) % nbk, bz = b / (nbk * nbk);
    tstart[b] = bscan[brick_pos(bx * bB, by * bB, bz * bB, nc, bB)];
}

__global__ __launch_bounds__(DB_BLOCK) void k_permute(int n, Bank src, Bank dst, int* __restrict__ list,
                                                       const int* __restrict__ newslot, int* __restrict__ slot_of_gid,
                                                       double4* __restrict__ xsave, double* __restrict__ vsave,
                                                       float4* __restrict__ xs) {
    int s = blockIdx.x * DB_BLOCK + threadIdx.x;   // position in cell order
    if (s >= n) return;
    int o = list[s];
    const int d = newslot[o];   // the bead's new slot
    double4 x = src.x[o];
    double vx = src.v[o], vy = src.v[n + o], vz = src.v[2 * n + o];
    dst.x[d] = x;
    dst.v[d] = vx;
    dst.v[n + d] = vy;
    dst.v[2 * n + d] = vz;
    if (xsave) {   // copy kept for re-running the block
        xsave[d] = x;
        vsave[d] = vx;
        vsave[n + d] = vy;
        vsave[2 * n + d] = vz;
    }
    slot_of_gid[meta_gid(x)] = d;
    int nb = src.nb[o];
    dst.nb[d] = (uint8_t)nb;
    for (int k = 0; k < nb; ++k) {
        dst.bp[k * n + d] = newslot[src.bp[k * n + o]];
        dst.bt[k * n + d] = src.bt[k * n + o];
    }
    int na = src.na[o];
    dst.na[d] = (uint8_t)na;
    for (int k = 0; k < na; ++k) {
        int4 e = src.ang[k * n + o];
        dst.ang[k * n + d] = make_int4(newslot[e.x], newslot[e.y], newslot[e.z], e.w);
    }
    int nd = src.nd[o];
    dst.nd[d] = (uint8_t)nd;
    for (int k = 0; k < nd; ++k) {
        int4 e = src.dih[k * n + o];
        dst.dih[k * n + d] = make_int4(newslot[e.x], newslot[e.y], newslot[e.z], newslot[e.w]);
        dst.dt[k * n + d] = src.dt[k * n + o];
    }
    list[s] = d;   // the cell list now names the new slots
    xs[s].w = xs_word(d, meta_word(x));
}

void launch_permute(db_ctx* c, bool save) {
    const int n = c->n;
    if (n == 0) return;
    hipStream_t s = c->stream;
    unsigned nb = (unsigned)((n + DB_BLOCK - 1) / DB_BLOCK);
    int* newslot = c->cells.cellid;   // the bin ids are no longer needed
    const bool tiled = tiles_enabled(c);
    if (tiled) {
        // brick order: the bin counts (zero between builds) serve as scan space and
        // are cleared again afterwards; the new slots go to the sweep's free flag
        // array, since the bin ids are read
        const int nc = c->hp.box.nc, bB = c->tile_bB, ncell = c->hp.ncell;
        int* bscan = c->cells.cnt;
        unsigned cb = (unsigned)((ncell + DB_BLOCK - 1) / DB_BLOCK);
        hipLaunchKernelGGL(k_brick_counts, dim3(cb), dim3(DB_BLOCK), 0, s, nc, bB, c->cells.start, bscan);
        launch_exclusive_scan(bscan, ncell, nullptr, c->cells.blocksum, s);
        newslot = c->sw.act;
        hipLaunchKernelGGL(k_newslot_brick, dim3(nb), dim3(DB_BLOCK), 0, s, n, nc, bB, c->cells.list,
                           c->cells.cellid, c->cells.start, bscan, newslot);
        const int nbk = (nc + bB - 1) / bB;
        unsigned tb = (unsigned)((nbk * nbk * nbk + 1 + DB_BLOCK - 1) / DB_BLOCK);
        hipLaunchKernelGGL(k_tile_starts, dim3(tb), dim3(DB_BLOCK), 0, s, n, nc, bB, bscan, c->tiles.tstart);
        launch_fill_int(bscan, 0, (size_t)ncell + 1, s);
    } else if (c->nrep == 0) {
        // bonded beads first within each XCD's share; the sweep's flag and offset
        // arrays are free while the cells are reordered
        hipLaunchKernelGGL(k_bonded_flags, dim3(nb), dim3(DB_BLOCK), 0, s, n, c->cells.list, c->bank[c->cur].nb,
                           c->sw.act);
        launch_scan_total(c->sw.act, c->sw.aoff, n, c->cells.blocksum, s);
        hipLaunchKernelGGL(k_newslot_bonded_first, dim3(nb), dim3(DB_BLOCK), 0, s, n, c->cells.list, c->sw.aoff,
                           newslot);
    } else {
        hipLaunchKernelGGL(k_newslot, dim3(nb), dim3(DB_BLOCK), 0, s, n, c->cells.list, newslot);
    }
    hipLaunchKernelGGL(k_permute, dim3(nb), dim3(DB_BLOCK), 0, s, n, c->bank[c->cur], c->bank[1 - c->cur],
                       c->cells.list, newslot, c->slot_of_gid, save ? c->xsave : (double4*)nullptr,
                       save ? c->vsave : (double*)nullptr, c->cells.xs);
    c->cur = 1 - c->cur;
    c->halo_force = true;
    c->tiles_valid = tiled;
    c->regions_valid = false;
}

}  // namespace db
