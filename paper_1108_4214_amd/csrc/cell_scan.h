// Neighbour scan over the cell list.  The cell sort also writes a float copy of
// every position in list order (x, y, z and a word holding the slot, the type and
// the reactive flag), so the beads of the 27
// cells around a bead are nine contiguous runs of that array (the three cells of
// an x-row are adjacent unless the row wraps).  Runs are read four entries at a
// time so that several loads are in flight per thread.  The float distance only
// prefilters: the visitor re-checks in double whatever it decides on.
#pragma once
#include "db_device.h"

#ifndef DB_SCAN_W
#define DB_SCAN_W 4   // candidates requested together per run
#endif
static_assert(DB_SCAN_W <= DB_XS_PAD, "a run's last group of loads stays within the padded position copy");

namespace db {

__device__ __forceinline__ float fmin_image(float d, float L, float hL) {
    const float lo = d - L, hi = d + L;
    float r = d > hL ? lo : d;
    return d < -hL ? hi : r;
}

// f(j, w) for every slot j != i in the cells around xi with float r2 < cut2; w is
// the entry's word (slot, type, reactive flag: xs_slot / xs_type / xs_reactive).
// With three or more cells per edge, the periodic image of a neighbour cell is
// fixed by whether its index wrapped, so the bead's own coordinates are shifted
// once per run and the candidates need no minimum-image test (the true nearest
// image is that one for every candidate within one cell edge).  Runs are read
// four entries at a time.  Smaller grids visit every cell once and take the
// per-candidate minimum image.  The visitor has a single call site per grid
// case, which keeps it inlined once.
// PARTS > 1 splits one bead's scan over PARTS threads: on grids of three or more
// cells per edge every thread walks all nine rows and takes the entries of each
// run whose place in the run is part modulo PARTS (neighbouring threads read
// neighbouring entries, and the shares differ by at most one entry per row); on
// small grids the thread takes the cells whose index is part modulo PARTS.
// Together the threads visit every candidate once.
template <int PARTS = 1, class F>
__device__ __forceinline__ void scan_cells(const Box& X, const int* __restrict__ cstart,
                                           const float4* __restrict__ xs, int i, const double4& xi, float cut2,
                                           F&& f, int part = 0) {
    static_assert(PARTS >= 1 && PARTS <= 64, "a bead's threads lie within a wavefront");
    // entries requested together per run: a thread of a split scan takes a few of
    // each run, so fewer at a time
    constexpr int SW = PARTS == 1 ? DB_SCAN_W : 2;
    const int nc = X.nc;
    const int cx = cell_coord(xi.x, X.cell_scale, nc);
    const int cy = cell_coord(xi.y, X.cell_scale, nc);
    const int cz = cell_coord(xi.z, X.cell_scale, nc);
    const float Lf = (float)X.L, hLf = (float)X.hL;
    const float px = (float)xi.x, py = (float)xi.y, pz = (float)xi.z;
    cstart += X.cell_off;
    if (X.noff == 3) {
        // Nine x-rows of three cells.  The x-part of a row is the same for every
        // row: cells [a0, a1), and only when it wraps in x a second range [b0, b1)
        // seen through its image; both are read as one run.  The bounds of the
        // next row are requested before the current row is scanned.
        auto shift = [&](int c) { return c < 0 ? -Lf : (c >= nc ? Lf : 0.0f); };
        int a0, a1, b0 = 0, b1 = 0;
        float qx1 = px;
        if (cx >= 1 && cx <= nc - 2) {
            a0 = cx - 1;
            a1 = cx + 2;
        } else if (cx == 0) {
            a0 = 0;
            a1 = 2;
            b0 = nc - 1;
            b1 = nc;
            qx1 = px + Lf;
        } else {
            a0 = nc - 2;
            a1 = nc;
            b0 = 0;
            b1 = 1;
            qx1 = px - Lf;
        }
        const bool wrapx = b1 > b0;
        auto row_of = [&](int r) {
            return (wrap_cell(cz + r / 3 - 1, nc) * nc + wrap_cell(cy + r % 3 - 1, nc)) * nc;
        };
        int row = row_of(0);
        int s0 = cstart[row + a0], s1 = cstart[row + a1];
        int t0 = wrapx ? cstart[row + b0] : 0, t1 = wrapx ? cstart[row + b1] : 0;
        for (int r = 0; r < 9; ++r) {
            const float qz = pz - shift(cz + r / 3 - 1), qy = py - shift(cy + r % 3 - 1);
            const int c0 = s0, d0 = t0;
            const int len0 = s1 - s0, len = len0 + (t1 - t0);
            if (r + 1 < 9) {
                row = row_of(r + 1);
                s0 = cstart[row + a0];
                s1 = cstart[row + a1];
                t0 = wrapx ? cstart[row + b0] : 0;
                t1 = wrapx ? cstart[row + b1] : 0;
            }
            for (int p = PARTS == 1 ? 0 : part; p < len; p += SW * PARTS) {
                float4 e[SW];
#pragma unroll
                for (int q = 0; q < SW; ++q) {
                    const int k = min(p + q * PARTS, len - 1);
                    e[q] = xs[k < len0 ? c0 + k : d0 + (k - len0)];
                }
#pragma unroll
                for (int q = 0; q < SW; ++q) {
                    // one branch per candidate: range, self and distance folded into one predicate
                    const int k = p + q * PARTS;
                    const int w = __float_as_int(e[q].w);
                    const int j = xs_slot(w);
                    const float dx = e[q].x - (k < len0 ? px : qx1), dy = e[q].y - qy, dz = e[q].z - qz;
                    const float r2 = (dx * dx + dy * dy) + dz * dz;
                    const bool hit = (k < len) & (j != i) & (r2 < cut2);
                    if (hit) f(j, w);
                }
            }
        }
        return;
    }
    int cell_no = 0;
    for (int oz = 0; oz < X.noff; ++oz) {
        const int zz = wrap_cell(cz + box_off(X, oz), nc);
        for (int oy = 0; oy < X.noff; ++oy) {
            const int row = (zz * nc + wrap_cell(cy + box_off(X, oy), nc)) * nc;
            for (int ox = 0; ox < X.noff; ++ox) {
                if (PARTS > 1 && cell_no++ % PARTS != part) continue;
                const int c = row + wrap_cell(cx + box_off(X, ox), nc);
                const int s0 = cstart[c], s1 = cstart[c + 1];
                for (int p = s0; p < s1; ++p) {
                    const float4 e = xs[p];
                    const int w = __float_as_int(e.w);
                    const int j = xs_slot(w);
                    const float dx = fmin_image(e.x - px, Lf, hLf);
                    const float dy = fmin_image(e.y - py, Lf, hLf);
                    const float dz = fmin_image(e.z - pz, Lf, hLf);
                    const float r2 = (dx * dx + dy * dy) + dz * dz;
                    if ((j != i) & (r2 < cut2)) f(j, w);
                }
            }
        }
    }
}

// The candidates of scan_cells (grids of three or more cells per edge only), each
// passed as f(w, hit) with w the entry's word (xs_slot(w) is its slot) and hit =
// (slot != i and float r2 < cut2), in scan_cells' order.  f runs for every
// candidate, so a visitor without branches (one that writes every candidate and
// advances its count by hit) keeps the lanes of a wave together; the x-range of a
// row and its wrapped part are separate loops, so the common range needs no
// per-candidate choice of image.  The bead's own entry is told apart by its whole
// word (the slot bits differ for every other bead), and r2 is formed with fused
// multiply-adds, whose rounding is within the relative margin of cut2.
template <class F>
__device__ __forceinline__ void scan_cells_all(const Box& X, const int* __restrict__ cstart,
                                               const float4* __restrict__ xs, int i, const double4& xi, float cut2,
                                               F&& f) {
    const int nc = X.nc;
    const int cx = cell_coord(xi.x, X.cell_scale, nc);
    const int cy = cell_coord(xi.y, X.cell_scale, nc);
    const int cz = cell_coord(xi.z, X.cell_scale, nc);
    const float Lf = (float)X.L;
    const float px = (float)xi.x, py = (float)xi.y, pz = (float)xi.z;
    const int wi = __float_as_int(xs_word(i, meta_word(xi)));
    cstart += X.cell_off;
    auto shift = [&](int c) { return c < 0 ? -Lf : (c >= nc ? Lf : 0.0f); };
    int a0, a1, b0 = 0, b1 = 0;
    float qx1 = px;
    if (cx >= 1 && cx <= nc - 2) {
        a0 = cx - 1;
        a1 = cx + 2;
    } else if (cx == 0) {
        a0 = 0;
        a1 = 2;
        b0 = nc - 1;
        b1 = nc;
        qx1 = px + Lf;
    } else {
        a0 = nc - 2;
        a1 = nc;
        b0 = 0;
        b1 = 1;
        qx1 = px - Lf;
    }
    const bool wrapx = b1 > b0;
    auto row_of = [&](int r) { return (wrap_cell(cz + r / 3 - 1, nc) * nc + wrap_cell(cy + r % 3 - 1, nc)) * nc; };
    // one run [s, e) of consecutive entries seen from (qx, qy, qz); a group of
    // loads may run past e (into the next cells' entries, or into the padding after
    // the last entry), and those candidates are masked
    auto run = [&](int s, int e, float qx, float qy, float qz) {
        for (int p = s; p < e; p += DB_SCAN_W) {
            float4 c[DB_SCAN_W];
            const float4* src = xs + p;
#pragma unroll
            for (int q = 0; q < DB_SCAN_W; ++q) c[q] = src[q];
            const int rem = e - p;
#pragma unroll
            for (int q = 0; q < DB_SCAN_W; ++q) {
                const int w = __float_as_int(c[q].w);
                const float dx = c[q].x - qx, dy = c[q].y - qy, dz = c[q].z - qz;
                const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                f(w, (q < rem) & (w != wi) & (r2 < cut2));
            }
        }
    };
    int row = row_of(0);
    int s0 = cstart[row + a0], s1 = cstart[row + a1];
    int t0 = wrapx ? cstart[row + b0] : 0, t1 = wrapx ? cstart[row + b1] : 0;
    for (int r = 0; r < 9; ++r) {
        const float qz = pz - shift(cz + r / 3 - 1), qy = py - shift(cy + r % 3 - 1);
        const int c0 = s0, c1 = s1, d0 = t0, d1 = t1;
        if (r + 1 < 9) {   // the next row's bounds are requested before this row is scanned
            row = row_of(r + 1);
            s0 = cstart[row + a0];
            s1 = cstart[row + a1];
            t0 = wrapx ? cstart[row + b0] : 0;
            t1 = wrapx ? cstart[row + b1] : 0;
        }
        run(c0, c1, px, qy, qz);
        run(d0, d1, qx1, qy, qz);
    }
}

// f(j, w) for every slot j != i with float r2 < cut2 in the 5 x 5 x 5 cells
// around xi: a reach of two cell edges, for lists redone with a cutoff beyond one
// edge.  Needs at least five cells per edge (no cell is visited twice).  Each
// candidate takes the minimum image; this serves the beads whose lists are redone
// after a sweep, and creation scans with a creation distance beyond one edge.  The
// outer layer of cells on a side is visited only when the bead lies within the
// cutoff of it (for a cutoff just beyond one edge, most beads need the inner
// 3 x 3 x 3 cells alone), and the x-cells of a row are read as one run unless the
// row wraps.  PARTS and part split the rows by their index modulo PARTS.  GW
// entries of a run are requested together (a patched list is redone for few
// beads, one thread each, so their loads in flight set its time; the creation scan
// takes one at a time, to keep its registers).
template <int PARTS = 1, int GW = DB_SCAN_W, class F>
__device__ void scan_cells_wide(const Box& X, const int* __restrict__ cstart, const float4* __restrict__ xs,
                                int i, const double4& xi, float cut2, F&& f, int part = 0) {
    const int nc = X.nc;
    const int cx = cell_coord(xi.x, X.cell_scale, nc);
    const int cy = cell_coord(xi.y, X.cell_scale, nc);
    const int cz = cell_coord(xi.z, X.cell_scale, nc);
    const float Lf = (float)X.L, hLf = (float)X.hL;
    const float px = (float)xi.x, py = (float)xi.y, pz = (float)xi.z;
    cstart += X.cell_off;
    // the outer layer on a side: needed when the bead is nearer than the reach
    // (the prefilter's radius, widened for rounding) to that layer's inner face
    const double edge = X.L / (double)nc;
    const double reach = sqrt((double)cut2) * (1.0 + 1e-6) + 1e-9 * X.L;
    auto lo_of = [&](double x, int c) { return (x * X.cell_scale - c + 1.0) * edge < reach ? -2 : -1; };
    auto hi_of = [&](double x, int c) { return (2.0 - (x * X.cell_scale - c)) * edge < reach ? 2 : 1; };
    const int lox = lo_of(xi.x, cx), hix = hi_of(xi.x, cx);
    const int loy = lo_of(xi.y, cy), hiy = hi_of(xi.y, cy);
    const int loz = lo_of(xi.z, cz), hiz = hi_of(xi.z, cz);
    const bool xrun = cx + lox >= 0 && cx + hix < nc;   // the row's x-cells are contiguous
    // a run is read GW entries at a time, all in flight together; the last group
    // may read past the run (into the next cells, or the padding after the copy),
    // and those entries are masked
    static_assert(GW >= 1 && GW <= DB_XS_PAD, "a group stays within the padded position copy");
    auto run = [&](int s0, int s1) {
        for (int p = s0; p < s1; p += GW) {
            float4 e[GW];
            const float4* src = xs + p;
#pragma unroll
            for (int q = 0; q < GW; ++q) e[q] = src[q];
            const int rem = s1 - p;
#pragma unroll
            for (int q = 0; q < GW; ++q) {
                const int w = __float_as_int(e[q].w);
                const int j = xs_slot(w);
                const float dx = fmin_image(e[q].x - px, Lf, hLf);
                const float dy = fmin_image(e[q].y - py, Lf, hLf);
                const float dz = fmin_image(e[q].z - pz, Lf, hLf);
                const float r2 = (dx * dx + dy * dy) + dz * dz;
                if ((q < rem) & (j != i) & (r2 < cut2)) f(j, w);
            }
        }
    };
    // rows in z-major order; with contiguous x-cells the next row's bounds are
    // requested before the current row is scanned
    const int ny = hiy - loy + 1, nrow = (hiz - loz + 1) * ny;
    auto row_of = [&](int r) { return (wrap_cell(cz + loz + r / ny, nc) * nc + wrap_cell(cy + loy + r % ny, nc)) * nc; };
    int r = PARTS > 1 ? part : 0;
    int a0 = 0, a1 = 0;
    if (xrun && r < nrow) {
        const int row = row_of(r);
        a0 = cstart[row + cx + lox];
        a1 = cstart[row + cx + hix + 1];
    }
    for (; r < nrow; r += PARTS) {
        if (xrun) {
            const int s0 = a0, s1 = a1;
            if (r + PARTS < nrow) {
                const int row = row_of(r + PARTS);
                a0 = cstart[row + cx + lox];
                a1 = cstart[row + cx + hix + 1];
            }
            run(s0, s1);
        } else {
            const int row = row_of(r);
            for (int ox = lox; ox <= hix; ++ox) {
                const int c = row + wrap_cell(cx + ox, nc);
                run(cstart[c], cstart[c + 1]);
            }
        }
    }
}

}  // namespace db
