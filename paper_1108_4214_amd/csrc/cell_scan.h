// Neighbour scan over the cell list.  The cell sort also writes a float copy of
// every position in list order (x, y, z and the slot), so the beads of the 27
// cells around a bead are nine contiguous runs of that array (the three cells of
// an x-row are adjacent unless the row wraps).  Runs are read four entries at a
// time so that several loads are in flight per thread.  The float distance only
// prefilters: the visitor re-checks in double whatever it decides on.
#pragma once
#include "db_device.h"

namespace db {

__device__ __forceinline__ float fmin_image(float d, float L, float hL) {
    const float lo = d - L, hi = d + L;
    float r = d > hL ? lo : d;
    return d < -hL ? hi : r;
}

// f(j, r2f) for every j != i in the cells around xi with float r2 < cut2.
// With three or more cells per edge, the periodic image of a neighbour cell is
// fixed by whether its index wrapped, so the bead's own coordinates are shifted
// once per run and the candidates need no minimum-image test (the true nearest
// image is that one for every candidate within one cell edge).  Smaller grids
// visit every cell once and take the per-candidate minimum image.  The visitor
// has a single call site per grid case, which keeps it inlined once.
template <class F>
__device__ __forceinline__ void scan_run(const float4* __restrict__ xs, int s0, int s1, int i, float qx, float qy,
                                         float qz, float cut2, F&& f) {
    for (int p = s0; p < s1; p += 4) {
        float4 e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = xs[min(p + q, s1 - 1)];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // one branch per candidate: range, self and distance folded into one predicate
            const int j = __float_as_int(e[q].w);
            const float dx = e[q].x - qx, dy = e[q].y - qy, dz = e[q].z - qz;
            const float r2 = (dx * dx + dy * dy) + dz * dz;
            const bool hit = (p + q < s1) & (j != i) & (r2 < cut2);
            if (hit) f(j, r2);
        }
    }
}

template <class F>
__device__ __forceinline__ void scan_cells(const Box& X, const int* __restrict__ cstart,
                                           const float4* __restrict__ xs, int i, const double4& xi, float cut2,
                                           F&& f) {
    const int nc = X.nc;
    const int cx = cell_coord(xi.x, X.cell_scale, nc);
    const int cy = cell_coord(xi.y, X.cell_scale, nc);
    const int cz = cell_coord(xi.z, X.cell_scale, nc);
    const float Lf = (float)X.L, hLf = (float)X.hL;
    const float px = (float)xi.x, py = (float)xi.y, pz = (float)xi.z;
    cstart += X.cell_off;
    if (X.noff == 3) {
        // nine x-rows of three cells; a row that wraps in x splits into two runs
        // (the wrapped cell seen through its image, and the two contiguous ones),
        // so each row is visited as two runs, the second empty unless it wraps
        auto shift = [&](int c) { return c < 0 ? -Lf : (c >= nc ? Lf : 0.0f); };
        for (int r = 0; r < 18; ++r) {
            const int zr = cz + r / 6 - 1, yr = cy + (r >> 1) % 3 - 1, part = r & 1;
            const float qz = pz - shift(zr), qy = py - shift(yr);
            const int row = (wrap_cell(zr, nc) * nc + wrap_cell(yr, nc)) * nc;
            int a0, a1;          // cell range [a0, a1) of the row, contiguous in the list
            float qx = px;
            if (cx >= 1 && cx <= nc - 2) {
                a0 = part ? 0 : cx - 1;
                a1 = part ? 0 : cx + 2;
            } else if (cx == 0) {
                a0 = part ? 0 : nc - 1;
                a1 = part ? 2 : nc;
                if (!part) qx = px + Lf;
            } else {
                a0 = part ? 0 : nc - 2;
                a1 = part ? 1 : nc;
                if (part) qx = px - Lf;
            }
            const int s0 = a1 > a0 ? cstart[row + a0] : 0;
            const int s1 = a1 > a0 ? cstart[row + a1] : 0;
            scan_run(xs, s0, s1, i, qx, qy, qz, cut2, f);
        }
        return;
    }
    for (int oz = 0; oz < X.noff; ++oz) {
        const int zz = wrap_cell(cz + X.off[oz], nc);
        for (int oy = 0; oy < X.noff; ++oy) {
            const int row = (zz * nc + wrap_cell(cy + X.off[oy], nc)) * nc;
            for (int ox = 0; ox < X.noff; ++ox) {
                const int c = row + wrap_cell(cx + X.off[ox], nc);
                const int s0 = cstart[c], s1 = cstart[c + 1];
                for (int p = s0; p < s1; ++p) {
                    const float4 e = xs[p];
                    const int j = __float_as_int(e.w);
                    const float dx = fmin_image(e.x - px, Lf, hLf);
                    const float dy = fmin_image(e.y - py, Lf, hLf);
                    const float dz = fmin_image(e.z - pz, Lf, hLf);
                    const float r2 = (dx * dx + dy * dy) + dz * dz;
                    if ((j != i) & (r2 < cut2)) f(j, r2);
                }
            }
        }
    }
}

}  // namespace db
