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

// f(j, r2f) for every j != i in the 27 cells around xi with float r2 < cut2
template <class F>
__device__ __forceinline__ void scan_cells(const Params& P, const int* __restrict__ cstart,
                                           const float4* __restrict__ xs, int i, const double4& xi, float cut2,
                                           F&& f) {
    const int nc = P.nc;
    const int cx = cell_coord(xi.x, P.cell_scale, nc);
    const int cy = cell_coord(xi.y, P.cell_scale, nc);
    const int cz = cell_coord(xi.z, P.cell_scale, nc);
    const float Lf = (float)P.L, hLf = (float)P.hL;
    const float px = (float)xi.x, py = (float)xi.y, pz = (float)xi.z;
    const bool rowmerge = (P.noff == 3) && cx >= 1 && cx <= nc - 2;
    for (int oz = 0; oz < P.noff; ++oz) {
        const int zz = wrap_cell(cz + P.off[oz], nc);
        for (int oy = 0; oy < P.noff; ++oy) {
            const int row = (zz * nc + wrap_cell(cy + P.off[oy], nc)) * nc;
            const int nseg = rowmerge ? 1 : P.noff;
            for (int ox = 0; ox < nseg; ++ox) {
                int s0, s1;
                if (rowmerge) {
                    s0 = cstart[row + cx - 1];
                    s1 = cstart[row + cx + 2];
                } else {
                    const int c = row + wrap_cell(cx + P.off[ox], nc);
                    s0 = cstart[c];
                    s1 = cstart[c + 1];
                }
                for (int p = s0; p < s1; p += 4) {
                    float4 e[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) e[q] = xs[min(p + q, s1 - 1)];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // one branch per candidate: range, self and distance folded into one predicate
                        const int j = __float_as_int(e[q].w);
                        const float dx = fmin_image(e[q].x - px, Lf, hLf);
                        const float dy = fmin_image(e[q].y - py, Lf, hLf);
                        const float dz = fmin_image(e[q].z - pz, Lf, hLf);
                        const float r2 = (dx * dx + dy * dy) + dz * dz;
                        const bool hit = (p + q < s1) & (j != i) & (r2 < cut2);
                        if (hit) f(j, r2);
                    }
                }
            }
        }
    }
}

}  // namespace db
