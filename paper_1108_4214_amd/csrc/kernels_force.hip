// Per-step force pass: one thread per bead gathers its own force (Newton's third
// law is not used for bonded terms: every bead evaluates each bond, angle and
// dihedral it takes part in, as in the paper's directional-bond storage, section 2
// and appendix), so nothing is accumulated across threads.  Pair forces: WCA over
// the 27 surrounding cells of the bead's current position.  Bonded: harmonic
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
template <>
__device__ __forceinline__ float r_atan2<float>(float y, float x) { return atan2f(y, x); }

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
__device__ __forceinline__ void pair_term(const Params& P, const double4& xi, const double4& xj, Acc<R>& a) {
    double dx, dy, dz;
    dx = min_image(xj.x - xi.x, P.L, P.hL);
    dy = min_image(xj.y - xi.y, P.L, P.hL);
    dz = min_image(xj.z - xi.z, P.L, P.hL);
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

template <typename R, int MODE>
__device__ void pair_forces(const Params& P, const Bank& B, const int* __restrict__ cstart,
                            const int* __restrict__ clist, int i, const double4& xi, int nb, int p0, int p1, int p2,
                            int p3, Acc<R>& a) {
    const int nc = P.nc;
    int cx = cell_coord(xi.x, P.cell_scale, nc);
    int cy = cell_coord(xi.y, P.cell_scale, nc);
    int cz = cell_coord(xi.z, P.cell_scale, nc);
    const R rc2 = (R)P.rc2;
    const bool rowmerge = (P.noff == 3) && cx >= 1 && cx <= nc - 2;
    for (int oz = 0; oz < P.noff; ++oz) {
        int zz = wrap_cell(cz + P.off[oz], nc);
        for (int oy = 0; oy < P.noff; ++oy) {
            int yy = wrap_cell(cy + P.off[oy], nc);
            int row = (zz * nc + yy) * nc;
            // the three cells of one x-row are contiguous in the list unless the row wraps
            int nseg = rowmerge ? 1 : P.noff;
            for (int ox = 0; ox < nseg; ++ox) {
                int s0, s1;
                if (rowmerge) {
                    s0 = cstart[row + cx - 1];
                    s1 = cstart[row + cx + 2];
                } else {
                    int c = row + wrap_cell(cx + P.off[ox], nc);
                    s0 = cstart[c];
                    s1 = cstart[c + 1];
                }
                for (int p = s0; p < s1; ++p) {
                    int j = clist[p];
                    if (j == i) continue;
                    double4 xj = B.x[j];
                    double dx = min_image(xj.x - xi.x, P.L, P.hL);
                    double dy = min_image(xj.y - xi.y, P.L, P.hL);
                    double dz = min_image(xj.z - xi.z, P.L, P.hL);
                    R rx = (R)dx, ry = (R)dy, rz = (R)dz;
                    R r2 = (rx * rx + ry * ry) + rz * rz;
                    if (!(r2 < rc2)) continue;
                    if (P.excl_depth >= 1 && in_list4(j, nb, p0, p1, p2, p3)) continue;
                    if (P.excl_depth >= 2 && two_bonds_apart(B, P.n, j, nb, p0, p1, p2, p3)) continue;
                    pair_term<R, MODE>(P, xi, xj, a);
                }
            }
        }
    }
}

// Verlet list of bead i: every bead within the list cutoff (pair cutoff plus a
// skin) that is not excluded, from the 27 cells of the current cell list.  The
// float prefilter carries a 1e-4 relative margin, so the list is a superset of
// the pairs within the cutoff in double.
__global__ __launch_bounds__(DB_BLOCK) void k_build_nlist(const Params* __restrict__ Pp, Bank B,
                                                          const int* __restrict__ cstart,
                                                          const float4* __restrict__ xs, NList NL,
                                                          int* __restrict__ err) {
    const Params& P = *Pp;
    const int n = P.n;
    const int i = xcd_tile(blockIdx.x, gridDim.x) * DB_BLOCK + threadIdx.x;
    if (i >= n) return;
    const double4 xi = B.x[i];
    const int nb = B.nb[i];
    const int p0 = nb > 0 ? B.bp[i] : -1;
    const int p1 = nb > 1 ? B.bp[n + i] : -1;
    const int p2 = nb > 2 ? B.bp[2 * n + i] : -1;
    const int p3 = nb > 3 ? B.bp[3 * n + i] : -1;
    int cnt = 0;
    scan_cells(P, cstart, xs, i, xi, (float)(P.rnl2 * 1.0001), [&](int j, float) {
        if (P.excl_depth >= 1 && in_list4(j, nb, p0, p1, p2, p3)) return;
        if (P.excl_depth >= 2 && two_bonds_apart(B, n, j, nb, p0, p1, p2, p3)) return;
        if (cnt < DB_NLCAP) NL.nl[cnt * n + i] = j;
        ++cnt;
    });
    if (cnt > DB_NLCAP) {
        atomicOr(err, ERR_NLIST);
        cnt = DB_NLCAP;
    }
    NL.cnt[i] = (uint8_t)cnt;
}

// pair forces from the Verlet list (exclusions were applied when it was built).
// Entries are taken four at a time: the four indices, then the four positions are
// requested before any of them is used, so one bead keeps several loads in flight.
template <typename R>
__device__ __forceinline__ void pair_one(const Params& P, const double4& xi, const double4& xj, R rc2, Acc<R>& a) {
    R rx = (R)min_image(xj.x - xi.x, P.L, P.hL);
    R ry = (R)min_image(xj.y - xi.y, P.L, P.hL);
    R rz = (R)min_image(xj.z - xi.z, P.L, P.hL);
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

template <typename R>
__device__ __forceinline__ void list_pair_forces(const Params& P, const Bank& B, const NList& NL, int i,
                                                 const double4& xi, Acc<R>& a) {
    const int n = P.n;
    const R rc2 = (R)P.rc2;
    const int m = NL.cnt[i];
    for (int k0 = 0; k0 < m; k0 += 4) {
        int j[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) j[q] = (k0 + q < m) ? NL.nl[(k0 + q) * n + i] : i;
        double4 xj[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) xj[q] = B.x[j[q]];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (k0 + q < m) pair_one<R>(P, xi, xj[q], rc2, a);
    }
}

// harmonic bond U = K (r - r0)^2 with the type bead i stores (all partners requested at once)
template <typename R, int MODE>
__device__ __forceinline__ void bond_terms(const Params& P, const Bank& B, int i, const double4& xi, int nb,
                                           Acc<R>& a) {
    const int n = P.n;
    int jj[DB_MAXB], tt[DB_MAXB];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) {
        jj[k] = k < nb ? B.bp[k * n + i] : i;
        tt[k] = k < nb ? (int)B.bt[k * n + i] : 0;
    }
    double4 xs[DB_MAXB];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) xs[k] = B.x[jj[k]];
#pragma unroll
    for (int k = 0; k < DB_MAXB; ++k) {
        if (k >= nb) continue;
        const double4& xj = xs[k];
        const int t = tt[k];
        double dx = min_image(xj.x - xi.x, P.L, P.hL);
        double dy = min_image(xj.y - xi.y, P.L, P.hL);
        double dz = min_image(xj.z - xi.z, P.L, P.hL);
        R rx = (R)dx, ry = (R)dy, rz = (R)dz;
        R rr2 = (rx * rx + ry * ry) + rz * rz;
        if (!(rr2 > (R)0)) continue;
        R ir = r_rsqrt<R>(rr2);
        R r = rr2 * ir;
        R K = (R)P.bK[t], r0 = (R)P.bR0[t];
        R g = (R)2.0 * K * (r - r0) * ir;   // F_i = g * (x_j - x_i)
        a.fx += (double)(g * rx);
        a.fy += (double)(g * ry);
        a.fz += (double)(g * rz);
        if (MODE == MODE_ENERGY) {
            a.e_bond += 0.5 * (double)(K * (r - r0) * (r - r0));
            a.vir -= 0.5 * (double)(g * r * r);
        }
    }
}

// harmonic angle U = K (theta - theta0)^2; bead i takes the force of its role
template <typename R, int MODE>
__device__ __forceinline__ void angle_terms(const Params& P, const Bank& B, int i, const double4& xi, int na,
                                            Acc<R>& a) {
    const int n = P.n;
    for (int k = 0; k < na; ++k) {
        int4 e = B.ang[k * n + i];
        double4 xa = B.x[e.x];
        double4 xb = B.x[e.y];
        double4 xc = B.x[e.z];
        R ux = (R)min_image(xa.x - xb.x, P.L, P.hL), uy = (R)min_image(xa.y - xb.y, P.L, P.hL),
          uz = (R)min_image(xa.z - xb.z, P.L, P.hL);
        R wx = (R)min_image(xc.x - xb.x, P.L, P.hL), wy = (R)min_image(xc.y - xb.y, P.L, P.hL),
          wz = (R)min_image(xc.z - xb.z, P.L, P.hL);
        R ru2 = (ux * ux + uy * uy) + uz * uz;
        R rw2 = (wx * wx + wy * wy) + wz * wz;
        if (!(ru2 > (R)0) || !(rw2 > (R)0)) continue;
        R iru = r_rsqrt<R>(ru2), irw = r_rsqrt<R>(rw2);
        R cux = ux * iru, cuy = uy * iru, cuz = uz * iru;
        R cwx = wx * irw, cwy = wy * irw, cwz = wz * irw;
        R cs = (cux * cwx + cuy * cwy) + cuz * cwz;
        R crx = cuy * cwz - cuz * cwy, cry = cuz * cwx - cux * cwz, crz = cux * cwy - cuy * cwx;
        R sn = r_sqrt<R>((crx * crx + cry * cry) + crz * crz);
        int t = e.w;
        R K = (R)P.aK[t];
        R th = r_atan2<R>(sn, cs);
        // dU/dtheta / sin(theta), finite at theta = pi when theta0 = pi
        R del = r_atan2<R>(sn, -cs);   // pi - theta
        R isn = r_rcp<R>(sn > (R)1e-8 ? sn : (R)1e-8);
        R ratio = del < (R)1e-6 ? (R)1.0 + del * del * (R)(1.0 / 6.0) : del * isn;
        R pth = (R)P.aPiMinusT0[t];
        R A = (R)2.0 * K * (-ratio + (pth != (R)0 ? pth * isn : (R)0));
        R Au = -A * iru, Aw = -A * irw;
        R fax = Au * (cs * cux - cwx), fay = Au * (cs * cuy - cwy), faz = Au * (cs * cuz - cwz);
        R fcx = Aw * (cs * cwx - cux), fcy = Aw * (cs * cwy - cuy), fcz = Aw * (cs * cwz - cuz);
        if (e.x == i) {
            a.fx += (double)fax; a.fy += (double)fay; a.fz += (double)faz;
        } else if (e.z == i) {
            a.fx += (double)fcx; a.fy += (double)fcy; a.fz += (double)fcz;
        } else {
            a.fx -= (double)(fax + fcx); a.fy -= (double)(fay + fcy); a.fz -= (double)(faz + fcz);
        }
        if (MODE == MODE_ENERGY) {
            R th0 = (R)P.aT0[t];
            a.e_ang += (double)(K * (th - th0) * (th - th0)) / 3.0;
            a.vir += (double)((ux * fax + uy * fay + uz * faz) + (wx * fcx + wy * fcy + wz * fcz)) / 3.0;
        }
    }
}

// cosine dihedral U = K [1 - cos(phi - phi0)], phi = atan2(|b2| b1.(b2 x b3), (b1 x b2).(b2 x b3))
template <typename R, int MODE>
__device__ __forceinline__ void dihedral_terms(const Params& P, const Bank& B, int i, const double4& xi, int nd,
                                               Acc<R>& a) {
    const int n = P.n;
    for (int k = 0; k < nd; ++k) {
        int4 e = B.dih[k * n + i];
        int t = B.dt[k * n + i];
        double4 xa = B.x[e.x];
        double4 xb = B.x[e.y];
        double4 xc = B.x[e.z];
        double4 xd = B.x[e.w];
        R b1x = (R)min_image(xb.x - xa.x, P.L, P.hL), b1y = (R)min_image(xb.y - xa.y, P.L, P.hL),
          b1z = (R)min_image(xb.z - xa.z, P.L, P.hL);
        R b2x = (R)min_image(xc.x - xb.x, P.L, P.hL), b2y = (R)min_image(xc.y - xb.y, P.L, P.hL),
          b2z = (R)min_image(xc.z - xb.z, P.L, P.hL);
        R b3x = (R)min_image(xd.x - xc.x, P.L, P.hL), b3y = (R)min_image(xd.y - xc.y, P.L, P.hL),
          b3z = (R)min_image(xd.z - xc.z, P.L, P.hL);
        R mx = b1y * b2z - b1z * b2y, my = b1z * b2x - b1x * b2z, mz = b1x * b2y - b1y * b2x;
        R nx = b2y * b3z - b2z * b3y, ny = b2z * b3x - b2x * b3z, nz = b2x * b3y - b2y * b3x;
        R m2 = (mx * mx + my * my) + mz * mz;
        R n2 = (nx * nx + ny * ny) + nz * nz;
        R b22 = (b2x * b2x + b2y * b2y) + b2z * b2z;
        if (m2 < (R)1e-24 || n2 < (R)1e-24 || b22 < (R)1e-24) continue;   // collinear: no defined plane
        R nb2 = r_sqrt<R>(b22);
        R inv = r_rsqrt<R>(m2 * n2);
        R cphi = ((mx * nx + my * ny) + mz * nz) * inv;
        R sphi = nb2 * ((b1x * nx + b1y * ny) + b1z * nz) * inv;
        R K = (R)P.dK[t], c0 = (R)P.dC0[t], s0 = (R)P.dS0[t];
        R dU = K * (sphi * c0 - cphi * s0);   // dU/dphi
        R sa = -nb2 * r_rcp<R>(m2), sd = nb2 * r_rcp<R>(n2), ib22 = r_rcp<R>(b22);
        R gax = sa * mx, gay = sa * my, gaz = sa * mz;
        R gdx = sd * nx, gdy = sd * ny, gdz = sd * nz;
        R pp = ((b1x * b2x + b1y * b2y) + b1z * b2z) * ib22;
        R qq = ((b3x * b2x + b3y * b2y) + b3z * b2z) * ib22;
        R fx, fy, fz;
        if (e.x == i) {
            fx = -dU * gax; fy = -dU * gay; fz = -dU * gaz;
        } else if (e.w == i) {
            fx = -dU * gdx; fy = -dU * gdy; fz = -dU * gdz;
        } else if (e.y == i) {
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
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double temperature(const Params& P, int64_t step) {
    if (P.ramp <= 0) return P.T0;
    int64_t k = step < P.ramp ? step : P.ramp;
    return P.T0 + (P.T1 - P.T0) * (double)k / (double)P.ramp;
}

template <typename R, int MODE>
__global__ __launch_bounds__(DB_BLOCK) void k_step(const Params* __restrict__ Pp, Bank B,
                                                    NList NL, double4* __restrict__ xout, int64_t step, double pref,
                                                    unsigned int* __restrict__ vmax2_slot,
                                                    double* __restrict__ fout, int* __restrict__ err) {
    static_assert(MODE == MODE_STEP || MODE == MODE_FORCES, "energies use k_energy");
    const Params& P = *Pp;
    const int n = P.n;
    int tile = xcd_tile(blockIdx.x, gridDim.x);
    int i = tile * DB_BLOCK + threadIdx.x;
    bool active = i < n;
    Acc<R> a;
    double4 xi = make_double4(0, 0, 0, 0);
    double vx = 0, vy = 0, vz = 0;
    if (active) {
        xi = B.x[i];
        int nb = B.nb[i];
        if (P.have_pair) list_pair_forces<R>(P, B, NL, i, xi, a);
        bond_terms<R, MODE>(P, B, i, xi, nb, a);
        angle_terms<R, MODE>(P, B, i, xi, B.na[i], a);
        dihedral_terms<R, MODE>(P, B, i, xi, B.nd[i], a);
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
        double Fx = a.fx, Fy = a.fy, Fz = a.fz;
        if (P.gamma != 0.0) {
            uint4 w = rng_draw(P, (uint32_t)meta_gid(xi), 0u, step, RNG_LANGEVIN);
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
            xo.x = wrap1(nxp, P.L);
            xo.y = wrap1(nyp, P.L);
            xo.z = wrap1(nzp, P.L);
            xo.w = xi.w;
            bool bad = !(xo.x >= 0.0 && xo.x < P.L && xo.y >= 0.0 && xo.y < P.L && xo.z >= 0.0 && xo.z < P.L);
            if (bad) atomicOr(err, ERR_NONFINITE);
            xout[i] = xo;
            B.v[i] = vx;
            B.v[n + i] = vy;
            B.v[2 * n + i] = vz;
        }
    }
    if (MODE == MODE_STEP) {
        // largest speed of the workgroup; one atomic per workgroup, spread over
        // 64 words so that the workgroups of one step do not serialise on one address
        __shared__ float wmax[DB_BLOCK / 64];
        double v2 = active ? (vx * vx + vy * vy) + vz * vz : 0.0;
        v2 = wave_max(v2);
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = (float)v2 * 1.0001f;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = wmax[0];
            for (int w = 1; w < DB_BLOCK / 64; ++w) m = fmaxf(m, wmax[w]);
            atomicMax(vmax2_slot + (blockIdx.x & (DB_VMAX_SPREAD - 1)), __float_as_uint(m));
        }
    }
}

// energy reduction: a separate, simpler kernel keeps the step kernel lean
template <typename R>
__global__ __launch_bounds__(DB_BLOCK) void k_energy(const Params* __restrict__ Pp, Bank B,
                                                      const int* __restrict__ cstart, const int* __restrict__ clist,
                                                      int64_t step, double* __restrict__ epart) {
    const Params& P = *Pp;
    const int n = P.n;
    int i = blockIdx.x * DB_BLOCK + threadIdx.x;
    double vals[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        Acc<R> a;
        double4 xi = B.x[i];
        int nb = B.nb[i];
        int p0 = nb > 0 ? B.bp[i] : -1;
        int p1 = nb > 1 ? B.bp[n + i] : -1;
        int p2 = nb > 2 ? B.bp[2 * n + i] : -1;
        int p3 = nb > 3 ? B.bp[3 * n + i] : -1;
        if (P.have_pair) pair_forces<R, MODE_ENERGY>(P, B, cstart, clist, i, xi, nb, p0, p1, p2, p3, a);
        bond_terms<R, MODE_ENERGY>(P, B, i, xi, nb, a);
        angle_terms<R, MODE_ENERGY>(P, B, i, xi, B.na[i], a);
        dihedral_terms<R, MODE_ENERGY>(P, B, i, xi, B.nd[i], a);
        double vx = B.v[i], vy = B.v[n + i], vz = B.v[2 * n + i];
        double Fx = a.fx, Fy = a.fy, Fz = a.fz;
        if (P.gamma != 0.0) {
            double pref = sqrt(24.0 * P.gamma * temperature(P, step) / P.dt);
            uint4 w = rng_draw(P, (uint32_t)meta_gid(xi), 0u, step, RNG_LANGEVIN);
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

void launch_build_nlist(db_ctx* c) {
    if (c->n == 0) return;
    hipLaunchKernelGGL(k_build_nlist, dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream, c->dp, c->bank[c->cur],
                       c->cells.start, c->cells.xs, c->nlist, c->err_d);
}

// sqrt(24 gamma T(step) / dt), the amplitude of the uniform Langevin noise
static double langevin_prefactor(const Params& P, int64_t step) {
    if (P.gamma == 0.0) return 0.0;
    double T = P.T0;
    if (P.ramp > 0) {
        int64_t k = step < P.ramp ? step : P.ramp;
        T = P.T0 + (P.T1 - P.T0) * (double)k / (double)P.ramp;
    }
    return sqrt(24.0 * P.gamma * T / P.dt);
}

void launch_step(db_ctx* c, int64_t step, int slot_in_block) {
    if (c->n == 0) return;
    const double pref = langevin_prefactor(c->hp, step);
    Bank& B = c->bank[c->cur];
    unsigned* vm = (unsigned*)(c->vmax2 + (size_t)slot_in_block * DB_VMAX_SPREAD);
    if (c->precision == DB_MIXED)
        hipLaunchKernelGGL((k_step<float, MODE_STEP>), dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream, c->dp, B,
                           c->nlist, c->xnext, step, pref, vm, (double*)nullptr, c->err_d);
    else
        hipLaunchKernelGGL((k_step<double, MODE_STEP>), dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream, c->dp,
                           B, c->nlist, c->xnext, step, pref, vm, (double*)nullptr, c->err_d);
    double4* t = B.x;
    B.x = c->xnext;
    c->xnext = t;
}

void launch_forces(db_ctx* c, double* f) {
    if (c->n == 0) return;
    Bank& B = c->bank[c->cur];
    if (c->precision == DB_MIXED)
        hipLaunchKernelGGL((k_step<float, MODE_FORCES>), dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream, c->dp,
                           B, c->nlist, (double4*)nullptr, (int64_t)0, 0.0, (unsigned*)nullptr, f, c->err_d);
    else
        hipLaunchKernelGGL((k_step<double, MODE_FORCES>), dim3(grid_for(c->n)), dim3(DB_BLOCK), 0, c->stream,
                           c->dp, B, c->nlist, (double4*)nullptr, (int64_t)0, 0.0,
                           (unsigned*)nullptr, f, c->err_d);
}

void launch_energy(db_ctx* c, double* out6) {
    unsigned nb = grid_for(c->n);
    Bank& B = c->bank[c->cur];
    if (c->n > 0) {
        if (c->precision == DB_MIXED)
            hipLaunchKernelGGL((k_energy<float>), dim3(nb), dim3(DB_BLOCK), 0, c->stream, c->dp, B, c->cells.start,
                               c->cells.list, c->step, c->red);
        else
            hipLaunchKernelGGL((k_energy<double>), dim3(nb), dim3(DB_BLOCK), 0, c->stream, c->dp, B, c->cells.start,
                               c->cells.list, c->step, c->red);
    }
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, c->stream, c->red, (int)(c->n > 0 ? nb : 0), out6);
}

}  // namespace db
