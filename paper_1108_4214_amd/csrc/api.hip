// Host side of libdynbond: the C-ABI entry points, argument validation, the
// device memory arena, host <-> device transfer of the system, and the step
// scheduler.
//
// Scheduling.  Time is advanced in blocks.  A block starts with a fresh cell
// list (and, every `permute_every` blocks, a reordering of all per-bead state
// into cell order), runs the sweep if the block's first step is a sweep step,
// and then runs up to `rebuild_interval` fused step kernels without rebuilding.
// Each step kernel records the largest speed; after the block the host bounds
// the largest displacement by the sum of dt * max speed.  If that bound exceeds
// half the skin (list cutoff minus pair cutoff) some pair could have been
// missed, so the block's positions and velocities are restored and the block is
// re-run with a fresh list at every step.  The interval adapts to the speeds
// seen.  With DPD the pair friction decorrelates velocities within a few steps,
// so the motion is diffusive and the speed bound far too cautious: there the
// step kernels record the largest displacement from the block's first position
// itself, which is the exact test, and the interval follows its growth.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "db_device.h"

using namespace db;

// ------------------------------------------------------------------------------------
// Scratch of db_energy_noalloc: the per-workgroup partial sums of the energy kernel
// and the six final sums, in a fixed device array (each device holds its own copy for
// the life of the process).  Host code never uses the array's name as an address: the
// device address of each device's copy is looked up once, with that device current,
// when the first handle on it sets up its memory, and kept in noalloc_ptr.
#define DB_NOALLOC_MAX_BLOCKS 65536   // energy workgroups: n <= 65536 * DB_BLOCK beads
static __device__ __align__(256) double scratch[6 * DB_NOALLOC_MAX_BLOCKS + 8];
static constexpr int kMaxDevices = 64;
static double* noalloc_ptr[kMaxDevices];
static std::mutex noalloc_mutex;

namespace {

const int kMaxBlock = 64;
const double kSkinDefault = 0.55;
// DPD at density 3 with the pair friction of the paper moves some bead far enough
// to need a new list after about every step whatever the skin, so the thinnest
// skin (shortest lists, cells of edge r_c) costs least per step
const double kSkinDefaultDPD = 0.02;

// host memory the device writes its end-of-block report into (mapped, pinned)
struct Pinned {
    int err;
    int pad;
    float vmax2[kMaxBlock];        // largest |v|^2 (DPD: squared displacement) after each step of the block
    unsigned long long stats[8];
    double energy[6];
    int total[4];
    double ledger[12];             // energies before and after the sweep of the block
};

// the block's maxima go to the host and their words are cleared for the next block
__global__ void k_report(float* __restrict__ vmax2, int len, const int* __restrict__ err,
                         const unsigned long long* __restrict__ stats, int with_stats, Pinned* __restrict__ out) {
    int q = threadIdx.x;
    if (q < len) {
        float m = 0.0f;
        for (int w = 0; w < DB_VMAX_SPREAD; ++w) {
            m = fmaxf(m, vmax2[q * DB_VMAX_SPREAD + w]);
            vmax2[q * DB_VMAX_SPREAD + w] = 0.0f;
        }
        out->vmax2[q] = m;
    }
    if (q == 0) out->err = *err;
    if (with_stats && q < 8) out->stats[q] = stats[q];
}

struct HostSys {
    std::vector<double> x, v;
    std::vector<int32_t> type;
    std::vector<uint8_t> reactive;
    std::vector<int32_t> bonds;   // 4 per bond: i, j, t_ij, t_ji
    std::vector<int32_t> ang;     // 4 per angle: type, a, b, c (a < c)
    std::vector<int32_t> dih;     // 5 per dihedral: type, a, b, c, d (a < d)
    std::vector<uint16_t> rep;    // replica of each bead (batches only)
};

}  // namespace

struct db_host_ext {
    HostSys h;
    bool host_valid = true;   // host copies reflect the current state
    bool dev_valid = false;   // device holds the current state
    int dev_error = 0;        // latched device error code
    Pinned* pin = nullptr;
    Pinned* pin_dev = nullptr;   // device view of pin
    int* tmp_n1 = nullptr;    // n + 1 ints
};

static db_host_ext& ext(db_ctx* c) { return *c->hx; }

static int fail(db_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
static int fail(db_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(c, expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail((c), DB_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------------------------
// arena layout

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// cell budget: at most 2 n + 64 cells per box
static int ncell_cap(const db_ctx* c) { return 2 * c->n + 64 * std::max(1, c->nrep); }

// brick tiles the arena holds: bricks average ~200 beads; a grid needing more
// tiles than this runs without them
static int tile_cap_of(const db_ctx* c) { return c->nrep > 0 ? 1 : (c->n + DB_BLOCK - 1) / DB_BLOCK + 1; }

// scan scratch: the tile sums of the longest scanned array (one int per tile of
// 4096 items)
static int blocksum_ints(int count) { return (count + 4095) / 4096 + 64; }

struct Layout {
    size_t off[64];
    int k = 0;
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t o = total;
        off[k++] = o;
        total = align256(total + (bytes ? bytes : 1));
        return o;
    }
};

static size_t layout(db_ctx* c, bool assign) {
    const size_t n = (size_t)std::max(c->n, 1);
    const size_t nc = (size_t)ncell_cap(c);
    Layout L;
    auto put = [&](auto*& p, size_t bytes) {
        size_t o = L.add(bytes);
        if (assign) p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(c->arena + o);
    };
    for (int b = 0; b < 2; ++b) {
        Bank& B = c->bank[b];
        put(B.x, 32 * n);
        put(B.v, 24 * n);
        put(B.nb, n);
        put(B.bp, 4 * DB_MAXB * n);
        put(B.bt, DB_MAXB * n);
        put(B.na, n);
        put(B.ang, 16 * DB_MAXA * n);
        put(B.nd, n);
        put(B.dih, 16 * DB_MAXD * n);
        put(B.dt, DB_MAXD * n);
    }
    put(c->xnext, 32 * n);
    put(c->vnext, 24 * n);
    put(c->xref, 32 * n);
    put(c->fext, 24 * n);
    put(c->xsave, 32 * n);
    put(c->vsave, 24 * n);
    SweepBuf& S = c->sw;
    put(S.nomC, 4 * n);
    put(S.ruleC, n);
    put(S.btC, n);
    put(S.nomK, 4 * n);
    put(S.ruleK, n);
    put(S.rmcnt, n);
    put(S.rmlist, 4 * DB_MAXB * n);
    put(S.conv, n);
    put(S.newp, 4 * n);
    put(S.stats, 8 * 8);
    put(S.aoff, 4 * (n + 1));
    put(S.act, 4 * n);
    put(S.chg, n);
    put(S.tchg, n);
    put(S.npurge, n);
    put(S.ngen, n);
    put(c->nlist.nl, 4 * (size_t)DB_NLCAP * n);
    put(c->nlist.cnt, n);
    put(c->halo.nu, n);
    put(c->halo.u, 4 * (size_t)DB_MAXU * n);
    put(c->halo.acode, 4 * (size_t)DB_MAXA * n);
    put(c->halo.dcode, 4 * (size_t)DB_MAXD * n);
    put(c->cells.cnt, 4 * (nc + 1));
    put(c->cells.start, 4 * (nc + 1));
    put(c->cells.list, 4 * n);
    put(c->cells.xs, 16 * (n + DB_XS_PAD));
    put(c->cells.cellid, 4 * n);
    put(c->cells.rank, 4 * n);
    put(c->cells.unsorted, 4 * n);
    put(c->cells.blocksum, 4 * (size_t)blocksum_ints((int)std::max(n, nc) + 1));
    put(c->slot_of_gid, 4 * n);
    if (assign) c->tile_cap = tile_cap_of(c);
    const size_t tcap = (size_t)tile_cap_of(c);
    put(c->tiles.tstart, 4 * ((size_t)ncell_cap(c) + 1));
    put(c->tiles.rcount, 4 * tcap);
    put(c->tiles.rslot, 4 * tcap * DB_RCAP);
    put(c->tiles.nl16, 2 * (size_t)DB_NLCAP * n);
    put(c->tiles.hu16, 2 * (size_t)DB_MAXU * n);
    put(c->tiles.rec, 16 * n);
    put(c->tiles.code8, 32 * n);
    put(c->tiles.itemA, 8 * tcap * DB_CAPA);
    put(c->tiles.itemD, 8 * tcap * DB_CAPD);
    put(c->tiles.nitems, 4 * tcap);
    put(c->err_d, 64);
    put(c->step_dev, 64);
    put(c->vmax2, 4 * (size_t)kMaxBlock * DB_VMAX_SPREAD);
    put(c->red, 8 * 6 * ((n + DB_BLOCK - 1) / DB_BLOCK + 1));
    put(c->ledger_d, 8 * 16);
    put(c->dp, sizeof(Params));
    put(c->rep_d, sizeof(Box) * (size_t)std::max(1, c->nrep));
    int* t1 = nullptr;
    put(t1, 4 * (n + 1));
    if (assign) ext(c).tmp_n1 = t1;
    return L.total;
}

// the device address of this device's copy of the no-allocation scratch, once per device
static int noalloc_setup(db_ctx* c) {
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, DB_EDEVICE, "device ordinal %d beyond %d", dev, kMaxDevices);
    c->device = dev;
    std::lock_guard<std::mutex> lock(noalloc_mutex);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        noalloc_ptr[dev] = (double*)p;
    }
    return DB_OK;
}

static int ensure_memory(db_ctx* c) {
    if (c->allocated) return DB_OK;
    int rc0 = noalloc_setup(c);
    if (rc0) return rc0;
    size_t need = layout(c, false);
    if (!c->arena) {
        void* p = nullptr;
        HIPCHK(c, hipMalloc(&p, need));
        c->arena = (char*)p;
        c->arena_bytes = need;
        c->arena_owned = true;
    }
    layout(c, true);
    if (!ext(c).pin) {
        void* p = nullptr;
        HIPCHK(c, hipHostMalloc(&p, sizeof(Pinned), hipHostMallocMapped));
        ext(c).pin = (Pinned*)p;
        memset(p, 0, sizeof(Pinned));
        void* dptr = nullptr;
        HIPCHK(c, hipHostGetDevicePointer(&dptr, p, 0));
        ext(c).pin_dev = (Pinned*)dptr;
    }
    // zero the counters that kernels assume start at zero
    launch_fill_int(c->cells.cnt, 0, (size_t)ncell_cap(c), c->stream);
    launch_fill_int(c->err_d, 0, 16, c->stream);
    launch_fill_int((int*)c->vmax2, 0, (size_t)kMaxBlock * DB_VMAX_SPREAD, c->stream);
    HIPCHK(c, hipEventCreateWithFlags(&c->ev_report, hipEventDisableTiming));
    c->allocated = true;
    HIPCHK(c, hipGetLastError());
    return DB_OK;
}

// ------------------------------------------------------------------------------------
// parameters and the cell grid

namespace db {
// the step kernel runs on brick tiles: a single box with WCA pairs whose grid has tiles
bool tiles_enabled(const db_ctx* c) {
    return c->tile_mode && c->nrep == 0 && c->ntile > 0 && c->hp.have_pair && c->hp.pair_style == PAIR_WCA;
}
}  // namespace db

// cells of edge >= amin, at most ncap of them
static void box_grid(Box& X, double amin, int ncap) {
    if (!(amin > 0)) amin = X.L;
    int nc = (int)std::floor(X.L / (amin * (1.0 + 1e-9)));
    if (nc < 1) nc = 1;
    while ((long long)nc * nc * nc > ncap && nc > 1) --nc;
    X.nc = nc;
    X.cell_scale = nc / X.L;
    if (nc >= 3) {
        X.noff = 3;
        X.off[0] = -1; X.off[1] = 0; X.off[2] = 1;
    } else if (nc == 2) {
        X.noff = 2;
        X.off[0] = 0; X.off[1] = 1; X.off[2] = 0;
    } else {
        X.noff = 1;
        X.off[0] = 0; X.off[1] = 0; X.off[2] = 0;
    }
}

// 4 sqrt(3) float ulps of 2L: bounds the length error of a separation formed in
// float from coordinates in [0, L) (each rounded once, one of them shifted by the
// rounded edge), so that the float prefilters of the cell scans never drop a pair
// the double test would keep
static double prefilter_slack(double L) {
    int e = 0;
    std::frexp(2.0 * L, &e);                   // 2L = m 2^e, m in [1/2, 1)
    return 4.0 * std::sqrt(3.0) * std::ldexp(1.0, e - 24);
}

static void compute_grid(db_ctx* c) {
    Params& P = c->hp;
    double rc = P.have_pair ? std::sqrt(P.rc2) : 0.0;
    double rcr = std::sqrt(std::max(P.rmax2_create, 0.0));
    double rnl = P.have_pair ? rc + c->skin : 0.0;
    P.rnl2 = rnl * rnl;
    // Cells no narrower than the list cutoff and the creation distance; when the
    // creation distance is the larger one and the box holds five cells of at least
    // half that distance per edge, the cells follow the list cutoff instead and the
    // creation scan reaches two cells (the list build, run every few steps, then
    // scans far fewer candidates).
    auto grid = [&](Box& X, int cap) {
        box_grid(X, std::max(rnl, rcr), cap);
        X.wide_create = 0;
        if (rcr > rnl) {
            Box W = X;
            box_grid(W, std::max(rnl, 0.5 * rcr), cap);
            if (W.nc >= 5 && W.nc > X.nc) {
                X = W;
                X.wide_create = X.L / X.nc < rcr ? 1 : 0;
            }
        }
        X.pf_slack = prefilter_slack(X.L);
        X.pf_create2 = (float)((rcr + X.pf_slack) * (rcr + X.pf_slack) * 1.0001);
        X.pf_list2 = (float)((rnl + X.pf_slack) * (rnl + X.pf_slack) * 1.0001);
    };
    if (c->nrep == 0) {
        grid(P.box, ncell_cap(c));
        P.box.cell_off = 0;
        P.ncell = P.box.nc * P.box.nc * P.box.nc;
        // tiles of DB_BLOCK slots in brick order: bricks of about 200 beads (or the
        // tuned edge), three or more cells per edge
        int bB = 0, ntile = 0;
        const int nc = P.box.nc;
        if (c->tile_mode && nc >= 3 && c->n > 0) {
            const double per_cell = (double)c->n / (double)P.ncell;
            bB = c->brick_edge > 0 ? c->brick_edge : (int)std::floor(std::cbrt(224.0 / per_cell));
            bB = std::max(2, std::min(bB, nc));
            ntile = (c->n + DB_BLOCK - 1) / DB_BLOCK;
        }
        if (ntile != c->ntile || bB != c->tile_bB) {
            c->tiles_valid = false;
            c->regions_valid = false;
        }
        c->ntile = ntile;
        c->tile_bB = bB;
        return;
    }
    int off = 0;
    for (int r = 0; r < c->nrep; ++r) {
        Box& X = c->reps[r];
        grid(X, 2 * c->rep_n[r] + 64);
        X.cell_off = off;
        off += X.nc * X.nc * X.nc;
    }
    P.ncell = off;
}

// Largest displacement any bead may make between neighbour-list builds: a pair
// that comes within the cutoff was within cutoff + skin when the list was built
// as long as neither bead moved more than half the skin.
static double skin_of(const db_ctx* c) {
    if (!c->hp.have_pair) return INFINITY;
    return 0.5 * c->skin;
}

static int upload_params(db_ctx* c) {
    if (!c->params_dirty) return DB_OK;
    compute_grid(c);
    c->hp.n = c->n;
    c->hp.fext = c->fext;
    c->hp.nrep = c->nrep;
    c->hp.rep = c->nrep > 0 ? c->rep_d : nullptr;
    if (c->nrep > 0)
        HIPCHK(c, hipMemcpyAsync(c->rep_d, c->reps.data(), sizeof(Box) * c->reps.size(), hipMemcpyHostToDevice,
                                 c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dp, &c->hp, sizeof(Params), hipMemcpyHostToDevice, c->stream));
    c->params_dirty = false;
    c->list_valid = false;   // the grid or the cutoffs may have changed
    return DB_OK;
}

// ------------------------------------------------------------------------------------
// host <-> device transfer of the whole system (slot = bead id after an upload)

static int upload_system(db_ctx* c) {
    db_host_ext& X = ext(c);
    HostSys& h = X.h;
    const int n = c->n;
    int rc = ensure_memory(c);
    if (rc) return rc;
    c->tiles_valid = false;   // slots follow the input order until the next reordering
    c->regions_valid = false;
    std::vector<double4> x4(n);
    std::vector<double> v(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        x4[i].x = h.x[3 * i];
        x4[i].y = h.x[3 * i + 1];
        x4[i].z = h.x[3 * i + 2];
        x4[i].w = pack_meta(i, h.type[i], h.reactive[i], h.rep.empty() ? 0 : (int)h.rep[i]);
        v[i] = h.v[3 * i];
        v[n + i] = h.v[3 * i + 1];
        v[2 * (size_t)n + i] = h.v[3 * i + 2];
    }
    std::vector<uint8_t> nb(n, 0), na(n, 0), nd(n, 0);
    std::vector<int> bp((size_t)DB_MAXB * n, -1);
    std::vector<int8_t> bt((size_t)DB_MAXB * n, 0);
    std::vector<int4> ang((size_t)DB_MAXA * n);
    std::vector<int4> dih((size_t)DB_MAXD * n);
    std::vector<uint8_t> dt((size_t)DB_MAXD * n, 0);
    const size_t nbonds = h.bonds.size() / 4;
    for (size_t k = 0; k < nbonds; ++k) {
        int i = h.bonds[4 * k], j = h.bonds[4 * k + 1];
        if (nb[i] >= DB_MAXB || nb[j] >= DB_MAXB)
            return fail(c, DB_ECAPACITY, "bead %d or %d has more than %d bonds", i, j, DB_MAXB);
        bp[(size_t)nb[i] * n + i] = j;
        bt[(size_t)nb[i] * n + i] = (int8_t)h.bonds[4 * k + 2];
        ++nb[i];
        bp[(size_t)nb[j] * n + j] = i;
        bt[(size_t)nb[j] * n + j] = (int8_t)h.bonds[4 * k + 3];
        ++nb[j];
    }
    const size_t nang = h.ang.size() / 4;
    for (size_t k = 0; k < nang; ++k) {
        int t = h.ang[4 * k], a = h.ang[4 * k + 1], b = h.ang[4 * k + 2], cc = h.ang[4 * k + 3];
        int mem[3] = {a, b, cc};
        for (int m = 0; m < 3; ++m) {
            int s = mem[m];
            if (na[s] >= DB_MAXA) return fail(c, DB_ECAPACITY, "bead %d is in more than %d angles", s, DB_MAXA);
            ang[(size_t)na[s] * n + s] = make_int4(a, b, cc, t);
            ++na[s];
        }
    }
    const size_t ndih = h.dih.size() / 5;
    for (size_t k = 0; k < ndih; ++k) {
        int t = h.dih[5 * k];
        int mem[4] = {h.dih[5 * k + 1], h.dih[5 * k + 2], h.dih[5 * k + 3], h.dih[5 * k + 4]};
        for (int m = 0; m < 4; ++m) {
            int s = mem[m];
            if (nd[s] >= DB_MAXD) return fail(c, DB_ECAPACITY, "bead %d is in more than %d dihedrals", s, DB_MAXD);
            dih[(size_t)nd[s] * n + s] = make_int4(mem[0], mem[1], mem[2], mem[3]);
            dt[(size_t)nd[s] * n + s] = (uint8_t)t;
            ++nd[s];
        }
    }
    c->cur = 0;
    Bank& B = c->bank[0];
    hipStream_t s = c->stream;
    if (n == 0) {
        X.dev_valid = true;
        X.dev_error = 0;
        return DB_OK;
    }
    HIPCHK(c, hipMemcpyAsync(B.x, x4.data(), 32 * (size_t)n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.v, v.data(), 24 * (size_t)n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.nb, nb.data(), n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.bp, bp.data(), 4 * (size_t)DB_MAXB * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.bt, bt.data(), (size_t)DB_MAXB * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.na, na.data(), n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.ang, ang.data(), 16 * (size_t)DB_MAXA * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.nd, nd.data(), n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.dih, dih.data(), 16 * (size_t)DB_MAXD * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(B.dt, dt.data(), (size_t)DB_MAXD * n, hipMemcpyHostToDevice, s));
    std::vector<int> ident(n);
    std::iota(ident.begin(), ident.end(), 0);
    HIPCHK(c, hipMemcpyAsync(c->slot_of_gid, ident.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    X.dev_valid = true;
    X.dev_error = 0;
    c->halo_force = true;
    c->list_valid = false;
    launch_fill_int(c->err_d, 0, 16, s);
    return DB_OK;
}

namespace db {
void launch_owned_offsets(db_ctx* c, int kind, int* buf);
void launch_write_owned(db_ctx* c, int kind, const int* off, int32_t* tup, int32_t* typ);
}  // namespace db

__global__ void k_gather_state(int n, Bank B, double* __restrict__ xo, double* __restrict__ vo) {
    int s = blockIdx.x * DB_BLOCK + threadIdx.x;
    if (s >= n) return;
    double4 x = B.x[s];
    int g = meta_gid(x);
    if (xo) {
        xo[3 * (size_t)g] = x.x;
        xo[3 * (size_t)g + 1] = x.y;
        xo[3 * (size_t)g + 2] = x.z;
    }
    if (vo) {
        vo[3 * (size_t)g] = B.v[s];
        vo[3 * (size_t)g + 1] = B.v[n + s];
        vo[3 * (size_t)g + 2] = B.v[2 * (size_t)n + s];
    }
}

// scratch for gathers: the per-bead storage of the inactive bank (free between reorders)
static char* gather_scratch(db_ctx* c, size_t bytes) {
    Bank& O = c->bank[1 - c->cur];
    size_t avail = (size_t)((char*)O.nd - (char*)O.ang);
    (void)avail;
    (void)bytes;
    return (char*)O.ang;
}
static size_t gather_scratch_bytes(db_ctx* c) {
    Bank& O = c->bank[1 - c->cur];
    return (size_t)((char*)O.nd - (char*)O.ang);
}

static int read_owned(db_ctx* c, int kind, std::vector<int32_t>& tup, std::vector<int32_t>& typ, int64_t* count) {
    const int n = c->n;
    const int width = kind == 0 ? 2 : (kind == 1 ? 3 : 4);
    const int twidth = kind == 0 ? 2 : 1;
    if (n == 0) {
        *count = 0;
        tup.clear();
        typ.clear();
        return DB_OK;
    }
    int* off = ext(c).tmp_n1;
    launch_owned_offsets(c, kind, off);
    HIPCHK(c, hipMemcpyAsync(&ext(c).pin->total[0], off + n, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int64_t m = ext(c).pin->total[0];
    *count = m;
    size_t need = (size_t)m * 4 * (width + twidth);
    if (need > gather_scratch_bytes(c)) return fail(c, DB_ECAPACITY, "topology list larger than the gather scratch");
    int32_t* dtup = (int32_t*)gather_scratch(c, need);
    int32_t* dtyp = dtup + (size_t)m * width;
    launch_write_owned(c, kind, off, dtup, dtyp);
    tup.resize((size_t)m * width);
    typ.resize((size_t)m * twidth);
    if (m) {
        HIPCHK(c, hipMemcpyAsync(tup.data(), dtup, 4 * (size_t)m * width, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(typ.data(), dtyp, 4 * (size_t)m * twidth, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    return DB_OK;
}

// device -> host copies in bead-id order, canonical and sorted topology
static int download_system(db_ctx* c) {
    db_host_ext& X = ext(c);
    if (X.host_valid || !X.dev_valid) return DB_OK;
    const int n = c->n;
    HostSys& h = X.h;
    if (n > 0) {
        double* d = (double*)gather_scratch(c, 48 * (size_t)n);
        hipLaunchKernelGGL(k_gather_state, dim3((n + DB_BLOCK - 1) / DB_BLOCK), dim3(DB_BLOCK), 0, c->stream, n,
                           c->bank[c->cur], d, d + 3 * (size_t)n);
        HIPCHK(c, hipMemcpyAsync(h.x.data(), d, 24 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(h.v.data(), d + 3 * (size_t)n, 24 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    std::vector<int32_t> tup, typ;
    int64_t m;
    int rc = read_owned(c, 0, tup, typ, &m);
    if (rc) return rc;
    h.bonds.resize(4 * (size_t)m);
    for (int64_t k = 0; k < m; ++k) {
        h.bonds[4 * k] = tup[2 * k];
        h.bonds[4 * k + 1] = tup[2 * k + 1];
        h.bonds[4 * k + 2] = typ[2 * k];
        h.bonds[4 * k + 3] = typ[2 * k + 1];
    }
    rc = read_owned(c, 1, tup, typ, &m);
    if (rc) return rc;
    h.ang.resize(4 * (size_t)m);
    for (int64_t k = 0; k < m; ++k) {
        h.ang[4 * k] = typ[k];
        for (int q = 0; q < 3; ++q) h.ang[4 * k + 1 + q] = tup[3 * k + q];
    }
    rc = read_owned(c, 2, tup, typ, &m);
    if (rc) return rc;
    h.dih.resize(5 * (size_t)m);
    for (int64_t k = 0; k < m; ++k) {
        h.dih[5 * k] = typ[k];
        for (int q = 0; q < 4; ++q) h.dih[5 * k + 1 + q] = tup[4 * k + q];
    }
    X.host_valid = true;
    return DB_OK;
}

// make the device state current (upload once after host-side edits)
static int ready(db_ctx* c) {
    db_host_ext& X = ext(c);
    if (!c->have_state) return fail(c, DB_ESTATE, "db_set_state has not been called");
    if (X.dev_error) return fail(c, X.dev_error, "a previous device error left the state undefined: %s", c->err.c_str());
    int rc = ensure_memory(c);
    if (rc) return rc;
    rc = upload_params(c);
    if (rc) return rc;
    if (!X.dev_valid) {
        rc = upload_system(c);
        if (rc) return rc;
    }
    return DB_OK;
}

// host-side edits start from a current host copy
static int editable(db_ctx* c) {
    db_host_ext& X = ext(c);
    if (X.dev_valid && !X.host_valid && !X.dev_error) {
        int rc = download_system(c);
        if (rc) return rc;
    }
    X.dev_valid = false;
    return DB_OK;
}

static int check_device_error(db_ctx* c) {
    db_host_ext& X = ext(c);
    int e = X.pin->err;
    if (!e) return DB_OK;
    int code = (e & (ERR_BOND_CAP | ERR_ANGLE_CAP | ERR_DIH_CAP | ERR_NLIST)) ? DB_ECAPACITY : DB_ENONFINITE;
    X.dev_error = code;
    return fail(c, code, "device reported %s%s%s%s%s",
                (e & ERR_BOND_CAP) ? "bond-table overflow " : "", (e & ERR_ANGLE_CAP) ? "angle-table overflow " : "",
                (e & ERR_DIH_CAP) ? "dihedral-table overflow " : "",
                (e & ERR_NLIST) ? "neighbour-list overflow " : "",
                (e & ERR_NONFINITE) ? "non-finite or escaping position" : "");
}

// cells_ready: the cell list was already built for the current positions
static void rebuild(db_ctx* c, bool permute, bool save = false, bool cells_ready = false) {
    if (!cells_ready) launch_build_cells(c);
    if (permute) launch_permute(c, save);
    c->rebuilds++;
}

// rows of src: tuple then types (typ_first = 0) or types then tuple (typ_first = 1);
// written sorted by tuple, then type
template <int W, int TW>
static void sorted_copy(const std::vector<int32_t>& src, int32_t* tup, int32_t* typ, int typ_first) {
    // src rows: [typ_first ? type, tuple : tuple, types]
    const size_t rows = src.size() / (W + TW);
    std::vector<size_t> idx(rows);
    std::iota(idx.begin(), idx.end(), 0);
    auto key = [&](size_t r, int q) { return src[r * (W + TW) + (typ_first ? TW : 0) + q]; };
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
        for (int q = 0; q < W; ++q)
            if (key(a, q) != key(b, q)) return key(a, q) < key(b, q);
        for (int q = 0; q < TW; ++q) {
            int ta = src[a * (W + TW) + (typ_first ? q : W + q)], tb = src[b * (W + TW) + (typ_first ? q : W + q)];
            if (ta != tb) return ta < tb;
        }
        return false;
    });
    for (size_t k = 0; k < rows; ++k) {
        size_t r = idx[k];
        for (int q = 0; q < W; ++q) tup[k * W + q] = key(r, q);
        for (int q = 0; q < TW; ++q) typ[k * TW + q] = src[r * (W + TW) + (typ_first ? q : W + q)];
    }
}

// ------------------------------------------------------------------------------------
// C-ABI

extern "C" {

int db_create(db_ctx** out, int32_t n, double L, uint64_t seed, int precision, void* stream) {
    if (!out) return DB_EINVAL;
    *out = nullptr;
    if (n < 0 || n > DB_MAX_BEADS || !(L > 0) || !(L <= DB_MAX_BOX_EDGE)) return DB_EINVAL;
    if (precision != DB_FP64 && precision != DB_MIXED) return DB_EINVAL;
    db_ctx* c = new db_ctx();
    c->hx = new db_host_ext();
    c->n = n;
    c->L = L;
    c->seed = seed;
    c->precision = precision;
    c->stream = (hipStream_t)stream;
    c->device = -1;
    c->step_dev = nullptr;
    c->step_base_d = nullptr;
    c->use_graph = false;
    c->graphs = new std::vector<GraphEntry>();
    c->cap_stream = nullptr;
    c->tile_mode = 0;   // db_tile_shape / db_autotune switch the tile kernel on
    c->brick_edge = 0;
    c->ntile = 0;
    c->tile_bB = 0;
    c->tile_cap = 0;
    c->tiles_valid = false;
    c->regions_valid = false;
    memset(&c->hp, 0, sizeof(Params));
    Params& P = c->hp;
    P.n = n;
    P.box.L = L;
    P.box.hL = 0.5 * L;
    P.box.invL = 1.0 / L;
    P.box.seed_lo = (uint32_t)seed;
    P.box.seed_hi = (uint32_t)(seed >> 32);
    P.box.T0 = P.box.T1 = 1.0;
    P.dt = 0.005;
    P.excl_depth = 1;
    for (int t = 0; t < DB_MAXT; ++t) P.bRc2[t] = INFINITY;
    c->params_dirty = true;
    c->skin = kSkinDefault;
    c->skin_tuned = false;
    c->profile = false;
    c->ev_report = nullptr;
    c->profile_every = 1;
    c->profile_count = 0;
    c->list_valid = false;
    c->list_disp = 0.0;
    c->disp_rate = 0.0;
    c->patches = 0;
    c->swept_step = -1;
    c->rebuild_interval = 8;
    c->permute_every = 8;
    c->vmax_est = 0;
    HostSys& h = c->hx->h;
    h.x.assign(3 * (size_t)n, 0.0);
    h.v.assign(3 * (size_t)n, 0.0);
    h.type.assign(n, 1);
    h.reactive.assign(n, 1);
    *out = c;
    return DB_OK;
}

int db_workspace_bytes(const db_ctx* c, size_t* bytes) {
    if (!c || !bytes) return DB_EINVAL;
    *bytes = layout(const_cast<db_ctx*>(c), false);
    return DB_OK;
}

int db_bind_workspace(db_ctx* c, void* p, size_t bytes) {
    if (!c) return DB_EINVAL;
    if (c->allocated) return fail(c, DB_ESTATE, "workspace already allocated");
    size_t need = layout(c, false);
    if (!p || bytes < need || ((uintptr_t)p & 255))
        return fail(c, DB_EINVAL, "workspace needs %zu bytes, 256-byte aligned", need);
    c->arena = (char*)p;
    c->arena_bytes = bytes;
    c->arena_owned = false;
    return DB_OK;
}

int db_destroy(db_ctx* c) {
    if (!c) return DB_EINVAL;
    db_host_ext& X = ext(c);
    if (c->allocated) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->ev_report) (void)hipEventDestroy(c->ev_report);
    for (GraphEntry& e : *c->graphs) {
        (void)hipGraphExecDestroy(e.exec);
        (void)hipGraphDestroy(e.graph);
    }
    delete c->graphs;
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->arena_owned && c->arena) (void)hipFree(c->arena);
    if (X.pin) (void)hipHostFree(X.pin);
    delete c->hx;
    delete c;
    return DB_OK;
}

const char* db_last_error(const db_ctx* c) { return c ? c->err.c_str() : "null handle"; }

int db_set_state(db_ctx* c, const double* x, const double* v, const int32_t* type, int on_device) {
    if (!c || !x || !type) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_ESTATE, "a batch takes its state and topology from its replicas");
    int rc = editable(c);
    if (rc) return rc;
    HostSys& h = ext(c).h;
    const size_t n = (size_t)c->n;
    std::vector<double> xs(3 * n), vs(3 * n, 0.0);
    std::vector<int32_t> ts(n);
    if (on_device) {
        if (n) {
            HIPCHK(c, hipMemcpy(xs.data(), x, 24 * n, hipMemcpyDeviceToHost));
            if (v) HIPCHK(c, hipMemcpy(vs.data(), v, 24 * n, hipMemcpyDeviceToHost));
            HIPCHK(c, hipMemcpy(ts.data(), type, 4 * n, hipMemcpyDeviceToHost));
        }
    } else {
        std::copy(x, x + 3 * n, xs.begin());
        if (v) std::copy(v, v + 3 * n, vs.begin());
        std::copy(type, type + n, ts.begin());
    }
    for (size_t i = 0; i < 3 * n; ++i) {
        if (!std::isfinite(xs[i]) || xs[i] < 0 || xs[i] >= c->L)
            return fail(c, DB_EINVAL, "position %zu = %g outside [0, L)", i / 3, xs[i]);
        if (!std::isfinite(vs[i])) return fail(c, DB_EINVAL, "velocity of bead %zu not finite", i / 3);
    }
    for (size_t i = 0; i < n; ++i)
        if (ts[i] < 1 || ts[i] > 31) return fail(c, DB_EINVAL, "bead %zu has type %d outside 1..31", i, ts[i]);
    h.x.swap(xs);
    h.v.swap(vs);
    h.type.swap(ts);
    c->have_state = true;
    ext(c).dev_error = 0;
    return DB_OK;
}

int db_set_reactive(db_ctx* c, const uint8_t* flag) {
    if (!c || !flag) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_ESTATE, "a batch takes its state and topology from its replicas");
    int rc = editable(c);
    if (rc) return rc;
    HostSys& h = ext(c).h;
    for (int i = 0; i < c->n; ++i) h.reactive[i] = flag[i] ? 1 : 0;
    return DB_OK;
}

int db_set_bonds(db_ctx* c, int64_t nb, const int32_t* ij, const int32_t* tij, const int32_t* tji) {
    if (!c || nb < 0 || (nb > 0 && (!ij || !tij || !tji))) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_ESTATE, "a batch takes its state and topology from its replicas");
    int rc = editable(c);
    if (rc) return rc;
    std::vector<int> deg(c->n, 0);
    std::vector<int32_t> b(4 * (size_t)nb);
    for (int64_t k = 0; k < nb; ++k) {
        int i = ij[2 * k], j = ij[2 * k + 1];
        if (i < 0 || j < 0 || i >= c->n || j >= c->n || i == j)
            return fail(c, DB_EINVAL, "bond %lld joins invalid beads %d, %d", (long long)k, i, j);
        if (tij[k] < 1 || tij[k] >= DB_MAXT || tji[k] < 1 || tji[k] >= DB_MAXT)
            return fail(c, DB_EINVAL, "bond %lld has a type outside 1..%d", (long long)k, DB_MAXT - 1);
        if (++deg[i] > DB_MAXB || ++deg[j] > DB_MAXB)
            return fail(c, DB_ECAPACITY, "a bead has more than %d bonds", DB_MAXB);
        int a = i, bb = j, ta = tij[k], tb = tji[k];
        if (a > bb) {
            std::swap(a, bb);
            std::swap(ta, tb);
        }
        b[4 * k] = a;
        b[4 * k + 1] = bb;
        b[4 * k + 2] = ta;
        b[4 * k + 3] = tb;
    }
    HostSys& h = ext(c).h;
    h.bonds.swap(b);
    h.ang.clear();
    h.dih.clear();
    return DB_OK;
}

int db_set_angles(db_ctx* c, int64_t na, const int32_t* abc, const int32_t* type) {
    if (!c || na < 0 || (na > 0 && (!abc || !type))) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_ESTATE, "a batch takes its state and topology from its replicas");
    int rc = editable(c);
    if (rc) return rc;
    std::vector<int32_t> a(4 * (size_t)na);
    for (int64_t k = 0; k < na; ++k) {
        int x = abc[3 * k], y = abc[3 * k + 1], z = abc[3 * k + 2];
        if (x < 0 || y < 0 || z < 0 || x >= c->n || y >= c->n || z >= c->n || x == y || y == z || x == z)
            return fail(c, DB_EINVAL, "angle %lld has invalid beads", (long long)k);
        if (type[k] < 1 || type[k] >= DB_MAXT) return fail(c, DB_EINVAL, "angle %lld has an invalid type", (long long)k);
        if (x > z) std::swap(x, z);
        a[4 * k] = type[k];
        a[4 * k + 1] = x;
        a[4 * k + 2] = y;
        a[4 * k + 3] = z;
    }
    ext(c).h.ang.swap(a);
    return DB_OK;
}

int db_set_dihedrals(db_ctx* c, int64_t nd, const int32_t* abcd, const int32_t* type) {
    if (!c || nd < 0 || (nd > 0 && (!abcd || !type))) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_ESTATE, "a batch takes its state and topology from its replicas");
    int rc = editable(c);
    if (rc) return rc;
    std::vector<int32_t> d(5 * (size_t)nd);
    for (int64_t k = 0; k < nd; ++k) {
        int m[4] = {abcd[4 * k], abcd[4 * k + 1], abcd[4 * k + 2], abcd[4 * k + 3]};
        for (int q = 0; q < 4; ++q)
            if (m[q] < 0 || m[q] >= c->n) return fail(c, DB_EINVAL, "dihedral %lld has invalid beads", (long long)k);
        if (type[k] < 1 || type[k] >= DB_MAXT)
            return fail(c, DB_EINVAL, "dihedral %lld has an invalid type", (long long)k);
        if (m[0] > m[3]) {
            std::swap(m[0], m[3]);
            std::swap(m[1], m[2]);
        }
        d[5 * k] = type[k];
        for (int q = 0; q < 4; ++q) d[5 * k + 1 + q] = m[q];
    }
    ext(c).h.dih.swap(d);
    return DB_OK;
}

int db_generate_angles_dihedrals(db_ctx* c) {
    if (!c) return DB_EINVAL;
    int rc = ready(c);
    if (rc) return rc;
    launch_generate_all(c);
    HIPCHK(c, hipMemcpyAsync(&ext(c).pin->err, c->err_d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    ext(c).host_valid = false;
    return check_device_error(c);
}

// ---- force field ----
int db_pair_wca(db_ctx* c, double eps, double sigma, double rc, int depth) {
    if (!c || !(rc > 0) || !(sigma > 0) || eps < 0 || depth < 0 || depth > 2) return DB_EINVAL;
    if (2.0 * rc > c->L) return fail(c, DB_EINVAL, "box edge must exceed twice the pair cutoff");
    Params& P = c->hp;
    P.have_pair = 1;
    P.pair_style = PAIR_WCA;
    if (!c->skin_tuned) c->skin = kSkinDefault;
    P.eps = eps;
    P.sig2 = sigma * sigma;
    P.rc2 = rc * rc;
    P.rc = rc;
    P.inv_rc = 1.0 / rc;
    P.excl_depth = depth;
    c->params_dirty = true;
    return DB_OK;
}

int db_pair_dpd(db_ctx* c, double a, double gamma, double rc, int depth) {
    if (!c || !(rc > 0) || !std::isfinite(a) || !(gamma >= 0) || !std::isfinite(gamma) || depth < 0 || depth > 2)
        return DB_EINVAL;
    if (2.0 * rc > c->L) return fail(c, DB_EINVAL, "box edge must exceed twice the pair cutoff");
    Params& P = c->hp;
    P.have_pair = 1;
    P.pair_style = PAIR_DPD;
    if (!c->skin_tuned) c->skin = kSkinDefaultDPD;
    P.dpd_a = a;
    P.dpd_gamma = gamma;
    P.rc2 = rc * rc;
    P.rc = rc;
    P.inv_rc = 1.0 / rc;
    P.excl_depth = depth;
    c->params_dirty = true;
    return DB_OK;
}

int db_external_force(db_ctx* c, int64_t count, const int32_t* ids, const double* f) {
    if (!c || count < 0 || (count > 0 && (!ids || !f))) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_ESTATE, "a batch takes no external forces");
    std::vector<double> t(3 * (size_t)c->n, 0.0);
    for (int64_t k = 0; k < count; ++k) {
        const int i = ids[k];
        if (i < 0 || i >= c->n) return fail(c, DB_EINVAL, "external force %lld on invalid bead %d", (long long)k, i);
        for (int q = 0; q < 3; ++q) {
            if (!std::isfinite(f[3 * k + q])) return fail(c, DB_EINVAL, "non-finite external force %lld", (long long)k);
            t[3 * (size_t)i + q] += f[3 * k + q];
        }
    }
    int rc = ensure_memory(c);
    if (rc) return rc;
    if (c->n > 0) {
        HIPCHK(c, hipMemcpyAsync(c->fext, t.data(), 24 * (size_t)c->n, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->hp.has_ext = count > 0 ? 1 : 0;
    c->params_dirty = true;
    return DB_OK;
}

int db_bond_harmonic(db_ctx* c, int32_t t, double K, double r0) {
    if (!c || t < 1 || t >= DB_MAXT || !std::isfinite(K) || !std::isfinite(r0)) return DB_EINVAL;
    c->hp.bK[t] = K;
    c->hp.bR0[t] = r0;
    c->hp.bE0[t] = 0.0;
    c->hp.bRc2[t] = INFINITY;
    c->params_dirty = true;
    return DB_OK;
}

// the well is the harmonic bond K (r - r_w)^2 with K = U_min / (r_z - r_w)^2,
// shifted by -U_min, and cut at r_cut
int db_bond_well(db_ctx* c, int32_t t, double umin, double rw, double rz, double rcut) {
    if (!c || t < 1 || t >= DB_MAXT || !std::isfinite(umin) || !std::isfinite(rw) || !std::isfinite(rz) || rz == rw ||
        !(rcut > 0))
        return DB_EINVAL;
    c->hp.bK[t] = umin / ((rz - rw) * (rz - rw));
    c->hp.bR0[t] = rw;
    c->hp.bE0[t] = -umin;
    c->hp.bRc2[t] = std::isfinite(rcut) ? rcut * rcut : INFINITY;
    c->params_dirty = true;
    return DB_OK;
}

int db_angle_harmonic(db_ctx* c, int32_t t, double K, double th0) {
    if (!c || t < 1 || t >= DB_MAXT || !std::isfinite(K) || !std::isfinite(th0)) return DB_EINVAL;
    c->hp.aK[t] = K;
    c->hp.aT0[t] = th0;
    c->hp.aPiMinusT0[t] = 3.14159265358979323846 - th0;
    c->params_dirty = true;
    return DB_OK;
}

int db_dihedral_cosine(db_ctx* c, int32_t t, double K, double p0) {
    if (!c || t < 1 || t >= DB_MAXT || !std::isfinite(K) || !std::isfinite(p0)) return DB_EINVAL;
    c->hp.dK[t] = K;
    c->hp.dC0[t] = std::cos(p0);
    c->hp.dS0[t] = std::sin(p0);
    c->params_dirty = true;
    return DB_OK;
}

// the temperature schedule of a single system, or of every replica of a batch
static void set_schedule(db_ctx* c, double T0, double T1, int64_t n) {
    c->hp.box.T0 = T0;
    c->hp.box.T1 = T1;
    c->hp.box.ramp = n;
    for (Box& X : c->reps) {
        X.T0 = T0;
        X.T1 = T1;
        X.ramp = n;
    }
}

int db_langevin(db_ctx* c, double T, double gamma, double dt) {
    if (!c || !(dt > 0) || gamma < 0 || T < 0) return DB_EINVAL;
    set_schedule(c, T, T, 0);
    c->hp.gamma = gamma;
    c->hp.dt = dt;
    c->params_dirty = true;
    return DB_OK;
}

int db_temperature_ramp(db_ctx* c, double T0, double T1, int64_t n) {
    if (!c || n < 0 || T0 < 0 || T1 < 0) return DB_EINVAL;
    set_schedule(c, T0, T1, n);
    c->params_dirty = true;
    return DB_OK;
}

// ---- rules ----
static void note_create_types(Params& P, int b1, int b2) {
    if (b1 == 0 || b2 == 0) P.create_types = 0xFFFFFFFFu;
    else P.create_types |= (1u << (b1 & 31)) | (1u << (b2 & 31));
}

static int add_rule(db_ctx* c, Rule r) {
    Params& P = c->hp;
    if (P.nrule >= DB_MAXRULES) return fail(c, DB_ECAPACITY, "at most %d bond rules", DB_MAXRULES);
    P.rule[P.nrule++] = r;
    if (r.kind == RK_CREATE || r.kind == RK_CREATEDIR) {
        double rmax = std::sqrt(r.r2);
        if (2.0 * rmax > c->L) {
            --P.nrule;
            return fail(c, DB_EINVAL, "box edge must exceed twice the reaction distance");
        }
        P.rmax2_create = std::max(P.rmax2_create, r.r2);
        note_create_types(P, r.b1, r.b2);
    }
    if (r.kind == RK_BREAK || r.kind == RK_CONVERT) P.has_break_class = 1;
    if (r.kind == RK_KILL) P.has_kill = 1;
    if (r.kind == RK_BREAK || r.kind == RK_CONVERT || r.kind == RK_KILL) P.break_types |= 1u << r.bt1;
    c->params_dirty = true;
    return DB_OK;
}

static bool bad_bt(int t) { return t < 1 || t >= DB_MAXT; }
static bool bad_bead(int b) { return b < 0 || b > 31; }
static bool bad_p(double p) { return !(p >= 0.0 && p <= 1.0); }

int db_sweep_every(db_ctx* c, int32_t every, int pc13, int pc14) {
    if (!c || every < 0) return DB_EINVAL;
    c->hp.every = every;
    c->hp.pc13 = pc13 ? 1 : 0;
    c->hp.pc14 = pc14 ? 1 : 0;
    c->params_dirty = true;
    return DB_OK;
}

int db_acceptance(db_ctx* c, int mode) {
    if (!c) return DB_EINVAL;
    if (mode != DB_ACCEPT_PAIR && mode != DB_ACCEPT_AVERAGE) return fail(c, DB_EINVAL, "acceptance mode %d", mode);
    c->hp.accept_average = mode == DB_ACCEPT_AVERAGE ? 1 : 0;
    c->params_dirty = true;
    return DB_OK;
}

int db_bond_create(db_ctx* c, int32_t bt, int32_t b1, int32_t b2, double rmax, double p) {
    if (!c || bad_bt(bt) || bad_bead(b1) || bad_bead(b2) || !(rmax > 0) || bad_p(p)) return DB_EINVAL;
    return add_rule(c, Rule{RK_CREATE, bt, bt, b1, b2, rmax * rmax, p});
}

int db_bond_create_dir(db_ctx* c, int32_t bt1, int32_t bt2, int32_t b1, int32_t b2, double rmax, double p) {
    if (!c || bad_bt(bt1) || bad_bt(bt2) || bad_bead(b1) || bad_bead(b2) || !(rmax > 0) || bad_p(p)) return DB_EINVAL;
    return add_rule(c, Rule{RK_CREATEDIR, bt1, bt2, b1, b2, rmax * rmax, p});
}

int db_bond_break(db_ctx* c, int32_t bt, double rmin, double p) {
    if (!c || bad_bt(bt) || !(rmin >= 0) || bad_p(p)) return DB_EINVAL;
    return add_rule(c, Rule{RK_BREAK, bt, bt, 0, 0, rmin * rmin, p});
}

int db_bond_kill(db_ctx* c, int32_t bt, double rmin) {
    if (!c || bad_bt(bt) || !(rmin >= 0)) return DB_EINVAL;
    return add_rule(c, Rule{RK_KILL, bt, bt, 0, 0, rmin * rmin, 1.0});
}

int db_bond_convert(db_ctx* c, int32_t bf, int32_t bto, double rmin, double p) {
    if (!c || bad_bt(bf) || bad_bt(bto) || !(rmin >= 0) || bad_p(p)) return DB_EINVAL;
    return add_rule(c, Rule{RK_CONVERT, bf, bto, 0, 0, rmin * rmin, p});
}

int db_max_bonds(db_ctx* c, int32_t bt, int32_t bead, int32_t max) {
    if (!c || bad_bt(bt) || bad_bead(bead) || max < 0) return DB_EINVAL;
    Params& P = c->hp;
    if (P.nmax >= DB_MAXRULES) return fail(c, DB_ECAPACITY, "at most %d maxbond rules", DB_MAXRULES);
    P.maxr[P.nmax++] = MaxRule{bt, bead, max};
    c->params_dirty = true;
    return DB_OK;
}

int db_angle_pattern(db_ctx* c, int32_t t, const int32_t b[3], const uint32_t m[2]) {
    if (!c || !b || !m || bad_bt(t)) return DB_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (bad_bead(b[k])) return DB_EINVAL;
    Params& P = c->hp;
    if (P.narule >= DB_MAXRULES) return fail(c, DB_ECAPACITY, "at most %d angle rules", DB_MAXRULES);
    AngRule r;
    r.type = t;
    for (int k = 0; k < 3; ++k) r.b[k] = b[k];
    r.m[0] = m[0];
    r.m[1] = m[1];
    P.arule[P.narule++] = r;
    c->params_dirty = true;
    return DB_OK;
}

int db_dihedral_pattern(db_ctx* c, int32_t t, const int32_t b[4], const uint32_t m[3]) {
    if (!c || !b || !m || bad_bt(t)) return DB_EINVAL;
    for (int k = 0; k < 4; ++k)
        if (bad_bead(b[k])) return DB_EINVAL;
    Params& P = c->hp;
    if (P.ndrule >= DB_MAXRULES) return fail(c, DB_ECAPACITY, "at most %d dihedral rules", DB_MAXRULES);
    DihRule r;
    r.type = t;
    for (int k = 0; k < 4; ++k) r.b[k] = b[k];
    for (int k = 0; k < 3; ++k) r.m[k] = m[k];
    P.drule[P.ndrule++] = r;
    c->params_dirty = true;
    return DB_OK;
}

// ---- running ----
static void record_sweep_stats(db_ctx* c) {
    Pinned* pin = ext(c).pin;
    for (int q = 0; q < 8; ++q) {
        c->stat_last[q] = (int64_t)pin->stats[q];
        c->stat_cum[q] += (int64_t)pin->stats[q];
    }
    if (c->ledger) {
        double du = 0.0;
        for (int k = 1; k <= 4; ++k) du += pin->ledger[6 + k] - pin->ledger[k];
        c->du_last = du;
        c->du_cum += du;
    }
    c->sweeps++;
}

// the sweep of a step, bracketed by potential-energy evaluations when the ledger is on
static int run_sweep(db_ctx* c, int64_t step) {
    if (c->ledger) launch_energy(c, c->ledger_d);
    launch_sweep(c, step);
    if (c->ledger) {
        launch_energy(c, c->ledger_d + 6);
        HIPCHK(c, hipMemcpyAsync(ext(c).pin->ledger, c->ledger_d, 96, hipMemcpyDeviceToHost, c->stream));
    }
    return DB_OK;
}

static int launch_timed_step(db_ctx* c, int64_t step, int slot, bool save) {
    if (c->profile && (c->profile_count++ % c->profile_every) == 0) {
        if ((size_t)c->ev_used + 2 > c->ev_pool.size()) {
            for (int k = 0; k < 2 * kMaxBlock; ++k) {
                hipEvent_t e;
                HIPCHK(c, hipEventCreate(&e));
                c->ev_pool.push_back(e);
            }
        }
        HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used], c->stream));
        launch_step(c, step, slot, save);
        HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used + 1], c->stream));
        c->ev_used += 2;
    } else {
        launch_step(c, step, slot, save);
    }
    return DB_OK;
}

static int harvest_events(db_ctx* c) {
    for (int k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
        c->prof_ms += ms;
        c->prof_launches++;
    }
    c->ev_used = 0;
    return DB_OK;
}

__global__ void k_set_step(int64_t* __restrict__ p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// The len step launches of a block from a captured graph: captured once per
// (length, rollback copy, buffers, kernel) and replayed with the block's first step
// written to the device beforehand.  Only kernel nodes are captured.
static int run_steps_graph(db_ctx* c, int64_t k0, int len, bool save) {
    Bank& B = c->bank[c->cur];
    const bool tiled = tiles_enabled(c) && c->tiles_valid && c->regions_valid;
    GraphEntry* hit = nullptr;
    for (GraphEntry& e : *c->graphs)
        if (e.len == len && e.save == save && e.tiled == tiled && e.cur == c->cur && e.x == B.x &&
            e.xnext == c->xnext && e.v == B.v && e.vnext == c->vnext) {
            hit = &e;
            break;
        }
    if (!hit) {
        if (c->graphs->size() >= 64) {   // a bounded cache: start afresh
            for (GraphEntry& e : *c->graphs) {
                (void)hipGraphExecDestroy(e.exec);
                (void)hipGraphDestroy(e.graph);
            }
            c->graphs->clear();
        }
        GraphEntry e{};
        e.len = len;
        e.save = save;
        e.tiled = tiled;
        e.cur = c->cur;
        e.x = B.x;
        e.xnext = c->xnext;
        e.v = B.v;
        e.vnext = c->vnext;
        // the null stream cannot be captured: capture on a stream of the handle's own
        hipStream_t run = c->stream;
        if (!run && !c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t cap = run ? run : c->cap_stream;
        double4* x0 = B.x;
        double4* xn0 = c->xnext;
        double* v0 = B.v;
        double* vn0 = c->vnext;
        c->stream = cap;
        c->step_base_d = c->step_dev;
        hipError_t st = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (st == hipSuccess) {
            for (int q = 0; q < len; ++q) launch_step(c, q, q, save && q == 0);
            st = hipStreamEndCapture(cap, &e.graph);
        }
        c->step_base_d = nullptr;
        c->stream = run;
        e.x_after = B.x;
        e.xnext_after = c->xnext;
        e.v_after = B.v;
        e.vnext_after = c->vnext;
        B.x = x0;   // nothing ran yet: the buffers swap when the graph runs
        c->xnext = xn0;
        B.v = v0;
        c->vnext = vn0;
        if (st != hipSuccess) return fail(c, DB_EDEVICE, "graph capture: %s", hipGetErrorString(st));
        HIPCHK(c, hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
        c->graphs->push_back(e);
        hit = &c->graphs->back();
    }
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, c->stream, c->step_dev, k0);
    HIPCHK(c, hipGraphLaunch(hit->exec, c->stream));
    B.x = (double4*)hit->x_after;
    c->xnext = (double4*)hit->xnext_after;
    B.v = (double*)hit->v_after;
    c->vnext = (double*)hit->vnext_after;
    return DB_OK;
}

// The list can be kept across sweeps when pairs interact and every box has at
// least five cells per edge (the patched lists scan two cell edges around a bead).
static bool list_reuse_allowed(const db_ctx* c) {
    if (!c->hp.have_pair || c->hp.every <= 0 || !std::isfinite(skin_of(c))) return false;
    if (c->nrep == 0) return c->hp.box.nc >= 5;
    for (const Box& X : c->reps)
        if (X.nc < 5) return false;
    return true;
}

int db_step(db_ctx* c, int64_t nsteps) {
    if (!c || nsteps < 0) return DB_EINVAL;
    int rc = ready(c);
    if (rc) return rc;
    db_host_ext& X = ext(c);
    Pinned* pin = X.pin;
    const double dt = c->hp.dt;
    const int every = c->hp.every;
    const double skin = skin_of(c);
    const bool track = c->hp.have_pair && c->hp.pair_style == PAIR_DPD;   // displacement, not speed
    const bool reuse_ok = list_reuse_allowed(c);
    // widest cutoff of a redone list whose expected length, at the densest box's
    // density, stays within half the list's capacity
    double dens = (double)c->n / (c->L * c->L * c->L);
    for (size_t r = 0; r < c->reps.size(); ++r)
        dens = std::max(dens, (double)c->rep_n[r] / (c->reps[r].L * c->reps[r].L * c->reps[r].L));
    const double reuse_cut_max = dens > 0 ? std::cbrt(0.5 * DB_NLCAP / (4.18879020478639 * dens)) : INFINITY;
    hipStream_t s = c->stream;
    bool cells_ready = false;   // built after the previous block's report, while the host waited
    while (nsteps > 0) {
        const int64_t k0 = c->step;
        const bool sweep_due = every > 0 && k0 % every == 0 && c->swept_step != k0;
        int64_t len = std::min<int64_t>(nsteps, std::min(c->rebuild_interval, kMaxBlock));
        if (every > 0) len = std::min<int64_t>(len, every - (k0 % every));
        // A block cut short by its sweep keeps the Verlet list when the displacement
        // bound since the list's full build, grown by this block, stays within half
        // the skin: only the lists of beads whose exclusions the sweep changed are
        // redone, with the cutoff widened by twice that bound (so that every list
        // stays valid while the bound does).
        const double grow = (track ? c->disp_rate : dt * c->vmax_est) * (double)len;
        const double patch_cut = std::sqrt(c->hp.rc2) + c->skin + 2.0 * c->list_disp;
        const bool reuse = reuse_ok && sweep_due && c->list_valid && c->list_disp + 1.25 * grow <= skin &&
                           patch_cut <= reuse_cut_max;
        const double d0 = reuse ? c->list_disp : 0.0;   // bound at the block's input
        bool permute = false;
        const bool guard = std::isfinite(skin) && len > 1;
        if (reuse) {
            rebuild(c, false, false, cells_ready);   // current cells for the sweep and the patched lists
            rc = run_sweep(c, k0);
            if (rc) return rc;
            c->swept_step = k0;
            launch_patch_nlist(c, patch_cut);
            c->patches++;
        } else {
            permute = (c->rebuild_count++ % c->permute_every) == 0;
            rebuild(c, permute, guard, cells_ready);
            if (sweep_due) {
                rc = run_sweep(c, k0);
                if (rc) return rc;
                c->swept_step = k0;
            }
            launch_build_nlist(c);   // after the sweep: exclusions follow the new bonds
        }
        // the block's input state is kept for a re-run: by the reorder, or else by
        // the first step kernel of the block
        if (c->use_graph && !c->profile) {
            rc = run_steps_graph(c, k0, (int)len, guard && !permute);
            if (rc) return rc;
        } else {
            for (int64_t q = 0; q < len; ++q) {
                rc = launch_timed_step(c, k0 + q, (int)q, guard && !permute && q == 0);
                if (rc) return rc;
            }
        }
        hipLaunchKernelGGL(k_report, dim3(1), dim3(kMaxBlock), 0, s, c->vmax2, (int)len, c->err_d, c->sw.stats,
                           sweep_due ? 1 : 0, X.pin_dev);
        HIPCHK(c, hipEventRecord(c->ev_report, s));
        // the next block's cell list (it needs only this block's positions) is built
        // while the host waits for the report; a re-run of this block discards it
        cells_ready = nsteps > len;
        if (cells_ready) launch_build_cells(c);
        HIPCHK(c, hipEventSynchronize(c->ev_report));
        HIPCHK(c, hipGetLastError());
        if (c->profile) {
            rc = harvest_events(c);
            if (rc) return rc;
        }
        if (sweep_due) record_sweep_stats(c);
        X.host_valid = false;
        rc = check_device_error(c);
        if (rc) return rc;
        // bound: how far any bead may be from where the list was built, at the
        // input of the block's last step; dlast: the same at the block's output
        double bound = d0, vmax = 0.0, dlast = d0;
        for (int64_t q = 0; q < len; ++q) {
            double v = std::sqrt((double)pin->vmax2[q]);
            if (track) {   // measured from the full build's positions
                if (q + 1 < len) bound = std::max(bound, v);
                dlast = v;
            } else {
                vmax = std::max(vmax, v);
                if (q + 1 < len) bound += dt * v;
                dlast += dt * v;
            }
        }
        if (guard && bound > skin) {
            // some bead may have left the reach of the cell list: redo with a fresh list every step
            c->rollbacks++;
            Bank& Bc = c->bank[c->cur];
            cells_ready = false;
            HIPCHK(c, hipMemcpyAsync(Bc.x, c->xsave, 32 * (size_t)c->n, hipMemcpyDeviceToDevice, s));
            HIPCHK(c, hipMemcpyAsync(Bc.v, c->vsave, 24 * (size_t)c->n, hipMemcpyDeviceToDevice, s));
            for (int64_t q = 0; q < len; ++q) {
                rebuild(c, false);
                launch_build_nlist(c);
                launch_step(c, k0 + q, 0);
            }
            // the re-run steps wrote their maxima into the first word row: clear it
            launch_fill_int((int*)c->vmax2, 0, DB_VMAX_SPREAD, s);
            HIPCHK(c, hipMemcpyAsync(&pin->err, c->err_d, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            rc = check_device_error(c);
            if (rc) return rc;
            c->rebuild_interval = std::max<int>(1, (int)(len / 2));
            c->list_valid = false;
        } else if (reuse) {
            // the interval follows full builds only
            c->list_disp = dlast;
            c->disp_rate = std::max(0.0, dlast - d0) / (double)len;
        } else if (track && std::isfinite(skin)) {
            // extrapolate the largest displacement linearly in time from the block's
            // end (exact for ballistic motion, cautious for diffusive motion, so the
            // interval keeps growing while the test passes)
            int want = dlast > 0 ? (int)std::floor(0.8 * skin * (double)len / dlast) + 1 : kMaxBlock;
            c->rebuild_interval = std::max(1, std::min(kMaxBlock, want));
        } else if (std::isfinite(skin) && vmax > 0) {
            int want = (int)std::floor(0.8 * skin / (dt * vmax));
            c->rebuild_interval = std::max(1, std::min(kMaxBlock, want));
        } else if (!std::isfinite(skin)) {
            c->rebuild_interval = kMaxBlock;
        }
        if (!reuse && !(guard && bound > skin)) {
            c->list_valid = true;
            c->list_disp = dlast;
            c->disp_rate = dlast / (double)len;
        }
        c->vmax_est = vmax;
        c->step += len;
        nsteps -= len;
    }
    return DB_OK;
}

int db_sweep_now(db_ctx* c) {
    if (!c) return DB_EINVAL;
    int rc = ready(c);
    if (rc) return rc;
    if (c->swept_step == c->step) return fail(c, DB_ESTATE, "the sweep of step %lld was already done", (long long)c->step);
    rebuild(c, (c->rebuild_count++ % c->permute_every) == 0);
    c->list_valid = false;
    rc = run_sweep(c, c->step);
    if (rc) return rc;
    Pinned* pin = ext(c).pin;
    HIPCHK(c, hipMemcpyAsync(pin->stats, c->sw.stats, 64, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&pin->err, c->err_d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    record_sweep_stats(c);
    c->swept_step = c->step;
    ext(c).host_valid = false;
    return check_device_error(c);
}

int db_forces(db_ctx* c, double* f, int on_device) {
    if (!c || !f) return DB_EINVAL;
    int rc = ready(c);
    if (rc) return rc;
    rebuild(c, false);
    launch_build_nlist(c);
    double* d = on_device ? f : (double*)gather_scratch(c, 24 * (size_t)c->n);
    launch_forces(c, d);
    if (!on_device && c->n) HIPCHK(c, hipMemcpyAsync(f, d, 24 * (size_t)c->n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&ext(c).pin->err, c->err_d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    return check_device_error(c);
}

int db_energy(db_ctx* c, double out[6]) {
    if (!c || !out) return DB_EINVAL;
    int rc = ready(c);
    if (rc) return rc;
    rebuild(c, false);
    double* d = (double*)gather_scratch(c, 64);
    launch_energy(c, d);
    HIPCHK(c, hipMemcpyAsync(ext(c).pin->energy, d, 48, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    memcpy(out, ext(c).pin->energy, 48);
    return DB_OK;
}

int db_energy_noalloc(db_ctx* c, double out[6]) {
    if (!c || !out) return DB_EINVAL;
    if ((int64_t)c->n > (int64_t)DB_NOALLOC_MAX_BLOCKS * DB_BLOCK)
        return fail(c, DB_EINVAL, "db_energy_noalloc takes at most %d beads (%d given)",
                    DB_NOALLOC_MAX_BLOCKS * DB_BLOCK, c->n);
    db_host_ext& X = ext(c);
    if (!c->have_state) return fail(c, DB_ESTATE, "db_set_state has not been called");
    if (X.dev_error) return fail(c, X.dev_error, "a previous device error left the state undefined: %s", c->err.c_str());
    // everything an allocating call would set up first must already be in place
    if (!c->allocated || !X.dev_valid || c->params_dirty)
        return fail(c, DB_ESTATE, "db_energy_noalloc needs device state and parameters that are current: "
                                  "run db_step, db_forces or db_energy once after the last change");
    double* part = (c->device >= 0 && c->device < kMaxDevices) ? noalloc_ptr[c->device] : nullptr;
    if (!part) return fail(c, DB_ESTATE, "no scratch address for device %d", c->device);
    double* sums = part + 6 * (size_t)DB_NOALLOC_MAX_BLOCKS;
    rebuild(c, false);
    launch_energy(c, sums, part);
    HIPCHK(c, hipMemcpyAsync(X.pin->energy, sums, 48, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    memcpy(out, X.pin->energy, 48);
    return DB_OK;
}

int db_get_state(db_ctx* c, double* x, double* v, int on_device) {
    if (!c) return DB_EINVAL;
    db_host_ext& X = ext(c);
    const size_t n = (size_t)c->n;
    if (!X.dev_valid || X.host_valid) {
        if (!c->have_state) return fail(c, DB_ESTATE, "no state");
        if (on_device) {
            if (x && n) HIPCHK(c, hipMemcpy(x, X.h.x.data(), 24 * n, hipMemcpyHostToDevice));
            if (v && n) HIPCHK(c, hipMemcpy(v, X.h.v.data(), 24 * n, hipMemcpyHostToDevice));
        } else {
            if (x) std::copy(X.h.x.begin(), X.h.x.end(), x);
            if (v) std::copy(X.h.v.begin(), X.h.v.end(), v);
        }
        return DB_OK;
    }
    if (n == 0) return DB_OK;
    double* d = (double*)gather_scratch(c, 48 * n);
    hipLaunchKernelGGL(k_gather_state, dim3((unsigned)((n + DB_BLOCK - 1) / DB_BLOCK)), dim3(DB_BLOCK), 0, c->stream,
                       (int)n, c->bank[c->cur], d, d + 3 * n);
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (x) HIPCHK(c, hipMemcpyAsync(x, d, 24 * n, kind, c->stream));
    if (v) HIPCHK(c, hipMemcpyAsync(v, d + 3 * n, 24 * n, kind, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    return DB_OK;
}

int db_topology_counts(db_ctx* c, int64_t* nb, int64_t* na, int64_t* nd) {
    if (!c) return DB_EINVAL;
    db_host_ext& X = ext(c);
    if (X.host_valid) {
        if (nb) *nb = (int64_t)(X.h.bonds.size() / 4);
        if (na) *na = (int64_t)(X.h.ang.size() / 4);
        if (nd) *nd = (int64_t)(X.h.dih.size() / 5);
        return DB_OK;
    }
    int rc = download_system(c);
    if (rc) return rc;
    return db_topology_counts(c, nb, na, nd);
}

int db_get_bonds(db_ctx* c, int32_t* ij, int32_t* tij, int32_t* tji) {
    if (!c) return DB_EINVAL;
    int rc = download_system(c);
    if (rc) return rc;
    const std::vector<int32_t>& b = ext(c).h.bonds;
    const size_t m = b.size() / 4;
    std::vector<int32_t> tt(2 * m);
    sorted_copy<2, 2>(b, ij, tt.data(), 0);
    for (size_t k = 0; k < m; ++k) {
        if (tij) tij[k] = tt[2 * k];
        if (tji) tji[k] = tt[2 * k + 1];
    }
    return DB_OK;
}

int db_get_angles(db_ctx* c, int32_t* abc, int32_t* type) {
    if (!c) return DB_EINVAL;
    int rc = download_system(c);
    if (rc) return rc;
    sorted_copy<3, 1>(ext(c).h.ang, abc, type, 1);
    return DB_OK;
}

int db_get_dihedrals(db_ctx* c, int32_t* abcd, int32_t* type) {
    if (!c) return DB_EINVAL;
    int rc = download_system(c);
    if (rc) return rc;
    sorted_copy<4, 1>(ext(c).h.dih, abcd, type, 1);
    return DB_OK;
}

int db_get_stats(db_ctx* c, db_stats* o) {
    if (!c || !o) return DB_EINVAL;
    int64_t* p = &o->bonds_created;
    for (int q = 0; q < 8; ++q) {
        p[q] = c->stat_last[q];
        p[8 + q] = c->stat_cum[q];
    }
    o->sweeps = c->sweeps;
    o->steps = c->step;
    o->rebuilds = c->rebuilds;
    o->rollbacks = c->rollbacks;
    o->du_topo_last = c->du_last;
    o->du_topo_cum = c->du_cum;
    o->list_patches = c->patches;
    return DB_OK;
}

int db_track_topology_energy(db_ctx* c, int enable) {
    if (!c) return DB_EINVAL;
    c->ledger = enable != 0;
    return DB_OK;
}

int db_set_step(db_ctx* c, int64_t step) {
    if (!c || step < 0) return DB_EINVAL;
    c->step = step;
    c->swept_step = -1;
    return DB_OK;
}

// ------------------------------------------------------------------------------------
// checkpoints: the whole device arena (state, tables, lists, cells, sweep buffers,
// in slot order) and the scheduler's host state, so that a run resumed from one
// continues as the saved run would have, bit for bit

namespace {
struct CkptHead {
    char magic[8];
    int32_t version, n, precision, nrep;
    uint64_t seed;
    double L;
    uint64_t arena_bytes;
    double skin;
    int32_t permute_every, tile_mode, brick_edge, cur;
    int32_t rebuild_interval, ntile, tile_bB, pad0;
    int64_t step, swept_step, rebuilds, rollbacks, sweeps, patches, rebuild_count;
    int64_t stat_last[8], stat_cum[8];
    uint8_t list_valid, tiles_valid, regions_valid, halo_force, halo_sweep, have_topology, ledger, pad1;
    double list_disp, disp_rate, vmax_est, du_last, du_cum;
    // the step kernel writes positions (and with DPD velocities) into a second
    // buffer and the pointers are exchanged: which arena buffer each one names
    uint64_t off_x[3], off_v[3];   // bank[0], bank[1], next
};
const char kCkptMagic[8] = {'D', 'B', 'C', 'K', 'P', 'T', '1', 0};
const int32_t kCkptVersion = 1;
}  // namespace

int db_checkpoint_bytes(db_ctx* c, size_t* bytes) {
    if (!c || !bytes) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_EINVAL, "checkpoints are taken of single systems");
    *bytes = sizeof(CkptHead) + layout(c, false);
    return DB_OK;
}

int db_checkpoint_save(db_ctx* c, void* buf, size_t bytes) {
    if (!c || !buf) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_EINVAL, "checkpoints are taken of single systems");
    int rc = ready(c);
    if (rc) return rc;
    const size_t arena = layout(c, false);
    if (bytes < sizeof(CkptHead) + arena)
        return fail(c, DB_EINVAL, "checkpoint needs %zu bytes", sizeof(CkptHead) + arena);
    CkptHead h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, kCkptMagic, 8);
    h.version = kCkptVersion;
    h.n = c->n;
    h.precision = c->precision;
    h.nrep = c->nrep;
    h.seed = c->seed;
    h.L = c->L;
    h.arena_bytes = arena;
    h.skin = c->skin;
    h.permute_every = c->permute_every;
    h.tile_mode = c->tile_mode;
    h.brick_edge = c->brick_edge;
    h.cur = c->cur;
    h.rebuild_interval = c->rebuild_interval;
    h.ntile = c->ntile;
    h.tile_bB = c->tile_bB;
    h.step = c->step;
    h.swept_step = c->swept_step;
    h.rebuilds = c->rebuilds;
    h.rollbacks = c->rollbacks;
    h.sweeps = c->sweeps;
    h.patches = c->patches;
    h.rebuild_count = c->rebuild_count;
    memcpy(h.stat_last, c->stat_last, sizeof h.stat_last);
    memcpy(h.stat_cum, c->stat_cum, sizeof h.stat_cum);
    h.list_valid = c->list_valid;
    h.tiles_valid = c->tiles_valid;
    h.regions_valid = c->regions_valid;
    h.halo_force = c->halo_force;
    h.halo_sweep = c->halo_sweep;
    h.have_topology = c->have_topology;
    h.ledger = c->ledger;
    h.list_disp = c->list_disp;
    h.disp_rate = c->disp_rate;
    h.vmax_est = c->vmax_est;
    h.du_last = c->du_last;
    h.du_cum = c->du_cum;
    const double4* xp[3] = {c->bank[0].x, c->bank[1].x, c->xnext};
    const double* vp[3] = {c->bank[0].v, c->bank[1].v, c->vnext};
    for (int k = 0; k < 3; ++k) {
        h.off_x[k] = (uint64_t)((const char*)xp[k] - c->arena);
        h.off_v[k] = (uint64_t)((const char*)vp[k] - c->arena);
    }
    memcpy(buf, &h, sizeof h);
    HIPCHK(c, hipMemcpyAsync((char*)buf + sizeof h, c->arena, arena, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DB_OK;
}

int db_checkpoint_load(db_ctx* c, const void* buf, size_t bytes) {
    if (!c || !buf) return DB_EINVAL;
    if (c->nrep > 0) return fail(c, DB_EINVAL, "checkpoints are taken of single systems");
    if (bytes < sizeof(CkptHead)) return fail(c, DB_EINVAL, "checkpoint too short");
    CkptHead h;
    memcpy(&h, buf, sizeof h);
    if (memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != kCkptVersion)
        return fail(c, DB_EINVAL, "not a checkpoint of this library version");
    if (h.n != c->n || h.precision != c->precision || h.nrep != 0 || h.seed != c->seed || h.L != c->L)
        return fail(c, DB_EINVAL, "checkpoint of another system (beads, precision, seed or box edge differ)");
    if (h.skin != c->skin || h.permute_every != c->permute_every || h.tile_mode != c->tile_mode ||
        h.brick_edge != c->brick_edge)
        return fail(c, DB_EINVAL, "checkpoint taken with another skin, reorder cadence or step-kernel shape");
    const size_t arena = layout(c, false);
    if (h.arena_bytes != arena || bytes < sizeof h + arena)
        return fail(c, DB_EINVAL, "checkpoint of another memory layout");
    db_host_ext& X = ext(c);
    int rc = ensure_memory(c);
    if (rc) return rc;
    // the buffers named by the saved pointers: the same three in some order
    {
        const char* xb[3] = {(const char*)c->bank[0].x, (const char*)c->bank[1].x, (const char*)c->xnext};
        const char* vb[3] = {(const char*)c->bank[0].v, (const char*)c->bank[1].v, (const char*)c->vnext};
        auto same_set = [&](const uint64_t* off, const char* const* bufs) {
            for (int k = 0; k < 3; ++k) {
                int hits = 0;
                for (int q = 0; q < 3; ++q) hits += off[q] == (uint64_t)(bufs[k] - c->arena);
                if (hits != 1) return false;
            }
            return true;
        };
        if (!same_set(h.off_x, xb) || !same_set(h.off_v, vb))
            return fail(c, DB_EINVAL, "checkpoint of another memory layout");
    }
    c->params_dirty = true;
    rc = upload_params(c);   // the grid of this handle's parameters
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->arena, (const char*)buf + sizeof h, arena, hipMemcpyHostToDevice, c->stream));
    // the parameter block in the arena holds the saving handle's addresses: write ours
    c->params_dirty = true;
    rc = upload_params(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->bank[0].x = (double4*)(c->arena + h.off_x[0]);
    c->bank[1].x = (double4*)(c->arena + h.off_x[1]);
    c->xnext = (double4*)(c->arena + h.off_x[2]);
    c->bank[0].v = (double*)(c->arena + h.off_v[0]);
    c->bank[1].v = (double*)(c->arena + h.off_v[1]);
    c->vnext = (double*)(c->arena + h.off_v[2]);
    c->cur = h.cur;
    c->rebuild_interval = h.rebuild_interval;
    c->ntile = h.ntile;
    c->tile_bB = h.tile_bB;
    c->step = h.step;
    c->swept_step = h.swept_step;
    c->rebuilds = h.rebuilds;
    c->rollbacks = h.rollbacks;
    c->sweeps = h.sweeps;
    c->patches = h.patches;
    c->rebuild_count = h.rebuild_count;
    memcpy(c->stat_last, h.stat_last, sizeof h.stat_last);
    memcpy(c->stat_cum, h.stat_cum, sizeof h.stat_cum);
    c->list_valid = h.list_valid;
    c->tiles_valid = h.tiles_valid;
    c->regions_valid = h.regions_valid;
    c->halo_force = h.halo_force;
    c->halo_sweep = h.halo_sweep;
    c->have_state = true;
    c->have_topology = h.have_topology;
    c->ledger = h.ledger;
    c->list_disp = h.list_disp;
    c->disp_rate = h.disp_rate;
    c->vmax_est = h.vmax_est;
    c->du_last = h.du_last;
    c->du_cum = h.du_cum;
    X.dev_valid = true;
    X.host_valid = false;
    X.dev_error = 0;
    X.pin->err = 0;
    return DB_OK;
}

int db_graph(db_ctx* c, int enable) {
    if (!c || (enable != 0 && enable != 1)) return DB_EINVAL;
    c->use_graph = enable == 1;
    return DB_OK;
}

int db_tile_shape(db_ctx* c, int enable, int32_t brick_edge) {
    if (!c || (enable != 0 && enable != 1) || brick_edge < 0 || brick_edge > 64) return DB_EINVAL;
    c->tile_mode = enable;
    c->brick_edge = brick_edge;
    c->params_dirty = true;
    c->tiles_valid = false;
    c->regions_valid = false;
    c->rebuild_count = 0;   // the next block reorders, into brick order when tiles are on
    return DB_OK;
}

int db_tile_stats(db_ctx* c, int64_t out[4]) {
    if (!c || !out) return DB_EINVAL;
    for (int k = 0; k < 4; ++k) out[k] = 0;
    if (!c->allocated || !tiles_enabled(c) || !c->regions_valid) return DB_OK;
    const int nt = c->ntile;
    std::vector<int> rc(nt);
    HIPCHK(c, hipMemcpyAsync(rc.data(), c->tiles.rcount, 4 * (size_t)nt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int64_t staged = 0, sum = 0, mx = 0;
    for (int v : rc) {
        if (v <= DB_RCAP) {
            ++staged;
            sum += v;
        }
        mx = std::max<int64_t>(mx, v);
    }
    out[0] = nt;
    out[1] = staged;
    out[2] = sum;
    out[3] = mx;
    return DB_OK;
}

int db_tune(db_ctx* c, double skin, int32_t permute_every) {
    if (!c || !(skin > 0) || !std::isfinite(skin) || permute_every < 1) return DB_EINVAL;
    c->skin = skin;
    c->skin_tuned = true;
    c->permute_every = permute_every;
    c->params_dirty = true;
    return DB_OK;
}

// steps_per_trial steps after one untimed step (which sets up a new grid or order)
static int timed_trial(db_ctx* c, int64_t steps_per_trial, double* t) {
    int rc = db_step(c, 1);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    auto t0 = std::chrono::steady_clock::now();
    rc = db_step(c, steps_per_trial);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return DB_OK;
}

int db_autotune(db_ctx* c, int64_t steps_per_trial, double* best_skin, int32_t* best_permute) {
    if (!c || steps_per_trial < 1) return DB_EINVAL;
    // DPD at density 3 favours thinner skins than the WCA workloads
    const bool dpd = c->hp.have_pair && c->hp.pair_style == PAIR_DPD;
    const double wca_skins[4] = {0.4, 0.5, 0.6, 0.8}, dpd_skins[4] = {0.02, 0.05, 0.1, 0.3};
    const double* skins_of = dpd ? dpd_skins : wca_skins;
    const double skins[4] = {skins_of[0], skins_of[1], skins_of[2], skins_of[3]};
    const int perms[4] = {1, 2, 4, 8};
    double best_t = INFINITY, bs = c->skin;
    int bp = c->permute_every;
    for (double sk : skins) {
        for (int pe : perms) {
            int rc = db_tune(c, sk, pe);
            if (rc) return rc;
            double t = 0;
            rc = timed_trial(c, steps_per_trial, &t);
            if (rc) return rc;
            if (t < best_t) {
                best_t = t;
                bs = sk;
                bp = pe;
            }
        }
    }
    int rc = db_tune(c, bs, bp);
    if (rc) return rc;
    // then the step kernel's shape: per-bead gathers, or tiles over bricks of 3, 4
    // or 5 cells (single systems with WCA pairs); then graphs off or on
    const bool can_tile = c->nrep == 0 && c->hp.have_pair && c->hp.pair_style == PAIR_WCA;
    int best_mode = 0, best_edge = 0;
    double shape_t = INFINITY;
    const int edges[4] = {0, 3, 4, 5};
    for (int k = 0; k < (can_tile ? 4 : 1); ++k) {
        const int mode = k == 0 ? 0 : 1, edge = edges[k];
        rc = db_tile_shape(c, mode, edge);
        if (rc) return rc;
        double t = 0;
        rc = timed_trial(c, steps_per_trial, &t);
        if (rc) return rc;
        if (t < shape_t) {
            shape_t = t;
            best_mode = mode;
            best_edge = edge;
        }
    }
    rc = db_tile_shape(c, best_mode, best_edge);
    if (rc) return rc;
    int best_graph = 0;
    double graph_t = INFINITY;
    for (int gr = 0; gr < 2; ++gr) {
        c->use_graph = gr == 1;
        double t = 0;
        rc = timed_trial(c, steps_per_trial, &t);
        if (rc) return rc;
        if (t < graph_t) {
            graph_t = t;
            best_graph = gr;
        }
    }
    c->use_graph = best_graph == 1;
    if (best_skin) *best_skin = bs;
    if (best_permute) *best_permute = bp;
    return DB_OK;
}

int db_get_shape(db_ctx* c, int32_t out[3]) {
    if (!c || !out) return DB_EINVAL;
    out[0] = c->tile_mode;
    out[1] = c->brick_edge;
    out[2] = c->use_graph ? 1 : 0;
    return DB_OK;
}

// the force field, thermostat and rules two handles would run with
static bool same_physics(const Params& a, const Params& b) {
    auto eq = [](const void* x, const void* y, size_t n) { return memcmp(x, y, n) == 0; };
    if (a.have_pair != b.have_pair || a.excl_depth != b.excl_depth || a.pair_style != b.pair_style ||
        a.eps != b.eps || a.sig2 != b.sig2 || a.rc2 != b.rc2 || a.dpd_a != b.dpd_a || a.dpd_gamma != b.dpd_gamma)
        return false;
    if (!eq(a.bK, b.bK, sizeof a.bK) || !eq(a.bR0, b.bR0, sizeof a.bR0) || !eq(a.bE0, b.bE0, sizeof a.bE0) ||
        !eq(a.bRc2, b.bRc2, sizeof a.bRc2) || !eq(a.aK, b.aK, sizeof a.aK) ||
        !eq(a.aT0, b.aT0, sizeof a.aT0) || !eq(a.dK, b.dK, sizeof a.dK) || !eq(a.dC0, b.dC0, sizeof a.dC0) ||
        !eq(a.dS0, b.dS0, sizeof a.dS0))
        return false;
    if (a.gamma != b.gamma || a.dt != b.dt || a.every != b.every || a.pc13 != b.pc13 || a.pc14 != b.pc14 ||
        a.accept_average != b.accept_average)
        return false;
    if (a.nrule != b.nrule || a.nmax != b.nmax || a.narule != b.narule || a.ndrule != b.ndrule) return false;
    for (int q = 0; q < a.nrule; ++q) {
        const Rule &x = a.rule[q], &y = b.rule[q];
        if (x.kind != y.kind || x.bt1 != y.bt1 || x.bt2 != y.bt2 || x.b1 != y.b1 || x.b2 != y.b2 || x.r2 != y.r2 ||
            x.p != y.p)
            return false;
    }
    for (int q = 0; q < a.nmax; ++q)
        if (a.maxr[q].bt != b.maxr[q].bt || a.maxr[q].bead != b.maxr[q].bead || a.maxr[q].max != b.maxr[q].max)
            return false;
    for (int q = 0; q < a.narule; ++q)
        if (a.arule[q].type != b.arule[q].type || !eq(a.arule[q].b, b.arule[q].b, sizeof a.arule[q].b) ||
            !eq(a.arule[q].m, b.arule[q].m, sizeof a.arule[q].m))
            return false;
    for (int q = 0; q < a.ndrule; ++q)
        if (a.drule[q].type != b.drule[q].type || !eq(a.drule[q].b, b.drule[q].b, sizeof a.drule[q].b) ||
            !eq(a.drule[q].m, b.drule[q].m, sizeof a.drule[q].m))
            return false;
    return true;
}

int db_batch_create(db_ctx** out, db_ctx* const* reps, int32_t nrep, void* stream) {
    if (!out) return DB_EINVAL;
    *out = nullptr;
    if (!reps || nrep < 1 || nrep > 65535) return DB_EINVAL;
    int64_t ntot = 0;
    double Lmin = INFINITY, Lmax = 0;
    for (int r = 0; r < nrep; ++r) {
        db_ctx* q = reps[r];
        if (!q || !q->have_state || q->nrep > 0) return DB_EINVAL;
        if (q->precision != reps[0]->precision || q->step != reps[0]->step) return DB_EINVAL;
        if (!same_physics(q->hp, reps[0]->hp)) return DB_EINVAL;
        if (q->hp.has_ext) return DB_EINVAL;   // external forces are tied to one system's bead ids
        db_host_ext& X = ext(q);
        if (X.dev_error) return DB_ESTATE;
        if (X.dev_valid && !X.host_valid) {
            int rc = download_system(q);
            if (rc) return rc;
        }
        ntot += q->n;
        Lmin = std::min(Lmin, q->L);
        Lmax = std::max(Lmax, q->L);
    }
    if (ntot > INT32_MAX) return DB_EINVAL;
    db_ctx* c = nullptr;
    int rc = db_create(&c, (int32_t)ntot, Lmax, reps[0]->seed, reps[0]->precision, stream);
    if (rc) return rc;
    const db_ctx* r0 = reps[0];
    c->hp = r0->hp;   // force field, thermostat, rules
    c->hp.n = (int)ntot;
    c->L = Lmin;      // the argument checks of later calls hold for every box
    c->nrep = nrep;
    c->reps.resize(nrep);
    c->rep_n.resize(nrep);
    c->step = r0->step;
    c->swept_step = r0->swept_step;
    HostSys& h = ext(c).h;
    h.x.clear();
    h.v.clear();
    h.type.clear();
    h.reactive.clear();
    h.rep.clear();
    int off = 0;
    for (int r = 0; r < nrep; ++r) {
        const db_ctx* q = reps[r];
        const HostSys& g = ext(const_cast<db_ctx*>(q)).h;
        Box X = q->hp.box;
        X.gid_off = off;
        c->reps[r] = X;
        c->rep_n[r] = q->n;
        h.x.insert(h.x.end(), g.x.begin(), g.x.end());
        h.v.insert(h.v.end(), g.v.begin(), g.v.end());
        h.type.insert(h.type.end(), g.type.begin(), g.type.end());
        h.reactive.insert(h.reactive.end(), g.reactive.begin(), g.reactive.end());
        h.rep.insert(h.rep.end(), (size_t)q->n, (uint16_t)r);
        for (size_t k = 0; k < g.bonds.size(); k += 4) {
            h.bonds.push_back(g.bonds[k] + off);
            h.bonds.push_back(g.bonds[k + 1] + off);
            h.bonds.push_back(g.bonds[k + 2]);
            h.bonds.push_back(g.bonds[k + 3]);
        }
        for (size_t k = 0; k < g.ang.size(); k += 4) {
            h.ang.push_back(g.ang[k]);
            for (int m = 1; m < 4; ++m) h.ang.push_back(g.ang[k + m] + off);
        }
        for (size_t k = 0; k < g.dih.size(); k += 5) {
            h.dih.push_back(g.dih[k]);
            for (int m = 1; m < 5; ++m) h.dih.push_back(g.dih[k + m] + off);
        }
        off += q->n;
    }
    c->have_state = true;
    c->params_dirty = true;
    *out = c;
    return DB_OK;
}

int db_batch_get_state(db_ctx* c, int32_t r, double* x, double* v, int on_device) {
    if (!c || c->nrep == 0 || r < 0 || r >= c->nrep) return DB_EINVAL;
    const size_t n = (size_t)c->n;
    const size_t off = (size_t)c->reps[r].gid_off, nr = (size_t)c->rep_n[r];
    db_host_ext& X = ext(c);
    if (!X.dev_valid || X.host_valid) {
        if (on_device) {
            if (x && nr) HIPCHK(c, hipMemcpy(x, X.h.x.data() + 3 * off, 24 * nr, hipMemcpyHostToDevice));
            if (v && nr) HIPCHK(c, hipMemcpy(v, X.h.v.data() + 3 * off, 24 * nr, hipMemcpyHostToDevice));
        } else {
            if (x) std::copy(X.h.x.begin() + 3 * off, X.h.x.begin() + 3 * (off + nr), x);
            if (v) std::copy(X.h.v.begin() + 3 * off, X.h.v.begin() + 3 * (off + nr), v);
        }
        return DB_OK;
    }
    if (nr == 0) return DB_OK;
    double* d = (double*)gather_scratch(c, 48 * n);
    hipLaunchKernelGGL(k_gather_state, dim3((unsigned)((n + DB_BLOCK - 1) / DB_BLOCK)), dim3(DB_BLOCK), 0, c->stream,
                       (int)n, c->bank[c->cur], d, d + 3 * n);
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (x) HIPCHK(c, hipMemcpyAsync(x, d + 3 * off, 24 * nr, kind, c->stream));
    if (v) HIPCHK(c, hipMemcpyAsync(v, d + 3 * n + 3 * off, 24 * nr, kind, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipGetLastError());
    return DB_OK;
}

int db_profile(db_ctx* c, int every) {
    if (!c || every < 0) return DB_EINVAL;
    c->profile = every > 0;
    c->profile_every = every > 0 ? every : 1;
    c->profile_count = 0;
    return DB_OK;
}

int db_step_kernel_time(db_ctx* c, double* mean_us, int64_t* launches) {
    if (!c) return DB_EINVAL;
    if (mean_us) *mean_us = c->prof_launches ? 1000.0 * c->prof_ms / (double)c->prof_launches : 0.0;
    if (launches) *launches = c->prof_launches;
    c->prof_ms = 0;
    c->prof_launches = 0;
    return DB_OK;
}

}  // extern "C"
