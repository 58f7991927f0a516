// Internal declarations of libdynbond: device-side parameter block, per-bead
// storage layout, the handle, and the kernel launchers shared by the .hip units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dynbond.h"

#define DB_MAXB DB_MAX_BONDS_PER_BEAD
#define DB_MAXA DB_MAX_ANGLES_PER_BEAD
#define DB_MAXD DB_MAX_DIHEDRALS_PER_BEAD
#define DB_MAXT 32
#define DB_MAXRULES 32
#define DB_BLOCK 256
#define DB_NLCAP 128         // neighbour-list entries per bead (DPD at density 3 lists ~50-80)
#define DB_MAXU 8            // bonded halo entries per bead (codes hold 3-bit indices)
#define DB_HALO_OVF 255      // halo marker: more than DB_MAXU distinct bonded partners
#define DB_VMAX_SPREAD 64    // words per step over which the speed maxima are spread
#define DB_RCAP 768          // region entries a tile of the step kernel stages in LDS
#define DB_CAPA 448          // angle work items of a tile
#define DB_CAPD 224          // dihedral work items of a tile
#define DB_XS_PAD 8          // entries after the float position copy that a run of the cell scan may read
#define DB_SLOT_BITS 26      // the float position copy packs slot | type << 26 | reactive << 31
#define DB_MAX_BEADS ((1 << DB_SLOT_BITS) - 1)

namespace db {

enum RuleKind { RK_CREATE = 1, RK_CREATEDIR = 2, RK_BREAK = 3, RK_KILL = 4, RK_CONVERT = 5 };

// random-number stream tags (top 4 bits of the last counter word)
enum RngKind : uint32_t { RNG_LANGEVIN = 0u, RNG_CREATE = 1u, RNG_BREAK = 2u, RNG_DPD = 3u };

// pair force styles
enum PairStyle { PAIR_WCA = 0, PAIR_DPD = 1 };

// counters of one sweep (SweepBuf::stats)
enum { ST_CREATED = 0, ST_BROKEN, ST_KILLED, ST_CONVERTED, ST_ANG_NEW, ST_ANG_DEL, ST_DIH_NEW, ST_DIH_DEL };

// device error word bits
enum ErrBit : int { ERR_BOND_CAP = 1, ERR_ANGLE_CAP = 2, ERR_DIH_CAP = 4, ERR_NONFINITE = 8, ERR_NLIST = 16 };

struct Rule {
    int kind, bt1, bt2, b1, b2;
    double r2, p;
};
struct MaxRule { int bt, bead, max; };
struct AngRule { int type; int b[3]; uint32_t m[2]; };
struct DihRule { int type; int b[4]; uint32_t m[3]; };

// One periodic box: its edge, cell grid and where its cells and bead ids start
// in the shared arrays, its random-number key and temperature schedule.  A
// single system has one box (Params::box); a batch of independent replicas has
// one per replica (Params::rep, indexed by the replica id in each bead's meta).
struct Box {
    double L, hL, invL;
    double cell_scale;   // nc / L
    int nc, noff;        // nc^3 cells of edge L/nc; neighbour offsets per dimension
    int off[3];
    int wide_create;     // the creation distance exceeds one cell edge: creation scans reach two cells
    int cell_off;        // first cell of the box in the shared cell arrays
    int gid_off;         // first global bead id of the box
    uint32_t seed_lo, seed_hi;
    double T0, T1;       // temperature T0 + (T1 - T0) min(step, ramp) / ramp
    int64_t ramp;
    // Float prefilters of the cell scans.  A separation formed from float copies
    // of coordinates below L, shifted by at most one float edge, is off by at most
    // 2.5 float ulps of 2L per component; pf_slack = 4 sqrt(3) ulp_f(2L) bounds
    // that in length, and the squared prefilter cutoffs carry it plus a relative
    // 1e-4 for the float products: a pair within a cutoff in double always passes
    // its prefilter.
    double pf_slack;
    float pf_create2;    // (creation distance + pf_slack)^2 (1 + 1e-4)
    float pf_list2;      // (list cutoff + pf_slack)^2 (1 + 1e-4)
};

// Read-only parameters, resident in device memory.
struct Params {
    int n;
    int ncell;           // cells over all boxes
    Box box;             // the box of a single system
    int nrep;            // replicas in a batch (0: single system)
    const Box* rep;      // [nrep] device table of a batch
    // pair force: WCA, or DPD (conservative a w, dissipative -gamma w^2 (e . v_ij),
    // random sigma w xi / sqrt(dt), w = 1 - r / rc)
    int have_pair, excl_depth, pair_style;
    double eps, sig2, rc2;
    double rc, inv_rc, dpd_a, dpd_gamma;
    double rnl2;         // neighbour-list cutoff squared (pair cutoff + skin)
    // bonded
    double bK[DB_MAXT], bR0[DB_MAXT];
    double bE0[DB_MAXT], bRc2[DB_MAXT];   // energy offset; squared cutoff (+inf: none)
    double aK[DB_MAXT], aT0[DB_MAXT], aPiMinusT0[DB_MAXT];
    double dK[DB_MAXT], dC0[DB_MAXT], dS0[DB_MAXT];
    // thermostat / integration
    double gamma, dt;
    // constant external forces, indexed by global bead id ([3n]; read only when has_ext)
    int has_ext;
    const double* fext;
    // rules, in call order
    int every, pc13, pc14;
    int accept_average;         // acceptance compares the mean of two per-bead uniforms with p
    int nrule, nmax, narule, ndrule;
    Rule rule[DB_MAXRULES];
    MaxRule maxr[DB_MAXRULES];
    AngRule arule[DB_MAXRULES];
    DihRule drule[DB_MAXRULES];
    double rmax2_create;        // largest creation distance squared
    uint32_t create_types;      // bit t: bead type t occurs in some creation rule
    int has_break_class;        // any breakbond / convertbond rule
    int has_kill;
    uint32_t break_types;       // bit t: some breakbond / killbond / convertbond rule acts on bond type t
};

// Per-bead storage in slot (cell-sorted) order.  Tables are column-major:
// entry k of bead s lives at [k * n + s], so a wavefront reads one row coalesced.
struct Bank {
    double4* x;       // x, y, z; w = bits {int gid, int meta}; meta = type | reactive << 8
    double* v;        // SoA: vx[n], vy[n], vz[n]
    uint8_t* nb;      // bond count
    int* bp;          // [MAXB][n] partner slot
    int8_t* bt;       // [MAXB][n] type this bead stores for the bond
    uint8_t* na;
    int4* ang;        // [MAXA][n] members (slots) a, b, c; .w = angle type
    uint8_t* nd;
    int4* dih;        // [MAXD][n] members (slots) a, b, c, d
    uint8_t* dt;      // [MAXD][n] dihedral type
};

// Scratch of the sweep, per bead in slot order.
struct SweepBuf {
    int* nomC;        // creation partner slot or -1
    int8_t* ruleC;    // rule index
    int8_t* btC;      // type this bead would store
    int* nomK;        // breakage partner slot or -1
    int8_t* ruleK;
    uint8_t* rmcnt;   // removed (killed / broken / converted) bond entries
    int* rmlist;      // [MAXB][n] partner slots of removed entries
    uint8_t* conv;    // bead takes part in an accepted conversion
    int* newp;        // partner slot of this bead's new (created or converted) bond, or -1
    unsigned long long* stats;   // [8] counters of the sweep
    int* aoff;        // [n + 1] the beads flagged in act, in slot order, aoff[n] = their number
                      // (also exclusive prefix sums of the bonded flags while the slots are reordered)
    int* act;         // [n] 0/1 flags: the beads that may nominate a creation partner (after
                      // the sweep: the beads whose Verlet list must be redone)
    uint8_t* chg;     // the sweep created or removed (not converted) a bond of the bead
    uint8_t* tchg;    // the sweep changed the bead's own bond, angle or dihedral table
    uint8_t* npurge;  // the bead lies within two bonds (old tables) of a bond the sweep removes
    uint8_t* ngen;    // the bead lies within two bonds (new tables) of a bond the sweep created or converted
};

// Verlet neighbour list: entry k of bead s at nl[k * n + s] (slots), count in cnt
struct NList {
    int* nl;          // [DB_NLCAP][n]
    uint8_t* cnt;     // [n]
};

// Bonded halo of each bead (built with the neighbour list): the distinct beads
// its bonds, angles and dihedrals reach, and those entries re-coded as the
// bead's role plus halo indices.  nu = DB_HALO_OVF marks a bead whose halo
// would exceed DB_MAXU; it reads the slot tables instead.
struct Halo {
    uint8_t* nu;        // [n]
    int* u;             // [DB_MAXU][n] slots, bond partners first in table order
    uint32_t* acode;    // [DB_MAXA][n]
    uint32_t* dcode;    // [DB_MAXD][n]
};

// Tiles of the step kernel.  The cells of the box are grouped into bricks of bB^3
// cells (the last brick of a dimension may be thinner); a reordering then places
// the beads brick by brick, so that a tile of DB_BLOCK consecutive slots is a
// compact piece of space.  After every list build the distinct beads that a
// tile's list and halo entries name (its region) are recorded in slot order, and
// those entries re-coded as 16-bit indices into the region; the step kernel
// stages the region's positions in LDS once per tile and reads every partner from
// there.  A tile whose region exceeds DB_RCAP, or a bead whose halo overflows,
// reads its partners from memory as before.
struct Tiles {
    int* tstart;      // [nbrick + 1] first slot of each brick (statistics only)
    int* rcount;      // [ntile] region entries (> DB_RCAP: too many to stage)
    int* rslot;       // [ntile][DB_RCAP] region slots, ascending
    uint16_t* nl16;   // list entries as region indices: the first 16 of a bead in one row, then column-major
    uint16_t* hu16;   // [n][DB_MAXU] halo entries as region indices
    uint4* rec;       // [n] the bead's words for the step: bond types; halo size, list length and table
                      // counts; its own region index and meta word; its global id
    uint4* code8;     // [n][2] its first four angle codes, then its first four dihedral codes (tiles with
                      // work items: the item and the bead's member role of each entry instead)
    // Work items: every angle and dihedral with a member in the tile, once per tile,
    // as the region indices of its members (10 bits each) and its type; the step
    // kernel evaluates each once for all of its members and the members collect
    // their forces from LDS
    uint2* itemA;     // [ntile][DB_CAPA]
    uint2* itemD;     // [ntile][DB_CAPD]
    uint32_t* nitems; // [ntile] angle items | dihedral items << 16; 0xFFFFFFFF: no items (per-bead terms)
};

// The step launches of one block captured as a HIP graph.  The key is everything
// the captured arguments depend on; the launches swap the position (and velocity)
// buffers, whose state after the block is kept for replays.
struct GraphEntry {
    int len;
    bool save, tiled;
    int cur;
    const void *x, *xnext, *v, *vnext;             // buffers before the block
    const void *x_after, *xnext_after, *v_after, *vnext_after;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

struct Cells {
    int* cnt;         // [ncell]
    int* start;       // [ncell + 1]
    int* list;        // [n] slots, cell by cell, ascending within a cell
    float4* xs;       // [n + DB_XS_PAD] in list order: float x, y, z and (bits) slot | type << 26 | reactive << 31
    int* cellid;      // [n]
    int* rank;        // [n] place of the bead among the beads of its cell
    int* unsorted;    // [n] the list before the ordering inside each cell
    int* blocksum;    // scan scratch
};

}  // namespace db

struct db_host_ext;   // host-side copies and staging, defined by the API unit

struct db_ctx {
    db_host_ext* hx;
    int n;
    double L;
    uint64_t seed;
    int precision;
    hipStream_t stream;
    int device;          // the HIP device current at creation
    std::string err;

    db::Params hp;       // host copy
    db::Params* dp;      // device copy
    bool params_dirty;

    // device memory arena
    char* arena;
    size_t arena_bytes;
    bool arena_owned;
    bool allocated;

    db::Bank bank[2];
    int cur;
    double4* xnext;      // double buffer of positions for the step kernel
    double4* xref;       // positions at the last full Verlet-list build (slot order)
    double* vnext;       // double buffer of velocities (DPD: the step reads neighbour velocities)
    double* fext;        // [3n] external force by global bead id
    double4* xsave;      // state at block start (rollback)
    double* vsave;
    db::SweepBuf sw;
    db::Cells cells;
    db::NList nlist;
    db::Halo halo;
    db::Tiles tiles;
    int tile_cap;        // tiles the arena holds
    int tile_mode;       // 1: brick tiles when the system allows them (default), 0: never
    int brick_edge;      // cells per brick edge chosen by the tuner (0: from the density)
    int ntile;           // tiles of the current grid (0: the step kernel reads partners from memory)
    int tile_bB;         // cells per brick edge of the current grid
    bool tiles_valid;    // slots are in brick order: the tiles are the bricks of the last reordering
    bool regions_valid;  // the regions and 16-bit entries match the current lists
    bool halo_force;     // slots or tables changed: rebuild the halo
    bool halo_sweep;     // a sweep ran since the last halo build: rebuild it if the sweep changed bonds
    // Verlet list kept across sweeps: valid for the current slots and topology, and
    // list_disp bounds how far any bead has moved since its full build
    bool list_valid;
    double list_disp;
    double disp_rate;    // growth of that bound per step seen lately
    int64_t patches;     // blocks that kept the list and redid only the changed beads' lists
    // a batch of independent replicas (nrep > 0): one box per replica
    int nrep;
    std::vector<db::Box> reps;   // host copy; cell_off and gid_off fixed at creation
    std::vector<int> rep_n;      // beads per replica
    db::Box* rep_d;              // device copy (Params::rep)
    double nl_skin;      // neighbour-list cutoff minus pair cutoff
    int* slot_of_gid;    // [n]
    int* err_d;          // device error word
    float* vmax2;        // [max block length][DB_VMAX_SPREAD] max |v|^2 after each step (float bits)
    double* red;         // reduction scratch
    double* ledger_d;    // [12] energies before and after the last sweep
    bool ledger;         // track the topology-energy ledger
    double du_last, du_cum;
    int64_t* cnt64;      // small device counters
    int64_t* step_dev;   // the first step of the block being replayed from a graph
    int64_t* step_base_d;   // step_dev while step launches are captured, else nullptr
    bool use_graph;      // blocks' step launches are replayed from captured HIP graphs
    std::vector<db::GraphEntry>* graphs;   // captured blocks, keyed by length and buffers
    hipStream_t cap_stream;   // capture stream when the handle's stream is the null stream
    void* pinned;        // pinned host staging
    int max_block;

    // topology on the host side until uploaded
    bool have_state, have_topology;
    int64_t step, swept_step;
    int64_t rebuilds, rollbacks, sweeps;
    int64_t stat_last[8], stat_cum[8];
    int rebuild_interval;     // steps between rebuilds inside a block
    int permute_every;        // permute the state every k-th rebuild
    int64_t rebuild_count;
    double skin;
    bool skin_tuned;          // set by db_tune: the pair style no longer picks the default
    double vmax_est;

    // profiling
    bool profile;
    hipEvent_t ev_report;     // recorded after each block's report
    int profile_every;        // time every profile_every-th step launch
    int64_t profile_count;
    std::vector<hipEvent_t> ev_pool;
    int ev_used;
    double prof_ms;
    int64_t prof_launches;
};

namespace db {

// kernels_cells.hip
void launch_fill_int(int* p, int value, size_t count, hipStream_t s);
void launch_build_cells(db_ctx* c);                  // bin + scan + scatter + in-cell sort
void launch_permute(db_ctx* c, bool save);           // reorder all per-bead state by the cell list
                                                     // (save: also copy x, v to the rollback buffers)
bool tiles_enabled(const db_ctx* c);                 // the step kernel runs on brick tiles
void launch_exclusive_scan(int* data, int count, int* total_out, int* blocksum, hipStream_t s);
// out[0..count) = exclusive prefix sums of in (in != out), out[count] = the total
void launch_scan_total(const int* in, int* out, int count, int* blocksum, hipStream_t s);
void launch_compact(const int* flags, int count, int* list, int* total, int* blocksum, hipStream_t s);

// kernels_force.hip
void launch_halo(db_ctx* c);                         // bonded halo, if slots or tables changed
void launch_build_nlist(db_ctx* c);                  // halo, then the Verlet list from the current cell list
void launch_regions(db_ctx* c);                      // tile regions and 16-bit entries of the current lists
// Verlet lists of the beads whose exclusions the last sweep changed, with cutoff
// cut (the list cutoff plus twice the displacement since the full build)
void launch_patch_nlist(db_ctx* c, double cut);
// save: keep the input x, v (the block's input state, for a re-run)
void launch_step(db_ctx* c, int64_t step, int slot_in_block, bool save = false);
void launch_forces(db_ctx* c, double* f_gid_order);
// partials: 6 doubles per workgroup of the energy kernel (nullptr: the arena's own)
void launch_energy(db_ctx* c, double* out6_device, double* partials = nullptr);

// kernels_sweep.hip
void launch_sweep(db_ctx* c, int64_t step);
void launch_generate_all(db_ctx* c);
void launch_count_topology(db_ctx* c, int64_t* nb_na_nd_device);
void launch_gather_topology(db_ctx* c, int kind, int32_t* out_tuples, int32_t* out_types, int64_t count);

}  // namespace db
