/*
 * dynbond.h -- C-ABI of libdynbond, the MI355X (gfx950) implementation of the
 * data-parallel hot path of dynamic-bonding molecular dynamics
 * (C. Svaneborg, "LAMMPS framework for dynamic bonding and an application
 * modeling DNA", Comput. Phys. Commun. 2012).
 *
 * The library owns one simulation box per handle: beads with positions and
 * velocities, a bond graph with per-direction bond types, per-bead angle and
 * dihedral tables, a force field (WCA pairs, harmonic bonds, harmonic angles,
 * cosine dihedrals, Langevin thermostat) and an ordered set of dynamic-bonding
 * rules.  Every step runs on the GPU: a counting-sort cell list, a fused
 * force + integrate kernel, and every `every` steps the bond create / break /
 * kill / convert sweep followed by the angle/dihedral update.
 *
 * Conventions shared by all calls
 *  - Bead ids are 0..N-1 and are the global ids used as random-number keys.
 *    The library reorders beads internally and never exposes that order.
 *  - Host pointers unless a call says otherwise (`on_device` = 1: the pointer
 *    is device memory on the handle's device).  Inputs are copied in; outputs
 *    are written into caller-allocated buffers of the documented size.
 *  - Arrays of 3-vectors are row-major N x 3 doubles.
 *  - Bead types are 1..31, wildcard DB_ANY (0).  Bond-type sets are 32-bit masks with bit
 *    t set for bond type t (types 1..31); DB_ALL_BONDTYPES matches any type.
 *  - Rule order is call order: when several rules apply to one bead pair the
 *    last one wins (section 2; appendix steps 2-3).
 *  - Every call returns DB_OK (0) or a negative DB_E* code; db_last_error()
 *    gives a message.  Device-side errors (table overflow, non-finite state)
 *    are latched on the device and reported by the next db_step /
 *    db_sweep_now; after one the state is undefined and must be reloaded.
 *  - A handle is not thread-safe and issues all work on its own stream.
 */
#ifndef DYNBOND_H
#define DYNBOND_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define DB_OK 0
#define DB_EINVAL (-1)      /* bad argument or rule */
#define DB_ECAPACITY (-2)   /* a per-bead table overflowed */
#define DB_ENONFINITE (-3)  /* non-finite or escaping position */
#define DB_EDEVICE (-4)     /* HIP runtime error */
#define DB_ESTATE (-5)      /* call out of order */

#define DB_ANY 0
#define DB_ALL_BONDTYPES 0xFFFFFFFFu
#define DB_MAX_BOX_EDGE 65536.0   /* largest box edge db_create accepts */

#define DB_FP64 0           /* all force arithmetic in double */
#define DB_MIXED 1          /* pair and bonded force arithmetic in float; positions,
                               differences, accumulation, integration in double */

/* per-bead capacities of the bond, angle and dihedral tables */
#define DB_MAX_BONDS_PER_BEAD 4
#define DB_MAX_ANGLES_PER_BEAD 12
#define DB_MAX_DIHEDRALS_PER_BEAD 16

typedef struct db_ctx db_ctx;

typedef struct {
    /* last sweep, then cumulative (appendix step 9 statistics) */
    int64_t bonds_created, bonds_broken, bonds_killed, bonds_converted;
    int64_t angles_created, angles_removed, dihedrals_created, dihedrals_removed;
    int64_t cum_bonds_created, cum_bonds_broken, cum_bonds_killed, cum_bonds_converted;
    int64_t cum_angles_created, cum_angles_removed, cum_dihedrals_created, cum_dihedrals_removed;
    int64_t sweeps;          /* sweeps performed */
    int64_t steps;           /* current step counter */
    int64_t rebuilds;        /* cell-list rebuilds */
    int64_t rollbacks;       /* blocks re-run because beads moved further than the skin */
    /* topology-energy ledger (appendix step 9 statistics, extended): change of the
     * potential energy (pair + bond + angle + dihedral, FP64) across the last sweep
     * at fixed positions, and its sum over all sweeps; 0 while not tracked
     * (db_track_topology_energy) */
    double du_topo_last, du_topo_cum;
    int64_t list_patches;    /* blocks that kept the Verlet list across their sweep and redid only the
                                lists of the beads whose exclusions changed */
} db_stats;

/* ---- lifecycle ---------------------------------------------------------------- */

/* Create a handle for n_beads beads (0 .. 2^26 - 1) in a periodic cube of edge
 * box_L (0 < box_L <= DB_MAX_BOX_EDGE; every cutoff decision is exact in double
 * at any such edge: the float prefilters of the cell scans widen their cutoffs
 * by 4 sqrt(3) float ulps of 2 box_L, 0.0017 sigma at box_L = 1000).  seed keys every random number (Langevin noise and bond acceptance).
 * precision: DB_FP64 or DB_MIXED.  hip_stream: a hipStream_t (NULL = the null
 * stream).  Allocates no device memory yet. */
int db_create(db_ctx** out, int32_t n_beads, double box_L, uint64_t seed, int precision, void* hip_stream);
/* Device bytes the handle needs; db_bind_workspace may hand it a caller-owned
 * buffer (>= that size, 256-byte aligned) before db_set_state; otherwise the
 * library allocates on first use. */
int db_workspace_bytes(const db_ctx* ctx, size_t* bytes);
int db_bind_workspace(db_ctx* ctx, void* dev_ptr, size_t bytes);
int db_destroy(db_ctx* ctx);
const char* db_last_error(const db_ctx* ctx);

/* ---- system / topology (section 2: directional bonds; appendix: init) --------- */

/* x: positions in [0, box_L); v: velocities (the leapfrog half-step velocity that
 * enters the next force evaluation; NULL = zero); type: bead types 1..31. */
int db_set_state(db_ctx* ctx, const double* x, const double* v, const int32_t* type, int on_device);
/* reactive group of the bonding rules (section 2, `beadgroup`): flag per bead */
int db_set_reactive(db_ctx* ctx, const uint8_t* flag);
/* nb bonds: ij[2k], ij[2k+1] bead ids; t_ij = type stored by the first bead,
 * t_ji = type stored by the second (equal for symmetric bonds).  Replaces the
 * bond graph and clears angles and dihedrals. */
int db_set_bonds(db_ctx* ctx, int64_t nb, const int32_t* ij, const int32_t* t_ij, const int32_t* t_ji);
/* explicit angle (a,b,c centre b) and dihedral (a,b,c,d) lists with types */
int db_set_angles(db_ctx* ctx, int64_t na, const int32_t* abc, const int32_t* type);
int db_set_dihedrals(db_ctx* ctx, int64_t nd, const int32_t* abcd, const int32_t* type);
/* replace the angle and dihedral lists by every path of the current bond graph
 * that matches the pattern rules (section 2 matching, applied with every bond
 * taken as new) */
int db_generate_angles_dihedrals(db_ctx* ctx);

/* ---- force field and thermostat (section 3 potentials) ------------------------- */

/* WCA U = 4 eps[(s/r)^12 - (s/r)^6] + eps for r < rc.  exclude_depth 1 removes
 * bonded pairs, 2 also pairs two bonds apart. */
int db_pair_wca(db_ctx* ctx, double eps, double sigma, double rc, int exclude_depth);
/* DPD (section 3), replacing WCA: for r = |r_ij| < rc, r_ij = x_i - x_j,
 * e = r_ij / r, w = 1 - r / rc, bead i receives (F^C + F^D + F^R) e with
 * F^C = a w, F^D = -gamma w^2 (e . v_ij), F^R = sigma w xi / sqrt(dt),
 * sigma = sqrt(2 T gamma), xi a standard normal drawn per unordered pair and
 * step (Philox stream tag 3, Box-Muller on its first two words); U = a rc w^2 / 2.
 * T and dt come from db_langevin / db_temperature_ramp (whose own gamma may be
 * 0, leaving the DPD pair thermostat alone).  exclude_depth as for WCA (the
 * paper's DNA runs exclude beads fewer than three bonds apart: depth 2).
 * gamma >= 0; gamma = 0 gives the conservative force only.  Box edge > 2 rc. */
int db_pair_dpd(db_ctx* ctx, double a, double gamma, double rc, int exclude_depth);
/* Constant external forces (the unzipping experiments of section 3, e.g. 28
 * opposite forces on the end pair of a duplex): bead ids[k] feels f[3k..3k+2]
 * in every force evaluation, db_forces included; a bead listed twice gets the
 * sum; count = 0 removes them all.  Host pointers; the table is indexed by bead
 * id, so it follows the beads through reorders.  No energy is attributed to it
 * (its potential is not periodic).  EINVAL for an id outside 0..N-1 or a
 * non-finite component; ESTATE on a batch, and db_batch_create refuses replicas
 * that carry external forces. */
int db_external_force(db_ctx* ctx, int64_t count, const int32_t* ids, const double* f);
/* U = K (r - r0)^2; a bead feels the potential of the type it stores.  Directional
 * types with different potentials (or K = 0 one way: a "half" bond) give a net
 * force along the bond (section 2 remark on active matter). */
int db_bond_harmonic(db_ctx* ctx, int32_t type, double K, double r0);
/* Bond well of the 1-bead DNA model (section 3: backbone U_min = 10, well 0.3,
 * zero 0.6; hybridization U_min = 1, well 0.6, zero and cutoff 1.0), in the
 * reading that makes the two printed forms consistent:
 * U = U_min [(r - r_well)^2 / (r_zero - r_well)^2 - 1] for r < r_cut, 0 beyond
 * (r_cut = +inf: no cutoff).  Replaces any harmonic setting of the type.
 * EINVAL for a type outside 1..31, non-finite U_min / r_well / r_zero,
 * r_zero == r_well or r_cut <= 0. */
int db_bond_well(db_ctx* ctx, int32_t type, double U_min, double r_well, double r_zero, double r_cut);
/* U = K (theta - theta0)^2 */
int db_angle_harmonic(db_ctx* ctx, int32_t type, double K, double theta0);
/* U = K [1 - cos(phi - phi0)], phi the signed dihedral with cis = 0 */
int db_dihedral_cosine(db_ctx* ctx, int32_t type, double K, double phi0);
/* Langevin force -gamma v + sqrt(24 gamma T/dt)(u - 1/2) per component, u uniform;
 * gamma = 0 gives NVE.  dt is the time step. */
int db_langevin(db_ctx* ctx, double T, double gamma, double dt);
/* T(step) = T0 + (T1 - T0) min(step, n_steps) / n_steps */
int db_temperature_ramp(db_ctx* ctx, double T0, double T1, int64_t n_steps);

/* ---- dynamic-bonding rules (Fig. 1 syntax, section 2 semantics) ---------------- */

/* sweep every `every` steps (0 = never); paircheck13/14 admit beads two / three
 * bonds apart as creation partners */
int db_sweep_every(db_ctx* ctx, int32_t every, int paircheck13, int paircheck14);
/* How a mutual pair's acceptance test draws its random number (appendix steps 5
 * and 7).  DB_ACCEPT_PAIR (default): one 53-bit uniform u per unordered pair,
 * Philox4x32-10 keyed by (lower id, higher id, step, stream tag 1 create / 2
 * break) and the seed; accept iff u < p, so the acceptance probability is p.
 * DB_ACCEPT_AVERAGE, the appendix's literal form: each bead draws its own
 * uniform (counter (id, id, step, tag)), the pair accepts iff the mean of the two
 * is below p; the probability is then 2p^2 for p <= 1/2 and 1 - 2(1-p)^2 above.
 * Either way both beads reach the same decision.  EINVAL for another mode. */
#define DB_ACCEPT_PAIR 0
#define DB_ACCEPT_AVERAGE 1
int db_acceptance(db_ctx* ctx, int mode);
/* createbond: symmetric bond of type bt between bead types bead1, bead2 when
 * r < r_max, with probability p */
int db_bond_create(db_ctx* ctx, int32_t bt, int32_t bead1, int32_t bead2, double r_max, double p);
/* createdirbond: the bead of type bead1 stores bt1, the bead of type bead2 stores bt2 */
int db_bond_create_dir(db_ctx* ctx, int32_t bt1, int32_t bt2, int32_t bead1, int32_t bead2, double r_max, double p);
/* breakbond: a symmetric bond of type bt longer than r_min breaks with probability p */
int db_bond_break(db_ctx* ctx, int32_t bt, double r_min, double p);
/* killbond: every symmetric bond of type bt longer than r_min is removed */
int db_bond_kill(db_ctx* ctx, int32_t bt, double r_min);
/* convertbond: a symmetric bond of type bt_from longer than r_min becomes bt_to
 * with probability p (r_min = 0: any length, as in Fig. 1) */
int db_bond_convert(db_ctx* ctx, int32_t bt_from, int32_t bt_to, double r_min, double p);
/* maxbond: a bead of type bead_type (DB_ANY: any) holds at most max bonds it stores as bt */
int db_max_bonds(db_ctx* ctx, int32_t bt, int32_t bead_type, int32_t max);
/* createangle: bead types bead[0..2] (DB_ANY wildcard), bond-type sets
 * bondmask[0] for the type the centre stores towards the first bead and
 * bondmask[1] towards the third; tested on ABC then CBA */
int db_angle_pattern(db_ctx* ctx, int32_t atype, const int32_t bead[3], const uint32_t bondmask[2]);
/* createdihedral: bead[0..3]; bondmask[0] for t(B->A), bondmask[1] for t(C->B) or
 * t(B->C), bondmask[2] for t(C->D); tested on ABCD then DCBA */
int db_dihedral_pattern(db_ctx* ctx, int32_t dtype, const int32_t bead[4], const uint32_t bondmask[3]);

/* ---- run and observe ----------------------------------------------------------- */

/* Advance n >= 0 steps.  Step k: if every > 0 and k % every == 0, the bond sweep
 * of the appendix (steps 2-9: nominations, mutual matching with stochastic
 * acceptance, purge, removal and conversion, creation, angle / dihedral
 * generation, statistics) on the positions after the previous drift; then the
 * forces of sections 2 and 3 (pairs, directional bonds, angles, dihedrals,
 * external forces), the thermostat (Langevin or the DPD pair forces) and the
 * velocity-Verlet update of section 3.  Runs on the handle's stream and returns
 * when the steps are done.  Errors: DB_ESTATE before db_set_state or after a
 * latched device error; DB_ENONFINITE when a position became non-finite or left
 * the box (latched: the state is undefined until db_set_state or
 * db_checkpoint_load); DB_ECAPACITY when a sweep overflowed a per-bead table or a
 * Verlet list (latched likewise); DB_EDEVICE on a HIP error.  n = 0 runs nothing
 * after those checks. */
int db_step(db_ctx* ctx, int64_t n);
/* The sweep of the current step (appendix steps 2-9), now, on the current
 * positions; db_step then does not repeat it for this step.  Errors as db_step. */
int db_sweep_now(db_ctx* ctx);
/* The conservative forces of sections 2 and 3 (pairs, bonds, angles, dihedrals,
 * and the external forces) at the current positions, no thermostat: f is N x 3
 * doubles in bead-id order, caller-owned, host memory (on_device = 0) or device
 * memory (on_device = 1, written on the handle's stream, complete on return).
 * Errors as db_step (DB_EINVAL for f == NULL). */
int db_forces(db_ctx* ctx, double* f, int on_device);
/* out (host, 6 doubles) = {kinetic energy from the full-step velocities, U_pair,
 * U_bond, U_angle, U_dihedral (section 3 potentials, FP64 sums in a fixed order),
 * virial sum over interactions of r . F (Clausius)}.  Errors as db_step. */
int db_energy(db_ctx* ctx, double out[6]);
/* db_energy for callers that cannot allocate device or pinned memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the same
 * kernels and the same result, bit for bit, with the energy kernel's partial
 * sums in a fixed device array of the library (3 MiB per device, held until the
 * process ends) instead of the handle's workspace.  Makes no allocation of any
 * kind.  At most 16,777,216 beads (DB_EINVAL beyond).  DB_ESTATE unless the
 * handle's device memory is set up and its state and parameters are current on
 * the device: after any setter, run one db_step, db_forces or db_energy first.
 * All handles on one device share that array, so calls that overlap on one
 * device (from several threads or streams) race; calls in sequence do not. */
int db_energy_noalloc(db_ctx* ctx, double out[6]);
/* Positions (in [0, box_L)) and velocities (as in db_set_state), N x 3 doubles
 * each in bead-id order, caller-owned, host or device memory as on_device says;
 * either may be NULL.  Errors as db_step. */
int db_get_state(db_ctx* ctx, double* x, double* v, int on_device);
/* Current numbers of bonds, angles and dihedrals (section 2 topology), host. */
int db_topology_counts(db_ctx* ctx, int64_t* nb, int64_t* na, int64_t* nd);
/* The topology as canonical sorted lists, into caller-owned host arrays sized by
 * db_topology_counts: bonds (i, j) with i < j, the type each end stores (t_ij by
 * i, t_ji by j: section 2 directional bonds); angles (a, b, c) with a < c and
 * dihedrals (a, b, c, d) with a < d (path reversed if needed), with their types. */
int db_get_bonds(db_ctx* ctx, int32_t* ij, int32_t* t_ij, int32_t* t_ji);
int db_get_angles(db_ctx* ctx, int32_t* abc, int32_t* type);
int db_get_dihedrals(db_ctx* ctx, int32_t* abcd, int32_t* type);
/* The sweep statistics (appendix step 9: bonds created / broken / killed /
 * converted, angles and dihedrals created / removed; last sweep and cumulative)
 * and the scheduler's counters, into a caller-owned struct. */
int db_get_stats(db_ctx* ctx, db_stats* out);
/* Checkpoints of a single system.  db_checkpoint_bytes gives the size of the
 * host buffer; db_checkpoint_save fills it with every device array of the handle
 * (positions, velocities and topology tables in slot order, the Verlet and cell
 * lists, the per-bead sweep buffers) and the step scheduler's state (step, list
 * validity and displacement bound, rebuild interval and count, statistics).  The
 * caller owns the buffer.  db_checkpoint_load restores one into a handle made by
 * db_create with the same bead count, box edge, seed and precision and given the
 * same force field, rules, db_tune and db_tile_shape settings (the buffer holds
 * state, not configuration); the run then continues bit for bit as the saved run
 * would have.  Random numbers are keyed by bead ids, step and seed (no generator
 * state to keep).  EINVAL: a batch handle, a buffer too small, or a checkpoint of
 * another system, version, layout or tuning; the loading handle is unchanged
 * then.  Saving needs a current state (ESTATE otherwise). */
int db_checkpoint_bytes(db_ctx* ctx, size_t* bytes);
int db_checkpoint_save(db_ctx* ctx, void* host_buf, size_t bytes);
int db_checkpoint_load(db_ctx* ctx, const void* host_buf, size_t bytes);
/* current step counter; db_set_step also allows the sweep of that step again */
int db_set_step(db_ctx* ctx, int64_t step);
/* tuning knobs of the step scheduler: the neighbour-list skin (list cutoff minus
 * pair cutoff, > 0; default 0.55 with WCA, 0.02 with DPD) and how many cell-list
 * rebuilds pass between reorderings of the per-bead state into cell order (>= 1;
 * default 8).  Once set here, the skin no longer follows the pair style. */
int db_tune(db_ctx* ctx, double skin, int32_t permute_every);
/* enable = 1: the step launches of each block (the steps between two cell-list
 * rebuilds) are captured once per block length as a HIP graph and replayed, the
 * block's first step written to the device before each replay; 0 (default):
 * launched one by one.  The kernels and their results are the same.  Not used
 * while db_profile times launches.  EINVAL for another value. */
int db_graph(db_ctx* ctx, int enable);
/* Shape of the fused step kernel.  enable = 1: for a single system with WCA
 * pairs, beads are reordered brick by brick (bricks of brick_edge^3 cells; 0:
 * chosen from the density, about 200 beads a brick), each workgroup takes 256
 * consecutive beads, loads the positions of every bead their lists and bonded
 * terms name into LDS once (each as its image next to the tile), and reads
 * partners from there; after every list build a region pass records those beads
 * and re-codes the entries as 16-bit indices.  In a tile whose beads hold at most
 * four angles and four dihedrals each (448 and 224 per tile at most), every angle
 * and dihedral is evaluated once, by one thread, and each member adds its share.
 * enable = 0 (default): one thread per bead gathers partners from memory and
 * evaluates its own terms.  The two agree to rounding (the staged separations are
 * differences of images instead of images of differences, and a bead's force is
 * summed in another order).  The arrays of this shape are part of the workspace
 * whether or not it is on.
 * Takes effect at the next block.  EINVAL for enable outside {0, 1} or
 * brick_edge outside 0..64. */
int db_tile_shape(db_ctx* ctx, int enable, int32_t brick_edge);
/* regions of the current tiles: out = {tiles, tiles whose region is staged in LDS,
 * sum of the staged regions' sizes, largest region}; all 0 while the step kernel
 * runs without tiles */
int db_tile_stats(db_ctx* ctx, int64_t out[4]);
/* HIP-event timing of the fused step kernel on the handle's stream: every
 * `every`-th launch is bracketed by two events (1 = every launch; 0 = off).
 * Each event pair leaves the GPU idle for a few microseconds between launches,
 * so sampling keeps the timed run close to an untimed one.  EINVAL if every < 0. */
int db_profile(db_ctx* ctx, int every);
/* mean GPU time per launch (microseconds) of the fused step kernel over the
 * launches timed since the last call, and their number; resets the tally */
int db_step_kernel_time(db_ctx* ctx, double* mean_us, int64_t* launches);

/* enable (1) / disable (0) the topology-energy ledger of db_stats: every sweep is
 * then bracketed by two potential-energy evaluations (costs about two force
 * passes per sweep) */
int db_track_topology_energy(db_ctx* ctx, int enable);
/* tries skin in {0.4, 0.5, 0.6, 0.8} (DPD: {0.02, 0.05, 0.1, 0.3}) x
 * permute_every in {1, 2, 4, 8}, then the step kernel's shape (db_tile_shape: per
 * bead, or tiles over bricks of 0 = density's choice, 3, 4, 5 cells; single
 * systems with WCA pairs), then graphs off and on (db_graph), running one untimed
 * and steps_per_trial timed steps of the trajectory with each (the system advances
 * (steps_per_trial + 1) x (16 + shapes + 2) steps, shapes = 4 or 1), and keeps the
 * fastest of each; best_skin / best_permute (either may be NULL) receive the
 * choice, db_get_shape the rest */
int db_autotune(db_ctx* ctx, int64_t steps_per_trial, double* best_skin, int32_t* best_permute);
/* out = {tile kernel on, brick edge (0: density's choice), graphs on} */
int db_get_shape(db_ctx* ctx, int32_t out[3]);

/* ---- batches of independent replicas ------------------------------------------ */
/* Not in the paper: many small boxes (replicas of a parameter ladder) are
 * advanced together so that every kernel launch covers all of them.
 *
 * db_batch_create builds a new handle holding copies of the n_rep configured
 * replica handles (state, reactive flags, topology, step counter).  The
 * replicas must agree on precision, force field, dt, gamma, rules and step
 * counter; each keeps its own bead count, box edge, seed and temperature
 * schedule, and evolves exactly as it would alone (bead ids and random numbers
 * are per replica).  The replica handles are not modified or referenced
 * afterwards.  Global bead ids of the batch are the replicas' ids offset by the
 * bead counts of the replicas before them, in the order given; db_get_bonds and
 * the other getters of the batch handle use global ids; db_batch_get_state
 * returns one replica's positions and velocities in its own ids.  State and
 * topology setters on a batch handle fail with DB_ESTATE; force-field, rule,
 * thermostat (applied to every replica) and tuning calls work as for a single
 * system.  Free with db_destroy.
 * Errors: DB_EINVAL for n_rep < 1 or > 65535, a NULL replica, a replica without
 * state or mismatched physics; device errors as for db_create. */
int db_batch_create(db_ctx** out, db_ctx* const* replicas, int32_t n_rep, void* hip_stream);
/* x, v: that replica's N_r x 3 arrays (either may be NULL), host or device */
int db_batch_get_state(db_ctx* batch, int32_t replica, double* x, double* v, int on_device);

#ifdef __cplusplus
}
#endif
#endif
