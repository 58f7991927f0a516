/*
 * oracle.h -- plain, slow FP64 CPU oracle of the dynamic-bonding hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; the two are
 * compared on identical seeded inputs.
 *
 * What it computes (paper: Svaneborg, "LAMMPS framework for dynamic bonding and
 * an application modeling DNA"):
 *   - forces of the WCA pair potential or the DPD conservative force, harmonic
 *     or well-shaped bonds with per-direction bond types (section 2,
 *     directional bonds), harmonic angles and cosine dihedrals (section 3
 *     potentials);
 *   - velocity-Verlet time stepping with a Langevin thermostat and/or the DPD
 *     dissipative and random pair forces (section 3);
 *   - the dynamic-bonding sweep (section 2 and the appendix "Implementation
 *     details", steps 2-9): creation and breakage nomination, mutual matching
 *     with stochastic acceptance, killbond, convertbond, removal of angles and
 *     dihedrals crossing broken bonds, bond creation and pattern-driven
 *     generation of angles and dihedrals.
 *
 * Representation: global lists of bonds (i<j, type stored by i, type stored by
 * j), angles (type, a, b, c with a<c) and dihedrals (type, a, b, c, d with
 * a<d); all ids are global bead ids.  No reordering, no per-bead tables.
 *
 * Every call returns 0 on success, a negative code on error (-1 invalid
 * argument, -2 capacity, -3 non-finite, -5 wrong call order).
 */
#ifndef DYNBOND_ORACLE_H
#define DYNBOND_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_sys or_sys;

or_sys* or_create(int32_t n, double box_L, uint64_t seed);
void or_destroy(or_sys* s);
int or_set_state(or_sys* s, const double* x, const double* v, const int32_t* type);
int or_set_reactive(or_sys* s, const uint8_t* flag);
int or_set_bonds(or_sys* s, int64_t nb, const int32_t* ij, const int32_t* t_ij, const int32_t* t_ji);
int or_set_angles(or_sys* s, int64_t na, const int32_t* abc, const int32_t* type);
int or_set_dihedrals(or_sys* s, int64_t nd, const int32_t* abcd, const int32_t* type);
int or_generate_angles_dihedrals(or_sys* s);

int or_pair_wca(or_sys* s, double eps, double sigma, double rc, int exclude_depth);
int or_pair_dpd(or_sys* s, double a, double gamma, double rc, int exclude_depth);
int or_bond_harmonic(or_sys* s, int32_t type, double K, double r0);
int or_bond_well(or_sys* s, int32_t type, double umin, double r_well, double r_zero, double r_cut);
int or_external_force(or_sys* s, int64_t count, const int32_t* ids, const double* f);
int or_angle_harmonic(or_sys* s, int32_t type, double K, double theta0);
int or_dihedral_cosine(or_sys* s, int32_t type, double K, double phi0);
int or_langevin(or_sys* s, double T, double gamma, double dt);
int or_temperature_ramp(or_sys* s, double T0, double T1, int64_t n_steps);

int or_sweep_every(or_sys* s, int32_t every, int paircheck13, int paircheck14);
/* 0: one uniform per pair (default); 1: the mean of one uniform per bead (appendix steps 5, 7) */
int or_acceptance(or_sys* s, int mode);
int or_bond_create(or_sys* s, int32_t bt, int32_t bead1, int32_t bead2, double r_max, double p);
int or_bond_create_dir(or_sys* s, int32_t bt1, int32_t bt2, int32_t bead1, int32_t bead2, double r_max, double p);
int or_bond_break(or_sys* s, int32_t bt, double r_min, double p);
int or_bond_kill(or_sys* s, int32_t bt, double r_min);
int or_bond_convert(or_sys* s, int32_t bt_from, int32_t bt_to, double r_min, double p);
int or_max_bonds(or_sys* s, int32_t bt, int32_t bead_type, int32_t max);
int or_angle_pattern(or_sys* s, int32_t atype, const int32_t bead[3], const uint32_t bondmask[2]);
int or_dihedral_pattern(or_sys* s, int32_t dtype, const int32_t bead[4], const uint32_t bondmask[3]);
int or_set_step(or_sys* s, int64_t step);

int or_step(or_sys* s, int64_t n);
int or_sweep_now(or_sys* s);
int or_forces(or_sys* s, double* f);
int or_energy(or_sys* s, double out[6]);
int or_get_state(or_sys* s, double* x, double* v);
int or_topology_counts(or_sys* s, int64_t* nb, int64_t* na, int64_t* nd);
int or_get_bonds(or_sys* s, int32_t* ij, int32_t* t_ij, int32_t* t_ji);
int or_get_angles(or_sys* s, int32_t* abc, int32_t* type);
int or_get_dihedrals(or_sys* s, int32_t* abcd, int32_t* type);
/* out[0..7]: bonds created, broken, killed, converted; angles created, removed;
 * dihedrals created, removed -- of the last sweep; out[8..15]: cumulative; out[16]: sweeps */
int or_get_stats(or_sys* s, int64_t out[17]);
/* nomination arrays of the last sweep: partner gid or -1 */
int or_last_nominations(or_sys* s, int32_t* nom_create, int32_t* nom_break);

/* test helpers */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* all pairs i<j with r^2 < rcut^2 (minimum image); brute=1: O(N^2), 0: cell list */
int64_t or_pairs_within(or_sys* s, double rcut, int brute, int32_t* out_ij, int64_t cap);
/* graph distance (number of bonds) between i and j, capped: returns 4 for >3 or disconnected */
int or_graph_distance(or_sys* s, int32_t i, int32_t j);

#ifdef __cplusplus
}
#endif
#endif
