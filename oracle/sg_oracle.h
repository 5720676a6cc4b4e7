/*
 * CPU oracle for checkerboard Metropolis / heat-bath sweeps of the 3D
 * Edwards-Anderson +-J Ising glass, the q = 4 +-J Potts glass and the q = 4
 * glassy (permutation) Potts model, driven by Parisi-Rapuano shift-register
 * random numbers.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * It is written for clarity: one site at a time, int8 / uint8 spins in the
 * canonical site order i = x + L*(y + L*z), a plain 61-entry ring per wheel,
 * exponentials evaluated in IEEE double on the host only.
 *
 * Paper passages followed (Belletti et al., "Simulating spin systems on
 * IANUS, an FPGA-based computer"):
 *   Eq. (1)  target distribution P ~ exp(-beta H)           (sec. 2.1)
 *   Eq. (2)  two-state Hamiltonian, EA case x = 1, h = 0     (sec. 2.1)
 *   Metropolis rule and heat bath, Eq. (4)                  (sec. 2.2)
 *   checkerboard (bipartite) parallel update                (sec. 3.1)
 *   Parisi-Rapuano generator, Eq. (5)                       (sec. 3.3)
 *   parallel tempering, named as an add-on                  (sec. 2.2)
 *   Eq. (3)  glassy Potts model with permutation couplings  (sec. 2.1)
 *            also on the 4D hypercubic lattice (OR_GPOTTS4)  (sec. 4.2)
 *   Eq. (2)  Ising-like models with dilution x_i and field h_i, e.g. the
 *            random-field Ising model (RFIM) and the diluted antiferromagnet
 *            in a field (DAFF)                               (sec. 2.1)
 * Two Potts models: the +-J glass H = -sum J_ij delta(s_i, s_j) (OR_POTTS)
 * and the glassy model of Eq. (3), H = -sum_<ij> delta(s_i, pi_ij(s_j))
 * (OR_GPOTTS).  For the latter the bond between i and j = i + e_d is stored
 * at i as the permutation pi of that term, one byte holding its images:
 * pi(v) = (byte >> 2v) & 3.
 */
#ifndef SG_ORACLE_H
#define SG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_ISING = 0, OR_POTTS = 1, OR_GPOTTS = 2, OR_ISING_GEN = 3, OR_GPOTTS4 = 4 };
enum { OR_METROPOLIS = 0, OR_HEATBATH = 1 };

/* Errors returned by or_run. */
enum { OR_OK = 0, OR_EINVAL = -1, OR_ENERGY_MISMATCH = -100 };

/* One Parisi-Rapuano wheel: ring[(pos + j) % 61] holds I(k - 61 + j),
 * j = 0..60, where k is the index of the next value to be produced. */
typedef struct {
  uint32_t ring[61];
  int32_t pos;
} or_wheel;

/* Load a wheel from its 61 words, oldest first (I(k-61) .. I(k-1)). */
void or_wheel_load(or_wheel *w, const uint32_t words[61]);
/* Store the 61 live words, oldest first. */
void or_wheel_store(const or_wheel *w, uint32_t words[61]);
/* Eq. (5): I(k) = I(k-24) + I(k-55) mod 2^32, R(k) = I(k) XOR I(k-61). */
uint32_t or_wheel_next(or_wheel *w);
/* n outputs of a wheel given by its 61 words; the words are not changed. */
void or_pr_stream(const uint32_t words[61], uint64_t n, uint32_t *out);

/* Integer thresholds, computed in IEEE double from the stated formulas.
 * Values are uint64 because 2^32 ("always") can occur. */
/* Metropolis, n = 0..2 unsatisfied bonds: floor(2^32 exp(-beta (12 - 4n))). */
void or_tables_metropolis(double beta, uint64_t T[3]);
/* Ising heat bath, k = 0..6 bonds with J s_j = +1, local field h = 2k - 6:
 * floor(2^32 / (1 + exp(-2 beta h))). */
void or_tables_heatbath(double beta, uint64_t T[7]);
/* Potts heat-bath weights W[d] = floor(2^28 exp(-beta d)), d = 0..12. */
void or_tables_potts(double beta, uint64_t W[13]);
/* Parallel-tempering factors F[b] = floor(2^32 exp(-|dbeta| 2^b)), b < 24. */
void or_tables_pt(double beta_a, double beta_b, uint64_t F[24]);
/* Integer acceptance threshold for an energy difference |D|:
 * T <- 2^32, then for every set bit b of |D| (ascending) T <- floor(T F[b] / 2^32);
 * |D| >= 2^24 gives 0. */
uint64_t or_pt_threshold(const uint64_t F[24], uint64_t absD);

/* Single-site updates (one random number r each); they return the energy
 * change and modify the spin in place.  T is the table of the algorithm. */
int32_t or_ising_update_site(int32_t L, int32_t algo, int8_t *s, const int8_t *J,
                             int64_t i, uint32_t r, const uint64_t *T);
int32_t or_potts_update_site(int32_t L, uint8_t *s, const int8_t *J, int64_t i,
                             uint32_t r, const uint64_t W[13]);
/* Glassy Potts: J holds the permutation bytes [3][N] (bond i -> i + e_d). */
int32_t or_gpotts_update_site(int32_t L, uint8_t *s, const uint8_t *P, int64_t i,
                              uint32_t r, const uint64_t W[13]);
/* Local fields h_a, a = 0..3, of site i of the glassy Potts model (the
 * number of bonds of i whose term is 1 when s_i = a). */
void or_gpotts_fields(int32_t L, const uint8_t *s, const uint8_t *P, int64_t i, int32_t h[4]);

/* 4D glassy Potts: periodic L^4, i = x + L (y + L (z + L u)), P = [4][N]
 * permutation bytes, P[d][i] on the bond i -> i + e_d (d = x, y, z, u),
 * term delta(s_i, pi(s_{i+e_d})) as in 3D; eight neighbours, h_a in 0..8.
 * Sweep order: colour (x + y + z + u) mod 2, even first; wheel
 * (g L + u) L + z serves rows g rho .. g rho + rho - 1 of the (z, u) plane,
 * rows ascending, x ascending (or_wheels_per_copy_4d(L) = L^3 / rho wheels). */
int32_t or_gpotts4_update_site(int32_t L, uint8_t *s, const uint8_t *P, int64_t i, uint32_t r,
                               const uint64_t W[13]);
void or_gpotts4_fields(int32_t L, const uint8_t *s, const uint8_t *P, int64_t i, int32_t h[4]);
int64_t or_gpotts4_energy(int32_t L, const uint8_t *s, const uint8_t *P);
int32_t or_wheels_per_copy_4d(int32_t L);

/* General Ising-like model of Eq. (2): D = [5][N] int8, rows J_x, J_y, J_z
 * (+-1, J[d][i] joins i and i + e_d), x (0 = empty site, 1 = spin) and f
 * (field sign +-1, h_i = field * f_i).  Empty sites are visited (and consume
 * their number) but never change.  Returns the change of the bond energy
 * E_b; *dM receives the change of M = sum_i x_i f_i s_i. */
int32_t or_isinggen_update_site(int32_t L, int32_t algo, int8_t *s, const int8_t *D, double field,
                                double beta, int64_t i, uint32_t r, int64_t *dM);
/* Bond energy E_b = -sum_<ij> J_ij x_i x_j s_i s_j and field sum
 * M = sum_i x_i f_i s_i; H = E_b - field * M. */
int64_t or_isinggen_bond_energy(int32_t L, const int8_t *s, const int8_t *D);
int64_t or_isinggen_field_sum(int32_t L, const int8_t *s, const int8_t *D);
/* Overlap over occupied sites, sum_i x_i s^a_i s^b_i. */
int64_t or_isinggen_overlap(int32_t L, const int8_t *a, const int8_t *b, const int8_t *D);

/* Energies and overlaps, by direct summation over the 3N bonds / N sites. */
int64_t or_ising_energy(int32_t L, const int8_t *s, const int8_t *J);
int64_t or_potts_energy(int32_t L, const uint8_t *s, const int8_t *J);
int64_t or_gpotts_energy(int32_t L, const uint8_t *s, const uint8_t *P);
int64_t or_ising_overlap(int32_t L, const int8_t *a, const int8_t *b);
int64_t or_potts_overlap(int32_t L, const uint8_t *a, const uint8_t *b);

/* Number of sweep wheels per copy: one per (z, group of rho = min(8, L) rows). */
int32_t or_wheels_per_copy(int32_t L);

typedef struct {
  int32_t model;          /* OR_ISING, OR_POTTS, OR_GPOTTS (q = 4), OR_ISING_GEN */
  int32_t algo;           /* OR_METROPOLIS or OR_HEATBATH (Potts: heat bath)     */
  int32_t L;              /* even side; 2, 4 or a multiple of 8                  */
  int32_t n_samples;      /* S disorder samples                                  */
  int32_t n_replicas;     /* R replicas per sample                               */
  int32_t n_temps;        /* K temperature slots per (sample, replica) chain     */
  int32_t pt_every;       /* sweeps between parallel-tempering steps, 0 = none   */
  int32_t measure_every;  /* sweeps between logged measurements, 0 = none        */
  int32_t check_energy;   /* 1: tracked energy == recomputed energy every sweep  */
  int32_t n_threads;      /* worker threads over copies (<= 0: one)              */
  double field;           /* OR_ISING_GEN: |h| (h_i = field * f_i); else unused  */
} or_spec;

/*
 * Run n_sweeps sweeps of every copy.  Copy (slot) c = (s R + r) K + k.
 *   betas         [K]            inverse temperatures, by temperature index
 *   J             [S][3][N]      int8 +-1 (glassy Potts: permutation bytes;
 *                                OR_ISING_GEN: [S][5][N], see above)
 *   spins         [C][N]         int8 +-1 (Ising) or uint8 0..3 (Potts), in/out
 *   wheels        [C][NW][61]    oldest first, in/out
 *   ptwheels      [S R][61]      one wheel per chain, in/out (unused if no PT)
 *   slot_of_temp  [S R][K]       slot holding temperature k, in/out
 *   sweeps_done   sweeps already performed (PT after sweeps that are
 *                 multiples of pt_every, counted from the start of the run)
 *   E_out         [C]            final energy of every slot (OR_ISING_GEN: E_b)
 *   M_out         [C]            OR_ISING_GEN: final field sum M of every slot
 *                                (may be NULL)
 *   E_log         [n_meas][S R][K] energy at each measurement, by chain and
 *                                temperature index (the slot holding it)
 *   Q_log         [n_meas][S][K] replica-0 / replica-1 overlap per
 *                                temperature (Ising sum s^a s^b, Potts models:
 *                                count of equal sites); needs R >= 2, else untouched
 *   pt_accepts    [S R][K-1]     accepted swaps per pair, accumulated
 * Measurements are taken after sweeps measure_every, 2 measure_every, ... of
 * this call, after any parallel-tempering step due at the same sweep.
 * OR_ISING_GEN runs without parallel tempering (its energy is not an integer
 * for a non-integer field); its overlap counts occupied sites only.
 */
int32_t or_run(const or_spec *sp, const double *betas, const int8_t *J, void *spins,
               uint32_t *wheels, uint32_t *ptwheels, int32_t *slot_of_temp,
               uint64_t sweeps_done, uint64_t n_sweeps, int64_t *E_out,
               int64_t *E_log, int64_t *Q_log, uint64_t *pt_accepts, int64_t *M_out);

#ifdef __cplusplus
}
#endif
#endif
