/*
 * CPU oracle -- TEST INFRASTRUCTURE ONLY (see sg_oracle.h).
 *
 * Plain reference implementation of the sweep described in the paper:
 * checkerboard single-spin updates (sec. 3.1), Metropolis and heat bath
 * (sec. 2.2, Eq. 4), one Parisi-Rapuano number per site update (sec. 3.3,
 * Eq. 5), compared against integer thresholds derived on the host in double.
 * Readings of points the paper leaves open are fixed in the project's design
 * notes; each is restated at the place it is used.
 */
#include "sg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Parisi-Rapuano wheel, Eq. (5).  The paper's "otimes" is read as a    */
/* bitwise XOR (it describes the last step as an XOR with a third       */
/* value).  Lags 24, 55, 61; words are 32 bits (sec. 3.3).             */
/* ------------------------------------------------------------------ */

void or_wheel_load(or_wheel *w, const uint32_t words[61]) {
  for (int j = 0; j < 61; j++) w->ring[j] = words[j];
  w->pos = 0; /* ring[pos] is the oldest live word, I(k-61) */
}

void or_wheel_store(const or_wheel *w, uint32_t words[61]) {
  for (int j = 0; j < 61; j++) words[j] = w->ring[(w->pos + j) % 61];
}

/* I(k-m) lives at ring[(pos + 61 - m) % 61] for m = 1..61. */
static uint32_t back(const or_wheel *w, int m) {
  int j = w->pos - m;
  return w->ring[j < 0 ? j + 61 : j];
}

uint32_t or_wheel_next(or_wheel *w) {
  uint32_t ik = back(w, 24) + back(w, 55); /* mod 2^32 by unsigned wrap */
  uint32_t out = ik ^ back(w, 61);
  w->ring[w->pos] = ik; /* I(k-61) is no longer needed; I(k) takes its place */
  w->pos = w->pos == 60 ? 0 : w->pos + 1;
  return out;
}

void or_pr_stream(const uint32_t words[61], uint64_t n, uint32_t *out) {
  or_wheel w;
  or_wheel_load(&w, words);
  for (uint64_t t = 0; t < n; t++) out[t] = or_wheel_next(&w);
}

/* ------------------------------------------------------------------ */
/* Thresholds.  A number r in [0, 2^32) is accepted when r < T, so the   */
/* acceptance probability is exactly T / 2^32.                          */
/* ------------------------------------------------------------------ */

static uint64_t scaled_floor(double p, int bits) { return (uint64_t)floor(ldexp(p, bits)); }

void or_tables_metropolis(double beta, uint64_t T[3]) {
  /* Flipping a spin with n unsatisfied bonds out of 6 changes the energy of
   * Eq. (2) (x = 1, h = 0) by dE = 12 - 4n; for n >= 3 dE <= 0 and the move is
   * always accepted, otherwise with probability exp(-beta dE) (sec. 2.2). */
  for (int n = 0; n < 3; n++) T[n] = scaled_floor(exp(-beta * (double)(12 - 4 * n)), 32);
}

void or_tables_heatbath(double beta, uint64_t T[7]) {
  /* Eq. (4) with E(+-1) = -+h, h = sum_j J_ij s_j = 2k - 6. */
  for (int k = 0; k < 7; k++) {
    double h = (double)(2 * k - 6);
    T[k] = scaled_floor(1.0 / (1.0 + exp(-2.0 * beta * h)), 32);
  }
}

void or_tables_potts(double beta, uint64_t W[13]) {
  for (int d = 0; d < 13; d++) W[d] = scaled_floor(exp(-beta * (double)d), 28);
}

void or_tables_pt(double beta_a, double beta_b, uint64_t F[24]) {
  double db = fabs(beta_a - beta_b);
  for (int b = 0; b < 24; b++) F[b] = scaled_floor(exp(-db * ldexp(1.0, b)), 32);
}

uint64_t or_pt_threshold(const uint64_t F[24], uint64_t absD) {
  if (absD >> 24) return 0;
  uint64_t T = (uint64_t)1 << 32;
  for (int b = 0; b < 24; b++)
    if ((absD >> b) & 1) T = (uint64_t)(((unsigned __int128)T * F[b]) >> 32);
  return T;
}

/* ------------------------------------------------------------------ */
/* Lattice: periodic L^3, i = x + L (y + L z); J[d][i] joins i, i + e_d. */
/* ------------------------------------------------------------------ */

static void neighbours_xyz(int32_t L, int64_t x, int64_t y, int64_t z, int64_t nb[6],
                           int64_t bond[6]) {
  int64_t N = (int64_t)L * L * L;
  int64_t i = x + L * (y + L * z);
  int64_t xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
  int64_t yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
  int64_t zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
  nb[0] = xp + L * (y + L * z);
  nb[1] = xm + L * (y + L * z);
  nb[2] = x + L * (yp + L * z);
  nb[3] = x + L * (ym + L * z);
  nb[4] = x + L * (y + L * zp);
  nb[5] = x + L * (y + L * zm);
  bond[0] = 0 * N + i;      /* bond to +x belongs to i          */
  bond[1] = 0 * N + nb[1];  /* bond to -x belongs to the -x site */
  bond[2] = 1 * N + i;
  bond[3] = 1 * N + nb[3];
  bond[4] = 2 * N + i;
  bond[5] = 2 * N + nb[5];
}

static void neighbours(int32_t L, int64_t i, int64_t nb[6], int64_t bond[6]) {
  neighbours_xyz(L, i % L, (i / L) % L, i / ((int64_t)L * L), nb, bond);
}

static int32_t ising_update(int32_t algo, int8_t *s, const int8_t *J, int64_t i,
                            const int64_t nb[6], const int64_t bond[6], uint32_t r,
                            const uint64_t *T) {
  int32_t h = 0; /* local field sum_j J_ij s_j */
  int32_t n = 0; /* unsatisfied bonds: J s_i s_j = -1 */
  for (int d = 0; d < 6; d++) {
    int32_t js = J[bond[d]] * s[nb[d]];
    h += js;
    if (js * s[i] == -1) n++;
  }
  int32_t old = s[i];
  if (algo == OR_METROPOLIS) {
    /* flip if dE <= 0 (n >= 3) or r < T[n]; e^0 = 1 at n = 3 */
    if (n >= 3 || (uint64_t)r < T[n]) {
      s[i] = (int8_t)(-old);
      return 2 * old * h; /* = 12 - 4n */
    }
    return 0;
  }
  /* heat bath: s = +1 with probability T[k] / 2^32, k = (h + 6) / 2 */
  int32_t k = (h + 6) / 2;
  int32_t nw = ((uint64_t)r < T[k]) ? 1 : -1;
  s[i] = (int8_t)nw;
  return -(nw - old) * h;
}

/* Heat bath over the four states given their local fields h_a (the energy
 * of state a is -h_a): P(a) ~ exp(beta h_a), drawn with the integer weights
 * w_a = W[h_max - h_a] and t = floor(r S / 2^32), S = sum w_a: the new state
 * is the first a with t < w_0 + ... + w_a.  Returns the energy change. */
static int32_t potts_heat_bath(uint8_t *s, int64_t i, const int32_t h[4], uint32_t r,
                               const uint64_t W[13]) {
  int32_t hmax = h[0];
  for (int a = 1; a < 4; a++)
    if (h[a] > hmax) hmax = h[a];
  /* Boltzmann weight of state a relative to the best one: exp(-beta (hmax - h_a)) */
  uint64_t w[4], S = 0;
  for (int a = 0; a < 4; a++) {
    w[a] = W[hmax - h[a]];
    S += w[a];
  }
  uint64_t t = ((uint64_t)r * S) >> 32; /* uniform on [0, S) up to rounding */
  uint64_t cum = 0;
  int32_t nw = 3;
  for (int a = 0; a < 4; a++) {
    cum += w[a];
    if (t < cum) {
      nw = a;
      break;
    }
  }
  int32_t old = s[i];
  s[i] = (uint8_t)nw;
  return -(h[nw] - h[old]);
}

static int32_t potts_update(uint8_t *s, const int8_t *J, int64_t i, const int64_t nb[6],
                            const int64_t bond[6], uint32_t r, const uint64_t W[13]) {
  int32_t h[4] = {0, 0, 0, 0}; /* h_a = sum_j J_ij delta(a, s_j) */
  for (int d = 0; d < 6; d++) h[s[nb[d]]] += J[bond[d]];
  return potts_heat_bath(s, i, h, r, W);
}

/* Glassy Potts, Eq. (3).  The term of the bond between i and j = i + e_d
 * (stored at i as pi) is delta(s_i, pi(s_j)).  For the fields of i:
 *   bond to j = i + e_d (stored at i):   s_i = a scores iff a = pi(s_j);
 *   bond to j = i - e_d (stored at j):   s_i = a scores iff pi(a) = s_j. */
static int perm_image(uint8_t P, int v) { return (P >> (2 * v)) & 3; }

static void gpotts_fields_n(int nd, const uint8_t *s, const uint8_t *P, const int64_t *nb,
                            const int64_t *bond, int32_t h[4]) {
  for (int a = 0; a < 4; a++) h[a] = 0;
  for (int d = 0; d < nd; d++) {
    uint8_t pi = P[bond[d]];
    int sj = s[nb[d]];
    if ((d & 1) == 0) {
      h[perm_image(pi, sj)] += 1;
    } else {
      for (int a = 0; a < 4; a++)
        if (perm_image(pi, a) == sj) h[a] += 1;
    }
  }
}

static void gpotts_fields(const uint8_t *s, const uint8_t *P, const int64_t nb[6],
                          const int64_t bond[6], int32_t h[4]) {
  gpotts_fields_n(6, s, P, nb, bond, h);
}

static int32_t gpotts_update(uint8_t *s, const uint8_t *P, int64_t i, const int64_t nb[6],
                             const int64_t bond[6], uint32_t r, const uint64_t W[13]) {
  int32_t h[4];
  gpotts_fields(s, P, nb, bond, h);
  return potts_heat_bath(s, i, h, r, W);
}

/* ------------------------------------------------------------------ */
/* 4D glassy Potts (Eq. 3 on the hypercubic lattice, sec. 4.2): periodic */
/* L^4, i = x + L (y + L (z + L u)); P[d][i] (d = x, y, z, u) is the bond */
/* between i and i + e_d, stored at i as for 3D.  Neighbour d = 2a is    */
/* i + e_a (bond stored at i), d = 2a + 1 is i - e_a (stored there).     */
/* ------------------------------------------------------------------ */
static void neighbours4(int32_t L, int64_t x, int64_t y, int64_t z, int64_t u, int64_t nb[8],
                        int64_t bond[8]) {
  int64_t N = (int64_t)L * L * L * L;
  int64_t c[4] = {x, y, z, u}, stride[4] = {1, L, (int64_t)L * L, (int64_t)L * L * L};
  int64_t i = x + stride[1] * y + stride[2] * z + stride[3] * u;
  for (int a = 0; a < 4; a++) {
    int64_t up = c[a] + 1 == L ? 0 : c[a] + 1, dn = c[a] == 0 ? L - 1 : c[a] - 1;
    nb[2 * a] = i + (up - c[a]) * stride[a];
    nb[2 * a + 1] = i + (dn - c[a]) * stride[a];
    bond[2 * a] = a * N + i;
    bond[2 * a + 1] = a * N + nb[2 * a + 1];
  }
}

static void neighbours4_i(int32_t L, int64_t i, int64_t nb[8], int64_t bond[8]) {
  int64_t L2 = (int64_t)L * L;
  neighbours4(L, i % L, (i / L) % L, (i / L2) % L, i / (L2 * L), nb, bond);
}

int32_t or_gpotts4_update_site(int32_t L, uint8_t *s, const uint8_t *P, int64_t i, uint32_t r,
                               const uint64_t W[13]) {
  int64_t nb[8], bond[8];
  int32_t h[4];
  neighbours4_i(L, i, nb, bond);
  gpotts_fields_n(8, s, P, nb, bond, h);
  return potts_heat_bath(s, i, h, r, W);
}

void or_gpotts4_fields(int32_t L, const uint8_t *s, const uint8_t *P, int64_t i, int32_t h[4]) {
  int64_t nb[8], bond[8];
  neighbours4_i(L, i, nb, bond);
  gpotts_fields_n(8, s, P, nb, bond, h);
}

/* each of the 4N bonds once, as the term stored at its lower site */
int64_t or_gpotts4_energy(int32_t L, const uint8_t *s, const uint8_t *P) {
  int64_t N = (int64_t)L * L * L * L, E = 0;
  for (int64_t i = 0; i < N; i++) {
    int64_t nb[8], bond[8];
    neighbours4_i(L, i, nb, bond);
    for (int d = 0; d < 8; d += 2)
      if (s[i] == perm_image(P[bond[d]], s[nb[d]])) E -= 1;
  }
  return E;
}

/* General Ising-like model, Eq. (2): H = -sum J_ij x_i x_j s_i s_j
 * - sum h_i x_i s_i with h_i = field * f_i.  For an occupied site the local
 * field is b + h_i with b = sum_j J_ij x_j s_j (an integer in [-6, 6]).
 *   Metropolis: dE = 2 s_i (b + h_i) = 2c + 2 field (1 - 2 phi), c = s_i b,
 *     phi = [s_i f_i = -1]; flip if dE <= 0, else iff r < floor(2^32 exp(-beta dE)).
 *   Heat bath (Eq. 4 with E(+-1) = -+(b + h_i)): s_i = +1 iff
 *     r < floor(2^32 / (1 + exp(-2 beta (b + field f_i)))).
 * Empty sites (x_i = 0) consume their number and keep their value. */
static int32_t isinggen_update(int32_t algo, int8_t *s, const int8_t *D, int64_t N, double field,
                               double beta, int64_t i, const int64_t nb[6], const int64_t bond[6],
                               uint32_t r, int64_t *dM) {
  const int8_t *x = D + 3 * N, *f = D + 4 * N;
  *dM = 0;
  if (!x[i]) return 0;
  int32_t b = 0;
  for (int d = 0; d < 6; d++) b += D[bond[d]] * x[nb[d]] * s[nb[d]];
  int32_t old = s[i], nw;
  if (algo == OR_METROPOLIS) {
    int32_t c = old * b;
    int phi = old * f[i] == -1;
    double dE = 2.0 * (double)c + 2.0 * field * (phi ? -1.0 : 1.0);
    uint64_t T = dE <= 0.0 ? ((uint64_t)1 << 32) : scaled_floor(exp(-beta * dE), 32);
    nw = (uint64_t)r < T ? -old : old;
  } else {
    double hl = (double)b + field * (double)f[i];
    uint64_t T = scaled_floor(1.0 / (1.0 + exp(-2.0 * beta * hl)), 32);
    nw = (uint64_t)r < T ? 1 : -1;
  }
  s[i] = (int8_t)nw;
  *dM = (int64_t)(nw - old) * f[i];
  return -(nw - old) * b;
}

int32_t or_isinggen_update_site(int32_t L, int32_t algo, int8_t *s, const int8_t *D, double field,
                                double beta, int64_t i, uint32_t r, int64_t *dM) {
  int64_t nb[6], bond[6];
  neighbours(L, i, nb, bond);
  return isinggen_update(algo, s, D, (int64_t)L * L * L, field, beta, i, nb, bond, r, dM);
}

int64_t or_isinggen_bond_energy(int32_t L, const int8_t *s, const int8_t *D) {
  int64_t N = (int64_t)L * L * L, E = 0;
  const int8_t *x = D + 3 * N;
  for (int64_t i = 0; i < N; i++) {
    int64_t nb[6], bond[6];
    neighbours(L, i, nb, bond);
    for (int d = 0; d < 6; d += 2) E -= (int64_t)D[bond[d]] * x[i] * x[nb[d]] * s[i] * s[nb[d]];
  }
  return E;
}

int64_t or_isinggen_field_sum(int32_t L, const int8_t *s, const int8_t *D) {
  int64_t N = (int64_t)L * L * L, M = 0;
  const int8_t *x = D + 3 * N, *f = D + 4 * N;
  for (int64_t i = 0; i < N; i++) M += (int64_t)x[i] * f[i] * s[i];
  return M;
}

int64_t or_isinggen_overlap(int32_t L, const int8_t *a, const int8_t *b, const int8_t *D) {
  int64_t N = (int64_t)L * L * L, Q = 0;
  const int8_t *x = D + 3 * N;
  for (int64_t i = 0; i < N; i++) Q += (int64_t)x[i] * a[i] * b[i];
  return Q;
}

int32_t or_ising_update_site(int32_t L, int32_t algo, int8_t *s, const int8_t *J,
                             int64_t i, uint32_t r, const uint64_t *T) {
  int64_t nb[6], bond[6];
  neighbours(L, i, nb, bond);
  return ising_update(algo, s, J, i, nb, bond, r, T);
}

int32_t or_potts_update_site(int32_t L, uint8_t *s, const int8_t *J, int64_t i, uint32_t r,
                             const uint64_t W[13]) {
  int64_t nb[6], bond[6];
  neighbours(L, i, nb, bond);
  return potts_update(s, J, i, nb, bond, r, W);
}

int32_t or_gpotts_update_site(int32_t L, uint8_t *s, const uint8_t *P, int64_t i, uint32_t r,
                              const uint64_t W[13]) {
  int64_t nb[6], bond[6];
  neighbours(L, i, nb, bond);
  return gpotts_update(s, P, i, nb, bond, r, W);
}

void or_gpotts_fields(int32_t L, const uint8_t *s, const uint8_t *P, int64_t i, int32_t h[4]) {
  int64_t nb[6], bond[6];
  neighbours(L, i, nb, bond);
  gpotts_fields(s, P, nb, bond, h);
}

int64_t or_ising_energy(int32_t L, const int8_t *s, const int8_t *J) {
  int64_t N = (int64_t)L * L * L, E = 0;
  for (int64_t i = 0; i < N; i++) {
    int64_t nb[6], bond[6];
    neighbours(L, i, nb, bond);
    for (int d = 0; d < 6; d += 2) E -= (int64_t)J[bond[d]] * s[i] * s[nb[d]];
  }
  return E;
}

int64_t or_potts_energy(int32_t L, const uint8_t *s, const int8_t *J) {
  int64_t N = (int64_t)L * L * L, E = 0;
  for (int64_t i = 0; i < N; i++) {
    int64_t nb[6], bond[6];
    neighbours(L, i, nb, bond);
    for (int d = 0; d < 6; d += 2)
      if (s[i] == s[nb[d]]) E -= J[bond[d]];
  }
  return E;
}

/* Eq. (3): each bond once, as the term stored at its lower site. */
int64_t or_gpotts_energy(int32_t L, const uint8_t *s, const uint8_t *P) {
  int64_t N = (int64_t)L * L * L, E = 0;
  for (int64_t i = 0; i < N; i++) {
    int64_t nb[6], bond[6];
    neighbours(L, i, nb, bond);
    for (int d = 0; d < 6; d += 2)
      if (s[i] == perm_image(P[bond[d]], s[nb[d]])) E -= 1;
  }
  return E;
}

int64_t or_ising_overlap(int32_t L, const int8_t *a, const int8_t *b) {
  int64_t N = (int64_t)L * L * L, Q = 0;
  for (int64_t i = 0; i < N; i++) Q += (int64_t)a[i] * b[i];
  return Q;
}

int64_t or_potts_overlap(int32_t L, const uint8_t *a, const uint8_t *b) {
  int64_t N = (int64_t)L * L * L, Q = 0;
  for (int64_t i = 0; i < N; i++) Q += (a[i] == b[i]);
  return Q;
}

int32_t or_wheels_per_copy(int32_t L) {
  int32_t rho = L < 8 ? L : 8;
  return L * (L / rho);
}

/* 4D: one wheel per (z, u, group of rho rows), index (g L + u) L + z */
int32_t or_wheels_per_copy_4d(int32_t L) { return L * or_wheels_per_copy(L); }

static int32_t is_4d(const or_spec *sp) { return sp->model == OR_GPOTTS4; }
static int64_t sites_of(const or_spec *sp) {
  int64_t N = (int64_t)sp->L * sp->L * sp->L;
  return is_4d(sp) ? N * sp->L : N;
}
static int32_t wheels_of(const or_spec *sp) {
  return is_4d(sp) ? or_wheels_per_copy_4d(sp->L) : or_wheels_per_copy(sp->L);
}

/* 4D sweep: colour p = (x + y + z + u) mod 2, even colour first; wheel
 * (g L + u) L + z serves rows y = g rho .. g rho + rho - 1 of the (z, u)
 * plane, one number per visited site, colour, then row, then increasing x. */
static void copy_sweep_4d(const or_spec *sp, uint8_t *spins, const uint8_t *P, or_wheel *wheels,
                          const uint64_t *W, int64_t *E) {
  int32_t L = sp->L, rho = L < 8 ? L : 8, nG = L / rho;
  for (int p = 0; p < 2; p++)
    for (int g = 0; g < nG; g++)
      for (int u = 0; u < L; u++)
        for (int z = 0; z < L; z++) {
          or_wheel *w = &wheels[((int64_t)g * L + u) * L + z];
          for (int y = g * rho; y < g * rho + rho; y++)
            for (int x = 0; x < L; x++) {
              if (((x + y + z + u) & 1) != p) continue;
              uint32_t r = or_wheel_next(w);
              int64_t i = x + (int64_t)L * (y + (int64_t)L * (z + (int64_t)L * u));
              int64_t nb[8], bond[8];
              int32_t h[4];
              neighbours4(L, x, y, z, u, nb, bond);
              gpotts_fields_n(8, spins, P, nb, bond, h);
              *E += potts_heat_bath(spins, i, h, r, W);
            }
        }
}

/* ------------------------------------------------------------------ */
/* One sweep of one copy.  Colour p = (x + y + z) mod 2; the even colour */
/* is updated first (sec. 3.1: all sites of one colour, then the other). */
/* Wheel w = g L + z serves rows y = g rho .. g rho + rho - 1 of plane z, */
/* drawing one number per visited site in the order: colour, then row,   */
/* then increasing x.  Every visit consumes exactly one number.          */
/* ------------------------------------------------------------------ */

static void copy_sweep(const or_spec *sp, void *spins, const int8_t *J, or_wheel *wheels,
                       const uint64_t *T, double beta, int64_t *E, int64_t *M) {
  int32_t L = sp->L, rho = L < 8 ? L : 8, nG = L / rho;
  for (int p = 0; p < 2; p++)
    for (int g = 0; g < nG; g++)
      for (int z = 0; z < L; z++) {
        or_wheel *w = &wheels[g * L + z];
        for (int y = g * rho; y < g * rho + rho; y++)
          for (int x = 0; x < L; x++) {
            if (((x + y + z) & 1) != p) continue;
            uint32_t r = or_wheel_next(w);
            int64_t i = x + (int64_t)L * (y + (int64_t)L * z);
            int64_t nb[6], bond[6];
            neighbours_xyz(L, x, y, z, nb, bond);
            if (sp->model == OR_ISING)
              *E += ising_update(sp->algo, (int8_t *)spins, J, i, nb, bond, r, T);
            else if (sp->model == OR_POTTS)
              *E += potts_update((uint8_t *)spins, J, i, nb, bond, r, T);
            else if (sp->model == OR_GPOTTS)
              *E += gpotts_update((uint8_t *)spins, (const uint8_t *)J, i, nb, bond, r, T);
            else {
              int64_t dM;
              *E += isinggen_update(sp->algo, (int8_t *)spins, J, (int64_t)L * L * L, sp->field,
                                    beta, i, nb, bond, r, &dM);
              *M += dM;
            }
          }
      }
}

static int64_t copy_energy(const or_spec *sp, const void *spins, const int8_t *J) {
  if (sp->model == OR_GPOTTS4) return or_gpotts4_energy(sp->L, (const uint8_t *)spins, (const uint8_t *)J);
  if (sp->model == OR_ISING) return or_ising_energy(sp->L, (const int8_t *)spins, J);
  if (sp->model == OR_POTTS) return or_potts_energy(sp->L, (const uint8_t *)spins, J);
  if (sp->model == OR_GPOTTS) return or_gpotts_energy(sp->L, (const uint8_t *)spins, (const uint8_t *)J);
  return or_isinggen_bond_energy(sp->L, (const int8_t *)spins, J);
}

static int64_t copy_field_sum(const or_spec *sp, const void *spins, const int8_t *J) {
  return sp->model == OR_ISING_GEN ? or_isinggen_field_sum(sp->L, (const int8_t *)spins, J) : 0;
}

/* coupling rows per sample: J_x, J_y, J_z (+ x, f for the general model) */
static int64_t coupling_rows(const or_spec *sp) {
  return sp->model == OR_ISING_GEN ? 5 : (sp->model == OR_GPOTTS4 ? 4 : 3);
}

static void copy_tables(const or_spec *sp, double beta, uint64_t T[13]) {
  if (sp->model == OR_POTTS || sp->model == OR_GPOTTS || sp->model == OR_GPOTTS4)
    or_tables_potts(beta, T);
  else if (sp->algo == OR_METROPOLIS)
    or_tables_metropolis(beta, T);
  else
    or_tables_heatbath(beta, T);
}

typedef struct {
  const or_spec *sp;
  const double *betas;
  const int8_t *J;
  uint8_t *spins;
  or_wheel *wheels;
  const int32_t *temp_of_slot;
  int64_t *E, *M;
  uint64_t nsw;
  int64_t c_begin, c_end;
  int32_t err;
} worker_arg;

#include <pthread.h>

static void *sweep_worker(void *p) {
  worker_arg *a = (worker_arg *)p;
  const or_spec *sp = a->sp;
  int64_t N = sites_of(sp);
  int32_t NW = wheels_of(sp);
  int64_t RK = (int64_t)sp->n_replicas * sp->n_temps;
  for (int64_t c = a->c_begin; c < a->c_end; c++) {
    const int8_t *Jc = a->J + (c / RK) * coupling_rows(sp) * N;
    uint8_t *sc = a->spins + c * N;
    const double beta = a->betas[a->temp_of_slot[c]];
    uint64_t T[13];
    copy_tables(sp, beta, T);
    for (uint64_t t = 0; t < a->nsw; t++) {
      if (is_4d(sp))
        copy_sweep_4d(sp, sc, (const uint8_t *)Jc, a->wheels + c * NW, T, &a->E[c]);
      else
        copy_sweep(sp, sc, Jc, a->wheels + c * NW, T, beta, &a->E[c], &a->M[c]);
      if (sp->check_energy &&
          (a->E[c] != copy_energy(sp, sc, Jc) || a->M[c] != copy_field_sum(sp, sc, Jc))) {
        a->err = OR_ENERGY_MISMATCH;
        return NULL;
      }
    }
  }
  return NULL;
}

static int32_t sweep_all(const or_spec *sp, const double *betas, const int8_t *J, uint8_t *spins,
                         or_wheel *wheels, const int32_t *temp_of_slot, int64_t *E, int64_t *M,
                         uint64_t nsw) {
  int64_t C = (int64_t)sp->n_samples * sp->n_replicas * sp->n_temps;
  int nt = sp->n_threads > 0 ? sp->n_threads : 1;
  if (nt > C) nt = (int)C;
  worker_arg args[256];
  pthread_t th[256];
  if (nt > 256) nt = 256;
  for (int t = 0; t < nt; t++) {
    args[t] = (worker_arg){sp, betas, J, spins, wheels, temp_of_slot, E, M, nsw,
                           C * t / nt, C * (t + 1) / nt, 0};
  }
  for (int t = 1; t < nt; t++) pthread_create(&th[t], NULL, sweep_worker, &args[t]);
  sweep_worker(&args[0]);
  for (int t = 1; t < nt; t++) pthread_join(th[t], NULL);
  for (int t = 0; t < nt; t++)
    if (args[t].err) return args[t].err;
  return OR_OK;
}

/* Parallel tempering (only named in sec. 2.2).  Reading used here: for
 * every (sample, replica) chain, pairs of neighbouring temperatures
 * i = 0..K-2 in ascending order; slots keep their configuration and wheels
 * and exchange temperatures; the swap is accepted with probability
 * min(1, exp((beta_i - beta_{i+1}) (E_a - E_b))) evaluated as an integer
 * threshold; one number of the chain's own wheel per pair, always drawn. */
static void pt_step(const or_spec *sp, const double *betas, or_wheel *ptw, int32_t *sot,
                    const int64_t *E, uint64_t *acc) {
  int32_t K = sp->n_temps;
  int64_t chains = (int64_t)sp->n_samples * sp->n_replicas;
  for (int64_t ch = 0; ch < chains; ch++) {
    int32_t *so = sot + ch * K;
    for (int i = 0; i + 1 < K; i++) {
      int64_t a = ch * K + so[i], b = ch * K + so[i + 1];
      int64_t D = E[b] - E[a];
      double dbeta = betas[i] - betas[i + 1];
      uint32_t r = or_wheel_next(&ptw[ch]);
      int accept;
      if (dbeta * (double)D <= 0.0) {
        accept = 1;
      } else {
        uint64_t F[24];
        or_tables_pt(betas[i], betas[i + 1], F);
        uint64_t absD = (uint64_t)(D < 0 ? -D : D);
        accept = (uint64_t)r < or_pt_threshold(F, absD);
      }
      if (accept) {
        int32_t t = so[i];
        so[i] = so[i + 1];
        so[i + 1] = t;
        if (acc) acc[ch * (K - 1) + i]++;
      }
    }
  }
}

static void measure(const or_spec *sp, const int8_t *J, const uint8_t *spins, const int32_t *sot,
                    const int64_t *E, int64_t *E_log, int64_t *Q_log) {
  int64_t N = sites_of(sp);
  int32_t S = sp->n_samples, R = sp->n_replicas, K = sp->n_temps;
  if (E_log)
    for (int64_t ch = 0; ch < (int64_t)S * R; ch++)
      for (int k = 0; k < K; k++) E_log[ch * K + k] = E[ch * K + sot[ch * K + k]];
  if (!Q_log || R < 2) return;
  for (int s = 0; s < S; s++)
    for (int k = 0; k < K; k++) {
      int64_t ca = ((int64_t)s * R + 0) * K + sot[((int64_t)s * R + 0) * K + k];
      int64_t cb = ((int64_t)s * R + 1) * K + sot[((int64_t)s * R + 1) * K + k];
      if (sp->model == OR_ISING)
        Q_log[(int64_t)s * K + k] =
            or_ising_overlap(sp->L, (const int8_t *)spins + ca * N, (const int8_t *)spins + cb * N);
      else if (sp->model == OR_ISING_GEN)
        Q_log[(int64_t)s * K + k] = or_isinggen_overlap(sp->L, (const int8_t *)spins + ca * N,
                                                        (const int8_t *)spins + cb * N, J + s * 5 * N);
      else {
        int64_t Q = 0; /* Potts models: number of equal sites */
        for (int64_t i = 0; i < N; i++) Q += spins[ca * N + i] == spins[cb * N + i];
        Q_log[(int64_t)s * K + k] = Q;
      }
    }
}

static int valid_L(int32_t L) { return L == 2 || L == 4 || (L >= 8 && L % 8 == 0); }

int32_t or_run(const or_spec *sp, const double *betas, const int8_t *J, void *spins_v,
               uint32_t *wheels_words, uint32_t *ptwheels_words, int32_t *slot_of_temp,
               uint64_t sweeps_done, uint64_t n_sweeps, int64_t *E_out, int64_t *E_log,
               int64_t *Q_log, uint64_t *pt_accepts, int64_t *M_out) {
  if (!sp || !valid_L(sp->L) || sp->n_samples < 1 || sp->n_replicas < 1 || sp->n_temps < 1)
    return OR_EINVAL;
  if (sp->model < OR_ISING || sp->model > OR_GPOTTS4) return OR_EINVAL;
  if ((sp->model == OR_POTTS || sp->model == OR_GPOTTS || sp->model == OR_GPOTTS4) &&
      sp->algo != OR_HEATBATH)
    return OR_EINVAL;
  if (sp->model == OR_ISING_GEN && (sp->pt_every > 0 || !(sp->field >= 0.0))) return OR_EINVAL;
  uint8_t *spins = (uint8_t *)spins_v;
  int64_t N = sites_of(sp);
  int32_t NW = wheels_of(sp);
  int32_t K = sp->n_temps;
  int64_t chains = (int64_t)sp->n_samples * sp->n_replicas;
  int64_t C = chains * K;

  or_wheel *wheels = (or_wheel *)malloc(sizeof(or_wheel) * C * NW);
  or_wheel *ptw = (or_wheel *)malloc(sizeof(or_wheel) * (chains > 0 ? chains : 1));
  int32_t *tos = (int32_t *)malloc(sizeof(int32_t) * C);
  int64_t *E = (int64_t *)malloc(sizeof(int64_t) * C);
  int64_t *M = (int64_t *)malloc(sizeof(int64_t) * C);
  for (int64_t w = 0; w < C * NW; w++) or_wheel_load(&wheels[w], wheels_words + w * 61);
  if (sp->pt_every > 0)
    for (int64_t ch = 0; ch < chains; ch++) or_wheel_load(&ptw[ch], ptwheels_words + ch * 61);
  for (int64_t c = 0; c < C; c++) {
    const int8_t *Jc = J + (c / K / sp->n_replicas) * coupling_rows(sp) * N;
    E[c] = copy_energy(sp, spins + c * N, Jc);
    M[c] = copy_field_sum(sp, spins + c * N, Jc);
  }

  int32_t rc = OR_OK;
  uint64_t t = 0, n_meas = 0;
  while (t < n_sweeps) {
    uint64_t nsw = n_sweeps - t;
    if (sp->pt_every > 0) {
      uint64_t until = sp->pt_every - (sweeps_done + t) % sp->pt_every;
      if (until < nsw) nsw = until;
    }
    if (sp->measure_every > 0) {
      uint64_t until = sp->measure_every - t % sp->measure_every;
      if (until < nsw) nsw = until;
    }
    for (int64_t ch = 0; ch < chains; ch++)
      for (int k = 0; k < K; k++) tos[ch * K + slot_of_temp[ch * K + k]] = k;
    rc = sweep_all(sp, betas, J, spins, wheels, tos, E, M, nsw);
    if (rc != OR_OK) break;
    t += nsw;
    if (sp->pt_every > 0 && (sweeps_done + t) % sp->pt_every == 0)
      pt_step(sp, betas, ptw, slot_of_temp, E, pt_accepts);
    if (sp->measure_every > 0 && t % sp->measure_every == 0) {
      measure(sp, J, spins, slot_of_temp, E, E_log ? E_log + n_meas * C : NULL,
              Q_log ? Q_log + n_meas * sp->n_samples * K : NULL);
      n_meas++;
    }
  }
  for (int64_t w = 0; w < C * NW; w++) or_wheel_store(&wheels[w], wheels_words + w * 61);
  if (sp->pt_every > 0)
    for (int64_t ch = 0; ch < chains; ch++) or_wheel_store(&ptw[ch], ptwheels_words + ch * 61);
  if (E_out) memcpy(E_out, E, sizeof(int64_t) * C);
  if (M_out) memcpy(M_out, M, sizeof(int64_t) * C);
  free(M);
  free(wheels);
  free(ptw);
  free(tos);
  free(E);
  return rc;
}
