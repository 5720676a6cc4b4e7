// Device data layout of the checkerboard sweep: geometry constants shared by
// the host-side packing code and the gfx950 kernels.  (Internal header; the
// public boundary is include/sg.h.)
//
// Ising copy (bit-packed, 1 bit per spin, bit 1 <-> spin -1; igeom):
//   The sites of one colour of a z-plane, taken row by row (y ascending) and
//   within a row in increasing x, form a string of L * L/2 bits: site
//   (x = 2j + e, y) is string position s = y L/2 + j.  The string is cut
//   into 32-bit block words (B = min(32, L^2/2) sites each), most significant
//   bit first: position s sits in word wb = s / B at bit B - 1 - s mod B.
//   The rho = min(8, L) rows served by one Parisi-Rapuano wheel are the
//   NBLK = rho L / (2 B) consecutive words of its row group, so a block word
//   holds exactly B consecutive draws of the wheel; rows may straddle two
//   words (L = 24, 40, 48, 56).  Words are indexed [colour p][plane z]
//   [block word wb] with the wb stride padded to an odd count WZ (LDS bank
//   spread).  Unused high bits (B < 32) are zero.
// Ising couplings: six words per (colour, wb, z), one per bond direction
//   (x+, x-, y+, y-, z+, z-), same bit order, bit 1 <-> J = -1, laid out
//   [p][wb][d][z] so that the lanes of a wave (consecutive z) read one
//   contiguous segment.
// Potts copy: one byte per site holding 8 * sigma, ordered [y][x][z] (z
//   fastest: the lanes of a wave serve consecutive z planes).
// Potts couplings: one pattern byte per site whose bit d is set when the
//   bond in direction d (x+, x-, y+, y-, z+, z-) has J = -1, stored in the
//   order the wheels consume the sites: word ((p * NBLK + blk) * BQ + q) * NW
//   + wheel holds, in byte b, the pattern of the (4q + b)-th site of block blk
//   of half-sweep p of that wheel (BQ = ceil(B / 4) words per block), so one
//   dword load per lane serves four consecutive draws and a wave's loads are
//   contiguous.
// Wheels: M >= 62 slots per wheel, slot (k mod M) holds I(k); slots are
//   stored [slot][copy * NW + wheel] (coalesced across lanes).
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define SG_HD __host__ __device__
#else
#define SG_HD
#endif

namespace sg {

struct Geom {
  int L, RHO, NG, NW, H, RPB, B, NBLK, NWB, WZ, CS, M, V;
};

SG_HD constexpr Geom geom(int L) {
  Geom g{};
  g.L = L;
  g.RHO = L < 8 ? L : 8;             // rows per wheel
  g.NG = L / g.RHO;                  // row groups per plane
  g.NW = L * g.NG;                   // wheels per copy
  g.H = L / 2;                       // sites of one colour per row
  int r = g.H >= 32 ? 1 : 32 / g.H;  // rows per 32-bit block word
  g.RPB = r < g.RHO ? r : g.RHO;
  g.B = g.RPB * g.H;                 // sites (and draws) per block
  g.NBLK = g.RHO / g.RPB;            // blocks per half-sweep per wheel
  g.NWB = g.L / g.RPB;               // block words per (colour, plane)
  g.WZ = g.NWB | 1;                  // padded stride
  g.CS = 2 * g.L * g.WZ;             // words per Ising copy
  // ring slots: a multiple of B, at least 62, with an even number V of block
  // phases (an even cycle lets the register allocator keep every slot in place)
  g.V = (62 + g.B - 1) / g.B;
  g.V += g.V & 1;
  g.M = g.V * g.B;
  return g;
}

// Geometry of the bit-packed Ising copies (EA glass and the Ising-like
// models): one block word of B = min(32, L^2/2) draws, NBLK = L/8 words per
// row group for L >= 8 (one word per plane below).  RPB is not used.
SG_HD constexpr Geom igeom(int L) {
  Geom g{};
  g.L = L;
  g.RHO = L < 8 ? L : 8;
  g.NG = L / g.RHO;
  g.NW = L * g.NG;
  g.H = L / 2;
  g.RPB = 0;
  g.B = g.RHO * g.H < 32 ? g.RHO * g.H : 32;
  g.NBLK = g.RHO * g.H / g.B;
  g.NWB = g.NG * g.NBLK;
  g.WZ = g.NWB | 1;
  g.CS = 2 * g.L * g.WZ;
  g.V = (62 + g.B - 1) / g.B;
  g.V += g.V & 1;
  g.M = g.V * g.B;
  return g;
}

SG_HD constexpr bool supported_L(int L) {
  return L == 2 || L == 4 || L == 8 || L == 16 || L == 24 || L == 32 || L == 40 || L == 48 ||
         L == 56 || L == 64;
}

SG_HD constexpr bool potts_supported_L(int L) { return supported_L(L) && L <= 48; }

// Words of Ising couplings per sample.
SG_HD constexpr int ising_js(int L) { return 2 * igeom(L).NWB * 6 * L; }

// Potts pattern words per block and per sample.
SG_HD constexpr int potts_bq(int L) { return (geom(L).B + 3) / 4; }
SG_HD constexpr int potts_js(int L) { return 2 * geom(L).NBLK * potts_bq(L) * geom(L).NW; }

// Glassy Potts couplings (permutations of 0..3, Eq. 3 of the paper): one
// word per site, in the draw order of the +-J patterns with one site per
// word: word ((p * NBLK + blk) * B + k) * NW + wheel.  Bits 5d..5d+4 hold the
// number (lexicographic order, 0..23) of the permutation on the bond in
// direction d (x+, x-, y+, y-, z+, z-): for d even the bond stored at the
// site itself, for d odd the bond stored at the neighbour.
SG_HD constexpr int gpotts_js(int L) { return 2 * geom(L).NBLK * geom(L).B * geom(L).NW; }

// 4D glassy Potts model (Eq. 3 on the hypercubic lattice of side L, site
// i = x + L (y + L (z + L u))): one wheel per (z, u, group of rho rows),
// index (g L + u) L + z, drawing for its rows in the 3D order (colour, row,
// x).  Blocks hold at most 8 draws (each site needs two coupling words,
// prefetched a block ahead).
SG_HD constexpr Geom geom4(int L) {
  Geom g{};
  g.L = L;
  g.RHO = L < 8 ? L : 8;
  g.NG = L / g.RHO;
  g.NW = L * L * g.NG;
  g.H = L / 2;
  int r = g.H >= 8 ? 1 : 8 / g.H;
  g.RPB = r < g.RHO ? r : g.RHO;
  g.B = g.RPB * g.H;
  g.NBLK = g.RHO / g.RPB;
  g.NWB = g.L / g.RPB;
  g.WZ = g.NWB | 1;
  g.CS = 0;
  g.V = (62 + g.B - 1) / g.B;
  g.V += g.V & 1;
  g.M = g.V * g.B;
  return g;
}

SG_HD constexpr bool potts4_supported_L(int L) { return L == 2 || L == 4 || L == 8 || L == 16; }

// 4D copy: one byte per site holding 8 sigma, ordered [y][u][x][z] (z
// fastest).  In HBM the u planes are L^2 bytes apart; in LDS each u plane
// is padded to potts4_us(L) bytes, so that the lanes of a wave (consecutive
// z, then u) reading sites of both x parities (L bytes apart) touch a window
// of 2L bytes per u plane and the windows of the wave's u planes fall on
// distinct LDS banks.
SG_HD constexpr int potts4_us(int L) { return L * L + (L == 16 ? 32 : (L == 8 ? 16 : 0)); }
SG_HD constexpr int potts4_lds_copy(int L) { return L * L * potts4_us(L); }
// Couplings: per site two words in draw order, element
// ((p NBLK + blk) B + k) NW + wheel (8 bytes): word 0 holds the permutation
// numbers of directions x+, x-, y+, y-, z+, z- (bits 5d..5d+4, as in 3D),
// word 1 those of u+ (bits 0..4) and u- (bits 5..9).
SG_HD constexpr int gpotts4_js(int L) { return 4 * geom4(L).NBLK * geom4(L).B * geom4(L).NW; }
// Weights W[0..8] are used (h_a in 0..8); 12 words per copy.
constexpr int POTTS4_W_WORDS = 12;

// Potts work items: at most 512 lanes per workgroup (the kernel keeps up to
// 256 VGPRs per lane).  LDS = the 64-entry rotation-base table (6 words per
// coupling pattern at an odd stride of 7 words; the kernels with several
// lanes per wheel index it by the pattern's bits 0..4 only, so the 32
// entries a read can touch lie on 32 distinct banks, and form the sixth
// word from bit 5), then the copies, then per copy 8 weight words and 1
// counter.  In LDS a copy's row y starts at byte y L XS + (y / RHO) 2L (XS =
// potts_xs(L), the x stride; each row group is skewed by 2L bytes) and
// copies are potts_lds_copy(L) bytes apart (0 mod 4).  The lanes of one row
// group (consecutive z, sites x = 2j + e with e alternating in z) touch a
// 2 XS-byte window of a row; with these offsets the windows of the row
// groups and copies of a wave fall on distinct LDS banks.
constexpr int POTTS_MAX_TPB = 512;
// Lanes per wheel of the 3D Potts kernels (the wheel's outputs are formed S
// at a time, lane l taking those with index = l mod S): eight at L = 16
// (8 NW = 256 lanes per copy), four where L/2 is a multiple of 4 and a
// copy's 4 NW lanes fit one workgroup (L = 8, 24, 32), two at L = 40, 48
// (2 NW = 400, 576 lanes), else one.  S divides L/2 and 24.
SG_HD constexpr int potts_wheel_lanes(int L) {
  return L == 16 ? 8 : (L == 8 || L == 24 || L == 32 ? 4 : (L == 40 || L == 48 ? 2 : 1));
}
// Lanes per wheel a 3D Potts job may choose instead (the numbers drawn and
// every result stay the same): four at L = 16, where eight is the default
// (eight lanes fill more SIMDs when the batch is small, four spend fewer
// instructions per update when the device is full).
SG_HD constexpr bool potts_lanes_ok(int L, int S) { return S == potts_wheel_lanes(L) || (L == 16 && S == 4); }
// Workgroups of the two-lanes-per-wheel kernels hold up to 768 threads.
constexpr int POTTS_PAIR_MAX_TPB = 768;
// Launch groups of the several-lanes-per-wheel kernels (+-J and glassy),
// beside the model numbers 0..4 of the other sweep kernels.
constexpr int LAUNCH_POTTS_QUAD = 5, LAUNCH_GPOTTS_QUAD = 6, LAUNCH_POTTS_PAIR = 7,
              LAUNCH_GPOTTS_PAIR = 8;
// Launch group of the EA kernel at L = 2, 4 (a kernel of its own).
constexpr int LAUNCH_ISING_SMALL = 9;
constexpr int POTTS_TAB_STRIDE = 7;
constexpr int POTTS_TAB_WORDS = 64 * POTTS_TAB_STRIDE;
constexpr int POTTS_W_WORDS = 8;
// Byte stride of x in a copy's LDS rows (z fastest, then x, then y).  At
// L = 32 the four lanes of a wheel read sites 2 x-steps apart, 64 bytes with
// an x stride of L: 16 words, so lanes 0 and 2 of every wheel would share a
// bank.  The 64 lanes of a wave (16 wheels of consecutive z, four lanes
// each; even and odd z planes one x-step apart) read 32 distinct words;
// with a stride of 48 bytes they lie on 32 distinct banks.  At L = 16 the
// eight lanes of a wheel read sites 32 bytes apart with a stride of L, and
// lanes 0 and 4 share a bank; with a stride of 24 bytes the 32 words a wave
// reads lie on 32 distinct banks (the reads of the z neighbours, where one
// wheel of the wave wraps around in z, excepted).
SG_HD constexpr int potts_xs(int L) { return L == 32 ? 48 : (L == 16 ? 24 : L); }
SG_HD constexpr int potts_lds_copy(int L) {
  return (L * L * potts_xs(L) + 2 * geom(L).NG * L + 3) / 4 * 4;
}

// Ising-like models of Eq. (2) of the paper (dilution x_i, field h_i =
// |h| f_i): spins as for the EA glass.  Per (colour p, block word wb, plane z)
// 14 words in the site order of the spin words, laid out [p][wb][d][z]:
//   d = 0..5   bit 1 <-> J = -1 on the bond in direction x+, x-, y+, y-, z+, z-
//   d = 6..11  bit 1 <-> the neighbour in that direction is occupied
//   d = 12     bit 1 <-> the site is occupied (x_i = 1)
//   d = 13     bit 1 <-> f_i = -1
// followed, per sample, by the occupancy bits of every site in the spin-copy
// layout (CS words, pads zero) for the overlap.
constexpr int GEN_WORDS = 14;
SG_HD constexpr int gen_block_js(int L) { return 2 * igeom(L).NWB * GEN_WORDS * L; }
SG_HD constexpr int gen_js(int L) { return gen_block_js(L) + igeom(L).CS; }
// LDS threshold table of a copy: 32 words at an odd stride (bank spread).
constexpr int GEN_TAB_STRIDE = 33;

// Ising: LDS threshold table of a copy at a stride of 40 words (8-byte
// aligned; copies sharing a wave start on different banks).  Metropolis:
// thresholds of site pairs, with T[v] for v = n mod 4 of a site's
// unsatisfied-bond count n (T[3] = 0): entry e = 0..15 at words 2 e, 2 e + 1
// holds T[v1], T[v0] for the odd site (v1 = bit 1 of e + 2 * bit 3) and the
// even site (v0 = bit 0 of e + 2 * bit 2) of a pair of consecutive sites;
// heat bath: T_HB[6 - m] at words m = 0..6, then 0.
constexpr int ISING_TAB_STRIDE = 40;

// Per-temperature threshold row: 32 words.  Ising Metropolis uses [0..2],
// heat bath [0..6], Potts [0..12]; a threshold equal to 2^32 is stored as
// 0xFFFFFFFF with bit n of word 15 set ("always").  Ising-like models: word
// k + 16 phi holds the threshold of class (k, phi), k = 0..12, and words 13
// and 29 the limits m_0, m_1 of the classes whose move is certain (Metropolis:
// k < m_phi flips; heat bath: k >= m_phi sets s = +1); those classes' words
// are 0.
constexpr int THR_WORDS = 32;

// One work item of a sweep launch: G complete copies of one job, served by
// G * NW lanes of one workgroup.
struct Work {
  uint32_t *spins;               // job spins (device layout), all copies
  const uint32_t *J;             // job couplings, all samples
  uint32_t *wheels;              // job wheel slots
  const int32_t *temp_of_slot;   // [C]
  const uint32_t *thr;           // [K][THR_WORDS]
  int64_t *E;                    // [C] energy per slot (written at the end)
  int32_t L, algo, model, copy0, ncopies, C, RK;
  int32_t nsweeps_cap;           // the item runs min(launch sweeps, cap) sweeps
  uint32_t spins_bytes, J_bytes, wheels_bytes;  // extents (buffer range checks)
  int32_t wl;                    // lanes per wheel (3D Potts kernels)
  const uint64_t *done;          // sweeps already performed by the job (device)
  int64_t *M;                    // [C] field sum per slot (Ising-like models), else null
};

// Size of the static device scratch of the no-allocation batch run (launch
// tables only: about 112 bytes per work item, 12 per job, 72 per
// parallel-tempering work item of up to PT_CHAINS_PER_ITEM chains), and the
// number of devices whose scratch address the library keeps.
constexpr uint64_t STATIC_SCRATCH_BYTES = 2u << 20;
constexpr int MAX_DEVICES = 64;

// Fused parallel tempering: chains per workgroup, and the largest number of
// temperatures it serves (more take the unfused kernel).
constexpr int PT_CHAINS_PER_ITEM = 16;
constexpr int PT_FUSED_KMAX = 64;

// Parallel-tempering work of one workgroup: up to PT_CHAINS_PER_ITEM chains of one job.
struct PtWork {
  const int64_t *E;          // [C] energy per slot
  int32_t *slot_of_temp;     // [chains][K]
  int32_t *temp_of_slot;     // [C]
  uint32_t *ptw;             // [chains][64]: 61 ring words + position
  const uint64_t *F;         // [K-1][24]
  const int32_t *sgn;        // [K-1]
  uint64_t *accepts;         // [chains][K-1]
  int32_t chain0, nchains, K, pad;
};

}  // namespace sg
