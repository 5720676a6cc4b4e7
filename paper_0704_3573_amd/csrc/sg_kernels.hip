// gfx950 kernels of the checkerboard spin-glass sweep.
//
// Paper: Belletti et al., "Simulating spin systems on IANUS, an FPGA-based
// computer".  Update rules of sec. 2.2 (Metropolis; heat bath, Eq. 4), the
// checkerboard schedule of sec. 3.1, the Parisi-Rapuano generator of sec. 3.3
// (Eq. 5).  Integer thresholds are computed on the host; no kernel evaluates
// an exponential.
//
// Mapping (one workgroup = G complete copies of one job):
//  * one lane per Parisi-Rapuano wheel; its live words sit in VGPRs as a ring
//    of M slots (slot k mod M holds I(k)); a block of B consecutive draws is
//    compiled for one of V = M / B ring phases, so every register index is
//    static (the paper's "wheel in logic, not memory", sec. 3.3);
//  * the B sites served by those draws are one 32-bit word of the bit-packed
//    lattice; the six-neighbour bond count is computed bit-sliced on whole
//    words (32 sites per operation) from LDS-resident neighbour words, and
//    the thresholds are read from the copy's small LDS table indexed by the
//    counts (the LUT of the paper's update cell; Metropolis reads the two
//    sites of a pair at once);
//  * each draw is compared with its site's threshold and the compare result
//    (a 64-lane mask) is shifted into a per-lane accumulator word with
//    add-with-carry, so the per-site work is draw + compare + insert + the
//    table address (half of one for Metropolis);
//  * the 3D Potts kernels share each wheel between four or two lanes (the
//    multi-output wheel of sec. 3.3, see PottsMK);
//  * the copies' spins stay in LDS for the whole launch; a workgroup barrier
//    separates the two colours (sec. 3.1: same-colour sites never interact).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_layout.h"
#include <mutex>
#include <type_traits>

#define DEV __device__ __forceinline__

namespace sg {

// Global memory goes through buffer resources: an SGPR descriptor plus a
// 32-bit per-lane byte offset; accesses outside the extent read 0 and are
// dropped on store.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
DEV rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
DEV uint32_t bload(rsrc_t r, uint32_t voff, uint32_t soff = 0) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}
DEV void bstore(rsrc_t r, uint32_t v, uint32_t voff, uint32_t soff = 0) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, soff, 0);
}

// Staging of n words from HBM into LDS by the whole workgroup with U loads
// in flight per thread (one wait per U words rather than one HBM round trip
// per word): load(i) reads word i (i < n), put(i, v) stores it.
template <int U, class Load, class Put>
DEV void stage_words(int n, Load load, Put put) {
  const int t = threadIdx.x, nthr = blockDim.x;
  for (int i0 = t; i0 < n; i0 += U * nthr) {
    uint32_t v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int i = i0 + u * nthr;
      v[u] = i < n ? load(i) : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int i = i0 + u * nthr;
      if (i < n) put(i, v[u]);
    }
  }
}

// Staging in two phases, for a workgroup of NT threads: load_words issues
// all U loads of a thread (word i = t + NT u of n, 1 <= n <= NT U; an index
// past the end re-reads the last word, so every load is valid and none is
// behind a branch), put_words stores the words that exist.  Loads of several
// arrays issued before any put wait for global memory together.
template <int NT, int U, class Load>
DEV void load_words(int n, Load load, uint32_t (&v)[U]) {
#pragma unroll
  for (int u = 0; u < U; u++) v[u] = load(min((int)threadIdx.x + NT * u, n - 1));
}
template <int NT, int U, class Put>
DEV void put_words(int n, const uint32_t (&v)[U], Put put) {
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int i = (int)threadIdx.x + NT * u;
    if (i < n) put(i, v[u]);
  }
}

// Compile-time geometry of the Potts kernels (row-aligned blocks of draws).
template <int L>
struct GC {
  static constexpr Geom g = geom(L);
  static constexpr int RHO = g.RHO, NG = g.NG, NW = g.NW, H = g.H, RPB = g.RPB, B = g.B,
                       NBLK = g.NBLK, NWB = g.NWB, WZ = g.WZ, CS = g.CS, M = g.M, V = g.V;
};

// Compile-time geometry of the bit-packed Ising copies (plane strings cut
// into B-bit block words, see sg_layout.h) and, per block word of a row
// group, the bits of the sites that end a row (in-row index L/2 - 1), start
// a row (index 0) and lie in an odd row (a row group starts at an even row,
// so these depend on the block's index within its group only).
template <int L>
struct IC {
  static constexpr Geom g = igeom(L);
  static constexpr int RHO = g.RHO, NG = g.NG, NW = g.NW, H = g.H, B = g.B, NBLK = g.NBLK,
                       NWB = g.NWB, WZ = g.WZ, CS = g.CS, M = g.M, V = g.V;
  static constexpr uint32_t MB = B == 32 ? 0xFFFFFFFFu : ((1u << B) - 1u);
  struct Masks {
    uint32_t ends[8], starts[8], odd[8];
  };
  static constexpr Masks masks() {
    Masks m{};
    for (int b = 0; b < NBLK; b++)
      for (int t = 0; t < B; t++) {
        const int s = b * B + t;
        const uint32_t bit = 1u << (B - 1 - t);
        if (s % H == H - 1) m.ends[b] |= bit;
        if (s % H == 0) m.starts[b] |= bit;
        if ((s / H) & 1) m.odd[b] |= bit;
      }
    return m;
  }
  static constexpr Masks MK = masks();
  static constexpr uint32_t mask(int kind, int b) {
    return b >= NBLK ? 0u : kind == 0 ? MK.ends[b] : kind == 1 ? MK.starts[b] : MK.odd[b];
  }
  static_assert(NBLK <= 8, "row groups hold at most 8 block words");
};

DEV uint32_t bfi(uint32_t m, uint32_t a, uint32_t b) { return (m & a) | (~m & b); }

// A compile-time mask in an SGPR, written next to its use (gfx9 VOP3
// instructions take no 32-bit literal; left to itself the compiler hoists
// every distinct mask of an unrolled loop into its own SGPR).
template <uint32_t V>
DEV uint32_t smask() {
  if constexpr (V == 0u || V == 0xFFFFFFFFu) {
    return V;
  } else {
    uint32_t r;
    asm volatile("s_mov_b32 %0, %1" : "=s"(r) : "i"(V));
    return r;
  }
}

// Row-end (kind 0), row-start (1) or odd-row (2) mask of block blk of an
// Ising row group; blk is a constant after unrolling, so the switch folds.
template <int L, int KIND>
DEV uint32_t imask(int blk) {
  using G = IC<L>;
  switch (blk) {
    case 0: return smask<G::mask(KIND, 0)>();
    case 1: return smask<G::mask(KIND, 1)>();
    case 2: return smask<G::mask(KIND, 2)>();
    case 3: return smask<G::mask(KIND, 3)>();
    case 4: return smask<G::mask(KIND, 4)>();
    case 5: return smask<G::mask(KIND, 5)>();
    case 6: return smask<G::mask(KIND, 6)>();
    default: return smask<G::mask(KIND, 7)>();
  }
}

// Shifts of a plane string cut into B-bit words (first position at bit
// B - 1), seen from word c with its successor n and predecessor q: bit of
// position s of the result holds position s + k (str_next) or s - k
// (str_prev), 0 <= k <= B.  Bits above B of the result are don't-care; the
// inputs have them zero.
template <int B>
DEV uint32_t str_next(uint32_t c, uint32_t n, int k) {
  if (k == 0) return c;
  if (k == B) return n;
  return (c << k) | (n >> (B - k));
}
template <int B>
DEV uint32_t str_prev(uint32_t c, uint32_t q, int k) {
  if (k == 0) return c;
  if (k == B) return q;
  return (c >> k) | (q << (B - k));
}

// Full adder on bit-sliced words: sum and majority carry.
DEV void fadd(uint32_t a, uint32_t b, uint32_t c, uint32_t &s, uint32_t &cy) {
  uint32_t t = a ^ b;
  s = t ^ c;
  cy = bfi(t, c, a);
}

// Bit-sliced count of six one-bit inputs: n = n0 + 2 n1 + 4 n2.
DEV void count6(const uint32_t u[6], uint32_t &n0, uint32_t &n1, uint32_t &n2) {
  uint32_t s1, c1, s2, c2;
  fadd(u[0], u[1], u[2], s1, c1);
  fadd(u[3], u[4], u[5], s2, c2);
  n0 = s1 ^ s2;
  uint32_t c3 = s1 & s2;
  fadd(c1, c2, c3, n1, n2);
}

// Word pointer into LDS: 32-bit address arithmetic (a generic pointer into a
// shared array costs 64-bit multiply-adds per access).
typedef __attribute__((address_space(3))) uint32_t lds_w32;
DEV lds_w32 *to_lds(uint32_t *p) { return (lds_w32 *)p; }

// Per-lane context of the Ising sweep.
struct IsingLane {
  lds_w32 *sp;         // LDS base of the lane's copy (lanes without a wheel: a
                       // scratch copy they may read and overwrite)
  lds_w32 *zb, *zpb, *zmb;  // first block word of the lane's row group in
                            // planes z, z + 1, z - 1 (colour 0)
  int nwrap, pwrap;    // word offsets from the group's last (first) block to
                       // the plane's next (previous) one, across the wrap
  rsrc_t rJ;           // couplings of the job
  uint32_t joff;       // byte offset of (sample, z) in the couplings
  int z, zp, zm, g;
  uint32_t zodd;       // all ones when z is odd
  uint32_t A;          // bits of the thresholds equal to 2^32 ("always")
};

// The six other-colour neighbour words of block blk of the lane's row group
// in colour p, and its own word.  With the other colour's plane string Q,
// the y neighbours of position s are Q[s + L/2] and Q[s - L/2]; in a row of
// parity e = (p + y + z) & 1, site j (x = 2j + e) has x+1 at index j + e and
// x-1 at index j + e - 1, periodic within the row: Q[s + 1] or, at a row's
// last site, Q[s + 1 - L/2]; Q[s - 1] or, at its first site, Q[s - 1 + L/2].
template <int L>
DEV void ising_neighbours(const IsingLane &ln, int p, int blk, uint32_t &S, uint32_t N[6],
                          lds_w32 *&own) {
  using G = IC<L>;
  if constexpr (G::NBLK == 1) blk = 0;
  const int q = p ^ 1;
  constexpr int PL = L * G::WZ;  // words per colour
  own = ln.zb + p * PL + blk;
  S = *own;
  const lds_w32 *oc = ln.zb + q * PL;
  const uint32_t Wc = oc[blk];
  N[4] = ln.zpb[q * PL + blk];  // z+
  N[5] = ln.zmb[q * PL + blk];  // z-
  uint32_t Wn = Wc, Wp = Wc;
  if constexpr (G::NWB > 1) {
    Wn = blk + 1 < G::NBLK ? oc[blk + 1] : oc[blk + 1 + ln.nwrap];
    Wp = blk > 0 ? oc[blk - 1] : oc[blk - 1 + ln.pwrap];
  }
  constexpr int B = G::B, H = G::H;
  N[2] = str_next<B>(Wc, Wn, H);  // y+
  N[3] = str_prev<B>(Wc, Wp, H);  // y-
  uint32_t rl, rr;                // other-colour index j + 1, j - 1
  if constexpr (H == B) {
    // one row per word: rotations
    rl = (Wc << 1) | (Wc >> (B - 1));
    rr = (Wc >> 1) | (Wc << (B - 1));
  } else {
    rl = bfi(imask<L, 0>(blk), str_prev<B>(Wc, Wp, H - 1), str_next<B>(Wc, Wn, 1));
    rr = bfi(imask<L, 1>(blk), str_next<B>(Wc, Wn, H - 1), str_prev<B>(Wc, Wp, 1));
  }
  // sites of rows with e = 1: odd rows when p + z is even, even rows otherwise
  const uint32_t em = imask<L, 2>(blk) ^ (p ? ~ln.zodd : ln.zodd);
  N[0] = bfi(em, rl, Wc);
  N[1] = bfi(em, Wc, rr);
}

template <int L>
DEV void ising_couplings(const IsingLane &ln, int p, int blk, uint32_t Jw[6]) {
  using G = IC<L>;
  // per-lane part (sample, row group, plane) in the VGPR offset, the
  // wave-uniform part (colour, block) in the SGPR offset, the direction in
  // the instruction's immediate offset
  const uint32_t voff = ln.joff + (uint32_t)(ln.g * G::NBLK * 6 * L) * 4u;
  const uint32_t soff =
      __builtin_amdgcn_readfirstlane((uint32_t)((p * G::NWB + blk) * 6 * L) * 4u);
#pragma unroll
  for (int d = 0; d < 6; d++) Jw[d] = bload(ln.rJ, voff + d * L * 4, soff);
}

// Per-draw ALU steps in inline assembly.  Each draw computes
// I(k) = I(k-24) + I(k-55) and r = I(k) xor I(k-61) (Eq. 5) and compares r
// with the site's threshold (a 64-lane mask in an SGPR pair); a second stage
// shifts the compare result into a per-lane accumulator word by
// add-with-carry (acc = 2 acc + c).
//
// On gfx94x / gfx950 a VALU instruction that reads an SGPR written by another
// VALU instruction (here: a compare mask used as carry-in) must issue at
// least two instructions after it.  The draws of a block are therefore
// issued as a software pipeline (volatile asm statements keep their order):
// stage 1 of draw 0, then for each draw i: stage 1 of draw i + 1, insert of
// draw i, so every mask is read at least two instructions after it was
// written; the block's last insert follows an explicit wait.
// r is a read-write operand so that one register holds it through the whole
// draw loop: left dead after the compare, its register would be handed to
// the next table address add, and an SDWA write to a register written by the
// previous instructions costs a wait state.
DEV void met_s1(uint32_t &inew, uint32_t a24, uint32_t a55, uint32_t a61, uint32_t T,
                uint32_t &r, uint64_t &m) {
  asm volatile("v_add_u32 %[n], %[a], %[b]\n\t"
               "v_xor_b32 %[r], %[n], %[c]\n\t"
               "v_cmp_lt_u32 %[m], %[r], %[T]"
               : [n] "=&v"(inew), [r] "+&v"(r), [m] "=&s"(m)
               : [a] "v"(a24), [b] "v"(a55), [c] "v"(a61), [T] "v"(T));
}

// (a & m) | c with the mask in a scalar register (one instruction).
DEV uint32_t and_or(uint32_t a, uint32_t m, uint32_t c) {
  uint32_t r;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(m), "v"(c));
  return r;
}

// x shifted right by s (left by -s); s is a compile-time constant.
DEV uint32_t shr(uint32_t x, int s) { return s >= 0 ? x >> s : x << -s; }

// Bit planes a, b interleaved by bit pairs: word 0 holds a[2i] at bit 2i and
// b[2i] at bit 2i + 1, word 1 holds a[2i + 1] at bit 2i and b[2i + 1] at
// bit 2i + 1.  Bit w + 8 j of a and b then sit at bits 8 j + 2 (w / 2) and
// 8 j + 2 (w / 2) + 1 of word w & 1: one shift and one mask move the pair of
// every site of a byte column into place (byte transposes below).
DEV void pair_planes(uint32_t a, uint32_t b, uint32_t &z0, uint32_t &z1) {
  z0 = bfi(0x55555555u, a, b << 1);
  z1 = bfi(0x55555555u, a >> 1, b);
}

// base + byte n of x (one instruction; n is a compile-time constant).
DEV uint32_t add_byte(int n, uint32_t base, uint32_t x) {
  uint32_t r;
  switch (n) {
    case 0:
      asm volatile("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
          : "=v"(r) : "v"(base), "v"(x));
      break;
    case 1:
      asm volatile("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
          : "=v"(r) : "v"(base), "v"(x));
      break;
    case 2:
      asm volatile("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
          : "=v"(r) : "v"(base), "v"(x));
      break;
    default:
      asm volatile("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
          : "=v"(r) : "v"(base), "v"(x));
      break;
  }
  return r;
}

// LDS words addressed by 32-bit byte offsets.
typedef __attribute__((address_space(3))) const uint32_t lds_u32;
DEV uint32_t lds_offset(const uint32_t *p) { return (uint32_t)(uintptr_t)(lds_u32 *)p; }

// Compile-time loop: f(std::integral_constant<int, I>) for I in [A, B).
template <int A, int B, class F>
DEV void static_for(F &&f) {
  if constexpr (A < B) {
    f(std::integral_constant<int, A>{});
    static_for<A + 1, B>(f);
  }
}

// Wait until at most N vector-memory operations are outstanding (lgkmcnt
// and expcnt left at their maxima).
template <int N>
DEV void vm_wait() {
  static_assert(N >= 0 && N <= 63, "vmcnt is a 6-bit field");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

// Wait until at most N LDS/scalar-memory operations are outstanding (gfx9
// s_waitcnt encoding: vmcnt and expcnt left at their maxima).
template <int N>
DEV void lgkm_wait() {
  static_assert(N >= 0 && N <= 15, "lgkmcnt is a 4-bit field");
  __builtin_amdgcn_s_waitcnt(0xC07F | (N << 8));
}

// Table reads run PF draws ahead of their compares.  Before the compare of
// draw J, every G draws (J = 1, G + 1, 2 G + 1, ...), one LDS wait covers the
// reads of draws J .. J + G - 1; the reads issued after them (up to draw
// J + PF - 2) stay in flight.  The compiler still adds a wait of its own
// wherever one of these is not enough, so the counts only save issue slots.
// Measured: the EA kernels are fastest with G = 2 (with G = 4 the compares
// wait on reads issued only five draws earlier), the Ising-like kernel,
// with more VALU work per block, with G = 4.
template <int G, int PF, int B, int J>
DEV void group_wait() {
  if constexpr ((J - 1) % G == 0) {
    constexpr int last = J + PF - 2 < B - 1 ? J + PF - 2 : B - 1;
    constexpr int need = J + G - 1 < B - 1 ? J + G - 1 : B - 1;
    lgkm_wait<(last - need > 0 ? last - need : 0)>();
  }
}

// Single compare-result insert: acc = 2 acc + c (first: acc = c).  The
// carry-out goes to an SGPR pair co that the draw loop holds for it alone
// (not VCC, and never a compare mask's register): the compiler pads a wait
// state after an SGPR write when the next statement is inline assembly
// that writes or reads the same register, or an SDWA instruction.
DEV void ins1(bool first, uint64_t m, uint32_t &acc, uint64_t &co) {
  if (first)
    asm volatile("v_addc_co_u32 %[a], %[co], 0, 0, %[m]" : [a] "=&v"(acc), [co] "+&s"(co) : [m] "s"(m));
  else
    asm volatile("v_addc_co_u32 %[a], %[co], %[a], %[a], %[m]"
                 : [a] "+v"(acc), [co] "+&s"(co)
                 : [m] "s"(m));
}

// Number of unsatisfied bonds touching the lane's colour-0 sites (every bond
// has exactly one colour-0 end, so the per-copy sum is U and E = 2U - 3N).
template <int L>
DEV int ising_lane_unsat(const IsingLane &ln) {
  using G = IC<L>;
  int U = 0;
#pragma unroll
  for (int blk = 0; blk < G::NBLK; blk++) {
    uint32_t S, N[6], Jw[6], u[6];
    lds_w32 *own;
    ising_neighbours<L>(ln, 0, blk, S, N, own);
    ising_couplings<L>(ln, 0, blk, Jw);
#pragma unroll
    for (int d = 0; d < 6; d++) u[d] = S ^ N[d] ^ Jw[d];
    uint32_t n0, n1, n2;
    count6(u, n0, n1, n2);
    U += __popc(n0 & G::MB) + 2 * __popc(n1 & G::MB) + 4 * __popc(n2 & G::MB);
  }
  return U;
}

// Ring residency.  Register slot r holds draw j = k0 + r (mod M); its memory
// slot is j mod M = (r + k0) mod M.  The launch always starts at register
// phase 0, so only the 61 live words I(k0-61) .. I(k0-1) (registers
// M-61 .. M-1) are loaded, and after the block of phase VI only the 61 words
// written last are stored back.
template <int M>
DEV void ring_load(uint32_t (&ring)[M], rsrc_t r, uint32_t voff, uint32_t stride, int kmod) {
#pragma unroll
  for (int i = M - 61; i < M; i++) {
    const uint32_t slot = __builtin_amdgcn_readfirstlane((uint32_t)((i + kmod) % M));
    ring[i] = bload(r, voff, slot * stride);
  }
}

template <int M, int LAST>
DEV void ring_store(const uint32_t (&ring)[M], rsrc_t r, uint32_t voff, uint32_t stride, int kmod) {
#pragma unroll
  for (int n = 0; n < 61; n++) {
    const int i = (LAST - n + M) % M;  // static
    const uint32_t slot = __builtin_amdgcn_readfirstlane((uint32_t)((i + kmod) % M));
    bstore(r, ring[i], voff, slot * stride);
  }
}

// Sweep driver shared by the kernels: the launch's blocks cycle through the V
// ring phases in order; a workgroup barrier closes every half-sweep.
struct Drive {
  int p, blk, s, nsweeps;
  bool active;
  rsrc_t rwh;
  uint32_t widx, wstride;
  int kmod;
};

// Kernels whose wheels are served by several lanes (K::QUAD) load and store
// their register rings themselves; the others use ring_load / ring_store.
template <class K, class = void>
struct is_quad : std::false_type {};
template <class K>
struct is_quad<K, std::void_t<decltype(K::QUAD)>> : std::bool_constant<K::QUAD> {};

template <class K>
DEV void ring_in(const K &k, uint32_t (&ring)[K::M], const Drive &d) {
  if constexpr (is_quad<K>::value)
    k.load_ring(ring, d);
  else
    ring_load<K::M>(ring, d.rwh, d.widx, d.wstride, d.kmod);
}

template <class K, int LAST>
DEV void ring_out(const K &k, const uint32_t (&ring)[K::M], const Drive &d) {
  if constexpr (is_quad<K>::value)
    k.template store_ring<LAST>(ring, d);
  else
    ring_store<K::M, LAST>(ring, d.rwh, d.widx, d.wstride, d.kmod);
}

template <class K, int VI>
DEV bool drive_chain(K &k, uint32_t (&ring)[K::M], Drive &d) {
  // every lane of a wave that holds at least one wheel runs the block (lanes
  // without a wheel compute on scratch data they alone write), so the ring
  // registers never flow around a divergent branch
  k.template block<VI>(ring, d.p, d.blk);
  if (++d.blk == K::NBLK) {
    d.blk = 0;
    __syncthreads();
    d.p ^= 1;
    if (d.p == 0 && ++d.s == d.nsweeps) {
      if (d.active) ring_out<K, (VI + 1) * K::B - 1>(k, ring, d);
      return true;
    }
  }
  if constexpr (VI + 1 < K::V)
    return drive_chain<K, VI + 1>(k, ring, d);
  else
    return false;
}

// When V divides NBLK every half-sweep starts at ring phase 0: the NBLK
// blocks of a half-sweep are unrolled (block b at phase b mod V, every block
// index a compile-time constant) and the launch has a single exit.
template <class K, int BLK>
DEV void drive_half(K &k, uint32_t (&ring)[K::M], int p) {
  k.template block<BLK % K::V>(ring, p, BLK);
  if constexpr (BLK + 1 < K::NBLK) drive_half<K, BLK + 1>(k, ring, p);
}

// When V divides 2 NBLK but not NBLK every sweep starts at ring phase 0:
// the 2 NBLK blocks of a sweep are unrolled (colour, block index and phase
// compile-time constants).
template <class K, int I>
DEV void drive_sweep(K &k, uint32_t (&ring)[K::M]) {
  k.template block<I % K::V>(ring, I / K::NBLK, I % K::NBLK);
  if constexpr (I % K::NBLK == K::NBLK - 1) __syncthreads();
  if constexpr (I + 1 < 2 * K::NBLK) drive_sweep<K, I + 1>(k, ring);
}

template <class K>
DEV void drive(K &k, Drive &d) {
  if (d.nsweeps <= 0) return;
  if (!__any(d.active)) {
    // a wave without wheels only keeps the workgroup barriers in step
    for (int i = 0; i < 2 * d.nsweeps; i++) __syncthreads();
    return;
  }
  uint32_t ring[K::M];
  if (d.active) ring_in(k, ring, d);
  // wait for the ring once here: with loads still in flight on entry, the
  // sweep loop would carry a vector-memory wait in front of every draw
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  if constexpr (K::NBLK % K::V == 0) {
    for (int s = 0; s < d.nsweeps; s++)
      for (int p = 0; p < 2; p++) {
        drive_half<K, 0>(k, ring, p);
        __syncthreads();
      }
    if (d.active) ring_out<K, K::M - 1>(k, ring, d);
  } else if constexpr ((2 * K::NBLK) % K::V == 0) {
    for (int s = 0; s < d.nsweeps; s++) drive_sweep<K, 0>(k, ring);
    if (d.active) ring_out<K, K::M - 1>(k, ring, d);
  } else {
    d.p = 0;
    d.blk = 0;
    d.s = 0;
    while (!drive_chain<K, 0>(k, ring, d)) {
    }
  }
}

// Metropolis with a per-copy threshold table (the LUT of the paper's update
// cell).  The number n of unsatisfied bonds of every site of the block is
// counted bit-sliced before the draws; the two sites of a pair (2 p + 1, 2 p)
// read their thresholds T[n mod 4] together, one 64-bit LDS read of the
// copy's pair table addressed by the four low count bits of the two sites
// (gathered into bytes, one byte-select add per pair), and the flips that
// are certain in advance (n >= 3, dE <= 0; or n >= m when the thresholds from
// m on equal 2^32, beta ~ 0) are one bit-sliced compare per block.  Per
// draw: add, xor, compare, insert and half an address add.  The block's
// couplings are loaded one block ahead.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) const u32x2 lds_u64;

template <int L>
struct IsingMetK {
  using G = IC<L>;
  static constexpr int M = G::M, B = G::B, V = G::V, NBLK = G::NBLK;
  IsingLane ln;
  const uint32_t *tab;  // LDS pair table of the lane's copy (8-byte aligned)
  uint32_t mlo, mhi;    // limit m in 0..3 of the certain flips, bits as lane masks
  uint32_t nextJ[6];    // coupling words of the next block

  DEV void fetch(int p, int blk) { ising_couplings<L>(ln, p, blk, nextJ); }

  template <int VI>
  DEV void block(uint32_t (&ring)[M], int p, int blk) {
    uint32_t Jw[6];
#pragma unroll
    for (int d = 0; d < 6; d++) Jw[d] = nextJ[d];
    if (blk + 1 < NBLK)
      fetch(p, blk + 1);
    else
      fetch(p ^ 1, 0);
    uint32_t S, N[6];
    lds_w32 *own;
    ising_neighbours<L>(ln, p, blk, S, N, own);
    uint32_t n0, n1, n2;
    {
      vm_wait<6>();  // this block's couplings; the next block's stay in flight
      uint32_t u[6];
#pragma unroll
      for (int d = 0; d < 6; d++) u[d] = S ^ N[d] ^ Jw[d];
      count6(u, n0, n1, n2);
    }
    // n >= m  <=>  n2 or (n1, n0) >= (mhi, mlo)
    const uint32_t below = bfi(n1 ^ mhi, mhi, ~n0 & mlo);
    const uint32_t cert = n2 | ~below;
    // pair p = 4 j + w (sites 8 j + 2 w + 1 and 8 j + 2 w): its table entry
    // e = n0[s] + 2 n0[s+1] + 4 n1[s] + 8 n1[s+1] (s = 8 j + 2 w) times 8,
    // the byte offset, sits in byte j of Kw[w].  X holds the nibbles of the
    // pairs w = 0 (bits 0..3 of each byte) and w = 2 (bits 4..7), Y those of
    // w = 1 and w = 3.
    uint32_t Kw[4];
    {
      const uint32_t X = bfi(0x33333333u, n0, n1 << 2);
      const uint32_t Y = bfi(0x33333333u, n0 >> 2, n1);
      Kw[0] = (X << 3) & 0x78787878u;
      Kw[1] = (Y << 3) & 0x78787878u;
      Kw[2] = (X >> 1) & 0x78787878u;
      Kw[3] = (Y >> 1) & 0x78787878u;
    }
    const uint32_t tbase = lds_offset(tab);
    constexpr int NP = B / 2;
    // thresholds of pair P in draw order (draws 2 P and 2 P + 1: sites
    // B - 1 - 2 P, odd, in .x and B - 2 - 2 P in .y), read PF pairs ahead
    u32x2 T[NP];
    uint32_t A[NP];
    auto addr = [&](int P) {
      const int pp = NP - 1 - P;
      A[P] = add_byte(pp >> 2, tbase, Kw[pp & 3]);
    };
    auto read = [&](int P) { T[P] = *(lds_u64 *)(uintptr_t)A[P]; };
    constexpr int PF = NP < 4 ? NP : 4;
#pragma unroll
    for (int P = 0; P < PF; P++) {
      addr(P);
      read(P);
    }
    __builtin_amdgcn_sched_barrier(0);

    static_assert(B >= 2 && B % 2 == 0, "the draw pipeline needs pairs of draws");
    uint32_t acc = 0, r = 0;
    uint64_t co = 0;
    uint64_t m[B];
    // per step: add, xor and compare of draw i + 1; the address add (i
    // even) or the read (i odd) of the pair PF - 1 pairs past the one that
    // draw i + 1 belongs to; the insert of draw i (an insert directly after
    // the compare that precedes it would cost a wait state).  The compiler
    // waits for each pair's read before its first compare.
    auto s1 = [&](int i) {
      const int k = VI * B + i;  // static after unrolling
      const uint32_t Ti = (i & 1) ? T[i >> 1].y : T[i >> 1].x;
      met_s1(ring[k % M], ring[(k + M - 24) % M], ring[(k + M - 55) % M], ring[(k + M - 61) % M],
             Ti, r, m[i]);
    };
    s1(0);
    static_for<0, B>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if constexpr (i + 1 < B) {
        s1(i + 1);
      } else {
        asm volatile("s_nop 1");
      }
      constexpr int Pn = i / 2 + PF;
      if constexpr (Pn < NP) {
        if constexpr (i % 2 == 0)
          addr(Pn);
        else
          read(Pn);
      }
      ins1(i == 0, m[i], acc, co);
    });
    __builtin_amdgcn_sched_barrier(0);
    *own = S ^ ((cert | acc) & G::MB);
  }
};

// Heat bath with the same table: with m = #{j : J_ij s_j = -1} counted
// bit-sliced (k = 6 - m bonds favour s_i = +1), the new spin is +1 iff
// r < T_HB[6 - m], read from the copy's 8-word LDS table at byte offset 4 m
// (three count planes transposed into bytes); the sites whose threshold is
// 2^32 (s = +1 certain, large local field at large beta) are m < m_lim.
template <int L>
struct IsingHbK {
  using G = IC<L>;
  static constexpr int M = G::M, B = G::B, V = G::V, NBLK = G::NBLK;
  IsingLane ln;
  const uint32_t *tab;      // LDS table of the lane's copy: T_HB[6 - m], m = 0..6, then 0
  uint32_t ml0, ml1, ml2;   // limit m_lim in 0..7 of the certain +1 sites, as lane masks
  uint32_t nextJ[6];        // coupling words of the next block

  DEV void fetch(int p, int blk) { ising_couplings<L>(ln, p, blk, nextJ); }

  template <int VI>
  DEV void block(uint32_t (&ring)[M], int p, int blk) {
    uint32_t Jw[6];
#pragma unroll
    for (int d = 0; d < 6; d++) Jw[d] = nextJ[d];
    if (blk + 1 < NBLK)
      fetch(p, blk + 1);
    else
      fetch(p ^ 1, 0);
    uint32_t S, N[6];
    lds_w32 *own;
    ising_neighbours<L>(ln, p, blk, S, N, own);
    uint32_t n0, n1, n2;
    {
      vm_wait<6>();  // this block's couplings; the next block's stay in flight
      uint32_t u[6];
#pragma unroll
      for (int d = 0; d < 6; d++) u[d] = N[d] ^ Jw[d];  // 1: J s_j = -1
      count6(u, n0, n1, n2);
    }
    // m < m_lim, bit-sliced over three bits
    uint32_t below = ~n0 & ml0;
    below = bfi(n1 ^ ml1, ml1, below);
    below = bfi(n2 ^ ml2, ml2, below);
    // byte j of word w = 4 m of the site at bit w + 8 j
    uint32_t Kw[8], z[2];
    pair_planes(n0, n1, z[0], z[1]);
#pragma unroll
    for (int w = 0; w < 8; w++)
      Kw[w] = and_or(shr(z[w & 1], 2 * (w >> 1) - 2), 0x0C0C0C0Cu, shr(n2, w - 4) & 0x10101010u);
    const uint32_t tbase = lds_offset(tab);
    uint32_t T[B];
    auto load = [&](int i) {
      const int q = B - 1 - i;
      T[i] = *(const lds_u32 *)(uintptr_t)add_byte(q >> 3, tbase, Kw[q & 7]);
    };
    constexpr int PF = B < 8 ? B : 8;
#pragma unroll
    for (int i = 0; i < PF; i++) load(i);
    __builtin_amdgcn_sched_barrier(0);

    static_assert(B >= 2, "the draw pipeline needs two draws per block");
    uint32_t acc = 0, r = 0;
    uint64_t co = 0;
    uint64_t m[B];
    // per step: add, xor and compare of draw i + 1; the address add and
    // read of draw i + PF; the insert of draw i (an insert directly before an
    // SDWA address add would cost a wait state)
    auto s1 = [&](int i) {
      const int k = VI * B + i;  // static after unrolling
      met_s1(ring[k % M], ring[(k + M - 24) % M], ring[(k + M - 55) % M], ring[(k + M - 61) % M],
             T[i], r, m[i]);
    };
    // one LDS wait per two draws (group_wait)
    s1(0);
    static_for<0, B>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if constexpr (i + 1 < B) {
        group_wait<2, PF, B, i + 1>();
        s1(i + 1);
      } else {
        asm volatile("s_nop 1");
      }
      if constexpr (i + PF < B) load(i + PF);
      ins1(i == 0, m[i], acc, co);
    });
    __builtin_amdgcn_sched_barrier(0);
    *own = ~(below | acc) & G::MB;  // bit 1 <-> spin -1
  }
};

template <int L, int ALGO>
struct IsingKernelOf {
  using type = IsingHbK<L>;
};
template <int L>
struct IsingKernelOf<L, 0> {
  using type = IsingMetK<L>;
};

template <int L, int ALGO>
DEV void ising_run(const Work &w, uint32_t *lds) {
  using G = IC<L>;
  const int t = threadIdx.x;
  const int nthr = blockDim.x;
  const int lanes = w.ncopies * G::NW;
  const bool active = t < lanes;
  int *Ucnt = (int *)(lds + w.ncopies * G::CS);
  // CS words; the counters take an even number of words, so the tables that
  // follow the scratch copy are 8-byte aligned (CS is even)
  uint32_t *scratch_copy = lds + w.ncopies * G::CS + ((w.ncopies + 1) & ~1);
  uint32_t *tabs = scratch_copy + G::CS;  // [ncopies][ISING_TAB_STRIDE] thresholds
  const rsrc_t rsp = make_rsrc(w.spins, w.spins_bytes);

  // stage the threshold tables and the copies in LDS
  const uint32_t sbase = (uint32_t)w.copy0 * G::CS * 4u;
  for (int i = t; i < w.ncopies; i += nthr) Ucnt[i] = 0;
  if constexpr (ALGO == 0)  // pair entry e: T[v1], T[v0] at words 2 e, 2 e + 1
    for (int i = t; i < w.ncopies * 32; i += nthr) {
      const int c = i >> 5, e = (i & 31) >> 1;
      const int v = (i & 1) ? (e & 1) | ((e >> 1) & 2) : ((e >> 1) & 1) | ((e >> 2) & 2);
      tabs[c * ISING_TAB_STRIDE + (i & 31)] =
          v < 3 ? w.thr[w.temp_of_slot[w.copy0 + c] * THR_WORDS + v] : 0u;
    }
  else  // heat bath: entry m holds T_HB[6 - m]
    for (int i = t; i < w.ncopies * 8; i += nthr) {
      const int c = i >> 3, e = i & 7;
      tabs[c * ISING_TAB_STRIDE + e] =
          e < 7 ? w.thr[w.temp_of_slot[w.copy0 + c] * THR_WORDS + 6 - e] : 0u;
    }
  stage_words<8>(
      w.ncopies * G::CS, [&](int i) { return bload(rsp, i * 4, sbase); },
      [&](int i, uint32_t v) { lds[i] = v; });

  // lanes without a wheel serve wheel (z = t mod L, row group 0) of the
  // scratch copy, so all their accesses stay inside it
  typename IsingKernelOf<L, ALGO>::type k;
  IsingLane &ln = k.ln;
  const int cl = active ? t / G::NW : 0;
  const int wl = active ? t - cl * G::NW : t % L;
  const int copy = w.copy0 + cl;
  ln.sp = to_lds(active ? lds + cl * G::CS : scratch_copy);
  ln.g = wl / L;
  ln.z = wl - ln.g * L;
  ln.zp = ln.z + 1 == L ? 0 : ln.z + 1;
  ln.zm = ln.z == 0 ? L - 1 : ln.z - 1;
  ln.zodd = (ln.z & 1) ? ~0u : 0u;
  ln.zb = ln.sp + ln.z * G::WZ + ln.g * G::NBLK;
  ln.zpb = ln.sp + ln.zp * G::WZ + ln.g * G::NBLK;
  ln.zmb = ln.sp + ln.zm * G::WZ + ln.g * G::NBLK;
  ln.nwrap = ln.g == G::NG - 1 ? -G::NWB : 0;
  ln.pwrap = ln.g == 0 ? G::NWB : 0;
  ln.rJ = make_rsrc(w.J, w.J_bytes);
  ln.joff = ((uint32_t)(copy / w.RK) * ising_js(L) + ln.z) * 4u;
  ln.A = active ? w.thr[w.temp_of_slot[copy] * THR_WORDS + 15] : 0u;
  if constexpr (ALGO == 0) {
    // certain flips from n = m on: m = 3 (dE <= 0), or the first n whose
    // threshold is 2^32 (thresholds grow with n)
    const int m = ln.A ? min(3, __ffs(ln.A) - 1) : 3;
    k.mlo = (m & 1) ? ~0u : 0u;
    k.mhi = (m & 2) ? ~0u : 0u;
  } else {
    // certain +1 for k >= k0 (first k whose threshold is 2^32; thresholds
    // grow with k), i.e. m = 6 - k < m_lim = 7 - k0
    const int mlim = ln.A ? 7 - (__ffs(ln.A) - 1) : 0;
    k.ml0 = (mlim & 1) ? ~0u : 0u;
    k.ml1 = (mlim & 2) ? ~0u : 0u;
    k.ml2 = (mlim & 4) ? ~0u : 0u;
  }
  k.tab = tabs + cl * ISING_TAB_STRIDE;

  Drive d;
  d.nsweeps = w.nsweeps_cap;
  d.active = active;
  d.rwh = make_rsrc(w.wheels, w.wheels_bytes);
  d.wstride = (uint32_t)w.C * G::NW * 4u;
  d.widx = ((uint32_t)copy * G::NW + wl) * 4u;
  d.kmod = (int)__builtin_amdgcn_readfirstlane((uint32_t)((*w.done * (uint64_t)(G::RHO * L)) % G::M));
  __syncthreads();
  k.fetch(0, 0);
  drive(k, d);

  // energy of every copy, then write back the spins
  if (active) atomicAdd(&Ucnt[cl], ising_lane_unsat<L>(ln));
  __syncthreads();
  if (w.nsweeps_cap > 0)
    for (int i = t; i < w.ncopies * G::CS; i += nthr) bstore(rsp, lds[i], i * 4, sbase);
  const int64_t N3 = (int64_t)L * L * L;
  for (int i = t; i < w.ncopies; i += nthr) w.E[w.copy0 + i] = 2 * (int64_t)Ucnt[i] - 3 * N3;
}

// ---------------------------------------------------------------------------
// Ising-like models of Eq. (2): H = -sum_<ij> J_ij x_i x_j s_i s_j
// - sum_i h_i x_i s_i with h_i = |h| f_i (random-field Ising model, diluted
// antiferromagnet in a field, and mixtures).  Copies, wheels and draw order
// are those of the EA glass; a block's 14 coupling words add the occupancy
// of the six neighbours, the site's own occupancy and its field sign to the
// six J words.
//
// Class of a site: k = n_e + 2 n_g in 0..12, with n_e the number of empty
// neighbours and n_g the number of occupied neighbours whose term is +1
// (Metropolis: J s_i s_j = +1, so k - 6 = s_i sum_j J_ij x_j s_j and a flip
// costs 2 (k - 6) + 2 h s_i f_i; heat bath: J s_j = +1, so the local field
// is k - 6 + h f_i), and a sign bit phi (Metropolis: s_i f_i = -1; heat bath:
// f_i = -1).  k is formed bit-sliced on whole words; each draw is then
// compared with the threshold of its site's class, read from the copy's LDS
// table at word k + 16 phi (the update cell of the paper likewise turns its
// inputs into a small LUT index).  Thresholds are monotone in k, so the
// classes whose move is certain (threshold 2^32) are k < m_phi (Metropolis)
// or k >= m_phi (heat bath): a bit-sliced compare with two per-temperature
// limits, which leaves 32-bit table entries.  Empty sites keep their spin
// and still consume their number.
// ---------------------------------------------------------------------------

// k = a < m for bit-sliced 4-bit a and a per-lane constant m given as four
// all-zero / all-one masks.
DEV uint32_t lt4(const uint32_t a[4], const uint32_t m[4]) {
  uint32_t t = ~a[0] & m[0];
#pragma unroll
  for (int b = 1; b < 4; b++) t = bfi(a[b] ^ m[b], m[b], t);
  return t;
}

// Class planes P[0..3] = k, P[4] = phi of the sites of one block word.
template <bool MET>
DEV void gen_classify(uint32_t S, const uint32_t N[6], const uint32_t Jw[GEN_WORDS],
                      uint32_t P[5]) {
  uint32_t gd[6], ed[6];
#pragma unroll
  for (int d = 0; d < 6; d++) {
    const uint32_t u = MET ? (S ^ N[d] ^ Jw[d]) : (N[d] ^ Jw[d]);  // 1: term -1
    gd[d] = bfi(u, 0u, Jw[6 + d]);                                 // occupied, term +1
    ed[d] = ~Jw[6 + d];                                            // empty
  }
  uint32_t g0, g1, g2, e0, e1, e2, c2;
  count6(gd, g0, g1, g2);
  count6(ed, e0, e1, e2);
  // n_e + 2 n_g <= 12: bit 3 receives at most one carry
  P[0] = e0;
  P[1] = e1 ^ g0;
  fadd(e2, g1, e1 & g0, P[2], c2);
  P[3] = g2 | c2;
  P[4] = MET ? (S ^ Jw[13]) : Jw[13];
}

template <int L, int ALGO>
struct GenK {
  using G = IC<L>;
  static constexpr int M = G::M, B = G::B, V = G::V, NBLK = G::NBLK, NWB = G::NWB;
  IsingLane ln;                // spins, couplings and position of the lane
  const uint32_t *tab;         // LDS threshold table of the lane's copy
  uint32_t m0[4], m1[4];       // limits of the certain classes (lane masks)
  uint32_t nextJ[GEN_WORDS];   // coupling words of the next block

  DEV void load(int p, int blk, uint32_t Jw[GEN_WORDS]) const {
    const uint32_t voff = ln.joff + (uint32_t)(ln.g * NBLK * GEN_WORDS * L) * 4u;
    const uint32_t s0 =
        __builtin_amdgcn_readfirstlane((uint32_t)((p * NWB + blk) * GEN_WORDS * L) * 4u);
#pragma unroll
    for (int d = 0; d < GEN_WORDS; d++) Jw[d] = bload(ln.rJ, voff + d * L * 4, s0);
  }
  DEV void fetch(int p, int blk) { load(p, blk, nextJ); }

  template <int VI>
  DEV void block(uint32_t (&ring)[M], int p, int blk) {
    uint32_t Jw[GEN_WORDS];
#pragma unroll
    for (int d = 0; d < GEN_WORDS; d++) Jw[d] = nextJ[d];
    if (blk + 1 < NBLK)
      fetch(p, blk + 1);
    else
      fetch(p ^ 1, 0);
    uint32_t S, N[6];
    lds_w32 *own;
    ising_neighbours<L>(ln, p, blk, S, N, own);
    uint32_t P[5];
    vm_wait<GEN_WORDS>();  // this block's words; the next block's stay in flight
    gen_classify<ALGO == 0>(S, N, Jw, P);
    const uint32_t lo = lt4(P, m0), hi = lt4(P, m1);
    const uint32_t cert = ALGO == 0 ? bfi(P[4], hi, lo) : ~bfi(P[4], hi, lo);

    // threshold of every site: the five class planes are transposed into
    // bytes, byte j of word w holding 4 (k + 16 phi) of the site at bit
    // q = w + 8 j, so each site's table address is one byte-select add
    uint32_t Kw[8], z01[2], z23[2];
    pair_planes(P[0], P[1], z01[0], z01[1]);
    pair_planes(P[2], P[3], z23[0], z23[1]);
#pragma unroll
    for (int w = 0; w < 8; w++) {
      const int t2 = 2 * (w >> 1);
      Kw[w] = and_or(shr(z01[w & 1], t2 - 2), 0x0C0C0C0Cu,
                     and_or(shr(z23[w & 1], t2 - 4), 0x30303030u, shr(P[4], w - 6) & 0x40404040u));
    }
    const uint32_t tbase = lds_offset(tab);
    uint32_t T[B];
    // threshold of draw i (site at bit B - 1 - i), read PF draws ahead
    auto load = [&](int i) {
      const int q = B - 1 - i;
      T[i] = *(const lds_u32 *)(uintptr_t)add_byte(q >> 3, tbase, Kw[q & 7]);
    };
    constexpr int PF = B < 8 ? B : 8;
#pragma unroll
    for (int i = 0; i < PF; i++) load(i);
    __builtin_amdgcn_sched_barrier(0);

    // draws: r = I(k) xor I(k-61), compare with the site's threshold, shift
    // the result into acc; per step the compare of draw i + 1, the table
    // read of draw i + PF and the insert of draw i, with one LDS wait per
    // four draws (group_wait)
    static_assert(B >= 2, "the draw pipeline needs two draws per block");
    uint32_t acc = 0, r = 0;
    uint64_t co = 0;
    uint64_t m[B];
    auto s1 = [&](int i) {
      const int k = VI * B + i;  // static after unrolling
      met_s1(ring[k % M], ring[(k + M - 24) % M], ring[(k + M - 55) % M], ring[(k + M - 61) % M],
             T[i], r, m[i]);
    };
    s1(0);
    static_for<0, B>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if constexpr (i + 1 < B) {
        group_wait<4, PF, B, i + 1>();
        s1(i + 1);
      } else {
        asm volatile("s_nop 1");
      }
      if constexpr (i + PF < B) load(i + PF);
      ins1(i == 0, m[i], acc, co);
    });
    __builtin_amdgcn_sched_barrier(0);

    const uint32_t X = Jw[12];
    if constexpr (ALGO == 0)
      *own = S ^ (X & (cert | acc));  // X is zero above the block's B bits
    else
      *own = bfi(X, ~(cert | acc), S) & G::MB;
  }

  // bond energy of the lane's colour-0 sites (every bond has one colour-0
  // end: E_b = -sum over them of x_i (k_i - 6)) and field sum of all its sites
  DEV void terms(int &Eb, int &Mf) const {
    Eb = 0;
    Mf = 0;
    for (int p = 0; p < 2; p++)
      for (int blk = 0; blk < NBLK; blk++) {
        uint32_t Jw[GEN_WORDS], S, N[6], P[5];
        lds_w32 *own;
        load(p, blk, Jw);
        ising_neighbours<L>(ln, p, blk, S, N, own);
        const uint32_t X = Jw[12];
        Mf += __popc(X) - 2 * __popc((S ^ Jw[13]) & X);
        if (p == 0) {
          gen_classify<true>(S, N, Jw, P);
          Eb -= __popc(P[0] & X) + 2 * __popc(P[1] & X) + 4 * __popc(P[2] & X) +
                8 * __popc(P[3] & X) - 6 * __popc(X);
        }
      }
  }
};

template <int L, int ALGO>
DEV void gen_run(const Work &w, uint32_t *lds) {
  using G = IC<L>;
  const int t = threadIdx.x;
  const int nthr = blockDim.x;
  const int lanes = w.ncopies * G::NW;
  const bool active = t < lanes;
  uint32_t *tabs = lds + w.ncopies * G::CS;                  // [ncopies][GEN_TAB_STRIDE]
  int *Ecnt = (int *)(tabs + w.ncopies * GEN_TAB_STRIDE);    // [ncopies]
  int *Mcnt = Ecnt + w.ncopies;                              // [ncopies]
  uint32_t *scratch_copy = (uint32_t *)(Mcnt + w.ncopies);   // CS words
  const rsrc_t rsp = make_rsrc(w.spins, w.spins_bytes);

  const uint32_t sbase = (uint32_t)w.copy0 * G::CS * 4u;
  for (int i = t; i < w.ncopies * 32; i += nthr) {
    const int c = i >> 5, e = i & 31;
    tabs[c * GEN_TAB_STRIDE + e] = w.thr[w.temp_of_slot[w.copy0 + c] * THR_WORDS + e];
  }
  for (int i = t; i < 2 * w.ncopies; i += nthr) Ecnt[i] = 0;
  stage_words<8>(
      w.ncopies * G::CS, [&](int i) { return bload(rsp, i * 4, sbase); },
      [&](int i, uint32_t v) { lds[i] = v; });

  // lanes without a wheel serve wheel (z = t mod L, row group 0) of the
  // scratch copy with the first copy's table
  GenK<L, ALGO> k;
  IsingLane &ln = k.ln;
  const int cl = active ? t / G::NW : 0;
  const int wl = active ? t - cl * G::NW : t % L;
  const int copy = w.copy0 + cl;
  ln.sp = to_lds(active ? lds + cl * G::CS : scratch_copy);
  ln.g = wl / L;
  ln.z = wl - ln.g * L;
  ln.zp = ln.z + 1 == L ? 0 : ln.z + 1;
  ln.zm = ln.z == 0 ? L - 1 : ln.z - 1;
  ln.zodd = (ln.z & 1) ? ~0u : 0u;
  ln.zb = ln.sp + ln.z * G::WZ + ln.g * G::NBLK;
  ln.zpb = ln.sp + ln.zp * G::WZ + ln.g * G::NBLK;
  ln.zmb = ln.sp + ln.zm * G::WZ + ln.g * G::NBLK;
  ln.nwrap = ln.g == G::NG - 1 ? -G::NWB : 0;
  ln.pwrap = ln.g == 0 ? G::NWB : 0;
  ln.rJ = make_rsrc(w.J, w.J_bytes);
  ln.joff = ((uint32_t)(copy / w.RK) * gen_js(L) + ln.z) * 4u;
  k.tab = tabs + cl * GEN_TAB_STRIDE;
  uint32_t lim0 = 0, lim1 = 0;
  if (active) {
    const uint32_t *tr = w.thr + w.temp_of_slot[copy] * THR_WORDS;
    lim0 = tr[13];
    lim1 = tr[29];
  }
#pragma unroll
  for (int b = 0; b < 4; b++) {
    k.m0[b] = (lim0 >> b) & 1u ? ~0u : 0u;
    k.m1[b] = (lim1 >> b) & 1u ? ~0u : 0u;
  }

  Drive d;
  d.nsweeps = w.nsweeps_cap;
  d.active = active;
  d.rwh = make_rsrc(w.wheels, w.wheels_bytes);
  d.wstride = (uint32_t)w.C * G::NW * 4u;
  d.widx = ((uint32_t)copy * G::NW + wl) * 4u;
  d.kmod = (int)__builtin_amdgcn_readfirstlane((uint32_t)((*w.done * (uint64_t)(G::RHO * L)) % G::M));
  __syncthreads();
  k.fetch(0, 0);
  drive(k, d);

  if (active) {
    int Eb, Mf;
    k.terms(Eb, Mf);
    atomicAdd(&Ecnt[cl], Eb);
    atomicAdd(&Mcnt[cl], Mf);
  }
  __syncthreads();
  if (w.nsweeps_cap > 0)
    for (int i = t; i < w.ncopies * G::CS; i += nthr) bstore(rsp, lds[i], i * 4, sbase);
  for (int i = t; i < w.ncopies; i += nthr) {
    w.E[w.copy0 + i] = Ecnt[i];
    w.M[w.copy0 + i] = Mcnt[i];
  }
}

// ---------------------------------------------------------------------------
// q = 4 +-J Potts heat bath.  One lane per wheel; each draw updates one site.
//
// Local field bytes.  With n- the number of J = -1 bonds of site i,
//   c_a = 4 (h_a + n-) = 4 (#{J = +1, sigma_j = a} + #{J = -1, sigma_j != a})
// lies in [0, 24] and differs from 4 h_a by a constant, so c_max - c_a is
// 4 (h_max - h_a).  Neighbour j adds rotr32(R, 8 sigma_j) with the rotation
// base R = 4 for J = +1 (a single 4 in byte (4 - sigma_j) & 3) or 0x04040400
// for J = -1 (a 4 in every other byte); byte (4 - a) & 3 of the sum is c_a.
// The six bases of a site come from an LDS table indexed by its coupling
// pattern.  Then w_a = W[h_max - h_a] is read from the lane's weight table
// (entries 4 bytes apart, so c_max - c_a is already the byte offset),
// S = sum w_a, t = (r S) >> 32 and sigma = #{a < 3 : w_0 + ... + w_a <= t},
// which is the sequential search for the first a with t < w_0 + ... + w_a.
//
// Glassy Potts model (Eq. 3, GLASSY = true): neighbour j votes for the state
// a = m_d(sigma_j), m_d = pi for the bond stored at the site (d = x+, y+, z+)
// and pi^-1 for the bond stored at the neighbour (d = x-, y-, z-).  The LDS
// table holds for each of the 24 permutations the words sum_v 8 pi(v) << 8v
// (entries 0..23) and sum_v 8 pi^-1(v) << 8v (entries 24..47); the site's
// coupling word holds the six permutation numbers, and neighbour j adds
// 4 << ((word >> 8 sigma_j) & 31): byte a of the sum is c_a = 4 h_a, in [0, 24].
// The rest (weights, draw, selection) is shared with the +-J glass.
//
// Same-colour sites are never neighbours, so the new spins of a row are kept
// in registers and stored after the row's last draw: every LDS read of the
// row can be scheduled ahead of any of its stores.
// ---------------------------------------------------------------------------
template <int L, bool GLASSY>
struct PottsK {
  using G = GC<L>;
  static_assert(potts_xs(L) == L, "the one-lane kernel uses an x stride of L bytes");
  static constexpr int M = G::M, B = G::B, V = G::V, NBLK = G::NBLK, H = G::H, RPB = G::RPB,
                       RHO = G::RHO, NW = G::NW, BQ = GLASSY ? G::B : potts_bq(L);
  uint8_t *sp;          // LDS bytes of the lane's copy, [y][x][z] (rows at row(y)), 8 sigma
  uint8_t *wp;          // where the lane stores its new spins: sp, or a dummy
                        // region for lanes without a wheel
  const uint32_t *tab;  // LDS table: rotation bases (+-J) or vote words (glassy)
  const uint8_t *Wb;    // LDS weight table of the lane's temperature
  rsrc_t rJ;            // coupling patterns of the job
  uint32_t voff;        // byte offset of the lane's pattern words
  bool active;          // the lane serves a wheel
  int z, zp, zm, g;
  uint32_t nextpat[BQ];  // coupling words of the next block, loaded one block ahead

  // LDS byte offset of row y (row groups skewed by 2L bytes)
  static DEV int row(int y) { return y * L * L + (y / RHO) * 2 * L; }

  DEV void fetch(int p, int blk) {
    const uint32_t s0 =
        __builtin_amdgcn_readfirstlane((uint32_t)((p * NBLK + blk) * BQ) * NW * 4u);
#pragma unroll
    for (int q = 0; q < BQ; q++) nextpat[q] = bload(rJ, voff, s0 + (uint32_t)q * NW * 4u);
  }

  template <int VI>
  DEV void block(uint32_t (&ring)[M], int p, int blk) {
    uint32_t pat[BQ];
#pragma unroll
    for (int q = 0; q < BQ; q++) pat[q] = nextpat[q];
    if (blk + 1 < NBLK)
      fetch(p, blk + 1);
    else
      fetch(p ^ 1, 0);
    rows<VI>(ring, pat, p, g * RHO + blk * RPB, sp, wp, tab, Wb);
  }

  // The block's spins are read through rd (the lane's copy) and written
  // through wr (the same copy, or the dummy region): every site read is of
  // the other colour and every site written of this one, so no byte is
  // accessed through both.  The B sites are software-pipelined in program
  // order: while site n is finished (draw, weights, multiply, select, store),
  // the fields of site n + 1 are formed and its weights requested, and the
  // neighbour bytes and rotation bases of site n + 2 are requested; the
  // scheduling barriers keep that order, so each LDS round trip overlaps the
  // work of other sites.
  template <int VI>
  DEV void rows(uint32_t (&ring)[M], const uint32_t (&pat)[BQ], int p, int y0,
                const uint8_t *__restrict__ rd, uint8_t *__restrict__ wr,
                const uint32_t *__restrict__ tb, const uint8_t *__restrict__ wt) const {
    int base[RPB], bxw[RPB], byp[RPB], bym[RPB];
#pragma unroll
    for (int rr = 0; rr < RPB; rr++) {
      const int y = y0 + rr;
      const int e = (p + y + z) & 1;
      const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
      base[rr] = row(y) + e * L + z;                        // site j = 0 of the row
      bxw[rr] = e ? base[rr] - L : base[rr] + (L - 1) * L;  // periodic x neighbour
      byp[rr] = row(yp) + e * L + z;
      bym[rr] = row(ym) + e * L + z;
    }
    const int dzp = zp - z, dzm = zm - z;
    uint32_t nb[B][6], rb[B][6], w[B][4];

    auto request_site = [&](int kb) {
      const int rr = kb / H, j = kb - rr * H, o = 2 * j * L;
      if constexpr (GLASSY) {
#pragma unroll
        for (int d = 0; d < 6; d++) rb[kb][d] = tb[(d & 1) * 24 + ((pat[kb] >> (5 * d)) & 31u)];
      } else {
        const uint32_t *r6 = tb + POTTS_TAB_STRIDE * ((pat[kb >> 2] >> (8 * (kb & 3))) & 0xFFu);
#pragma unroll
        for (int d = 0; d < 6; d++) rb[kb][d] = r6[d];
      }
      nb[kb][0] = rd[j == H - 1 ? bxw[rr] : base[rr] + o + L];
      nb[kb][1] = rd[j == 0 ? bxw[rr] : base[rr] + o - L];
      nb[kb][2] = rd[byp[rr] + o];
      nb[kb][3] = rd[bym[rr] + o];
      nb[kb][4] = rd[base[rr] + o + dzp];
      nb[kb][5] = rd[base[rr] + o + dzm];
    };
    auto request_weights = [&](int kb) {
      uint32_t c, c0, c1, c2, c3;
      if constexpr (GLASSY) {
        c = 0;
#pragma unroll
        for (int d = 0; d < 6; d++) c += 4u << ((rb[kb][d] >> nb[kb][d]) & 31u);
        c0 = c & 0xFFu, c1 = (c >> 8) & 0xFFu, c2 = (c >> 16) & 0xFFu, c3 = c >> 24;
      } else {
        c = __builtin_rotateright32(rb[kb][0], nb[kb][0]) +
            __builtin_rotateright32(rb[kb][1], nb[kb][1]) +
            __builtin_rotateright32(rb[kb][2], nb[kb][2]) +
            __builtin_rotateright32(rb[kb][3], nb[kb][3]) +
            __builtin_rotateright32(rb[kb][4], nb[kb][4]) +
            __builtin_rotateright32(rb[kb][5], nb[kb][5]);
        c0 = c & 0xFFu, c3 = (c >> 8) & 0xFFu, c2 = (c >> 16) & 0xFFu, c1 = c >> 24;
      }
      const uint8_t *wm = wt + max(max(c0, c3), max(c2, c1));
      w[kb][0] = *(const uint32_t *)(wm - c0);
      w[kb][1] = *(const uint32_t *)(wm - c1);
      w[kb][2] = *(const uint32_t *)(wm - c2);
      w[kb][3] = *(const uint32_t *)(wm - c3);
    };
    auto finish_site = [&](int kb) {
      const int rr = kb / H, j = kb - rr * H;
      const int k = VI * B + kb;  // ring slot (static)
      ring[k % M] = ring[(k + M - 24) % M] + ring[(k + M - 55) % M];
      const uint32_t r = ring[k % M] ^ ring[(k + M - 61) % M];
      const uint32_t C1 = w[kb][0] + w[kb][1], C2 = C1 + w[kb][2];
      const uint32_t t = __umulhi(r, C2 + w[kb][3]);
      // state = #{cumulative weights <= t}: weights are at most 2^28, so t
      // and the sums stay below 2^31 and [C <= t] is bit 31 of C + ~t (no
      // compare masks, whose reads by a select would cost wait states)
      const uint32_t nt = ~t;
      const uint32_t v = (((w[kb][0] + nt) >> 31) + ((C1 + nt) >> 31) + ((C2 + nt) >> 31)) << 3;
      wr[base[rr] + 2 * j * L] = (uint8_t)v;
    };

    request_site(0);
    if constexpr (B > 1) request_site(1);
    __builtin_amdgcn_sched_barrier(0);
    request_weights(0);
#pragma unroll
    for (int kb = 0; kb < B; kb++) {
      __builtin_amdgcn_sched_barrier(0);
      if (kb + 2 < B) request_site(kb + 2);
      __builtin_amdgcn_sched_barrier(0);
      if (kb + 1 < B) request_weights(kb + 1);
      __builtin_amdgcn_sched_barrier(0);
      finish_site(kb);
    }
    __builtin_amdgcn_sched_barrier(0);
  }

  // sum over the lane's colour-0 sites of h_{sigma_i} = sum_j J_ij delta(sigma_i, sigma_j):
  // every bond joins a colour-0 and a colour-1 site, so each is counted once
  DEV int lane_bond_sum() const {
    int hsum = 0;
    for (int blk = 0; blk < NBLK; blk++) {
      const int y0 = g * RHO + blk * RPB;
      for (int kb = 0; kb < B; kb++) {
        const int rr = kb / H, j = kb - rr * H;
        const int y = y0 + rr;
        const int e = (y + z) & 1;
        const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
        const int base = row(y) + e * L + z;
        const int bxw = e ? base - L : base + (L - 1) * L;
        const int o = 2 * j * L;
        const int nb[6] = {j == H - 1 ? bxw : base + o + L, j == 0 ? bxw : base + o - L,
                           row(yp) + e * L + z + o,         row(ym) + e * L + z + o,
                           base - z + zp + o,               base - z + zm + o};
        const uint32_t si = sp[base + o];
        if constexpr (GLASSY) {
          // the bond to neighbour d scores when sigma_i = m_d(sigma_j)
          const uint32_t pw = bload(rJ, voff + (uint32_t)((blk * BQ + kb) * NW) * 4u);
          for (int d = 0; d < 6; d++) {
            const uint32_t vote = tab[(d & 1) * 24 + ((pw >> (5 * d)) & 31u)];
            hsum += ((vote >> sp[nb[d]]) & 31u) == si;
          }
        } else {
          const uint32_t pw = bload(rJ, voff + (uint32_t)((blk * BQ + (kb >> 2)) * NW) * 4u);
          const uint32_t pat = (pw >> (8 * (kb & 3))) & 0xFFu;
          for (int d = 0; d < 6; d++)
            if (sp[nb[d]] == si) hsum += ((pat >> d) & 1u) ? -1 : 1;
        }
      }
    }
    return hsum;
  }
};

// LDS table of the Potts kernels: the vote words of the 24 permutations
// (glassy model) or the rotation bases of the 64 coupling patterns (+-J).
template <bool GLASSY>
DEV void potts_tables(uint32_t *tab) {
  const int t = threadIdx.x, nthr = blockDim.x;
  if constexpr (GLASSY) {
    // vote words of the 24 permutations (lexicographic order): pi, then pi^-1
    for (int i = t; i < 48; i += nthr) {
      const int k = i % 24;
      int avail[4] = {0, 1, 2, 3}, pi[4], inv[4];
      const int digit[3] = {k / 6, (k / 2) % 3, k % 2};
      int left = 4;
      for (int v = 0; v < 4; v++) {
        const int c = v < 3 ? digit[v] : 0;
        pi[v] = avail[c];
        for (int u = c; u + 1 < left; u++) avail[u] = avail[u + 1];
        left--;
      }
      for (int v = 0; v < 4; v++) inv[pi[v]] = v;
      uint32_t word = 0;
      for (int v = 0; v < 4; v++) word |= (uint32_t)(8 * (i < 24 ? pi[v] : inv[v])) << (8 * v);
      tab[i] = word;
    }
  } else {
    for (int i = t; i < POTTS_TAB_WORDS; i += nthr) {
      const int pat = i / POTTS_TAB_STRIDE, d = i - POTTS_TAB_STRIDE * pat;
      tab[i] = d < 6 && ((pat >> d) & 1) ? 0x04040400u : 4u;
    }
  }
}

template <int L, bool GLASSY>
DEV void potts_run(const Work &w, uint32_t *lds) {
  using G = GC<L>;
  constexpr int N3 = L * L * L;
  constexpr int CW = potts_lds_copy(L) / 4;  // LDS words per copy
  constexpr int GW = G::RHO * L * L / 4;     // HBM words per row group
  const int t = threadIdx.x;
  const int nthr = blockDim.x;
  const int lanes = w.ncopies * G::NW;
  const bool active = t < lanes;
  uint32_t *tab = lds;                                  // [64][7] rotation bases
  uint32_t *cp = lds + POTTS_TAB_WORDS;                 // [ncopies][CW] spins
  uint32_t *Wt = cp + w.ncopies * CW;                   // [ncopies][POTTS_W_WORDS]
  int *Hcnt = (int *)(Wt + w.ncopies * POTTS_W_WORDS);  // [ncopies]
  uint8_t *dummy = (uint8_t *)(Hcnt + w.ncopies);       // RHO L^2 bytes if NW % 64 != 0
  const rsrc_t rsp = make_rsrc(w.spins, w.spins_bytes);
  const uint32_t sbase = (uint32_t)w.copy0 * N3;
  potts_tables<GLASSY>(tab);
  for (int i = t; i < w.ncopies * POTTS_W_WORDS; i += nthr) {
    const int c = w.copy0 + i / POTTS_W_WORDS;
    Wt[i] = w.thr[w.temp_of_slot[c] * THR_WORDS + i % POTTS_W_WORDS];
  }
  // word u of a copy in HBM (rows at y L^2) -> LDS word u + (row group) L / 2
  stage_words<8>(
      w.ncopies * (N3 / 4), [&](int i) { return bload(rsp, i * 4, sbase); },
      [&](int i, uint32_t v) {
        const int c = i / (N3 / 4), u = i - c * (N3 / 4);
        cp[c * CW + u + (u / GW) * L / 2] = v;
      });
  for (int i = t; i < w.ncopies; i += nthr) Hcnt[i] = 0;

  // lanes without a wheel run the blocks of wheel (z = t mod L, row group 0)
  // of the first copy and store into the dummy region (the rows of row group
  // 0 span RHO L^2 bytes); distinct z keep their stores on distinct bytes
  PottsK<L, GLASSY> k;
  const int cl = active ? t / G::NW : 0;
  const int wl = active ? t - cl * G::NW : t % L;
  const int copy = w.copy0 + cl;
  k.sp = (uint8_t *)(cp + cl * CW);
  k.wp = active ? k.sp : dummy;
  k.tab = tab;
  k.Wb = (const uint8_t *)(Wt + cl * POTTS_W_WORDS);
  k.active = active;
  k.g = wl / L;
  k.z = wl - k.g * L;
  k.zp = k.z + 1 == L ? 0 : k.z + 1;
  k.zm = k.z == 0 ? L - 1 : k.z - 1;
  k.rJ = make_rsrc(w.J, w.J_bytes);
  k.voff = ((uint32_t)(copy / w.RK) * (GLASSY ? gpotts_js(L) : potts_js(L)) + wl) * 4u;

  Drive d;
  d.nsweeps = w.nsweeps_cap;
  d.active = active;
  d.rwh = make_rsrc(w.wheels, w.wheels_bytes);
  d.wstride = (uint32_t)w.C * G::NW * 4u;
  d.widx = ((uint32_t)copy * G::NW + wl) * 4u;
  d.kmod = (int)__builtin_amdgcn_readfirstlane((uint32_t)((*w.done * (uint64_t)(G::RHO * L)) % G::M));
  __syncthreads();
  k.fetch(0, 0);
  drive(k, d);

  if (active) atomicAdd(&Hcnt[cl], k.lane_bond_sum());
  __syncthreads();
  if (w.nsweeps_cap > 0)
    for (int i = t; i < w.ncopies * (N3 / 4); i += nthr) {
      const int c = i / (N3 / 4), u = i - c * (N3 / 4);
      bstore(rsp, cp[c * CW + u + (u / GW) * L / 2], i * 4, sbase);
    }
  for (int i = t; i < w.ncopies; i += nthr) w.E[w.copy0 + i] = -(int64_t)Hcnt[i];
}

// ---------------------------------------------------------------------------
// q = 4 Potts heat bath (+-J glass and glassy model) with S = 8, 4 or 2
// lanes per wheel.  Sec. 3.3 lets one wheel emit many numbers per clock,
// because the recurrence I(k) = I(k-24) + I(k-55) reaches back at least 24
// outputs: any 24 consecutive outputs can be formed at once.  Here the S
// lanes of a group share a wheel: lane l forms the outputs k = k0 + S s + l
// (step s), so the numbers, their order and every site's number are those of
// the one-lane kernel.  For a lag m = q S + r (0 <= r < S), I(k - m) is the
// output of step s - q of lane l - r if l >= r, else of step s - q - 1 of
// lane l - r + S: each lane exposes the word its reader needs (step s - q - 1
// in lanes l >= S - r, else s - q: one bit-select on lane-constant masks)
// and the reader takes it across lanes (a DPP quad permutation for S <= 4,
// two DPP row rotations and a select for S = 8); lag 24 (r = 0) stays in the
// lane.  Each lane keeps its outputs of the last D steps in registers (D = 8
// for S = 8, 16 for S = 4, 31 for S = 2; a ring of RL >= D words, static
// indices), and within a block of B draws (as in the one-lane kernel) lane l
// updates draws l, l + S, l + 2S, ...  Everything else (fields, weights,
// multiply, selection, the LDS layout and the HBM state) is the one-lane
// kernel's.  potts_wheel_lanes gives S: eight at L = 16, four at L = 8, 24,
// 32, two at L = 40, 48 (more lanes per wheel would not fit one workgroup
// there, or would not divide L/2).
// ---------------------------------------------------------------------------

// DPP quad-permutation control: lane i of a group of S (S | 4) reads lane
// (i - r) mod S of its group.
constexpr int qp_ctrl(int S, int r) {
  int c = 0;
  for (int i = 0; i < 4; i++) c |= ((i / S) * S + ((i % S) - r + S) % S) << (2 * i);
  return c;
}

template <int L, bool GLASSY, int S>
struct PottsMK {
  using G = GC<L>;
  static constexpr bool QUAD = true;  // loads and stores its own ring
  static_assert(S == 2 || S == 4 || S == 8, "two, four or eight lanes per wheel");
  static_assert(G::B % S == 0 && G::H % S == 0, "S lanes per wheel need B, L/2 multiples of S");
  static constexpr int B = G::B / S;                 // steps per block (draws per lane)
  static constexpr int Q24 = 24 / S, Q55 = 55 / S, R55 = 55 % S, Q61 = 61 / S, R61 = 61 % S;
  static_assert(24 % S == 0 && R55 > 0 && R61 > 0, "lag 24 in-lane, lags 55 and 61 across lanes");
  static constexpr int D = Q61 + 1;                  // steps of history a lane keeps
  static constexpr int RL = ((D + B - 1) / B) * B;   // register ring of a lane (steps)
  static constexpr int M = RL, V = RL / B;           // as the drive expects them
  static constexpr int NBLK = G::NBLK, H = G::H, RPB = G::RPB, RHO = G::RHO, NW = G::NW;
  static constexpr int MS = G::M;                    // HBM ring slots of a wheel
  // +-J patterns hold four draws per word: with S <= 4 every lane loads all
  // words of the block, with S = 8 each lane the word of each of its draws
  static constexpr bool OWNW = !GLASSY && S > 4;
  static constexpr int BQ = GLASSY || OWNW ? B : potts_bq(L);  // coupling words per block and lane
  static constexpr int XS = potts_xs(L);             // LDS byte stride of x
  uint8_t *sp;          // LDS bytes of the lane's copy, [y][x][z] (rows at row(y)), 8 sigma
  uint8_t *wp;          // where the lane stores its new spins: sp, or the dummy region
  const uint32_t *tab;  // LDS table: rotation bases (+-J) or vote words (glassy)
  const uint8_t *Wb;    // LDS weight table of the lane's temperature
  rsrc_t rJ;            // coupling words of the job
  uint32_t voff;        // byte offset of the lane's coupling words
  bool active;
  int z, zp, zm, g, sub;  // wheel plane, row group and the lane's place in its group
  uint32_t m0, mlast;     // all ones in lanes with sub == 0 (== S - 1)
  uint32_t x55, x61;      // all ones in lanes exposing the older word for lag 55 (61)
  uint32_t lo55, lo61;    // S = 8: all ones in lanes reading a lane below them (sub >= r)
  uint32_t sh;            // 8 (sub mod 4): the lane's byte of a +-J pattern word
  int kmod0, kmod1;       // first draw of the launch (and of the next one) mod MS
  uint32_t nextpat[BQ];

  static DEV int row(int y) { return y * L * XS + (y / RHO) * 2 * L; }

  DEV void init_lane(int t) {
    sub = t % S;
    m0 = sub == 0 ? ~0u : 0u;
    mlast = sub == S - 1 ? ~0u : 0u;
    x55 = sub >= S - R55 ? ~0u : 0u;
    x61 = sub >= S - R61 ? ~0u : 0u;
    lo55 = sub >= R55 ? ~0u : 0u;
    lo61 = sub >= R61 ? ~0u : 0u;
    sh = 8u * (uint32_t)(sub & 3);
  }

  // x of lane (sub - R) mod S of the lane's group.  S <= 4: one quad
  // permutation.  S = 8: the groups are the halves of the 16-lane DPP rows;
  // rotating the row by R serves the lanes with sub >= R, rotating it by
  // R + 8 the others.
  template <int R>
  DEV uint32_t from_lane(uint32_t x, uint32_t lo) const {
    if constexpr (S <= 4) {
      (void)lo;
      return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, qp_ctrl(S, R), 0xF, 0xF, false);
    } else {
      const uint32_t a = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x120 + R, 0xF, 0xF, false);
      const uint32_t b = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x120 + R + 8, 0xF, 0xF, false);
      return bfi(lo, a, b);
    }
  }

  DEV void fetch(int p, int blk) {
    if constexpr (GLASSY) {
      // one word per draw: the lane's draws S i + sub of the block
      const uint32_t s0 = __builtin_amdgcn_readfirstlane((uint32_t)((p * NBLK + blk) * G::B) * NW * 4u);
#pragma unroll
      for (int i = 0; i < B; i++) nextpat[i] = bload(rJ, voff, s0 + (uint32_t)(S * i) * NW * 4u);
    } else if constexpr (OWNW) {
      // draw S i + sub is in word S i / 4 + sub / 4 (sub / 4 is in voff)
      const uint32_t s0 =
          __builtin_amdgcn_readfirstlane((uint32_t)((p * NBLK + blk) * potts_bq(L)) * NW * 4u);
#pragma unroll
      for (int i = 0; i < B; i++) nextpat[i] = bload(rJ, voff, s0 + (uint32_t)(S / 4 * i) * NW * 4u);
    } else {
      // four draws per word
      const uint32_t s0 = __builtin_amdgcn_readfirstlane((uint32_t)((p * NBLK + blk) * BQ) * NW * 4u);
#pragma unroll
      for (int q = 0; q < BQ; q++) nextpat[q] = bload(rJ, voff, s0 + (uint32_t)q * NW * 4u);
    }
  }

  // HBM slot of the output at draw offset `off` from a launch's first draw
  DEV uint32_t slot_of(int kmod, int off) const { return (uint32_t)((kmod + 4 * MS + off) % MS); }

  // outputs of steps -D .. -1 (draws k0 + S st + sub); the oldest are dead
  // (before k0 - 61) in some lanes and never read
  DEV void load_ring(uint32_t (&ring)[RL], const Drive &d) const {
#pragma unroll
    for (int i = 0; i < D; i++) {
      const int st = i - D;
      ring[(st + RL) % RL] = bload(d.rwh, d.widx + slot_of(kmod0, S * st + sub) * d.wstride);
    }
  }

  // LAST: the register of the launch's last step; live words are those of
  // draws >= k_end - 61
  template <int LAST>
  DEV void store_ring(const uint32_t (&ring)[RL], const Drive &d) const {
#pragma unroll
    for (int ds = 0; ds < D; ds++) {
      const int i = (LAST - ds + RL) % RL;
      const int off = -S - S * ds + sub;
      if (off >= -61) bstore(d.rwh, ring[i], d.widx + slot_of(kmod1, off) * d.wstride);
    }
  }

  template <int VI>
  DEV void block(uint32_t (&ring)[M], int p, int blk) {
    uint32_t pat[BQ];
#pragma unroll
    for (int q = 0; q < BQ; q++) pat[q] = nextpat[q];
    if (blk + 1 < NBLK)
      fetch(p, blk + 1);
    else
      fetch(p ^ 1, 0);
    rows<VI>(ring, pat, p, g * RHO + blk * RPB, sp, wp, tab, Wb);
  }

  template <int VI>
  DEV void rows(uint32_t (&ring)[M], const uint32_t (&pat)[BQ], int p, int y0,
                const uint8_t *__restrict__ rd, uint8_t *__restrict__ wr,
                const uint32_t *__restrict__ tb, const uint8_t *__restrict__ wt) const {
    // per row of the block: the lane's first site (j = sub), the periodic x
    // neighbour at the row's ends, and the y neighbours' rows
    int base[RPB], bxw[RPB], byp[RPB], bym[RPB];
#pragma unroll
    for (int rr = 0; rr < RPB; rr++) {
      const int y = y0 + rr;
      const int e = (p + y + z) & 1;
      const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
      const int lane = 2 * sub * XS;
      base[rr] = row(y) + e * XS + z + lane;
      bxw[rr] = row(y) + z + (e ? 0 : (L - 1) * XS);
      byp[rr] = row(yp) + e * XS + z + lane;
      bym[rr] = row(ym) + e * XS + z + lane;
    }
    const int dzp = zp - z, dzm = zm - z;
    uint32_t nb[B][6], rb[B][6], w[B][4];

    // step i: draw S i + sub of the block, row rr = S i / H, in-row index
    // j = S i mod H + sub (H is a multiple of S)
    auto request_site = [&](int i) {
      const int rr = S * i / H, jb = S * i - rr * H, o = 2 * jb * XS;
      if constexpr (GLASSY) {
#pragma unroll
        for (int d = 0; d < 6; d++) rb[i][d] = tb[(d & 1) * 24 + ((pat[i] >> (5 * d)) & 31u)];
      } else {
        // word (S i + sub) / 4, byte (S i + sub) mod 4; the entry of the
        // pattern's bits 0..4 gives directions 0..4, bit 5 the sixth word
        const uint32_t pb = OWNW ? pat[i] >> sh : pat[(S * i) >> 2] >> (sh + 8 * ((S * i) & 3));
        const uint32_t *r5 = tb + POTTS_TAB_STRIDE * (pb & 31u);
#pragma unroll
        for (int d = 0; d < 5; d++) rb[i][d] = r5[d];
        rb[i][5] = bfi((uint32_t)((int32_t)(pb << 26) >> 31), 0x04040400u, 4u);
      }
      const int c = base[rr] + o;
      const int xp = jb == H - S ? (int)bfi(mlast, (uint32_t)bxw[rr], (uint32_t)(c + XS)) : c + XS;
      const int xm = jb == 0 ? (int)bfi(m0, (uint32_t)bxw[rr], (uint32_t)(c - XS)) : c - XS;
      nb[i][0] = rd[xp];
      nb[i][1] = rd[xm];
      nb[i][2] = rd[byp[rr] + o];
      nb[i][3] = rd[bym[rr] + o];
      nb[i][4] = rd[c + dzp];
      nb[i][5] = rd[c + dzm];
    };
    auto request_weights = [&](int i) {
      uint32_t c, c0, c1, c2, c3;
      if constexpr (GLASSY) {
        c = 0;
#pragma unroll
        for (int d = 0; d < 6; d++) c += 4u << ((rb[i][d] >> nb[i][d]) & 31u);
        c0 = c & 0xFFu, c1 = (c >> 8) & 0xFFu, c2 = (c >> 16) & 0xFFu, c3 = c >> 24;
      } else {
        c = __builtin_rotateright32(rb[i][0], nb[i][0]) + __builtin_rotateright32(rb[i][1], nb[i][1]) +
            __builtin_rotateright32(rb[i][2], nb[i][2]) + __builtin_rotateright32(rb[i][3], nb[i][3]) +
            __builtin_rotateright32(rb[i][4], nb[i][4]) + __builtin_rotateright32(rb[i][5], nb[i][5]);
        c0 = c & 0xFFu, c3 = (c >> 8) & 0xFFu, c2 = (c >> 16) & 0xFFu, c1 = c >> 24;
      }
      const uint8_t *wm = wt + max(max(c0, c3), max(c2, c1));
      w[i][0] = *(const uint32_t *)(wm - c0);
      w[i][1] = *(const uint32_t *)(wm - c1);
      w[i][2] = *(const uint32_t *)(wm - c2);
      w[i][3] = *(const uint32_t *)(wm - c3);
    };
    auto finish_site = [&](int i) {
      const int rr = S * i / H, jb = S * i - rr * H;
      const int st = VI * B + i;  // register of this step (static)
      const uint32_t e55 = bfi(x55, ring[(st + RL - Q55 - 1) % RL], ring[(st + RL - Q55) % RL]);
      const uint32_t e61 = bfi(x61, ring[(st + RL - Q61 - 1) % RL], ring[(st + RL - Q61) % RL]);
      const uint32_t y55 = from_lane<R55>(e55, lo55);
      const uint32_t y61 = from_lane<R61>(e61, lo61);
      ring[st % RL] = ring[(st + RL - Q24) % RL] + y55;
      const uint32_t r = ring[st % RL] ^ y61;
      const uint32_t C1 = w[i][0] + w[i][1], C2 = C1 + w[i][2];
      const uint32_t t = __umulhi(r, C2 + w[i][3]);
      const uint32_t nt = ~t;
      const uint32_t v = (((w[i][0] + nt) >> 31) + ((C1 + nt) >> 31) + ((C2 + nt) >> 31)) << 3;
      wr[base[rr] + 2 * jb * XS] = (uint8_t)v;
    };

    request_site(0);
    if constexpr (B > 1) request_site(1);
    __builtin_amdgcn_sched_barrier(0);
    request_weights(0);
#pragma unroll
    for (int i = 0; i < B; i++) {
      __builtin_amdgcn_sched_barrier(0);
      if (i + 2 < B) request_site(i + 2);
      __builtin_amdgcn_sched_barrier(0);
      if (i + 1 < B) request_weights(i + 1);
      __builtin_amdgcn_sched_barrier(0);
      finish_site(i);
    }
    __builtin_amdgcn_sched_barrier(0);
  }

  // sum over the lane's colour-0 sites of h_{sigma_i} = sum_j J_ij delta(sigma_i, sigma_j)
  DEV int lane_bond_sum() const {
    int hsum = 0;
    for (int blk = 0; blk < NBLK; blk++) {
      const int y0 = g * RHO + blk * RPB;
      for (int i = 0; i < B; i++) {
        const int kb = S * i + sub, rr = kb / H, j = kb - rr * H;
        const int y = y0 + rr;
        const int e = (y + z) & 1;
        const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
        const int c = row(y) + (2 * j + e) * XS + z;
        const int xpi = (2 * j + e + 1) % L, xmi = (2 * j + e + L - 1) % L;
        const int nb[6] = {row(y) + xpi * XS + z, row(y) + xmi * XS + z,
                           row(yp) + (2 * j + e) * XS + z, row(ym) + (2 * j + e) * XS + z,
                           c - z + zp, c - z + zm};
        const uint32_t si = sp[c];
        if constexpr (GLASSY) {
          const uint32_t pw = bload(rJ, voff + (uint32_t)((blk * G::B + S * i) * NW) * 4u);
          for (int d = 0; d < 6; d++) {
            const uint32_t vote = tab[(d & 1) * 24 + ((pw >> (5 * d)) & 31u)];
            hsum += ((vote >> sp[nb[d]]) & 31u) == si;
          }
        } else {
          // word kb / 4 of the block (voff holds sub / 4 when S = 8)
          const uint32_t v0 = OWNW ? voff - (uint32_t)((sub >> 2) * NW) * 4u : voff;
          const uint32_t pw = bload(rJ, v0 + (uint32_t)((blk * potts_bq(L) + (kb >> 2)) * NW) * 4u);
          const uint32_t pt = (pw >> (8 * (kb & 3))) & 0xFFu;
          for (int d = 0; d < 6; d++)
            if (sp[nb[d]] == si) hsum += ((pt >> d) & 1u) ? -1 : 1;
        }
      }
    }
    return hsum;
  }
};

template <int L, bool GLASSY, int S>
DEV void potts_multi_run(const Work &w, uint32_t *lds) {
  using G = GC<L>;
  using K = PottsMK<L, GLASSY, S>;
  constexpr int N3 = L * L * L;
  constexpr int CW = potts_lds_copy(L) / 4;  // LDS words per copy
  constexpr int XW = potts_xs(L) / 4;        // LDS words per x step
  constexpr int LPC = S * G::NW;             // lanes per copy
  // LDS word of HBM word u of a copy (u = (y L + x) L / 4 + z / 4)
  auto lds_word = [](int u) {
    const int y = u / (L * L / 4), x = (u / (L / 4)) % L;
    return (y * L * potts_xs(L) + (y / G::RHO) * 2 * L) / 4 + x * XW + u % (L / 4);
  };
  const int t = threadIdx.x;
  const int nthr = blockDim.x;
  const bool active = t < w.ncopies * LPC;
  uint32_t *tab = lds;
  uint32_t *cp = lds + POTTS_TAB_WORDS;
  uint32_t *Wt = cp + w.ncopies * CW;
  int *Hcnt = (int *)(Wt + w.ncopies * POTTS_W_WORDS);
  uint8_t *dummy = (uint8_t *)(Hcnt + w.ncopies);  // RHO L XS bytes if LPC % 64 != 0
  const rsrc_t rsp = make_rsrc(w.spins, w.spins_bytes);
  const uint32_t sbase = (uint32_t)w.copy0 * N3;
  potts_tables<GLASSY>(tab);
  for (int i = t; i < w.ncopies * POTTS_W_WORDS; i += nthr) {
    const int c = w.copy0 + i / POTTS_W_WORDS;
    Wt[i] = w.thr[w.temp_of_slot[c] * THR_WORDS + i % POTTS_W_WORDS];
  }
  stage_words<8>(
      w.ncopies * (N3 / 4), [&](int i) { return bload(rsp, i * 4, sbase); },
      [&](int i, uint32_t v) {
        const int c = i / (N3 / 4), u = i - c * (N3 / 4);
        cp[c * CW + lds_word(u)] = v;
      });
  for (int i = t; i < w.ncopies; i += nthr) Hcnt[i] = 0;

  // lanes without a wheel (whole groups of S) run wheel (z = (t / S) mod L,
  // row group 0) of the first copy and store into the dummy region
  K k;
  const int cl = active ? t / LPC : 0;
  const int rem = active ? t - cl * LPC : S * ((t / S) % L) + t % S;
  const int wl = rem / S;
  const int copy = w.copy0 + cl;
  k.init_lane(t);
  k.sp = (uint8_t *)(cp + cl * CW);
  k.wp = active ? k.sp : dummy;
  k.tab = tab;
  k.Wb = (const uint8_t *)(Wt + cl * POTTS_W_WORDS);
  k.active = active;
  k.g = wl / L;
  k.z = wl - k.g * L;
  k.zp = k.z + 1 == L ? 0 : k.z + 1;
  k.zm = k.z == 0 ? L - 1 : k.z - 1;
  k.rJ = make_rsrc(w.J, w.J_bytes);
  k.voff = ((uint32_t)(copy / w.RK) * (GLASSY ? gpotts_js(L) : potts_js(L)) + wl) * 4u;
  if constexpr (GLASSY) k.voff += (uint32_t)(k.sub * G::NW) * 4u;
  if constexpr (K::OWNW) k.voff += (uint32_t)((k.sub >> 2) * G::NW) * 4u;
  const uint64_t per_sweep = (uint64_t)G::RHO * L;
  const uint64_t done = *w.done;
  k.kmod0 = (int)__builtin_amdgcn_readfirstlane((uint32_t)((done * per_sweep) % G::M));
  k.kmod1 = (int)__builtin_amdgcn_readfirstlane(
      (uint32_t)(((done + (uint64_t)max(w.nsweeps_cap, 0)) * per_sweep) % G::M));

  Drive d;
  d.nsweeps = w.nsweeps_cap;
  d.active = active;
  d.rwh = make_rsrc(w.wheels, w.wheels_bytes);
  d.wstride = (uint32_t)w.C * G::NW * 4u;
  d.widx = ((uint32_t)copy * G::NW + wl) * 4u;
  d.kmod = k.kmod0;
  __syncthreads();
  k.fetch(0, 0);
  drive(k, d);

  if (active) atomicAdd(&Hcnt[cl], k.lane_bond_sum());
  __syncthreads();
  if (w.nsweeps_cap > 0)
    for (int i = t; i < w.ncopies * (N3 / 4); i += nthr) {
      const int c = i / (N3 / 4), u = i - c * (N3 / 4);
      bstore(rsp, cp[c * CW + lds_word(u)], i * 4, sbase);
    }
  for (int i = t; i < w.ncopies; i += nthr) w.E[w.copy0 + i] = -(int64_t)Hcnt[i];
}

template <bool GLASSY>
DEV void potts_quad_dispatch(const Work &w, uint32_t *lds) {
  switch (w.L) {
    case 8: potts_multi_run<8, GLASSY, 4>(w, lds); break;
    case 16:
      if (w.wl == 4)
        potts_multi_run<16, GLASSY, 4>(w, lds);
      else
        potts_multi_run<16, GLASSY, 8>(w, lds);
      break;
    case 24: potts_multi_run<24, GLASSY, 4>(w, lds); break;
    case 32: potts_multi_run<32, GLASSY, 4>(w, lds); break;
    default: break;
  }
}

template <bool GLASSY>
DEV void potts_pair_dispatch(const Work &w, uint32_t *lds) {
  switch (w.L) {
    case 40: potts_multi_run<40, GLASSY, 2>(w, lds); break;
    case 48: potts_multi_run<48, GLASSY, 2>(w, lds); break;
    default: break;
  }
}

__global__ __launch_bounds__(POTTS_MAX_TPB) void potts_quad_kernel(const Work *__restrict__ works,
                                                                   int nsweeps) {
  extern __shared__ uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  potts_quad_dispatch<false>(w, lds);
}

__global__ __launch_bounds__(POTTS_MAX_TPB) void gpotts_quad_kernel(const Work *__restrict__ works,
                                                                    int nsweeps) {
  extern __shared__ uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  potts_quad_dispatch<true>(w, lds);
}

__global__ __launch_bounds__(POTTS_PAIR_MAX_TPB) void potts_pair_kernel(const Work *__restrict__ works,
                                                                        int nsweeps) {
  extern __shared__ uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  potts_pair_dispatch<false>(w, lds);
}

__global__ __launch_bounds__(POTTS_PAIR_MAX_TPB) void gpotts_pair_kernel(const Work *__restrict__ works,
                                                                         int nsweeps) {
  extern __shared__ uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  potts_pair_dispatch<true>(w, lds);
}

template <bool GLASSY>
DEV void potts_dispatch(const Work &w, uint32_t *lds) {
  switch (w.L) {
    case 2: potts_run<2, GLASSY>(w, lds); break;
    case 4: potts_run<4, GLASSY>(w, lds); break;
    default: break;
  }
}

__global__ __launch_bounds__(POTTS_MAX_TPB) void potts_sweep_kernel(const Work *__restrict__ works,
                                                                    int nsweeps) {
  extern __shared__ uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  potts_dispatch<false>(w, lds);
}

__global__ __launch_bounds__(POTTS_MAX_TPB) void gpotts_sweep_kernel(const Work *__restrict__ works,
                                                                     int nsweeps) {
  extern __shared__ uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  potts_dispatch<true>(w, lds);
}
// ---------------------------------------------------------------------------
// 4D glassy Potts model (Eq. 3 on the hypercubic lattice), heat bath.  The
// 3D glassy kernel with eight neighbours: lanes serve the wheels of the
// (z, u) planes, neighbours u +- 1 are one padded u plane (US bytes) away,
// and each site's eight permutation numbers come in two coupling words (x,
// y, z in the first, u in the second).  Byte a of the vote sum is
// 4 h_a <= 32; the weight table holds W[0..8].
// ---------------------------------------------------------------------------
template <int L>
struct Potts4K {
  static constexpr Geom G4 = geom4(L);
  static constexpr int M = G4.M, B = G4.B, V = G4.V, NBLK = G4.NBLK, H = G4.H, RPB = G4.RPB,
                       RHO = G4.RHO, NW = G4.NW;
  static constexpr int US = potts4_us(L), YS = L * US;  // LDS strides of u and y
  uint8_t *sp;          // LDS bytes of the lane's copy (layout of sg_layout.h), 8 sigma
  uint8_t *wp;          // where the lane stores its new spins: sp, or the dummy region
  const uint32_t *tab;  // LDS vote words: pi (0..23), pi^-1 (24..47)
  const uint8_t *Wb;    // LDS weight table of the lane's temperature
  rsrc_t rJ;            // coupling words of the job
  uint32_t voff;        // byte offset of the lane's coupling words
  int z, dzp, dzm, dup, dum, g, inplane;  // inplane = u US + z
  uint32_t nextpat[2 * B];  // coupling words of the next block

  DEV void fetch(int p, int blk) {
    const uint32_t s0 = __builtin_amdgcn_readfirstlane((uint32_t)((p * NBLK + blk) * B) * NW * 8u);
#pragma unroll
    for (int q = 0; q < B; q++) {
      nextpat[2 * q] = bload(rJ, voff, s0 + (uint32_t)q * NW * 8u);
      nextpat[2 * q + 1] = bload(rJ, voff + 4, s0 + (uint32_t)q * NW * 8u);
    }
  }

  template <int VI>
  DEV void block(uint32_t (&ring)[M], int p, int blk) {
    uint32_t pat[2 * B];
#pragma unroll
    for (int q = 0; q < 2 * B; q++) pat[q] = nextpat[q];
    if (blk + 1 < NBLK)
      fetch(p, blk + 1);
    else
      fetch(p ^ 1, 0);
    rows<VI>(ring, pat, p, g * RHO + blk * RPB, sp, wp, tab, Wb);
  }

  // Offsets of row y's site j = 0 (x = e) of the lane's (z, u) plane, of the
  // x neighbour that wraps (x = L - 1 for e = 0, x = 0 for e = 1; it is also
  // the non-wrapping x+ of j = H - 1, e = 0 and x- of j = 0, e = 1) and of
  // the y neighbours; site j is 2 j L further.
  DEV void row_offsets(int p, int y, int &own, int &bxw, int &byp, int &bym) const {
    const int e = (p + y + g_parity) & 1;
    const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
    own = y * YS + inplane + e * L;
    bxw = e ? own - L : own + (L - 1) * L;
    byp = own + (yp - y) * YS;
    bym = own + (ym - y) * YS;
  }
  int g_parity;  // (z + u) & 1

  // Same pipeline as the 3D kernels: neighbour bytes and vote words of site
  // n + 2, fields and weight reads of site n + 1, draw and store of site n.
  template <int VI>
  DEV void rows(uint32_t (&ring)[M], const uint32_t (&pat)[2 * B], int p, int y0,
                const uint8_t *__restrict__ rd, uint8_t *__restrict__ wr,
                const uint32_t *__restrict__ tb, const uint8_t *__restrict__ wt) const {
    int own[RPB], bxw[RPB], byp[RPB], bym[RPB];
#pragma unroll
    for (int rr = 0; rr < RPB; rr++) row_offsets(p, y0 + rr, own[rr], bxw[rr], byp[rr], bym[rr]);
    uint32_t nb[B][8], rb[B][8], w[B][4];

    auto request_site = [&](int kb) {
      const int rr = kb / H, j = kb - rr * H, o = 2 * j * L;
      const uint32_t w0 = pat[2 * kb], w1 = pat[2 * kb + 1];
#pragma unroll
      for (int d = 0; d < 6; d++) rb[kb][d] = tb[(d & 1) * 24 + ((w0 >> (5 * d)) & 31u)];
      rb[kb][6] = tb[w1 & 31u];
      rb[kb][7] = tb[24 + ((w1 >> 5) & 31u)];
      const int s = own[rr] + o;
      nb[kb][0] = rd[j == H - 1 ? bxw[rr] : s + L];
      nb[kb][1] = rd[j == 0 ? bxw[rr] : s - L];
      nb[kb][2] = rd[byp[rr] + o];
      nb[kb][3] = rd[bym[rr] + o];
      nb[kb][4] = rd[s + dzp];
      nb[kb][5] = rd[s + dzm];
      nb[kb][6] = rd[s + dup];
      nb[kb][7] = rd[s + dum];
    };
    auto request_weights = [&](int kb) {
      uint32_t c = 0;
#pragma unroll
      for (int d = 0; d < 8; d++) c += 4u << ((rb[kb][d] >> nb[kb][d]) & 31u);
      const uint32_t c0 = c & 0xFFu, c1 = (c >> 8) & 0xFFu, c2 = (c >> 16) & 0xFFu, c3 = c >> 24;
      const uint8_t *wm = wt + max(max(c0, c3), max(c2, c1));
      w[kb][0] = *(const uint32_t *)(wm - c0);
      w[kb][1] = *(const uint32_t *)(wm - c1);
      w[kb][2] = *(const uint32_t *)(wm - c2);
      w[kb][3] = *(const uint32_t *)(wm - c3);
    };
    auto finish_site = [&](int kb) {
      const int rr = kb / H, j = kb - rr * H;
      const int k = VI * B + kb;  // ring slot (static)
      ring[k % M] = ring[(k + M - 24) % M] + ring[(k + M - 55) % M];
      const uint32_t r = ring[k % M] ^ ring[(k + M - 61) % M];
      const uint32_t C1 = w[kb][0] + w[kb][1], C2 = C1 + w[kb][2];
      const uint32_t t = __umulhi(r, C2 + w[kb][3]);
      // compare-and-select form: the 3D kernel's mask-free count measured
      // slightly slower here
      uint32_t v = t >= w[kb][0] ? 8u : 0u;
      v = t >= C1 ? 16u : v;
      v = t >= C2 ? 24u : v;
      wr[own[rr] + 2 * j * L] = (uint8_t)v;
    };

    request_site(0);
    if constexpr (B > 1) request_site(1);
    __builtin_amdgcn_sched_barrier(0);
    request_weights(0);
#pragma unroll
    for (int kb = 0; kb < B; kb++) {
      __builtin_amdgcn_sched_barrier(0);
      if (kb + 2 < B) request_site(kb + 2);
      __builtin_amdgcn_sched_barrier(0);
      if (kb + 1 < B) request_weights(kb + 1);
      __builtin_amdgcn_sched_barrier(0);
      finish_site(kb);
    }
    __builtin_amdgcn_sched_barrier(0);
  }

  // sum over the lane's colour-0 sites of the number of its eight bonds whose
  // term is 1 (every bond joins a colour-0 and a colour-1 site)
  DEV int lane_bond_sum() const {
    int hsum = 0;
    for (int blk = 0; blk < NBLK; blk++) {
      const int y0 = g * RHO + blk * RPB;
      for (int kb = 0; kb < B; kb++) {
        const int rr = kb / H, j = kb - rr * H, o = 2 * j * L;
        int own, bxw, byp, bym;
        row_offsets(0, y0 + rr, own, bxw, byp, bym);
        const int s = own + o;
        const int nbo[8] = {j == H - 1 ? bxw : s + L, j == 0 ? bxw : s - L, byp + o, bym + o,
                            s + dzp, s + dzm, s + dup, s + dum};
        const uint32_t el = voff + (uint32_t)((blk * B + kb) * NW) * 8u;
        const uint32_t w0 = bload(rJ, el), w1 = bload(rJ, el + 4);
        const uint32_t si = sp[s];
        for (int d = 0; d < 8; d++) {
          const uint32_t num = d < 6 ? (w0 >> (5 * d)) & 31u : (w1 >> (5 * (d - 6))) & 31u;
          const uint32_t vote = tab[(d & 1) * 24 + num];
          hsum += ((vote >> sp[nbo[d]]) & 31u) == si;
        }
      }
    }
    return hsum;
  }
};

template <int L>
DEV void potts4_run(const Work &w, uint32_t *lds) {
  using K4 = Potts4K<L>;
  constexpr int N4 = L * L * L * L;
  constexpr int CW = potts4_lds_copy(L) / 4;  // LDS words per copy
  constexpr int L2 = L * L, UW = potts4_us(L) / 4;  // HBM u-plane bytes, LDS u-plane words
  const int t = threadIdx.x;
  const int nthr = blockDim.x;
  const int lanes = w.ncopies * K4::NW;
  const bool active = t < lanes;
  uint32_t *tab = lds;                                   // [48] vote words
  uint32_t *cp = lds + 48;                               // [ncopies][CW] spins
  uint32_t *Wt = cp + w.ncopies * CW;                    // [ncopies][POTTS4_W_WORDS]
  int *Hcnt = (int *)(Wt + w.ncopies * POTTS4_W_WORDS);  // [ncopies]
  uint8_t *dummy = (uint8_t *)(Hcnt + w.ncopies);        // RHO L US bytes if NW % 64 != 0
  const rsrc_t rsp = make_rsrc(w.spins, w.spins_bytes);
  const uint32_t sbase = (uint32_t)w.copy0 * N4;
  // vote words of the 24 permutations (lexicographic order): pi, then pi^-1
  for (int i = t; i < 48; i += nthr) {
    const int k = i % 24;
    int avail[4] = {0, 1, 2, 3}, pi[4], inv[4];
    const int digit[3] = {k / 6, (k / 2) % 3, k % 2};
    int left = 4;
    for (int v = 0; v < 4; v++) {
      const int c = v < 3 ? digit[v] : 0;
      pi[v] = avail[c];
      for (int q = c; q + 1 < left; q++) avail[q] = avail[q + 1];
      left--;
    }
    for (int v = 0; v < 4; v++) inv[pi[v]] = v;
    uint32_t word = 0;
    for (int v = 0; v < 4; v++) word |= (uint32_t)(8 * (i < 24 ? pi[v] : inv[v])) << (8 * v);
    tab[i] = word;
  }
  // HBM word q of a copy ([y][u][x][z], u planes L^2 bytes apart) -> LDS
  // (u planes potts4_us(L) bytes apart)
  for (int i = t; i < w.ncopies * POTTS4_W_WORDS; i += nthr) {
    const int c = w.copy0 + i / POTTS4_W_WORDS;
    Wt[i] = w.thr[w.temp_of_slot[c] * THR_WORDS + i % POTTS4_W_WORDS];
  }
  stage_words<8>(
      w.ncopies * (N4 / 4), [&](int i) { return bload(rsp, i * 4, sbase); },
      [&](int i, uint32_t v) {
        const int c = i / (N4 / 4), q = i - c * (N4 / 4);
        const int yu = q / (L2 / 4), r = q - yu * (L2 / 4);
        cp[c * CW + yu * UW + r] = v;
      });
  for (int i = t; i < w.ncopies; i += nthr) Hcnt[i] = 0;

  // lanes without a wheel run the blocks of wheel (z = t mod L, u = 0, row
  // group 0) of the first copy and store into the dummy region
  K4 k;
  const int cl = active ? t / K4::NW : 0;
  const int wl = active ? t - cl * K4::NW : t % L;
  const int copy = w.copy0 + cl;
  k.sp = (uint8_t *)(cp + cl * CW);
  k.wp = active ? k.sp : dummy;
  k.tab = tab;
  k.Wb = (const uint8_t *)(Wt + cl * POTTS4_W_WORDS);
  const int u = (wl / L) % L;
  k.g = wl / L2;
  k.z = wl % L;
  k.g_parity = (k.z + u) & 1;
  k.inplane = u * K4::US + k.z;
  k.dzp = k.z + 1 == L ? 1 - L : 1;
  k.dzm = k.z == 0 ? L - 1 : -1;
  k.dup = u + 1 == L ? (1 - L) * K4::US : K4::US;
  k.dum = u == 0 ? (L - 1) * K4::US : -K4::US;
  k.rJ = make_rsrc(w.J, w.J_bytes);
  k.voff = ((uint32_t)(copy / w.RK) * gpotts4_js(L) + 2 * wl) * 4u;

  Drive d;
  d.nsweeps = w.nsweeps_cap;
  d.active = active;
  d.rwh = make_rsrc(w.wheels, w.wheels_bytes);
  d.wstride = (uint32_t)w.C * K4::NW * 4u;
  d.widx = ((uint32_t)copy * K4::NW + wl) * 4u;
  d.kmod = (int)__builtin_amdgcn_readfirstlane((uint32_t)((*w.done * (uint64_t)(K4::RHO * L)) % K4::M));
  __syncthreads();
  k.fetch(0, 0);
  drive(k, d);

  if (active) atomicAdd(&Hcnt[cl], k.lane_bond_sum());
  __syncthreads();
  if (w.nsweeps_cap > 0)
    for (int i = t; i < w.ncopies * (N4 / 4); i += nthr) {
      const int c = i / (N4 / 4), q = i - c * (N4 / 4);
      const int yu = q / (L2 / 4), r = q - yu * (L2 / 4);
      bstore(rsp, cp[c * CW + yu * UW + r], i * 4, sbase);
    }
  for (int i = t; i < w.ncopies; i += nthr) w.E[w.copy0 + i] = -(int64_t)Hcnt[i];
}

__global__ __launch_bounds__(POTTS_MAX_TPB) void gpotts4_sweep_kernel(const Work *__restrict__ works,
                                                                      int nsweeps) {
  extern __shared__ uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  switch (w.L) {
    case 2: potts4_run<2>(w, lds); break;
    case 4: potts4_run<4>(w, lds); break;
    case 8: potts4_run<8>(w, lds); break;
    case 16: potts4_run<16>(w, lds); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Overlap between replica 0 and replica 1 at every temperature.
//   Ising: Q = N - 2 popcount(a xor b) over the packed words (pads are zero);
//   Ising-like models: over occupied sites, Q = sum popcount(X) -
//   2 popcount((a xor b) and X) with X the sample's occupancy words;
//   Potts: C = number of equal site bytes.
// grid = S * K, one workgroup per (sample, temperature).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void overlap_kernel(const uint32_t *__restrict__ spins,
                                                      const int32_t *__restrict__ slot_of_temp,
                                                      int64_t *__restrict__ Q, int model, int L,
                                                      int R, int K, int copy_words,
                                                      const uint32_t *__restrict__ occ,
                                                      uint32_t occ_stride) {
  __shared__ int part[256];
  const int sk = blockIdx.x;
  const int s = sk / K, k = sk - s * K;
  const int ca = (s * R + 0) * K + slot_of_temp[(s * R + 0) * K + k];
  const int cb = (s * R + 1) * K + slot_of_temp[(s * R + 1) * K + k];
  const uint32_t *a = spins + (size_t)ca * copy_words;
  const uint32_t *b = spins + (size_t)cb * copy_words;
  const uint32_t *X = occ ? occ + (size_t)s * occ_stride : nullptr;
  int acc = 0;
  for (int i = threadIdx.x; i < copy_words; i += blockDim.x) {
    const uint32_t x = a[i] ^ b[i];
    if (X) {
      acc += __popc(X[i]) - 2 * __popc(x & X[i]);
    } else if (model == 0) {
      acc += __popc(x);
    } else {
      // count equal bytes: a byte of x is zero iff the two sites agree
      const uint32_t nz = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;
      acc += 4 - __popc(nz & 0x80808080u);
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t N = (int64_t)L * L * L;
    Q[sk] = model == 0 && !X ? N - 2 * (int64_t)part[0] : (int64_t)part[0];
  }
}

// ---------------------------------------------------------------------------
// Parallel tempering, one thread per (sample, replica) chain.  Pairs of
// neighbouring temperatures in ascending order; one number of the chain's own
// wheel per pair; accept when sign(dbeta) * D <= 0, else when r < T with T the
// integer product of the factors F[b] over the set bits of |D|.
// The chain wheel is stored as 61 words + the position of the oldest word.
// ---------------------------------------------------------------------------
DEV uint32_t ptw_next(uint32_t *w) {
  int pos = (int)w[61];
  auto back = [&](int m) { int j = pos - m; return w[j < 0 ? j + 61 : j]; };
  const uint32_t ik = back(24) + back(55);
  const uint32_t out = ik ^ w[pos];
  w[pos] = ik;
  w[61] = pos == 60 ? 0 : pos + 1;
  return out;
}

// The threshold of |D| (0 < |D| < 2^24): from T = 2^32, for each set bit b
// of |D|, lowest first, T <- floor(T Fi[b] / 2^32).  No factor exceeds
// 2^32 and one equal to 2^32 leaves T as it is, so with m = the set bits
// whose factor is below 2^32 (m != 0) the first step sets T to that factor
// and every later one is the high word of a 32 x 32-bit product; m = 0
// leaves T = 2^32.  F2: the pair's factors as (low, high) word pairs.
DEV uint32_t pt_threshold(const uint32_t *F2, uint32_t m) {
  uint32_t T = F2[2 * (__ffs(m) - 1)];
  for (m &= m - 1; m; m &= m - 1) T = __umulhi(T, F2[2 * (__ffs(m) - 1)]);
  return T;
}

// ptw_next with the position held by the caller (in a register)
DEV uint32_t ptw_draw(uint32_t *w, int &pos) {
  auto back = [&](int m) { int j = pos - m; return w[j < 0 ? j + 61 : j]; };
  const uint32_t ik = back(24) + back(55);
  const uint32_t out = ik ^ w[pos];
  w[pos] = ik;
  pos = pos == 60 ? 0 : pos + 1;
  return out;
}

__global__ __launch_bounds__(64) void pt_kernel(const int64_t *__restrict__ E,
                                                int32_t *__restrict__ slot_of_temp,
                                                int32_t *__restrict__ temp_of_slot,
                                                uint32_t *__restrict__ ptw,
                                                const uint64_t *__restrict__ F,
                                                const int32_t *__restrict__ sgn,
                                                uint64_t *__restrict__ accepts, int chains, int K) {
  const int ch = blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= chains) return;
  int32_t *so = slot_of_temp + (size_t)ch * K;
  uint32_t *w = ptw + (size_t)ch * 64;
  const int64_t *Ec = E + (size_t)ch * K;
  for (int i = 0; i + 1 < K; i++) {
    const int a = so[i], b = so[i + 1];
    const int64_t D = Ec[b] - Ec[a];
    const uint32_t r = ptw_next(w);
    const int sd = D > 0 ? 1 : (D < 0 ? -1 : 0);
    bool accept;
    if (sgn[i] * sd <= 0) {
      accept = true;
    } else {
      const uint64_t aD = (uint64_t)(D < 0 ? -D : D);
      uint64_t T = 0;
      if (aD < (1ull << 24)) {
        T = 1ull << 32;
        const uint64_t *Fi = F + (size_t)i * 24;
        for (int bb = 0; bb < 24; bb++)
          if ((aD >> bb) & 1) {
            // floor(T * F / 2^32), exact: T <= 2^32, F <= 2^32
            const uint64_t f = Fi[bb];
            T = __umul64hi(T, f) << 32 | ((T * f) >> 32);
          }
      }
      accept = (uint64_t)r < T;
    }
    if (accept) {
      so[i] = b;
      so[i + 1] = a;
      if (accepts) accepts[(size_t)ch * (K - 1) + i]++;
    }
  }
  for (int i = 0; i < K; i++) temp_of_slot[(size_t)ch * K + so[i]] = i;
}

// Fused variant: one workgroup per PT_CHAINS_PER_ITEM (at most) chains of
// one job, every job of a batch in one launch.  Wheels, energies,
// permutations, the factor table and the signs are staged in LDS, so the 31
// sequential swap decisions of a chain run on LDS latency instead of global
// memory latency.  Same decisions as pt_kernel.
// Workgroup 0 also adds min(cap[i], nsweeps) to the ncnt sweep counters
// *done[i] (the counter update of a period that ends in parallel tempering;
// nothing in the launch reads the counters).
__global__ __launch_bounds__(64) void pt_fused_kernel(const PtWork *__restrict__ works, int kmax,
                                                      uint64_t *const *__restrict__ done,
                                                      const int32_t *__restrict__ cap, int ncnt,
                                                      int nsweeps) {
  extern __shared__ uint32_t lds[];
  const PtWork w = works[blockIdx.x];
  const int t = threadIdx.x;
  if (blockIdx.x == 0)
    for (int i = t; i < ncnt; i += 64) *done[i] += (uint64_t)min(cap[i], nsweeps);
  const int K = w.K;
  uint32_t *ring = lds + t * 62;                                 // 61 words + position
  int32_t *Es = (int32_t *)(lds + 64 * 62) + t * kmax;           // energy by slot
  int32_t *so = (int32_t *)(lds + 64 * 62 + 64 * kmax) + t * kmax;  // slot by temperature
  uint64_t *Fl = (uint64_t *)(lds + 64 * 62 + 128 * kmax);       // [K-1][24]
  int32_t *sgl = (int32_t *)(Fl + (kmax - 1) * 24);              // [K-1] sign of dbeta
  uint32_t *onem = (uint32_t *)(sgl + (kmax - 1));               // [K-1] bits whose factor is 2^32
  // one staging pass: every load of the factor table (as 32-bit halves),
  // the signs and the wheels (64 words per chain in memory, 62 used),
  // energies (|E| <= 3 L^3: the low word of each int64) and permutations of
  // the workgroup's consecutive chains is issued before any is stored, so
  // the thread waits for global memory about once (not once per array and
  // chunk); each decision then reads LDS only
  const int nch = w.nchains;
  const int nF = (K - 1) * 48, nW = nch * 64, nE = nch * K;
  const uint32_t *F32 = (const uint32_t *)w.F;
  const uint32_t *gw0 = w.ptw + (size_t)w.chain0 * 64;
  const uint32_t *E0 = (const uint32_t *)(w.E + (size_t)w.chain0 * K);
  const uint32_t *S0 = (const uint32_t *)(w.slot_of_temp + (size_t)w.chain0 * K);
  constexpr int UF = (PT_FUSED_KMAX - 1) * 48 / 64 + 1, UW = PT_CHAINS_PER_ITEM,
                UE = (PT_CHAINS_PER_ITEM * PT_FUSED_KMAX + 63) / 64;
  uint32_t vF[UF], vW[UW], vE[UE], vS[UE];
  load_words<64>(nF, [&](int i) { return F32[i]; }, vF);
  const int32_t sg_t = t < K - 1 ? w.sgn[t] : 0;
  load_words<64>(nW, [&](int i) { return gw0[i]; }, vW);
  load_words<64>(nE, [&](int i) { return E0[2 * i]; }, vE);
  load_words<64>(nE, [&](int i) { return S0[i]; }, vS);
  put_words<64>(nF, vF, [&](int i, uint32_t v) { ((uint32_t *)Fl)[i] = v; });
  if (t < K - 1) sgl[t] = sg_t;
  put_words<64>(nW, vW, [&](int i, uint32_t v) {
    if ((i & 63) < 62) lds[(i >> 6) * 62 + (i & 63)] = v;
  });
  int32_t *EsAll = (int32_t *)(lds + 64 * 62);
  int32_t *soAll = (int32_t *)(lds + 64 * 62 + 64 * kmax);
  put_words<64>(nE, vE, [&](int i, uint32_t v) {
    const int c = i / K;
    EsAll[c * kmax + (i - c * K)] = (int32_t)v;
  });
  put_words<64>(nE, vS, [&](int i, uint32_t v) {
    const int c = i / K;
    soAll[c * kmax + (i - c * K)] = (int32_t)v;
  });
  __syncthreads();
  if (t < K - 1) {
    const uint32_t *Fh = (const uint32_t *)(Fl + t * 24) + 1;
    uint32_t m = 0;
    for (int bb = 0; bb < 24; bb++) m |= (Fh[2 * bb] != 0u ? 1u : 0u) << bb;
    onem[t] = m;
  }
  __syncthreads();
  if (t >= nch) return;
  const int ch = w.chain0 + t;
  uint64_t accepted = 0;  // bit i: the swap of temperatures i, i + 1 was accepted
  // the configuration at temperature i is carried upward: after step i it is
  // at i + 1 if the swap was accepted, else the one read from i + 1 is; so
  // the slot and energy read at i + 1 never depend on earlier decisions and
  // only (Sc, Ec) does
  int Sc = so[0];
  int32_t Ec = Es[Sc];
  int pos = (int)ring[61];
  for (int i = 0; i + 1 < K; i++) {
    const int a = Sc, b = so[i + 1];
    const int32_t Eb = Es[b];
    const int32_t D = Eb - Ec;
    const uint32_t r = ptw_draw(ring, pos);
    const int sd = D > 0 ? 1 : (D < 0 ? -1 : 0);
    bool accept;
    if (sgl[i] * sd <= 0) {
      accept = true;
    } else {
      const uint32_t aD = (uint32_t)(D < 0 ? -D : D);
      const uint32_t m = aD & ~onem[i];
      // |D| >= 2^24 gives T = 0
      accept = aD < (1u << 24) && (m == 0 || r < pt_threshold((const uint32_t *)(Fl + i * 24), m));
    }
    if (accept) {
      so[i] = b;
      accepted |= 1ull << i;
    } else {
      so[i] = a;
      Sc = b;
      Ec = Eb;
    }
  }
  so[K - 1] = Sc;
  ring[61] = (uint32_t)pos;
  // each counter belongs to this thread alone; atomics whose result is not
  // used leave the thread without a dependent load per accepted swap
  if (w.accepts)
    for (uint64_t m = accepted; m; m &= m - 1)
      atomicAdd((unsigned long long *)&w.accepts[(size_t)ch * (K - 1) + __ffsll((unsigned long long)m) - 1],
                1ull);
  uint32_t *gwo = w.ptw + (size_t)ch * 64;
  for (int j = 0; j < 62; j++) gwo[j] = ring[j];
  for (int k = 0; k < K; k++) {
    w.slot_of_temp[(size_t)ch * K + k] = so[k];
    w.temp_of_slot[(size_t)ch * K + so[k]] = k;
  }
}

// ---------------------------------------------------------------------------
// Next n outputs of one sweep wheel, state untouched (test hook).
// ---------------------------------------------------------------------------
__global__ void debug_rng_kernel(const uint32_t *__restrict__ wheels, uint32_t *__restrict__ out,
                                 uint64_t wstride_words, uint64_t widx, int M, uint64_t k0, int n) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t w[62];
  for (int j = 0; j < 61; j++) {
    const uint64_t kj = k0 + M - 61 + j;  // draw index k0 - 61 + j, shifted to stay >= 0
    w[j] = wheels[(kj % M) * wstride_words + widx];
  }
  w[61] = 0;
  for (int i = 0; i < n; i++) out[i] = ptw_next(w);
}

template <int ALGO>
__global__ __launch_bounds__(1024) void ising_sweep_kernel(const Work *__restrict__ works,
                                                          int nsweeps) {
  extern __shared__ __align__(16) uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  switch (w.L) {
    case 8: ising_run<8, ALGO>(w, lds); break;
    case 16: ising_run<16, ALGO>(w, lds); break;
    case 24: ising_run<24, ALGO>(w, lds); break;
    case 32: ising_run<32, ALGO>(w, lds); break;
    case 40: ising_run<40, ALGO>(w, lds); break;
    case 48: ising_run<48, ALGO>(w, lds); break;
    case 56: ising_run<56, ALGO>(w, lds); break;
    case 64: ising_run<64, ALGO>(w, lds); break;
    default: break;
  }
}

// L = 2 and 4 (blocks of 2 and 8 draws, so a register ring cycling through
// 31 and 8 block phases): a kernel of their own, so that their register
// needs do not set those of the large-lattice kernel
template <int ALGO>
__global__ __launch_bounds__(1024) void ising_small_kernel(const Work *__restrict__ works,
                                                          int nsweeps) {
  extern __shared__ __align__(16) uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  switch (w.L) {
    case 2: ising_run<2, ALGO>(w, lds); break;
    case 4: ising_run<4, ALGO>(w, lds); break;
    default: break;
  }
}

template __global__ void ising_sweep_kernel<0>(const Work *, int);
template __global__ void ising_sweep_kernel<1>(const Work *, int);
template __global__ void ising_small_kernel<0>(const Work *, int);
template __global__ void ising_small_kernel<1>(const Work *, int);

template <int ALGO>
__global__ __launch_bounds__(POTTS_MAX_TPB) void gen_sweep_kernel(const Work *__restrict__ works,
                                                                  int nsweeps) {
  extern __shared__ uint32_t lds[];
  Work w = works[blockIdx.x];
  w.nsweeps_cap = min(w.nsweeps_cap, nsweeps);
  switch (w.L) {
    case 2: gen_run<2, ALGO>(w, lds); break;
    case 4: gen_run<4, ALGO>(w, lds); break;
    case 8: gen_run<8, ALGO>(w, lds); break;
    case 16: gen_run<16, ALGO>(w, lds); break;
    case 24: gen_run<24, ALGO>(w, lds); break;
    case 32: gen_run<32, ALGO>(w, lds); break;
    case 40: gen_run<40, ALGO>(w, lds); break;
    case 48: gen_run<48, ALGO>(w, lds); break;
    case 56: gen_run<56, ALGO>(w, lds); break;
    case 64: gen_run<64, ALGO>(w, lds); break;
    default: break;
  }
}

template __global__ void gen_sweep_kernel<0>(const Work *, int);
template __global__ void gen_sweep_kernel<1>(const Work *, int);

}  // namespace sg

// ---------------------------------------------------------------------------
// Launchers used by the host library (same translation unit as the kernels).
// ---------------------------------------------------------------------------
namespace sg {

// done[j] += min(cap[j], nsweeps) for every job of a launch (sweep counters
// live on the device so that a captured graph can be replayed).
__global__ void advance_kernel(uint64_t *const *__restrict__ done, const int32_t *__restrict__ cap,
                               int n, int nsweeps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *done[i] += (uint64_t)min(cap[i], nsweeps);
}

__global__ void add_kernel(uint64_t *p, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += v;
}

hipError_t launch_add(uint64_t *p, uint64_t v, hipStream_t st) {
  hipLaunchKernelGGL(add_kernel, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_sweep(int model, int algo, const Work *d_works, int nworks, int tpb,
                        size_t lds, int nsweeps, hipStream_t st) {
  if (nworks <= 0) return hipSuccess;
  if (model == LAUNCH_POTTS_QUAD)
    hipLaunchKernelGGL(potts_quad_kernel, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == LAUNCH_GPOTTS_QUAD)
    hipLaunchKernelGGL(gpotts_quad_kernel, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == LAUNCH_POTTS_PAIR)
    hipLaunchKernelGGL(potts_pair_kernel, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == LAUNCH_GPOTTS_PAIR)
    hipLaunchKernelGGL(gpotts_pair_kernel, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == LAUNCH_ISING_SMALL && algo == 0)
    hipLaunchKernelGGL(ising_small_kernel<0>, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == LAUNCH_ISING_SMALL)
    hipLaunchKernelGGL(ising_small_kernel<1>, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == 4)
    hipLaunchKernelGGL(gpotts4_sweep_kernel, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == 3 && algo == 0)
    hipLaunchKernelGGL(gen_sweep_kernel<0>, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == 3)
    hipLaunchKernelGGL(gen_sweep_kernel<1>, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == 2)
    hipLaunchKernelGGL(gpotts_sweep_kernel, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (model == 1)
    hipLaunchKernelGGL(potts_sweep_kernel, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else if (algo == 0)
    hipLaunchKernelGGL(ising_sweep_kernel<0>, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  else
    hipLaunchKernelGGL(ising_sweep_kernel<1>, dim3(nworks), dim3(tpb), lds, st, d_works, nsweeps);
  return hipGetLastError();
}

hipError_t set_max_lds(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)potts_sweep_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)gpotts_sweep_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)potts_quad_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)gpotts_quad_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)potts_pair_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)gpotts_pair_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)gpotts4_sweep_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)gen_sweep_kernel<0>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)gen_sweep_kernel<1>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)ising_small_kernel<0>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)ising_small_kernel<1>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)ising_sweep_kernel<0>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)ising_sweep_kernel<1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_overlap(const uint32_t *spins, const int32_t *slot_of_temp, int64_t *Q, int model,
                          int L, int S, int R, int K, int copy_words, const uint32_t *occ,
                          uint32_t occ_stride, hipStream_t st) {
  if (S * K <= 0) return hipSuccess;
  hipLaunchKernelGGL(overlap_kernel, dim3(S * K), dim3(256), 0, st, spins, slot_of_temp, Q, model,
                     L, R, K, copy_words, occ, occ_stride);
  return hipGetLastError();
}

hipError_t launch_pt(const int64_t *E, int32_t *slot_of_temp, int32_t *temp_of_slot, uint32_t *ptw,
                     const uint64_t *F, const int32_t *sgn, uint64_t *accepts, int chains, int K,
                     hipStream_t st) {
  if (chains <= 0 || K < 2) return hipSuccess;
  hipLaunchKernelGGL(pt_kernel, dim3((chains + 63) / 64), dim3(64), 0, st, E, slot_of_temp,
                     temp_of_slot, ptw, F, sgn, accepts, chains, K);
  return hipGetLastError();
}

hipError_t launch_pt_fused(const PtWork *works, int nworks, int kmax, hipStream_t st,
                           uint64_t *const *done, const int32_t *cap, int ncnt, int nsweeps) {
  if (nworks <= 0) return hipSuccess;
  const size_t lds = (size_t)(64 * 62 + 128 * kmax) * 4 + (size_t)(kmax > 1 ? kmax - 1 : 1) * (24 * 8 + 8);
  hipLaunchKernelGGL(pt_fused_kernel, dim3(nworks), dim3(64), lds, st, works, kmax, done, cap, ncnt,
                     nsweeps);
  return hipGetLastError();
}

hipError_t launch_debug_rng(const uint32_t *wheels, uint32_t *out, uint64_t wstride_words,
                            uint64_t widx, int M, uint64_t k0, int n, hipStream_t st) {
  hipLaunchKernelGGL(debug_rng_kernel, dim3(1), dim3(64), 0, st, wheels, out, wstride_words, widx,
                     M, k0, n);
  return hipGetLastError();
}

hipError_t launch_advance(uint64_t *const *done, const int32_t *cap, int n, int nsweeps,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(advance_kernel, dim3((n + 63) / 64), dim3(64), 0, st, done, cap, n, nsweeps);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static scratch of the no-allocation batch run (sg_batch_run_static): the
// launch tables of a batch (work items, per-job sweep counters and caps,
// parallel-tempering work lists) go into this fixed device array instead of
// library-allocated buffers.  Each device holds its own copy until the
// process ends; host code uses only the address resolved here, never the
// array's name (on the host the name is a stand-in, not a device address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[STATIC_SCRATCH_BYTES];

// Device address of `scratch` on `device`, resolved once per device with that
// device current (the caller has made it current).
hipError_t scratch_address(int device, void **out) {
  static std::mutex mu;
  static void *addr[MAX_DEVICES] = {};
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

}  // namespace sg
