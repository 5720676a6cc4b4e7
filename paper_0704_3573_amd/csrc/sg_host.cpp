// Host side of libsg: argument checks, integer threshold tables (IEEE double,
// host only), canonical <-> device layout conversion, launch planning,
// batches replayed from captured hipGraphs.  The C-ABI is declared in
// include/sg.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "sg.h"
#include "sg_layout.h"

namespace sg {
hipError_t launch_sweep(int model, int algo, const Work *d_works, int nworks, int tpb, size_t lds,
                        int nsweeps, hipStream_t st);
hipError_t set_max_lds(int bytes);
hipError_t launch_overlap(const uint32_t *spins, const int32_t *slot_of_temp, int64_t *Q, int model,
                          int L, int S, int R, int K, int copy_words, const uint32_t *occ,
                          uint32_t occ_stride, hipStream_t st);
hipError_t launch_pt(const int64_t *E, int32_t *slot_of_temp, int32_t *temp_of_slot, uint32_t *ptw,
                     const uint64_t *F, const int32_t *sgn, uint64_t *accepts, int chains, int K,
                     hipStream_t st);
hipError_t launch_debug_rng(const uint32_t *wheels, uint32_t *out, uint64_t wstride_words,
                            uint64_t widx, int M, uint64_t k0, int n, hipStream_t st);
hipError_t launch_advance(uint64_t *const *done, const int32_t *cap, int n, int nsweeps,
                          hipStream_t st);
hipError_t launch_add(uint64_t *p, uint64_t v, hipStream_t st);
// with done != nullptr the launch also performs launch_advance(done, cap,
// ncnt, nsweeps)
hipError_t launch_pt_fused(const PtWork *works, int nworks, int kmax, hipStream_t st,
                           uint64_t *const *done = nullptr, const int32_t *cap = nullptr, int ncnt = 0,
                           int nsweeps = 0);
hipError_t scratch_address(int device, void **out);
}  // namespace sg

using sg::Geom;
using sg::PtWork;
using sg::Work;
using sg::PT_CHAINS_PER_ITEM;
using sg::PT_FUSED_KMAX;

// ---------------------------------------------------------------- errors --
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(x)                                                                    \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail(SG_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// Test hook: when the environment variable SG_TEST_INJECT_HIP_ERROR names
// an entry point that checks it, that call fails with SG_E_HIP before it
// touches any state, as if the device had reported an error.
static bool injected(const char *fn) {
  const char *e = std::getenv("SG_TEST_INJECT_HIP_ERROR");
  return e && std::strcmp(e, fn) == 0;
}
#define INJECTION_POINT()                                                               \
  if (injected(__func__))                                                               \
    return fail(SG_E_HIP, "%s: injected device error (SG_TEST_INJECT_HIP_ERROR)", __func__)

#define GUARD_BEGIN try {
#define GUARD_END                                     \
  }                                                   \
  catch (const std::bad_alloc &) {                    \
    return fail(SG_E_NOMEM, "host allocation failed"); \
  }                                                   \
  catch (...) {                                       \
    return fail(SG_E_INVALID, "internal error");      \
  }

static hipStream_t S_(void *s) { return (hipStream_t)s; }

// ---------------------------------------------------------------- tables --
// Thresholds of a number r in [0, 2^32): accepted when r < T, probability T / 2^32.
static uint64_t scaled_floor(double p, int bits) { return (uint64_t)std::floor(std::ldexp(p, bits)); }

// Ising-like models of Eq. 2: thresholds of the classes (k, phi), k = 0..12
// (see sg_layout.h), and the limits of the certain classes.  Metropolis: a
// flip of a site with s_i sum_j J x_j s_j = k - 6 changes the energy by
// dE = 2 (k - 6) + 2 field s_i f_i, phi = [s_i f_i = -1]; accepted when
// r < floor(2^32 min(1, exp(-beta dE))).  Heat bath: local field
// k - 6 + field f_i, phi = [f_i = -1]; s = +1 when r < floor(2^32 / (1 +
// exp(-2 beta h))).  The certain classes (threshold 2^32) must form a prefix
// (Metropolis) or a suffix (heat bath) of k = 0..12.
static int gen_threshold_row(int algo, double beta, double field, uint32_t row[sg::THR_WORDS]) {
  std::memset(row, 0, sizeof(uint32_t) * sg::THR_WORDS);
  for (int phi = 0; phi < 2; phi++) {
    uint64_t T[13];
    for (int k = 0; k < 13; k++) {
      const double c = (double)(k - 6);
      if (algo == SG_METROPOLIS) {
        const double dE = 2.0 * c + 2.0 * field * (phi ? -1.0 : 1.0);
        T[k] = dE <= 0.0 ? (1ull << 32) : scaled_floor(std::exp(-beta * dE), 32);
      } else {
        const double h = c + field * (phi ? -1.0 : 1.0);
        T[k] = scaled_floor(1.0 / (1.0 + std::exp(-2.0 * beta * h)), 32);
      }
    }
    int lim = 0;
    if (algo == SG_METROPOLIS) {
      while (lim < 13 && T[lim] >= (1ull << 32)) lim++;
      for (int k = lim; k < 13; k++)
        if (T[k] >= (1ull << 32)) return fail(SG_E_UNSUPPORTED, "non-monotone thresholds");
    } else {
      lim = 13;
      while (lim > 0 && T[lim - 1] >= (1ull << 32)) lim--;
      for (int k = 0; k < lim; k++)
        if (T[k] >= (1ull << 32)) return fail(SG_E_UNSUPPORTED, "non-monotone thresholds");
    }
    for (int k = 0; k < 13; k++) row[16 * phi + k] = T[k] >= (1ull << 32) ? 0u : (uint32_t)T[k];
    row[16 * phi + 13] = (uint32_t)lim;
  }
  return SG_OK;
}

// Row of THR_WORDS words for one temperature (see sg_layout.h).
static void threshold_row(int model, int algo, double beta, uint32_t row[sg::THR_WORDS]) {
  std::memset(row, 0, sizeof(uint32_t) * sg::THR_WORDS);
  uint64_t T[13];
  int n = 0;
  if (model != SG_ISING) {
    for (int d = 0; d < 13; d++) T[d] = scaled_floor(std::exp(-beta * (double)d), 28);
    n = 13;
  } else if (algo == SG_METROPOLIS) {
    // flip with n unsatisfied bonds costs dE = 12 - 4n (n = 0..2)
    for (int k = 0; k < 3; k++) T[k] = scaled_floor(std::exp(-beta * (double)(12 - 4 * k)), 32);
    n = 3;
  } else {
    // heat bath, local field h = 2k - 6: P(+1) = 1 / (1 + exp(-2 beta h))
    for (int k = 0; k < 7; k++) {
      const double h = (double)(2 * k - 6);
      T[k] = scaled_floor(1.0 / (1.0 + std::exp(-2.0 * beta * h)), 32);
    }
    n = 7;
  }
  uint32_t always = 0;
  for (int k = 0; k < n; k++) {
    if (T[k] >= (1ull << 32)) {
      row[k] = 0xFFFFFFFFu;
      always |= 1u << k;
    } else {
      row[k] = (uint32_t)T[k];
    }
  }
  if (model == SG_ISING) row[15] = always;
}

// ------------------------------------------------------------------- ctx --
// chains per fused PT work item: the decisions of a chain are sequential,
// so a launch's time is one chain's decisions plus the staging of its
// workgroup's wheels, energies and permutations; small items keep the
// staging short and spread it over many CUs

struct sg_ctx {
  int device;
  int max_lds;
  int cus;
  void *scratch;  // device address of the static scratch array on this device
};

// ------------------------------------------------------------------- job --
struct Layout {
  uint64_t spins, J, wheels, ptw, tos, sot, thr, F, sgn, E, Q, acc, done, Mf, dbg, works, ptworks, total;
  uint64_t spins_bytes, J_bytes, wheels_bytes;
};

static uint64_t al(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

static bool is_potts(int model) { return model == SG_POTTS || model == SG_GPOTTS || model == SG_GPOTTS4; }

// geometry of a model: 4D wheels for the 4D glassy Potts model, else 3D
static Geom geom_of(int model, int L) {
  if (model == SG_GPOTTS4) return sg::geom4(L);
  return model == SG_ISING || model == SG_ISING_GEN ? sg::igeom(L) : sg::geom(L);
}
// Lanes serving one copy, and the fused launch (sweep kernel) of a job: the
// 3D Potts models run several lanes per wheel where the layout allows it.
static int wheel_lanes(int model, int L) {
  return model == SG_POTTS || model == SG_GPOTTS ? sg::potts_wheel_lanes(L) : 1;
}
static int launch_group(int model, int L, int wl) {
  if (model == SG_ISING && L <= 4) return sg::LAUNCH_ISING_SMALL;
  if (wl >= 4) return model == SG_POTTS ? sg::LAUNCH_POTTS_QUAD : sg::LAUNCH_GPOTTS_QUAD;
  if (wl == 2) return model == SG_POTTS ? sg::LAUNCH_POTTS_PAIR : sg::LAUNCH_GPOTTS_PAIR;
  return model;
}

static uint64_t sites_of(int model, int L) {
  const uint64_t N = (uint64_t)L * L * L;
  return model == SG_GPOTTS4 ? N * L : N;
}

static int check_spec(const sg_job_spec *sp) {
  if (!sp) return fail(SG_E_INVALID, "spec is NULL");
  if (sp->model < SG_ISING || sp->model > SG_GPOTTS4) return fail(SG_E_INVALID, "bad model %d", sp->model);
  if (sp->algo != SG_METROPOLIS && sp->algo != SG_HEATBATH) return fail(SG_E_INVALID, "bad algo %d", sp->algo);
  if (is_potts(sp->model) && sp->algo != SG_HEATBATH)
    return fail(SG_E_UNSUPPORTED, "the Potts models are built for heat bath only");
  if (is_potts(sp->model) && sp->q != 4) return fail(SG_E_UNSUPPORTED, "Potts q must be 4");
  if (sp->model == SG_ISING_GEN) {
    if (!(sp->field >= 0.0) || std::isinf(sp->field))
      return fail(SG_E_INVALID, "field must be finite and >= 0");
    if (sp->pt_every > 0 && sp->n_temps > 1)
      return fail(SG_E_UNSUPPORTED, "no parallel tempering for the Ising-like models");
  }
  if (!sg::supported_L(sp->L)) return fail(SG_E_UNSUPPORTED, "L = %d is not built", sp->L);
  if (is_potts(sp->model) && !sg::potts_supported_L(sp->L))
    return fail(SG_E_UNSUPPORTED, "Potts L = %d is not built (L <= 48)", sp->L);
  if (sp->model == SG_GPOTTS4 && !sg::potts4_supported_L(sp->L))
    return fail(SG_E_UNSUPPORTED, "4D Potts L = %d is not built (2, 4, 8, 16)", sp->L);
  if (sp->n_samples < 1 || sp->n_replicas < 1 || sp->n_temps < 1)
    return fail(SG_E_INVALID, "S, R, K must be >= 1");
  if (sp->pt_every < 0) return fail(SG_E_INVALID, "pt_every must be >= 0");
  const uint64_t C = (uint64_t)sp->n_samples * sp->n_replicas * sp->n_temps;
  if (C > (1u << 24)) return fail(SG_E_INVALID, "too many copies");
  return SG_OK;
}

static Layout layout(const sg_job_spec *sp) {
  const Geom g = geom_of(sp->model, sp->L);
  const uint64_t S = sp->n_samples, R = sp->n_replicas, K = sp->n_temps, C = S * R * K;
  const uint64_t N = sites_of(sp->model, sp->L);
  const uint64_t K1 = K > 1 ? K - 1 : 1;
  Layout l{};
  uint64_t o = 0;
  l.spins_bytes = is_potts(sp->model) ? C * N : C * g.CS * 4;
  l.J_bytes = S * 4 *
              (uint64_t)(sp->model == SG_ISING       ? sg::ising_js(sp->L)
                         : sp->model == SG_POTTS     ? sg::potts_js(sp->L)
                         : sp->model == SG_ISING_GEN ? sg::gen_js(sp->L)
                         : sp->model == SG_GPOTTS4   ? sg::gpotts4_js(sp->L)
                                                     : sg::gpotts_js(sp->L));
  l.wheels_bytes = (uint64_t)g.M * C * g.NW * 4;
  l.spins = o; o = al(o + l.spins_bytes);
  l.J = o; o = al(o + l.J_bytes);
  l.wheels = o; o = al(o + l.wheels_bytes);
  l.ptw = o; o = al(o + S * R * 64 * 4);
  l.tos = o; o = al(o + C * 4);
  l.sot = o; o = al(o + S * R * K * 4);
  l.thr = o; o = al(o + K * sg::THR_WORDS * 4);
  l.F = o; o = al(o + K1 * 24 * 8);
  l.sgn = o; o = al(o + K1 * 4);
  l.E = o; o = al(o + C * 8);
  l.Q = o; o = al(o + S * K * 8);
  l.acc = o; o = al(o + S * R * K1 * 8);
  l.done = o; o = al(o + 8);
  l.Mf = o; o = al(o + C * 8);
  l.dbg = o; o = al(o + 4096 * 4);
  l.works = o; o = al(o + C * sizeof(Work));
  l.ptworks = o; o = al(o + ((S * R + PT_CHAINS_PER_ITEM - 1) / PT_CHAINS_PER_ITEM) * sizeof(PtWork));
  l.total = o;
  return l;
}

struct sg_job {
  sg_ctx *ctx;
  sg_job_spec sp;
  Geom g;
  int L, S, R, K, C, chains;
  uint64_t N;
  Layout lay;
  uint8_t *arena;
  std::vector<double> betas;
  std::vector<Work> works;  // host copy of the job's own launch plan
  int tpb;
  size_t lds;
  uint64_t sweeps_done;
  int wl = 1;         // lanes per wheel
  uint64_t gen = 0;   // changes of the job's launch shape (lanes per wheel)

  template <class T>
  T *at(uint64_t off) const {
    return (T *)(arena + off);
  }
  uint64_t *done_ptr() const { return at<uint64_t>(lay.done); }
  int lanes() const { return g.NW * wl; }                  // lanes per copy
  int group() const { return launch_group(sp.model, L, wl); }  // fused launch of the job
};

// lanes and LDS bytes of a work item of G copies
static size_t item_lds(const sg_job *j, int G) {
  // Ising: copies, per-copy counters (an even count of words, so that the
  // tables are 8-byte aligned), one scratch copy for lanes without a wheel
  // and the per-copy threshold tables; Potts: the
  // rotation-base table, copies, per-copy weight tables and counters, and
  // (when a wave can hold lanes without a wheel) the region those lanes
  // store into
  if (j->sp.model == SG_ISING)
    return (size_t)(G + 1) * j->g.CS * 4 + (size_t)((G + 1) & ~1) * 4 +
           (size_t)G * sg::ISING_TAB_STRIDE * 4;
  // Ising-like: copies, per-copy threshold tables and two counters, scratch copy
  if (j->sp.model == SG_ISING_GEN)
    return (size_t)(G + 1) * j->g.CS * 4 + (size_t)G * (sg::GEN_TAB_STRIDE + 2) * 4;
  if (j->sp.model == SG_GPOTTS4) {
    const size_t dummy4 = j->g.NW % 64 ? (size_t)j->g.RHO * j->L * sg::potts4_us(j->L) : 0;
    return (size_t)48 * 4 + (size_t)G * sg::potts4_lds_copy(j->L) + (size_t)G * sg::POTTS4_W_WORDS * 4 +
           (size_t)G * 4 + dummy4;
  }
  const size_t dummy = j->lanes() % 64 ? (size_t)j->g.RHO * j->L * sg::potts_xs(j->L) : 0;
  return (size_t)sg::POTTS_TAB_WORDS * 4 + (size_t)G * sg::potts_lds_copy(j->L) +
         (size_t)G * sg::POTTS_W_WORDS * 4 + (size_t)G * 4 + dummy;
}

// threads per workgroup of a launch group for a requested block size
static int model_tpb(int group, int tpb) {
  if (group == SG_ISING || group == sg::LAUNCH_ISING_SMALL) return tpb;
  if (group == sg::LAUNCH_POTTS_PAIR || group == sg::LAUNCH_GPOTTS_PAIR)
    return std::min(tpb, sg::POTTS_PAIR_MAX_TPB);
  return std::min(tpb, sg::POTTS_MAX_TPB);
}

// workgroup size of a job's items for a requested block size: the block,
// limited by the launch group, or one copy's lanes if a copy needs more
static int item_tpb(const sg_job *j, int tpb) {
  return std::max(model_tpb(j->group(), tpb), (j->lanes() + 63) / 64 * 64);
}

static int copies_per_item(const sg_job *j, int tpb) {
  int G = item_tpb(j, tpb) / j->lanes();
  G = std::min(G, j->C);
  while (G > 1 && item_lds(j, G) > (size_t)j->ctx->max_lds) G--;
  return G;
}

static void make_items(const sg_job *j, int G, std::vector<Work> &out) {
  for (int c0 = 0; c0 < j->C; c0 += G) {
    Work w{};
    w.spins = j->at<uint32_t>(j->lay.spins);
    w.J = j->at<uint32_t>(j->lay.J);
    w.wheels = j->at<uint32_t>(j->lay.wheels);
    w.temp_of_slot = j->at<int32_t>(j->lay.tos);
    w.thr = j->at<uint32_t>(j->lay.thr);
    w.E = j->at<int64_t>(j->lay.E);
    w.L = j->L;
    w.algo = j->sp.algo;
    w.model = j->sp.model;
    w.copy0 = c0;
    w.ncopies = std::min(G, j->C - c0);
    w.C = j->C;
    w.RK = j->R * j->K;
    w.nsweeps_cap = 0x7FFFFFFF;
    w.spins_bytes = (uint32_t)j->lay.spins_bytes;
    w.J_bytes = (uint32_t)j->lay.J_bytes;
    w.wheels_bytes = (uint32_t)j->lay.wheels_bytes;
    w.wl = j->wl;
    w.done = j->done_ptr();
    w.M = j->sp.model == SG_ISING_GEN ? j->at<int64_t>(j->lay.Mf) : nullptr;
    out.push_back(w);
  }
}

// Work items of one launch are dealt to the 8 XCDs round-robin by workgroup
// index, and each XCD has its own L2.  Items reading the same sample's
// couplings (consecutive in the list) are put on one XCD so that its L2
// serves the second reader: within each run of equal-size items (the list
// keeps its order), the run is cut into 8 contiguous parts and part x
// fills the run's positions p with p mod 8 = x.  Results do not depend on
// the order of the items.
static uint64_t work_size(const Work &w) { return (uint64_t)w.ncopies * w.L * w.L * w.L; }
// sites one lane of the item visits per sweep (its wheel's min(8, L) rows of
// L sites): the item's duration grows with it, whatever the item's copies
static uint64_t lane_work(const Work &w) { return (uint64_t)std::min(8, w.L) * w.L; }

static void xcd_order(std::vector<Work> &v) {
  const size_t NX = 8;
  size_t i = 0;
  while (i < v.size()) {
    size_t j = i;
    while (j < v.size() && work_size(v[j]) == work_size(v[i])) j++;
    const std::vector<Work> run(v.begin() + i, v.begin() + j);
    size_t r = 0;
    for (size_t x = 0; x < NX; x++)
      for (size_t p = i; p < j; p++)
        if (p % NX == x) v[p] = run[r++];
    i = j;
  }
}


// the job's own launch plan (job sweeps outside batches), uploaded on st
static int own_plan(sg_job *j, hipStream_t st) {
  int tpb = 512;
  if (j->lanes() > tpb) tpb = j->lanes();
  const int G = copies_per_item(j, tpb);
  if (G < 1 || item_lds(j, 1) > (size_t)j->ctx->max_lds)
    return fail(SG_E_UNSUPPORTED, "one copy of L = %d needs more LDS than the device offers", j->L);
  j->works.clear();
  make_items(j, G, j->works);
  xcd_order(j->works);
  j->tpb = ((G * j->lanes() + 63) / 64) * 64;
  j->lds = item_lds(j, G);
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.works), j->works.data(), j->works.size() * sizeof(Work),
                        hipMemcpyHostToDevice, st));
  return SG_OK;
}

static void make_pt_works(const sg_job *j, std::vector<PtWork> &out) {
  for (int c0 = 0; c0 < j->chains; c0 += PT_CHAINS_PER_ITEM) {
    PtWork w{};
    w.E = j->at<int64_t>(j->lay.E);
    w.slot_of_temp = j->at<int32_t>(j->lay.sot);
    w.temp_of_slot = j->at<int32_t>(j->lay.tos);
    w.ptw = j->at<uint32_t>(j->lay.ptw);
    w.F = j->at<uint64_t>(j->lay.F);
    w.sgn = j->at<int32_t>(j->lay.sgn);
    w.accepts = j->at<uint64_t>(j->lay.acc);
    w.chain0 = c0;
    w.nchains = std::min(PT_CHAINS_PER_ITEM, j->chains - c0);
    w.K = j->K;
    out.push_back(w);
  }
}

// --------------------------------------------------------------- packing --
// Site of bit t (draw order, 0 = most significant bit) of block word wb of
// colour p in plane z of an Ising copy: string position s = wb B + t, row
// y = s / (L/2), x = 2 (s mod L/2) + e.
struct BitSite {
  int x, y;
};
static BitSite bit_site(const Geom &g, int p, int z, int wb, int t) {
  const int s = wb * g.B + t;
  const int y = s / g.H;
  return {2 * (s % g.H) + ((p + y + z) & 1), y};
}

static void pack_ising_spins(const Geom &g, const int8_t *s, uint32_t *out) {
  const int L = g.L;
  std::memset(out, 0, sizeof(uint32_t) * g.CS);
  for (int p = 0; p < 2; p++)
    for (int z = 0; z < L; z++)
      for (int wb = 0; wb < g.NWB; wb++) {
        uint32_t word = 0;
        for (int t = 0; t < g.B; t++) {
          const BitSite b = bit_site(g, p, z, wb, t);
          if (s[b.x + L * (b.y + L * z)] < 0) word |= 1u << (g.B - 1 - t);
        }
        out[(p * L + z) * g.WZ + wb] = word;
      }
}

static void unpack_ising_spins(const Geom &g, const uint32_t *in, int8_t *s) {
  const int L = g.L;
  for (int p = 0; p < 2; p++)
    for (int z = 0; z < L; z++)
      for (int wb = 0; wb < g.NWB; wb++) {
        const uint32_t word = in[(p * L + z) * g.WZ + wb];
        for (int t = 0; t < g.B; t++) {
          const BitSite b = bit_site(g, p, z, wb, t);
          s[b.x + L * (b.y + L * z)] = ((word >> (g.B - 1 - t)) & 1u) ? -1 : 1;
        }
      }
}

// bond d of site (x, y, z): x+, x-, y+, y-, z+, z-
static int8_t bond(const int8_t *J, int L, int x, int y, int z, int d) {
  const uint64_t N = (uint64_t)L * L * L;
  auto idx = [&](int xx, int yy, int zz) { return (uint64_t)xx + L * ((uint64_t)yy + (uint64_t)L * zz); };
  switch (d) {
    case 0: return J[0 * N + idx(x, y, z)];
    case 1: return J[0 * N + idx((x + L - 1) % L, y, z)];
    case 2: return J[1 * N + idx(x, y, z)];
    case 3: return J[1 * N + idx(x, (y + L - 1) % L, z)];
    case 4: return J[2 * N + idx(x, y, z)];
    default: return J[2 * N + idx(x, y, (z + L - 1) % L)];
  }
}

static void pack_ising_J(const Geom &g, const int8_t *J, uint32_t *out) {
  const int L = g.L;
  for (int p = 0; p < 2; p++)
    for (int wb = 0; wb < g.NWB; wb++)
      for (int d = 0; d < 6; d++)
        for (int z = 0; z < L; z++) {
          uint32_t word = 0;
          for (int t = 0; t < g.B; t++) {
            const BitSite b = bit_site(g, p, z, wb, t);
            if (bond(J, L, b.x, b.y, z, d) < 0) word |= 1u << (g.B - 1 - t);
          }
          out[((p * g.NWB + wb) * 6 + d) * L + z] = word;
        }
}

// Ising-like models: D = [5][N] rows J_x, J_y, J_z, x, f -> the 14 words of
// every (colour, block word, plane) and the occupancy words in the spin-copy
// layout (see sg_layout.h)
static void pack_gen_J(const Geom &g, const int8_t *D, uint32_t *out) {
  const int L = g.L;
  const uint64_t N = (uint64_t)L * L * L;
  const int8_t *X = D + 3 * N, *F = D + 4 * N;
  auto idx = [&](int x, int y, int z) {
    return (uint64_t)((x + L) % L) + L * ((uint64_t)((y + L) % L) + (uint64_t)L * ((z + L) % L));
  };
  const int dx[6] = {1, -1, 0, 0, 0, 0}, dy[6] = {0, 0, 1, -1, 0, 0}, dz[6] = {0, 0, 0, 0, 1, -1};
  for (int p = 0; p < 2; p++)
    for (int wb = 0; wb < g.NWB; wb++)
      for (int z = 0; z < L; z++) {
        uint32_t w[sg::GEN_WORDS] = {};
        for (int t = 0; t < g.B; t++) {
          const BitSite b = bit_site(g, p, z, wb, t);
          const int x = b.x, y = b.y;
          const uint32_t bit = 1u << (g.B - 1 - t);
          for (int d = 0; d < 6; d++) {
            if (bond(D, L, x, y, z, d) < 0) w[d] |= bit;
            if (X[idx(x + dx[d], y + dy[d], z + dz[d])]) w[6 + d] |= bit;
          }
          if (X[idx(x, y, z)]) w[12] |= bit;
          if (F[idx(x, y, z)] < 0) w[13] |= bit;
        }
        for (int d = 0; d < sg::GEN_WORDS; d++)
          out[((p * g.NWB + wb) * sg::GEN_WORDS + d) * L + z] = w[d];
      }
  // occupancy in the spin layout: a copy whose spins are all -1 where occupied
  std::vector<int8_t> occ((size_t)N);
  for (uint64_t i = 0; i < N; i++) occ[i] = X[i] ? -1 : 1;
  pack_ising_spins(g, occ.data(), out + sg::gen_block_js(L));
}

// Potts: byte per site, order [y][x][z]
static uint64_t potts_idx(int L, int x, int y, int z) { return ((uint64_t)y * L + x) * L + z; }

static void pack_potts_spins(int L, const uint8_t *s, uint8_t *out) {
  for (int z = 0; z < L; z++)
    for (int y = 0; y < L; y++)
      for (int x = 0; x < L; x++) out[potts_idx(L, x, y, z)] = (uint8_t)(s[x + L * (y + L * z)] << 3);
}

static void unpack_potts_spins(int L, const uint8_t *in, uint8_t *s) {
  for (int z = 0; z < L; z++)
    for (int y = 0; y < L; y++)
      for (int x = 0; x < L; x++) s[x + L * (y + L * z)] = (uint8_t)(in[potts_idx(L, x, y, z)] >> 3);
}

// coupling pattern bytes in wheel draw order (see sg_layout.h)
static void pack_potts_J(const Geom &g, const int8_t *J, uint32_t *out) {
  const int L = g.L, BQ = sg::potts_bq(L);
  for (int p = 0; p < 2; p++)
    for (int blk = 0; blk < g.NBLK; blk++)
      for (int q = 0; q < BQ; q++)
        for (int w = 0; w < g.NW; w++) {
          const int gr = w / L, z = w % L;
          uint32_t word = 0;
          for (int b = 0; b < 4; b++) {
            const int kb = 4 * q + b;
            if (kb >= g.B) break;
            const int y = gr * g.RHO + blk * g.RPB + kb / g.H;
            const int x = 2 * (kb % g.H) + ((p + y + z) & 1);
            uint32_t pat = 0;
            for (int d = 0; d < 6; d++)
              if (bond(J, L, x, y, z, d) < 0) pat |= 1u << d;
            word |= pat << (8 * b);
          }
          out[((size_t)(p * g.NBLK + blk) * BQ + q) * g.NW + w] = word;
        }
}

// Glassy Potts: number (lexicographic order) of every permutation byte, -1 if
// the byte is not a permutation of (0, 1, 2, 3).
static void permutation_numbers(int num[256]) {
  for (int b = 0; b < 256; b++) num[b] = -1;
  int n = 0;
  for (int a = 0; a < 4; a++)
    for (int b = 0; b < 4; b++)
      for (int c = 0; c < 4; c++)
        for (int d = 0; d < 4; d++)
          if (a != b && a != c && a != d && b != c && b != d && c != d)
            num[a | b << 2 | c << 4 | d << 6] = n++;
}

// Glassy Potts couplings -> per-site words of six permutation numbers in
// wheel draw order (see sg_layout.h); P is [3][N] permutation bytes.
static void pack_gpotts_J(const Geom &g, const uint8_t *P, const int num[256], uint32_t *out) {
  const int L = g.L;
  const uint64_t N = (uint64_t)L * L * L;
  auto idx = [&](int x, int y, int z) { return (uint64_t)((x + L) % L) + L * ((uint64_t)((y + L) % L) + (uint64_t)L * ((z + L) % L)); };
  for (int p = 0; p < 2; p++)
    for (int blk = 0; blk < g.NBLK; blk++)
      for (int kb = 0; kb < g.B; kb++)
        for (int w = 0; w < g.NW; w++) {
          const int gr = w / L, z = w % L;
          const int y = gr * g.RHO + blk * g.RPB + kb / g.H;
          const int x = 2 * (kb % g.H) + ((p + y + z) & 1);
          const uint64_t own[3] = {idx(x, y, z), idx(x, y, z), idx(x, y, z)};
          const uint64_t low[3] = {idx(x - 1, y, z), idx(x, y - 1, z), idx(x, y, z - 1)};
          uint32_t word = 0;
          for (int a = 0; a < 3; a++) {
            word |= (uint32_t)num[P[a * N + own[a]]] << (5 * (2 * a));
            word |= (uint32_t)num[P[a * N + low[a]]] << (5 * (2 * a + 1));
          }
          out[((size_t)(p * g.NBLK + blk) * g.B + kb) * g.NW + w] = word;
        }
}

// 4D Potts spins: canonical i = x + L (y + L (z + L u)) -> bytes [y][u][x][z]
static uint64_t potts4_idx(int L, int x, int y, int z, int u) {
  return (((uint64_t)y * L + u) * L + x) * L + z;
}

static void pack_potts4_spins(int L, const uint8_t *s, uint8_t *out) {
  for (int u = 0; u < L; u++)
    for (int z = 0; z < L; z++)
      for (int y = 0; y < L; y++)
        for (int x = 0; x < L; x++)
          out[potts4_idx(L, x, y, z, u)] = (uint8_t)(s[x + L * (y + L * (z + (uint64_t)L * u))] << 3);
}

static void unpack_potts4_spins(int L, const uint8_t *in, uint8_t *s) {
  for (int u = 0; u < L; u++)
    for (int z = 0; z < L; z++)
      for (int y = 0; y < L; y++)
        for (int x = 0; x < L; x++)
          s[x + L * (y + L * (z + (uint64_t)L * u))] = (uint8_t)(in[potts4_idx(L, x, y, z, u)] >> 3);
}

// 4D glassy Potts couplings (P = [4][N] permutation bytes) -> two words per
// site in wheel draw order (see sg_layout.h)
static void pack_gpotts4_J(const Geom &g, const uint8_t *P, const int num[256], uint32_t *out) {
  const int L = g.L;
  const uint64_t N = (uint64_t)L * L * L * L;
  auto idx = [&](int x, int y, int z, int u) {
    return (uint64_t)((x + L) % L) +
           L * ((uint64_t)((y + L) % L) + L * ((uint64_t)((z + L) % L) + (uint64_t)L * ((u + L) % L)));
  };
  for (int p = 0; p < 2; p++)
    for (int blk = 0; blk < g.NBLK; blk++)
      for (int kb = 0; kb < g.B; kb++)
        for (int w = 0; w < g.NW; w++) {
          const int gr = w / (L * L), u = (w / L) % L, z = w % L;
          const int y = gr * g.RHO + blk * g.RPB + kb / g.H;
          const int x = 2 * (kb % g.H) + ((p + y + z + u) & 1);
          const uint64_t own = idx(x, y, z, u);
          const uint64_t low[4] = {idx(x - 1, y, z, u), idx(x, y - 1, z, u), idx(x, y, z - 1, u),
                                   idx(x, y, z, u - 1)};
          uint32_t w0 = 0, w1 = 0;
          for (int a = 0; a < 3; a++) {
            w0 |= (uint32_t)num[P[a * N + own]] << (5 * (2 * a));
            w0 |= (uint32_t)num[P[a * N + low[a]]] << (5 * (2 * a + 1));
          }
          w1 = (uint32_t)num[P[3 * N + own]] | (uint32_t)num[P[3 * N + low[3]]] << 5;
          const size_t e = ((size_t)(p * g.NBLK + blk) * g.B + kb) * g.NW + w;
          out[2 * e] = w0;
          out[2 * e + 1] = w1;
        }
}

// wheel words (oldest first) of a state that has drawn k0 numbers -> slots
static void pack_wheels(const sg_job *j, const uint32_t *wh, uint64_t k0, uint32_t *out) {
  const uint64_t M = j->g.M, NW = j->g.NW, C = j->C, stride = C * NW;
  for (uint64_t c = 0; c < C; c++)
    for (uint64_t w = 0; w < NW; w++) {
      const uint32_t *src = wh + (c * NW + w) * 61;
      for (int i = 0; i < 61; i++) {
        const uint64_t slot = (k0 + M - 61 + i) % M;  // draw index k0 - 61 + i
        out[slot * stride + c * NW + w] = src[i];
      }
    }
}

static void unpack_wheels(const sg_job *j, const uint32_t *in, uint64_t k0, uint32_t *wh) {
  const uint64_t M = j->g.M, NW = j->g.NW, C = j->C, stride = C * NW;
  for (uint64_t c = 0; c < C; c++)
    for (uint64_t w = 0; w < NW; w++) {
      uint32_t *dst = wh + (c * NW + w) * 61;
      for (int i = 0; i < 61; i++) dst[i] = in[((k0 + M - 61 + i) % M) * stride + c * NW + w];
    }
}

// Parallel-tempering factors of the pair (beta_i, beta_next):
// F[b] = floor(2^32 exp(-|dbeta| 2^b)), b < 24, and the sign of dbeta.
static void pt_factors(double bi, double bn, uint64_t F[24], int32_t *sgn) {
  const double db = bi - bn;
  *sgn = db > 0 ? 1 : (db < 0 ? -1 : 0);
  for (int b = 0; b < 24; b++) F[b] = scaled_floor(std::exp(-std::fabs(db) * std::ldexp(1.0, b)), 32);
}

static int tables_upload_host(const sg_job *j, std::vector<uint32_t> &thr, std::vector<uint64_t> &F,
                              std::vector<int32_t> &sgn) {
  const int K = j->K, K1 = K > 1 ? K - 1 : 1;
  thr.assign((size_t)K * sg::THR_WORDS, 0);
  for (int k = 0; k < K; k++) {
    uint32_t *row = &thr[(size_t)k * sg::THR_WORDS];
    if (j->sp.model == SG_ISING_GEN) {
      const int rc = gen_threshold_row(j->sp.algo, j->betas[k], j->sp.field, row);
      if (rc) return rc;
    } else {
      threshold_row(j->sp.model, j->sp.algo, j->betas[k], row);
    }
  }
  F.assign((size_t)K1 * 24, 0);
  sgn.assign((size_t)K1, 0);
  for (int i = 0; i + 1 < K; i++) pt_factors(j->betas[i], j->betas[i + 1], &F[(size_t)i * 24], &sgn[i]);
  return SG_OK;
}

static int upload_tables(sg_job *j, hipStream_t st) {
  std::vector<uint32_t> thr;
  std::vector<uint64_t> F;
  std::vector<int32_t> sgn;
  const int rc = tables_upload_host(j, thr, F, sgn);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.thr), thr.data(), thr.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.F), F.data(), F.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.sgn), sgn.data(), sgn.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return SG_OK;
}

static int check_betas(const double *betas, int K) {
  if (!betas) return fail(SG_E_INVALID, "betas is NULL");
  for (int k = 0; k < K; k++)
    if (!(betas[k] >= 0.0) || std::isinf(betas[k])) return fail(SG_E_INVALID, "beta[%d] must be finite and >= 0", k);
  return SG_OK;
}

// ------------------------------------------------------------- C-ABI ------
extern "C" {

const char *sg_last_error(void) { return g_err.c_str(); }

int32_t sg_wheels_per_copy(int32_t L) { return sg::supported_L(L) ? sg::geom(L).NW : 0; }

int32_t sg_model_wheels_per_copy(int32_t model, int32_t L) {
  if (model == SG_GPOTTS4) return sg::potts4_supported_L(L) ? sg::geom4(L).NW : 0;
  return sg_wheels_per_copy(L);
}

int sg_threshold_row(int32_t model, int32_t algo, double beta, double field, uint32_t row[32]) {
  GUARD_BEGIN
  INJECTION_POINT();
  if (!row) return fail(SG_E_INVALID, "row is NULL");
  if (model < SG_ISING || model > SG_GPOTTS4) return fail(SG_E_INVALID, "bad model %d", model);
  if (algo != SG_METROPOLIS && algo != SG_HEATBATH) return fail(SG_E_INVALID, "bad algo %d", algo);
  if (is_potts(model) && algo != SG_HEATBATH)
    return fail(SG_E_UNSUPPORTED, "the Potts models are built for heat bath only");
  if (!(beta >= 0.0) || std::isinf(beta)) return fail(SG_E_INVALID, "beta must be finite and >= 0");
  if (model == SG_ISING_GEN) {
    if (!(field >= 0.0) || std::isinf(field)) return fail(SG_E_INVALID, "field must be finite and >= 0");
    return gen_threshold_row(algo, beta, field, row);
  }
  threshold_row(model, algo, beta, row);
  return SG_OK;
  GUARD_END
}

int sg_pt_factors(double beta_i, double beta_next, uint64_t F[24], int32_t *sign) {
  if (!F || !sign) return fail(SG_E_INVALID, "NULL argument");
  if (!(beta_i >= 0.0) || !(beta_next >= 0.0) || std::isinf(beta_i) || std::isinf(beta_next))
    return fail(SG_E_INVALID, "betas must be finite and >= 0");
  pt_factors(beta_i, beta_next, F, sign);
  return SG_OK;
}

int sg_ctx_create(int device, sg_ctx **out) {
  GUARD_BEGIN
  if (!out) return fail(SG_E_INVALID, "out is NULL");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(SG_E_INVALID, "device %d of %d", device, n);
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SG_E_UNSUPPORTED, "device %d is %s, the kernels are built for gfx950", device, prop.gcnArchName);
  void *scratch = nullptr;
  HIPCHK(sg::scratch_address(device, &scratch));
  sg_ctx *c = new sg_ctx;
  c->device = device;
  c->scratch = scratch;
  c->max_lds = (int)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
  c->cus = prop.multiProcessorCount;
  if (sg::set_max_lds(c->max_lds) != hipSuccess) {
    (void)hipGetLastError();
    c->max_lds = 64 * 1024;
  }
  *out = c;
  return SG_OK;
  GUARD_END
}

int sg_ctx_destroy(sg_ctx *ctx) {
  delete ctx;
  return SG_OK;
}

int sg_job_bytes(const sg_job_spec *spec, uint64_t *bytes) {
  int rc = check_spec(spec);
  if (rc) return rc;
  if (!bytes) return fail(SG_E_INVALID, "bytes is NULL");
  *bytes = layout(spec).total;
  return SG_OK;
}

int sg_job_create(sg_ctx *ctx, const sg_job_spec *spec, const double *betas, const int8_t *J,
                  const void *spins, const uint32_t *wheels, const uint32_t *ptwheels,
                  const int32_t *slot_of_temp, uint64_t sweeps_done, void *d_arena,
                  uint64_t arena_bytes, void *stream, sg_job **out) {
  GUARD_BEGIN
  INJECTION_POINT();
  if (!ctx || !out) return fail(SG_E_INVALID, "ctx or out is NULL");
  int rc = check_spec(spec);
  if (rc) return rc;
  rc = check_betas(betas, spec->n_temps);
  if (rc) return rc;
  const Layout lay = layout(spec);
  if (!d_arena) return fail(SG_E_INVALID, "arena is NULL");
  if (arena_bytes < lay.total)
    return fail(SG_E_NOMEM, "arena of %llu bytes, job needs %llu", (unsigned long long)arena_bytes,
                (unsigned long long)lay.total);
  if (((uintptr_t)d_arena & 255) != 0) return fail(SG_E_INVALID, "arena must be 256-byte aligned");
  if (lay.spins_bytes >= (1ull << 32) || lay.wheels_bytes >= (1ull << 32) || lay.J_bytes >= (1ull << 32))
    return fail(SG_E_UNSUPPORTED, "job too large for one device buffer (split it into several jobs)");
  const uint64_t N = sites_of(spec->model, spec->L);
  const uint64_t S = spec->n_samples, R = spec->n_replicas, K = spec->n_temps, C = S * R * K;
  const uint64_t NW = (uint64_t)geom_of(spec->model, spec->L).NW;
  const bool pt = spec->pt_every > 0 && spec->n_temps > 1;
  // inputs passed as NULL come from the spec's seed
  const uint64_t rows = spec->model == SG_ISING_GEN ? 5 : spec->model == SG_GPOTTS4 ? 4 : 3;
  std::vector<int8_t> genJ;
  std::vector<uint8_t> genS;
  std::vector<uint32_t> genW, genP;
  if (!J) {
    genJ.resize(S * rows * N);
    J = genJ.data();
  }
  if (!spins) {
    genS.resize(C * N);
    spins = genS.data();
  }
  if (!wheels) {
    genW.resize(C * NW * 61);
    wheels = genW.data();
  }
  if (!ptwheels && pt) {
    genP.resize(S * R * 61);
    ptwheels = genP.data();
  }
  if (!genJ.empty() || !genS.empty() || !genW.empty() || !genP.empty()) {
    rc = sg_generate(spec, genJ.empty() ? nullptr : genJ.data(), genS.empty() ? nullptr : genS.data(),
                     genW.empty() ? nullptr : genW.data(), genP.empty() ? nullptr : genP.data());
    if (rc) return fail(rc, "instance generation failed");
  }
  // validate host inputs
  int perm_num[256];
  permutation_numbers(perm_num);
  if (spec->model == SG_GPOTTS || spec->model == SG_GPOTTS4) {
    const uint8_t *P = (const uint8_t *)J;
    for (uint64_t i = 0; i < S * rows * N; i++)
      if (perm_num[P[i]] < 0) return fail(SG_E_INVALID, "coupling byte %u is not a permutation", P[i]);
  } else if (spec->model == SG_ISING_GEN) {
    for (uint64_t s = 0; s < S; s++)
      for (uint64_t r = 0; r < 5; r++)
        for (uint64_t i = 0; i < N; i++) {
          const int8_t v = J[(s * 5 + r) * N + i];
          if (r == 3 ? (v != 0 && v != 1) : (v != 1 && v != -1))
            return fail(SG_E_INVALID, "row %d of the couplings must be %s", (int)r,
                        r == 3 ? "0 or 1" : "+1 or -1");
        }
  } else {
    for (uint64_t i = 0; i < S * 3 * N; i++)
      if (J[i] != 1 && J[i] != -1) return fail(SG_E_INVALID, "couplings must be +1 or -1");
  }
  if (!is_potts(spec->model)) {
    const int8_t *s = (const int8_t *)spins;
    for (uint64_t i = 0; i < C * N; i++)
      if (s[i] != 1 && s[i] != -1) return fail(SG_E_INVALID, "Ising spins must be +1 or -1");
  } else {
    const uint8_t *s = (const uint8_t *)spins;
    for (uint64_t i = 0; i < C * N; i++)
      if (s[i] > 3) return fail(SG_E_INVALID, "Potts spins must be in 0..3");
  }
  std::vector<int32_t> sot((size_t)S * R * K), tos((size_t)C);
  for (uint64_t ch = 0; ch < S * R; ch++) {
    std::vector<int> seen((size_t)K, 0);
    for (uint64_t k = 0; k < K; k++) {
      const int32_t v = slot_of_temp ? slot_of_temp[ch * K + k] : (int32_t)k;
      if (v < 0 || v >= (int32_t)K || seen[v]) return fail(SG_E_INVALID, "slot_of_temp is not a permutation");
      seen[v] = 1;
      sot[ch * K + k] = v;
      tos[ch * K + v] = (int32_t)k;
    }
  }

  // owned here until the job is complete: every early return frees it
  std::unique_ptr<sg_job> owner(new sg_job);
  sg_job *j = owner.get();
  j->ctx = ctx;
  j->sp = *spec;
  j->g = geom_of(spec->model, spec->L);
  j->L = spec->L;
  j->S = spec->n_samples;
  j->R = spec->n_replicas;
  j->K = spec->n_temps;
  j->C = (int)C;
  j->chains = (int)(S * R);
  j->N = N;
  j->lay = lay;
  j->arena = (uint8_t *)d_arena;
  j->betas.assign(betas, betas + K);
  j->sweeps_done = sweeps_done;
  hipStream_t st = S_(stream);
  HIPCHK(hipSetDevice(ctx->device));

  // pack on the host; every upload is ordered on the caller's stream and the
  // host buffers live until the final stream synchronisation
  std::vector<uint32_t> spw, jw, wv, pw((size_t)S * R * 64, 0);
  std::vector<uint8_t> spb;
  if (!is_potts(spec->model)) {
    spw.resize((size_t)C * j->g.CS);
    for (uint64_t c = 0; c < C; c++)
      pack_ising_spins(j->g, (const int8_t *)spins + c * N, &spw[c * j->g.CS]);
    jw.resize((size_t)lay.J_bytes / 4);
    if (spec->model == SG_ISING)
      for (uint64_t s = 0; s < S; s++) pack_ising_J(j->g, J + s * 3 * N, &jw[s * sg::ising_js(j->L)]);
    else
      for (uint64_t s = 0; s < S; s++) pack_gen_J(j->g, J + s * 5 * N, &jw[s * sg::gen_js(j->L)]);
    HIPCHK(hipMemcpyAsync(j->at<void>(lay.spins), spw.data(), lay.spins_bytes, hipMemcpyHostToDevice, st));
  } else {
    spb.resize((size_t)C * N);
    for (uint64_t c = 0; c < C; c++)
      if (spec->model == SG_GPOTTS4)
        pack_potts4_spins(j->L, (const uint8_t *)spins + c * N, &spb[c * N]);
      else
        pack_potts_spins(j->L, (const uint8_t *)spins + c * N, &spb[c * N]);
    jw.resize((size_t)lay.J_bytes / 4);
    if (spec->model == SG_POTTS) {
      for (uint64_t s = 0; s < S; s++) pack_potts_J(j->g, J + s * 3 * N, &jw[s * sg::potts_js(j->L)]);
    } else if (spec->model == SG_GPOTTS4) {
      for (uint64_t s = 0; s < S; s++)
        pack_gpotts4_J(j->g, (const uint8_t *)J + s * 4 * N, perm_num, &jw[s * sg::gpotts4_js(j->L)]);
    } else {
      for (uint64_t s = 0; s < S; s++)
        pack_gpotts_J(j->g, (const uint8_t *)J + s * 3 * N, perm_num, &jw[s * sg::gpotts_js(j->L)]);
    }
    HIPCHK(hipMemcpyAsync(j->at<void>(lay.spins), spb.data(), lay.spins_bytes, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipMemcpyAsync(j->at<void>(lay.J), jw.data(), lay.J_bytes, hipMemcpyHostToDevice, st));
  wv.assign((size_t)lay.wheels_bytes / 4, 0);
  pack_wheels(j, wheels, sweeps_done * (uint64_t)j->g.RHO * j->L, wv.data());
  HIPCHK(hipMemcpyAsync(j->at<void>(lay.wheels), wv.data(), lay.wheels_bytes, hipMemcpyHostToDevice, st));
  if (ptwheels)
    for (uint64_t ch = 0; ch < S * R; ch++) std::memcpy(&pw[ch * 64], ptwheels + ch * 61, 61 * 4);
  HIPCHK(hipMemcpyAsync(j->at<void>(lay.ptw), pw.data(), pw.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(lay.sot), sot.data(), sot.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(lay.tos), tos.data(), tos.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(lay.done), &j->sweeps_done, 8, hipMemcpyHostToDevice, st));
  std::vector<uint8_t> zero((size_t)(lay.done - lay.E), 0);  // E, Q, accepts
  HIPCHK(hipMemcpyAsync(j->at<void>(lay.E), zero.data(), zero.size(), hipMemcpyHostToDevice, st));
  j->wl = wheel_lanes(spec->model, spec->L);
  rc = own_plan(j, st);
  if (rc) return rc;
  std::vector<PtWork> ptw;
  make_pt_works(j, ptw);
  HIPCHK(hipMemcpyAsync(j->at<void>(lay.ptworks), ptw.data(), ptw.size() * sizeof(PtWork),
                        hipMemcpyHostToDevice, st));
  rc = upload_tables(j, st);  // ends with a synchronisation of the stream
  if (rc) return rc;
  *out = owner.release();
  return SG_OK;
  GUARD_END
}

int sg_job_set_betas(sg_job *job, const double *betas, void *stream) {
  GUARD_BEGIN
  if (!job) return fail(SG_E_INVALID, "job is NULL");
  int rc = check_betas(betas, job->K);
  if (rc) return rc;
  job->betas.assign(betas, betas + job->K);
  return upload_tables(job, S_(stream));
  GUARD_END
}

static int run_pt(sg_job *j, hipStream_t st) {
  if (j->K <= PT_FUSED_KMAX) {
    HIPCHK(sg::launch_pt_fused(j->at<PtWork>(j->lay.ptworks),
                               (j->chains + PT_CHAINS_PER_ITEM - 1) / PT_CHAINS_PER_ITEM, j->K, st));
    return SG_OK;
  }
  HIPCHK(sg::launch_pt(j->at<int64_t>(j->lay.E), j->at<int32_t>(j->lay.sot), j->at<int32_t>(j->lay.tos),
                       j->at<uint32_t>(j->lay.ptw), j->at<uint64_t>(j->lay.F), j->at<int32_t>(j->lay.sgn),
                       j->at<uint64_t>(j->lay.acc), j->chains, j->K, st));
  return SG_OK;
}

// own-plan sweep launch of `n` sweeps plus the counter update
static int launch_own(sg_job *j, int n, hipStream_t st) {
  HIPCHK(sg::launch_sweep(j->group(), j->sp.algo, j->at<Work>(j->lay.works), (int)j->works.size(), j->tpb,
                          j->lds, n, st));
  return SG_OK;
}

int sg_job_sweep(sg_job *job, uint64_t n_sweeps, void *stream) {
  GUARD_BEGIN
  INJECTION_POINT();
  if (!job) return fail(SG_E_INVALID, "job is NULL");
  hipStream_t st = S_(stream);
  uint64_t left = n_sweeps;
  while (left > 0) {
    uint64_t chunk = std::min<uint64_t>(left, 1u << 20);
    const int pe = job->sp.pt_every;
    if (pe > 0) chunk = std::min<uint64_t>(chunk, pe - job->sweeps_done % pe);
    int rc = launch_own(job, (int)chunk, st);
    if (rc) return rc;
    HIPCHK(sg::launch_add(job->done_ptr(), chunk, st));
    job->sweeps_done += chunk;
    left -= chunk;
    if (pe > 0 && job->sweeps_done % pe == 0 && job->K > 1) {
      rc = run_pt(job, st);
      if (rc) return rc;
    }
  }
  return SG_OK;
  GUARD_END
}

int sg_job_sweep_beta(sg_job *job, double beta, uint64_t n_sweeps, void *stream) {
  GUARD_BEGIN
  if (!job) return fail(SG_E_INVALID, "job is NULL");
  if (job->K != 1) return fail(SG_E_INVALID, "sweep(beta, n) is for jobs with one temperature (K = %d)", job->K);
  if (job->betas[0] != beta) {
    const int rc = sg_job_set_betas(job, &beta, stream);
    if (rc) return rc;
  }
  return sg_job_sweep(job, n_sweeps, stream);
  GUARD_END
}

int sg_job_measure(sg_job *job, int64_t *E, int64_t *Q, void *stream) {
  GUARD_BEGIN
  INJECTION_POINT();
  if (!job) return fail(SG_E_INVALID, "job is NULL");
  hipStream_t st = S_(stream);
  int rc = launch_own(job, 0, st);  // energy only
  if (rc) return rc;
  if (Q) {
    if (job->R < 2) return fail(SG_E_STATE, "overlaps need at least two replicas");
    const int cw = is_potts(job->sp.model) ? (int)(job->N / 4) : job->g.CS;
    const bool gen = job->sp.model == SG_ISING_GEN;
    const uint32_t *occ = gen ? job->at<uint32_t>(job->lay.J) + sg::gen_block_js(job->L) : nullptr;
    HIPCHK(sg::launch_overlap(job->at<uint32_t>(job->lay.spins), job->at<int32_t>(job->lay.sot),
                              job->at<int64_t>(job->lay.Q), job->sp.model, job->L, job->S, job->R, job->K, cw,
                              occ, gen ? (uint32_t)sg::gen_js(job->L) : 0u, st));
  }
  std::vector<int64_t> Es((size_t)job->C);
  std::vector<int32_t> sot((size_t)job->C);
  HIPCHK(hipMemcpyAsync(Es.data(), job->at<void>(job->lay.E), Es.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(sot.data(), job->at<void>(job->lay.sot), sot.size() * 4, hipMemcpyDeviceToHost, st));
  if (Q)
    HIPCHK(hipMemcpyAsync(Q, job->at<void>(job->lay.Q), (size_t)job->S * job->K * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (E)
    for (int ch = 0; ch < job->chains; ch++)
      for (int k = 0; k < job->K; k++)
        E[(size_t)ch * job->K + k] = Es[(size_t)ch * job->K + sot[(size_t)ch * job->K + k]];
  return SG_OK;
  GUARD_END
}

int sg_job_energies(sg_job *job, int64_t *E_slot, void *stream) {
  if (!job || !E_slot) return fail(SG_E_INVALID, "NULL argument");
  hipStream_t st = S_(stream);
  HIPCHK(hipMemcpyAsync(E_slot, job->at<void>(job->lay.E), (size_t)job->C * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return SG_OK;
}

int sg_job_field_sums(sg_job *job, int64_t *M, void *stream) {
  GUARD_BEGIN
  if (!job || !M) return fail(SG_E_INVALID, "NULL argument");
  if (job->sp.model != SG_ISING_GEN) return fail(SG_E_STATE, "field sums exist for the Ising-like models only");
  hipStream_t st = S_(stream);
  int rc = launch_own(job, 0, st);  // recompute from the current spins
  if (rc) return rc;
  std::vector<int64_t> Ms((size_t)job->C);
  std::vector<int32_t> sot((size_t)job->C);
  HIPCHK(hipMemcpyAsync(Ms.data(), job->at<void>(job->lay.Mf), Ms.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(sot.data(), job->at<void>(job->lay.sot), sot.size() * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int ch = 0; ch < job->chains; ch++)
    for (int k = 0; k < job->K; k++)
      M[(size_t)ch * job->K + k] = Ms[(size_t)ch * job->K + sot[(size_t)ch * job->K + k]];
  return SG_OK;
  GUARD_END
}

int sg_job_get_spins(sg_job *job, void *out, void *stream) {
  GUARD_BEGIN
  if (!job || !out) return fail(SG_E_INVALID, "NULL argument");
  hipStream_t st = S_(stream);
  std::vector<uint8_t> raw((size_t)job->lay.spins_bytes);
  HIPCHK(hipMemcpyAsync(raw.data(), job->at<void>(job->lay.spins), raw.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int c = 0; c < job->C; c++) {
    if (!is_potts(job->sp.model))
      unpack_ising_spins(job->g, (const uint32_t *)raw.data() + (size_t)c * job->g.CS, (int8_t *)out + (size_t)c * job->N);
    else if (job->sp.model == SG_GPOTTS4)
      unpack_potts4_spins(job->L, raw.data() + (size_t)c * job->N, (uint8_t *)out + (size_t)c * job->N);
    else
      unpack_potts_spins(job->L, raw.data() + (size_t)c * job->N, (uint8_t *)out + (size_t)c * job->N);
  }
  return SG_OK;
  GUARD_END
}

int sg_job_get_wheels(sg_job *job, uint32_t *wheels_out, uint32_t *ptwheels_out, void *stream) {
  GUARD_BEGIN
  if (!job) return fail(SG_E_INVALID, "job is NULL");
  hipStream_t st = S_(stream);
  if (wheels_out) {
    std::vector<uint32_t> raw((size_t)job->lay.wheels_bytes / 4);
    HIPCHK(hipMemcpyAsync(raw.data(), job->at<void>(job->lay.wheels), job->lay.wheels_bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    unpack_wheels(job, raw.data(), job->sweeps_done * (uint64_t)job->g.RHO * job->L, wheels_out);
  }
  if (ptwheels_out) {
    std::vector<uint32_t> raw((size_t)job->chains * 64);
    HIPCHK(hipMemcpyAsync(raw.data(), job->at<void>(job->lay.ptw), raw.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int ch = 0; ch < job->chains; ch++) {
      const uint32_t *w = &raw[(size_t)ch * 64];
      const uint32_t pos = w[61] % 61;
      for (int i = 0; i < 61; i++) ptwheels_out[(size_t)ch * 61 + i] = w[(pos + i) % 61];
    }
  }
  return SG_OK;
  GUARD_END
}

int sg_job_get_perm(sg_job *job, int32_t *out, void *stream) {
  if (!job || !out) return fail(SG_E_INVALID, "NULL argument");
  hipStream_t st = S_(stream);
  HIPCHK(hipMemcpyAsync(out, job->at<void>(job->lay.sot), (size_t)job->chains * job->K * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return SG_OK;
}

int sg_job_get_pt_accepts(sg_job *job, uint64_t *out, void *stream) {
  if (!job || !out) return fail(SG_E_INVALID, "NULL argument");
  hipStream_t st = S_(stream);
  const int K1 = job->K > 1 ? job->K - 1 : 1;
  HIPCHK(hipMemcpyAsync(out, job->at<void>(job->lay.acc), (size_t)job->chains * K1 * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return SG_OK;
}

int sg_job_sweeps_done(const sg_job *job, uint64_t *out) {
  if (!job || !out) return fail(SG_E_INVALID, "NULL argument");
  *out = job->sweeps_done;
  return SG_OK;
}

// ------------------------------------------------------------ checkpoint --
// Blob (8-byte items first, so every section is aligned in an aligned
// buffer): header, betas [K] (double), swap counters [S*R][max(K-1, 1)],
// energies per slot [C], canonical spins [C][N] (1 byte per site), sweep
// wheels [C][NW][61], parallel-tempering wheels [S*R][61], slot_of_temp
// [S*R][K].
struct CkHeader {
  char magic[8];
  uint32_t conventions, header_bytes;
  int32_t model, algo, q, L, S, R, K, pt_every;
  double field;
  uint64_t sweeps_done, J_digest, total_bytes;
};
static const char CK_MAGIC[8] = {'S', 'G', 'C', 'K', 'P', 'T', '0', '1'};
static const uint32_t CONVENTIONS_VERSION = 1;

static uint64_t ck_bytes(const sg_job *j) {
  const uint64_t K1 = j->K > 1 ? j->K - 1 : 1;
  return sizeof(CkHeader) + (uint64_t)j->K * 8 + (uint64_t)j->C * j->N +
         (uint64_t)j->C * j->g.NW * 61 * 4 + (uint64_t)j->chains * 61 * 4 +
         (uint64_t)j->chains * j->K * 4 + (uint64_t)j->chains * K1 * 8 + (uint64_t)j->C * 8;
}

// 64-bit FNV-1a of the job's device couplings (identifies the instance)
static int J_digest(sg_job *j, hipStream_t st, uint64_t *out) {
  std::vector<uint8_t> raw((size_t)j->lay.J_bytes);
  HIPCHK(hipMemcpyAsync(raw.data(), j->at<void>(j->lay.J), raw.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  uint64_t h = 0xcbf29ce484222325ull;
  for (uint8_t b : raw) h = (h ^ b) * 0x100000001b3ull;
  *out = h;
  return SG_OK;
}

int sg_job_checkpoint_bytes(const sg_job *job, uint64_t *bytes) {
  if (!job || !bytes) return fail(SG_E_INVALID, "NULL argument");
  *bytes = ck_bytes(job);
  return SG_OK;
}

int sg_job_checkpoint(sg_job *job, void *host_buf, uint64_t bytes, void *stream) {
  GUARD_BEGIN
  if (!job || !host_buf) return fail(SG_E_INVALID, "NULL argument");
  if (bytes < ck_bytes(job))
    return fail(SG_E_NOMEM, "checkpoint needs %llu bytes, buffer has %llu",
                (unsigned long long)ck_bytes(job), (unsigned long long)bytes);
  hipStream_t st = S_(stream);
  CkHeader h{};
  std::memcpy(h.magic, CK_MAGIC, 8);
  h.conventions = CONVENTIONS_VERSION;
  h.header_bytes = sizeof(CkHeader);
  h.model = job->sp.model;
  h.algo = job->sp.algo;
  h.q = job->sp.q;
  h.L = job->L;
  h.S = job->S;
  h.R = job->R;
  h.K = job->K;
  h.pt_every = job->sp.pt_every;
  h.field = job->sp.field;
  h.sweeps_done = job->sweeps_done;
  h.total_bytes = ck_bytes(job);
  int rc = J_digest(job, st, &h.J_digest);
  if (rc) return rc;
  uint8_t *p = (uint8_t *)host_buf;
  std::memcpy(p, &h, sizeof h);
  p += sizeof h;
  std::memcpy(p, job->betas.data(), (size_t)job->K * 8);
  p += (size_t)job->K * 8;
  rc = sg_job_get_pt_accepts(job, (uint64_t *)p, stream);
  if (rc) return rc;
  p += (size_t)job->chains * (job->K > 1 ? job->K - 1 : 1) * 8;
  rc = sg_job_energies(job, (int64_t *)p, stream);
  if (rc) return rc;
  p += (size_t)job->C * 8;
  rc = sg_job_get_spins(job, p, stream);
  if (rc) return rc;
  p += (size_t)job->C * job->N;
  uint32_t *wh = (uint32_t *)p;
  uint32_t *ptw = wh + (size_t)job->C * job->g.NW * 61;
  rc = sg_job_get_wheels(job, wh, ptw, stream);
  if (rc) return rc;
  return sg_job_get_perm(job, (int32_t *)(ptw + (size_t)job->chains * 61), stream);
  GUARD_END
}

int sg_job_restore(sg_job *j, const void *host_buf, uint64_t bytes, void *stream) {
  GUARD_BEGIN
  INJECTION_POINT();
  if (!j || !host_buf) return fail(SG_E_INVALID, "NULL argument");
  CkHeader h;
  if (bytes < sizeof h) return fail(SG_E_INVALID, "not a checkpoint (too short)");
  std::memcpy(&h, host_buf, sizeof h);
  if (std::memcmp(h.magic, CK_MAGIC, 8) != 0 || h.header_bytes != sizeof h)
    return fail(SG_E_INVALID, "not a checkpoint of this library");
  if (h.conventions != CONVENTIONS_VERSION)
    return fail(SG_E_STATE, "checkpoint of conventions version %u, library has %u", h.conventions,
                CONVENTIONS_VERSION);
  if (h.model != j->sp.model || h.algo != j->sp.algo || h.L != j->L || h.S != j->S || h.R != j->R ||
      h.K != j->K || h.pt_every != j->sp.pt_every || h.field != j->sp.field)
    return fail(SG_E_STATE, "checkpoint of another job specification");
  if (h.total_bytes != ck_bytes(j) || bytes < h.total_bytes)
    return fail(SG_E_INVALID, "checkpoint size %llu does not match the job", (unsigned long long)bytes);
  hipStream_t st = S_(stream);
  uint64_t dig = 0;
  int rc = J_digest(j, st, &dig);
  if (rc) return rc;
  if (dig != h.J_digest) return fail(SG_E_STATE, "checkpoint of other couplings");
  const uint8_t *p = (const uint8_t *)host_buf + sizeof h;
  std::vector<double> betas((size_t)j->K);
  std::memcpy(betas.data(), p, betas.size() * 8);
  rc = check_betas(betas.data(), j->K);
  if (rc) return rc;
  p += (size_t)j->K * 8;
  const int K1 = j->K > 1 ? j->K - 1 : 1;
  const uint8_t *acc = p;
  p += (size_t)j->chains * K1 * 8;
  const uint8_t *E = p;
  p += (size_t)j->C * 8;
  const uint8_t *spins = p;
  p += (size_t)j->C * j->N;
  const uint8_t *wh = p;
  p += (size_t)j->C * j->g.NW * 61 * 4;
  const uint8_t *ptw = p;
  p += (size_t)j->chains * 61 * 4;
  std::vector<int32_t> sot_in((size_t)j->chains * j->K);
  std::memcpy(sot_in.data(), p, sot_in.size() * 4);
  // validate before touching the device
  const bool ising = !is_potts(j->sp.model);
  for (uint64_t i = 0; i < (uint64_t)j->C * j->N; i++)
    if (ising ? ((int8_t)spins[i] != 1 && (int8_t)spins[i] != -1) : spins[i] > 3)
      return fail(SG_E_INVALID, "checkpoint holds invalid spins");
  std::vector<int32_t> sot((size_t)j->chains * j->K), tos((size_t)j->C);
  for (int ch = 0; ch < j->chains; ch++) {
    std::vector<int> seen((size_t)j->K, 0);
    for (int k = 0; k < j->K; k++) {
      const int32_t v = sot_in[(size_t)ch * j->K + k];
      if (v < 0 || v >= j->K || seen[v]) return fail(SG_E_INVALID, "checkpoint permutation is invalid");
      seen[v] = 1;
      sot[(size_t)ch * j->K + k] = v;
      tos[(size_t)ch * j->K + v] = k;
    }
  }
  // pack and upload, ordered on the stream
  std::vector<uint32_t> spw, wv((size_t)j->lay.wheels_bytes / 4, 0), pw((size_t)j->chains * 64, 0);
  std::vector<uint8_t> spb;
  if (ising) {
    spw.resize((size_t)j->C * j->g.CS);
    for (int c = 0; c < j->C; c++)
      pack_ising_spins(j->g, (const int8_t *)spins + (size_t)c * j->N, &spw[(size_t)c * j->g.CS]);
    HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.spins), spw.data(), j->lay.spins_bytes, hipMemcpyHostToDevice, st));
  } else {
    spb.resize((size_t)j->C * j->N);
    for (int c = 0; c < j->C; c++)
      if (j->sp.model == SG_GPOTTS4)
        pack_potts4_spins(j->L, spins + (size_t)c * j->N, &spb[(size_t)c * j->N]);
      else
        pack_potts_spins(j->L, spins + (size_t)c * j->N, &spb[(size_t)c * j->N]);
    HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.spins), spb.data(), j->lay.spins_bytes, hipMemcpyHostToDevice, st));
  }
  {
    std::vector<uint32_t> words((size_t)j->C * j->g.NW * 61);
    std::memcpy(words.data(), wh, words.size() * 4);
    pack_wheels(j, words.data(), h.sweeps_done * (uint64_t)j->g.RHO * j->L, wv.data());
  }
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.wheels), wv.data(), j->lay.wheels_bytes, hipMemcpyHostToDevice, st));
  for (int ch = 0; ch < j->chains; ch++) std::memcpy(&pw[(size_t)ch * 64], ptw + (size_t)ch * 61 * 4, 61 * 4);
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.ptw), pw.data(), pw.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.sot), sot.data(), sot.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.tos), tos.data(), tos.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.acc), acc, (size_t)j->chains * K1 * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.E), E, (size_t)j->C * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(j->at<void>(j->lay.done), &h.sweeps_done, 8, hipMemcpyHostToDevice, st));
  j->betas = betas;
  rc = upload_tables(j, st);  // ends with a synchronisation of the stream
  if (rc) return rc;
  j->sweeps_done = h.sweeps_done;
  return SG_OK;
  GUARD_END
}

int sg_job_debug_rng(sg_job *job, int32_t copy, int32_t wheel, uint32_t n, uint32_t *out, void *stream) {
  if (!job || !out) return fail(SG_E_INVALID, "NULL argument");
  if (copy < 0 || copy >= job->C || wheel < 0 || wheel >= job->g.NW || n > 4096)
    return fail(SG_E_INVALID, "copy, wheel or n out of range");
  hipStream_t st = S_(stream);
  const uint64_t stride = (uint64_t)job->C * job->g.NW;
  HIPCHK(sg::launch_debug_rng(job->at<uint32_t>(job->lay.wheels), job->at<uint32_t>(job->lay.dbg), stride,
                              (uint64_t)copy * job->g.NW + wheel, job->g.M,
                              job->sweeps_done * (uint64_t)job->g.RHO * job->L, (int)n, st));
  HIPCHK(hipMemcpyAsync(out, job->at<void>(job->lay.dbg), (size_t)n * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return SG_OK;
}

int sg_job_destroy(sg_job *job) {
  delete job;
  return SG_OK;
}

int sg_job_set_wheel_lanes(sg_job *job, int32_t lanes, void *stream) {
  GUARD_BEGIN
  if (!job) return fail(SG_E_INVALID, "job is NULL");
  const bool potts3 = job->sp.model == SG_POTTS || job->sp.model == SG_GPOTTS;
  if (!(potts3 ? sg::potts_lanes_ok(job->L, lanes) : lanes == 1))
    return fail(SG_E_INVALID, "%d lanes per wheel are not built for model %d at L = %d", (int)lanes,
                (int)job->sp.model, job->L);
  if (lanes == job->wl) return SG_OK;
  hipStream_t st = S_(stream);
  const int old = job->wl;
  job->wl = lanes;
  int rc = own_plan(job, st);
  if (rc) {
    job->wl = old;
    return rc;
  }
  job->gen++;
  HIPCHK(hipStreamSynchronize(st));
  return SG_OK;
  GUARD_END
}

int sg_job_wheel_lanes(sg_job *job, int32_t *lanes) {
  if (!job || !lanes) return fail(SG_E_INVALID, "NULL argument");
  *lanes = job->wl;
  return SG_OK;
}

}  // extern "C"

// ----------------------------------------------------------------- batch --
struct GraphKey {
  int nsw;
  std::vector<int> pt_jobs;
  bool operator<(const GraphKey &o) const {
    if (nsw != o.nsw) return nsw < o.nsw;
    return pt_jobs < o.pt_jobs;
  }
};

struct PtTable {
  PtWork *d;
  int n, kmax;
};

// One fused sweep launch of a period: the work items of one kernel (launch
// group: the five models, then the four-lanes-per-wheel Potts kernels; and
// algorithm) that run with one block size.  Items much smaller than the
// batch's block get workgroups of their own size, so that small jobs do not
// hold a large workgroup's wave slots for a few active lanes.
struct Launch {
  int group, algo, tpb;
  size_t lds;
  std::vector<Work> items;
};

struct sg_batch {
  sg_ctx *ctx;
  std::vector<sg_job *> jobs;
  std::vector<uint64_t> budget;  // remaining sweeps per job (UINT64_MAX = unlimited)
  std::vector<uint64_t> pcap;    // sweeps per run per job (UINT64_MAX = unlimited)
  std::vector<int32_t> run_cap;  // sweeps each job runs in the current period
  int block_req = 0;  // 0 = automatic
  // plan
  bool dirty = true;
  std::vector<uint64_t> gens;     // the jobs' launch shapes the plan was made for
  int tpb = 0;                    // the batch's block size
  std::vector<Launch> launches;   // fused launches of a period
  Work *d_items = nullptr;
  size_t d_items_cap = 0;
  uint64_t **d_done = nullptr;
  int32_t *d_cap = nullptr;
  size_t d_jobs_cap = 0;
  std::map<GraphKey, hipGraphExec_t> graphs;
  std::map<GraphKey, int> seen;  // periods launched directly per key since the last plan
  std::vector<void *> graph_bufs;  // device buffers referenced by captured graphs
  std::map<std::vector<int>, PtTable> pt_cache;
  hipStream_t cap_stream = nullptr;
  std::vector<hipStream_t> side;  // streams of the concurrent launches
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  bool timing = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the fused sweep launch
  bool ran = false;                // periods have been enqueued ...
  hipStream_t last_stream = nullptr;  // ... on this stream (by the last run)
  // host copy of the launch tables of the no-allocation run (uploaded into
  // the static device scratch; kept until the next call has waited for the
  // periods of this one)
  struct Static {
    std::vector<Launch> launches;
    int tpb = 0;
    std::vector<uint64_t *> done;
    std::vector<int32_t> cap;
    std::vector<PtWork> pt;                 // fused PT work of every PT job, job after job
    std::vector<int> pt_first, pt_count;    // per job (count 0: none or K > 64)
  } stat;
};

static void drop_graphs(sg_batch *b) {
  for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
  b->seen.clear();
  for (void *p : b->graph_bufs) (void)hipFree(p);
  b->graph_bufs.clear();
  b->pt_cache.clear();
}

// idle-lane fraction of a block size for the batch's jobs (lower is better)
static double idle_fraction(const sg_batch *b, int tpb) {
  double used = 0, total = 0;
  for (sg_job *j : b->jobs) {
    if (j->lanes() > tpb) return 2.0;
    const int G = copies_per_item(j, tpb);
    if (G < 1) return 2.0;
    const double items = std::ceil((double)j->C / G);
    const double per_lane = (double)j->g.RHO / j->wl;  // draws per lane, in L/2
    used += (double)j->C * j->lanes() * per_lane;
    total += items * item_tpb(j, tpb) * per_lane;
  }
  return total > 0 ? 1.0 - used / total : 0.0;
}

// Plan of the current membership.  Periods already enqueued (on the stream
// of the last run) may still read the launch tables and the parallel-
// tempering tables, so a re-plan first waits for them: the caller may add
// and remove jobs between runs without synchronising.
static int wait_enqueued(sg_batch *b) {
  if (b->ran) HIPCHK(hipStreamSynchronize(b->last_stream));
  return SG_OK;
}

// Host part of a plan: block size and the fused launches (work items
// longest first, XCD-aware order; each launch's LDS bytes).
static int plan_items(const sg_batch *b, int &tpb_out, std::vector<Launch> &launches) {
  int tpb = b->block_req;
  if (tpb <= 0) {
    double best = 3;
    for (int t = 64; t <= 1024; t += 64) {
      const double f = idle_fraction(b, t);
      if (f < best - 1e-9) {
        best = f;
        tpb = t;
      }
    }
    if (tpb <= 0) return fail(SG_E_UNSUPPORTED, "no block size fits the batch");
  }
  std::map<std::tuple<int, int, int>, Launch> by_key;
  for (sg_job *j : b->jobs) {
    const int G = copies_per_item(j, tpb);
    int blk = item_tpb(j, tpb);
    const int need = (G * j->lanes() + 63) / 64 * 64;
    if (need <= blk / 2) blk = need;
    Launch &l = by_key[std::make_tuple(j->group(), j->sp.algo, blk)];
    l.group = j->group();
    l.algo = j->sp.algo;
    l.tpb = blk;
    l.lds = std::max(l.lds, item_lds(j, G));
    make_items(j, G, l.items);
  }
  launches.clear();
  for (auto &kv : by_key) {
    Launch &l = kv.second;
    // longest items first (most sites per lane, then most sites): the launch
    // tail is then made of short items
    std::stable_sort(l.items.begin(), l.items.end(), [](const Work &x, const Work &y) {
      return lane_work(x) != lane_work(y) ? lane_work(x) > lane_work(y) : work_size(x) > work_size(y);
    });
    xcd_order(l.items);
    launches.push_back(std::move(l));
  }
  tpb_out = tpb;
  return SG_OK;
}

// a job of the batch changed its launch shape since the plan was made
static bool shapes_changed(const sg_batch *b) {
  if (b->gens.size() != b->jobs.size()) return true;
  for (size_t i = 0; i < b->jobs.size(); i++)
    if (b->jobs[i]->gen != b->gens[i]) return true;
  return false;
}

static int plan(sg_batch *b) {
  if (!b->dirty && !shapes_changed(b)) return SG_OK;
  int rc = wait_enqueued(b);
  if (rc) return rc;
  drop_graphs(b);
  int tpb = 0;
  rc = plan_items(b, tpb, b->launches);
  if (rc) return rc;
  size_t total = 0;
  for (auto &l : b->launches) total += l.items.size();
  // device tables grow geometrically: a serving loop adds jobs one by one,
  // and every hipFree waits for the whole device
  if (total > b->d_items_cap) {
    const size_t cap = std::max<size_t>({total, 2 * b->d_items_cap, 256});
    if (b->d_items) HIPCHK(hipFree(b->d_items));
    b->d_items = nullptr;
    HIPCHK(hipMalloc(&b->d_items, cap * sizeof(Work)));
    b->d_items_cap = cap;
  }
  size_t off = 0;
  for (auto &l : b->launches) {
    if (!l.items.empty())
      HIPCHK(hipMemcpy(b->d_items + off, l.items.data(), l.items.size() * sizeof(Work), hipMemcpyHostToDevice));
    off += l.items.size();
  }
  // one capture branch per launch beyond the first
  while (b->side.size() + 1 < b->launches.size()) {
    hipStream_t sst;
    hipEvent_t ev;
    HIPCHK(hipStreamCreateWithFlags(&sst, hipStreamNonBlocking));
    b->side.push_back(sst);
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    b->join.push_back(ev);
  }
  if (b->jobs.size() > b->d_jobs_cap) {
    const size_t cap = std::max<size_t>({b->jobs.size(), 2 * b->d_jobs_cap, 64});
    if (b->d_done) HIPCHK(hipFree(b->d_done));
    if (b->d_cap) HIPCHK(hipFree(b->d_cap));
    b->d_done = nullptr;
    b->d_cap = nullptr;
    HIPCHK(hipMalloc(&b->d_done, cap * sizeof(uint64_t *)));
    HIPCHK(hipMalloc(&b->d_cap, cap * sizeof(int32_t)));
    b->d_jobs_cap = cap;
  }
  std::vector<uint64_t *> done;
  std::vector<int32_t> cap;
  for (sg_job *j : b->jobs) {
    done.push_back(j->done_ptr());
    cap.push_back(0x7FFFFFFF);
  }
  if (!done.empty()) {
    HIPCHK(hipMemcpy(b->d_done, done.data(), done.size() * sizeof(uint64_t *), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_cap, cap.data(), cap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  b->run_cap.assign(b->jobs.size(), 0x7FFFFFFF);
  b->tpb = tpb;
  b->gens.clear();
  for (sg_job *j : b->jobs) b->gens.push_back(j->gen);
  b->dirty = false;
  return SG_OK;
}

// sweeps job i may still run in one run call (UINT64_MAX = no limit)
static uint64_t limit(const sg_batch *b, size_t i) { return std::min(b->budget[i], b->pcap[i]); }

static void account(sg_batch *b, uint64_t chunk) {
  for (size_t i = 0; i < b->jobs.size(); i++) {
    const uint64_t ran = std::min<uint64_t>(chunk, limit(b, i));
    b->jobs[i]->sweeps_done += ran;
    if (b->budget[i] != UINT64_MAX) b->budget[i] -= ran;
  }
}

// per-job sweep caps of one period; uploads item and counter caps if changed
static int apply_caps(sg_batch *b, uint64_t chunk, hipStream_t st) {
  std::vector<int32_t> cap(b->jobs.size());
  bool changed = false;
  for (size_t i = 0; i < b->jobs.size(); i++) {
    const uint64_t c = std::min<uint64_t>(chunk, limit(b, i));
    cap[i] = limit(b, i) == UINT64_MAX ? 0x7FFFFFFF : (int32_t)c;
    if (cap[i] != b->run_cap[i]) changed = true;
  }
  if (!changed) return SG_OK;
  (void)st;
  int rc = wait_enqueued(b);  // earlier periods may still read the tables
  if (rc) return rc;
  b->run_cap = cap;
  // items carry the job's arena pointers; find the job by its counter
  std::map<const uint64_t *, int32_t> by_counter;
  for (size_t i = 0; i < b->jobs.size(); i++) by_counter[b->jobs[i]->done_ptr()] = cap[i];
  size_t off = 0;
  for (auto &l : b->launches) {
    for (Work &w : l.items) w.nsweeps_cap = by_counter[w.done];
    if (!l.items.empty())
      HIPCHK(hipMemcpy(b->d_items + off, l.items.data(), l.items.size() * sizeof(Work), hipMemcpyHostToDevice));
    off += l.items.size();
  }
  HIPCHK(hipMemcpy(b->d_cap, cap.data(), cap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return SG_OK;
}

// enqueue one period: fused sweep launches, counters, due PT steps
static int enqueue_period(sg_batch *b, int nsw, const std::vector<int> &pt_jobs, hipStream_t st) {
  size_t off = 0;
  const bool capturing = st == b->cap_stream;
  const bool timed = b->timing && !capturing;
  if (timed) HIPCHK(hipEventRecord(b->ev0, st));
  // the fused launches run concurrently: side streams forked from and joined
  // back to the caller's stream (while capturing, parallel branches of the
  // graph).  A batch whose membership changes often (serving) launches its
  // periods directly, and one launch after another would last as long as the
  // sum of the launches' durations rather than the longest.
  const bool fork = b->launches.size() > 1;
  if (fork) HIPCHK(hipEventRecord(b->fork, st));
  for (size_t g = 0; g < b->launches.size(); g++) {
    const Launch &l = b->launches[g];
    hipStream_t s = st;
    if (fork && g > 0) {
      s = b->side[g - 1];
      HIPCHK(hipStreamWaitEvent(s, b->fork, 0));
    }
    HIPCHK(sg::launch_sweep(l.group, l.algo, b->d_items + off, (int)l.items.size(), l.tpb, l.lds, nsw, s));
    if (fork && g > 0) {
      HIPCHK(hipEventRecord(b->join[g - 1], s));
      HIPCHK(hipStreamWaitEvent(st, b->join[g - 1], 0));
    }
    off += l.items.size();
  }
  if (timed) HIPCHK(hipEventRecord(b->ev1, st));
  // parallel tempering of every due job in one fused launch (buffers prepared
  // before any capture starts), which also advances the sweep counters; a
  // period without it advances them in a launch of their own
  auto it = b->pt_cache.find(pt_jobs);
  const bool fused_pt = it != b->pt_cache.end() && it->second.n > 0;
  if (!fused_pt) HIPCHK(sg::launch_advance(b->d_done, b->d_cap, (int)b->jobs.size(), nsw, st));
  for (int ji : pt_jobs)
    if (b->jobs[ji]->K > PT_FUSED_KMAX) {
      int rc = run_pt(b->jobs[ji], st);
      if (rc) return rc;
    }
  if (fused_pt)
    HIPCHK(sg::launch_pt_fused(it->second.d, it->second.n, it->second.kmax, st, b->d_done, b->d_cap,
                               (int)b->jobs.size(), nsw));
  return SG_OK;
}

// device table of the fused PT launch for a set of due jobs
static int prepare_pt(sg_batch *b, const std::vector<int> &pt_jobs) {
  if (b->pt_cache.count(pt_jobs)) return SG_OK;
  std::vector<PtWork> pw;
  int kmax = 2;
  for (int ji : pt_jobs) {
    sg_job *j = b->jobs[ji];
    if (j->K > PT_FUSED_KMAX) continue;
    kmax = std::max(kmax, j->K);
    make_pt_works(j, pw);
  }
  PtTable t{nullptr, (int)pw.size(), kmax};
  if (!pw.empty()) {
    HIPCHK(hipMalloc(&t.d, pw.size() * sizeof(PtWork)));
    b->graph_bufs.push_back(t.d);
    HIPCHK(hipMemcpy(t.d, pw.data(), pw.size() * sizeof(PtWork), hipMemcpyHostToDevice));
  }
  b->pt_cache.emplace(pt_jobs, t);
  return SG_OK;
}

// capture stream, side streams and events of a new batch
static int batch_streams(sg_batch *b) {
  HIPCHK(hipSetDevice(b->ctx->device));
  HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  return SG_OK;
}

extern "C" {

int sg_batch_create(sg_ctx *ctx, sg_job *const *jobs, int32_t n, sg_batch **out) {
  GUARD_BEGIN
  if (!ctx || !out) return fail(SG_E_INVALID, "NULL argument");
  if (n < 0 || (n > 0 && !jobs)) return fail(SG_E_INVALID, "bad job list");
  sg_batch *b = new sg_batch;
  b->ctx = ctx;
  int rc = batch_streams(b);
  for (int32_t i = 0; rc == SG_OK && i < n; i++) rc = sg_batch_add(b, jobs[i]);
  if (rc) {
    const std::string msg = g_err;
    sg_batch_destroy(b);  // releases whatever was created
    g_err = msg;
    return rc;
  }
  *out = b;
  return SG_OK;
  GUARD_END
}

int sg_batch_add(sg_batch *b, sg_job *job) {
  GUARD_BEGIN
  if (!b || !job) return fail(SG_E_INVALID, "NULL argument");
  if (job->ctx != b->ctx) return fail(SG_E_INVALID, "job belongs to another context");
  if (std::find(b->jobs.begin(), b->jobs.end(), job) != b->jobs.end())
    return fail(SG_E_STATE, "job is already in the batch");
  b->jobs.push_back(job);
  b->budget.push_back(UINT64_MAX);
  b->pcap.push_back(UINT64_MAX);
  b->dirty = true;
  return SG_OK;
  GUARD_END
}

int sg_batch_remove(sg_batch *b, sg_job *job) {
  GUARD_BEGIN
  if (!b || !job) return fail(SG_E_INVALID, "NULL argument");
  auto it = std::find(b->jobs.begin(), b->jobs.end(), job);
  if (it == b->jobs.end()) return fail(SG_E_STATE, "job is not in the batch");
  b->budget.erase(b->budget.begin() + (it - b->jobs.begin()));
  b->pcap.erase(b->pcap.begin() + (it - b->jobs.begin()));
  b->jobs.erase(it);
  b->dirty = true;
  return SG_OK;
  GUARD_END
}

int sg_batch_set_budget(sg_batch *b, sg_job *job, uint64_t sweeps) {
  if (!b || !job) return fail(SG_E_INVALID, "NULL argument");
  auto it = std::find(b->jobs.begin(), b->jobs.end(), job);
  if (it == b->jobs.end()) return fail(SG_E_STATE, "job is not in the batch");
  if (sweeps != UINT64_MAX && job->sp.pt_every > 0 && job->K > 1)
    return fail(SG_E_INVALID, "sweep budgets are for jobs without parallel tempering");
  b->budget[it - b->jobs.begin()] = sweeps;
  return SG_OK;
}

int sg_batch_set_period_cap(sg_batch *b, sg_job *job, uint64_t sweeps) {
  if (!b || !job) return fail(SG_E_INVALID, "NULL argument");
  auto it = std::find(b->jobs.begin(), b->jobs.end(), job);
  if (it == b->jobs.end()) return fail(SG_E_STATE, "job is not in the batch");
  if (sweeps != UINT64_MAX && job->sp.pt_every > 0 && job->K > 1)
    return fail(SG_E_INVALID, "per-run caps are for jobs without parallel tempering");
  b->pcap[it - b->jobs.begin()] = sweeps;
  return SG_OK;
}

int sg_batch_get_budget(sg_batch *b, sg_job *job, uint64_t *sweeps) {
  if (!b || !job || !sweeps) return fail(SG_E_INVALID, "NULL argument");
  auto it = std::find(b->jobs.begin(), b->jobs.end(), job);
  if (it == b->jobs.end()) return fail(SG_E_STATE, "job is not in the batch");
  *sweeps = b->budget[it - b->jobs.begin()];
  return SG_OK;
}

int sg_batch_set_block(sg_batch *b, int32_t threads) {
  if (!b) return fail(SG_E_INVALID, "batch is NULL");
  if (threads != 0 && (threads < 64 || threads > 1024 || threads % 64 != 0))
    return fail(SG_E_INVALID, "block must be 0 or a multiple of 64 in [64, 1024]");
  b->block_req = threads;
  b->dirty = true;
  return SG_OK;
}

int sg_batch_block(sg_batch *b, int32_t *threads) {
  if (!b || !threads) return fail(SG_E_INVALID, "NULL argument");
  int rc = plan(b);
  if (rc) return rc;
  *threads = b->tpb;
  return SG_OK;
}

int sg_batch_run(sg_batch *b, uint64_t n_sweeps, void *stream) {
  GUARD_BEGIN
  INJECTION_POINT();
  if (!b) return fail(SG_E_INVALID, "batch is NULL");
  if (b->jobs.empty() || n_sweeps == 0) return SG_OK;
  hipStream_t st = S_(stream);
  // periods enqueued by earlier runs on another stream are waited for here;
  // those on `st` are waited for wherever the tables change
  if (b->ran && b->last_stream != st) HIPCHK(hipStreamSynchronize(b->last_stream));
  b->last_stream = st;
  b->ran = true;
  int rc = plan(b);
  if (rc) return rc;
  uint64_t left = n_sweeps;
  while (left > 0) {
    uint64_t chunk = std::min<uint64_t>(left, 1u << 20);
    for (sg_job *j : b->jobs)
      if (j->sp.pt_every > 0 && j->K > 1)
        chunk = std::min<uint64_t>(chunk, j->sp.pt_every - j->sweeps_done % j->sp.pt_every);
    GraphKey key;
    key.nsw = (int)chunk;
    for (size_t i = 0; i < b->jobs.size(); i++) {
      sg_job *j = b->jobs[i];
      if (j->sp.pt_every > 0 && j->K > 1 && (j->sweeps_done + chunk) % j->sp.pt_every == 0)
        key.pt_jobs.push_back((int)i);
    }
    rc = prepare_pt(b, key.pt_jobs);
    if (rc) return rc;
    rc = apply_caps(b, chunk, st);
    if (rc) return rc;
    if (b->timing) {
      // timing mode: the same period enqueued directly on the caller's stream,
      // with events around the fused sweep launch
      rc = enqueue_period(b, key.nsw, key.pt_jobs, st);
      if (rc) return rc;
      account(b, chunk);
      left -= chunk;
      continue;
    }
    auto it = b->graphs.find(key);
    if (it == b->graphs.end() && b->seen[key]++ == 0) {
      // first period with this membership and shape: launch directly; a graph
      // is captured only once the same period recurs (serving changes
      // membership often, the batched campaign repeats one period)
      rc = enqueue_period(b, key.nsw, key.pt_jobs, st);
      if (rc) return rc;
      account(b, chunk);
      left -= chunk;
      continue;
    }
    if (it == b->graphs.end()) {
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      rc = enqueue_period(b, key.nsw, key.pt_jobs, b->cap_stream);
      hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
      if (rc) return rc;
      if (e != hipSuccess) return fail(SG_E_HIP, "graph capture: %s", hipGetErrorString(e));
      hipGraphExec_t ge;
      e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(SG_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
      it = b->graphs.emplace(key, ge).first;
    }
    HIPCHK(hipGraphLaunch(it->second, st));
    account(b, chunk);
    left -= chunk;
  }
  return SG_OK;
  GUARD_END
}

// No-allocation run: the launch tables live in the static device scratch,
// laid out [work items][job sweep counters][job caps][parallel-tempering
// work], each part 256-byte aligned; periods are enqueued directly (no graph).
int sg_batch_run_static(sg_batch *b, uint64_t n_sweeps, void *stream) {
  GUARD_BEGIN
  INJECTION_POINT();
  if (!b) return fail(SG_E_INVALID, "batch is NULL");
  if (b->jobs.empty() || n_sweeps == 0) return SG_OK;
  if (!b->ctx->scratch) return fail(SG_E_STATE, "the context has no scratch address");
  hipStream_t st = S_(stream);
  // this batch's earlier periods may still read the scratch and the host
  // tables uploaded from: wait for them before rewriting either
  if (b->ran) HIPCHK(hipStreamSynchronize(b->last_stream));
  b->last_stream = st;
  b->ran = true;
  auto &T = b->stat;
  int rc = plan_items(b, T.tpb, T.launches);
  if (rc) return rc;
  const size_t nj = b->jobs.size();
  size_t nitems = 0;
  for (auto &l : T.launches) nitems += l.items.size();
  T.pt.clear();
  T.pt_first.assign(nj, 0);
  T.pt_count.assign(nj, 0);
  for (size_t i = 0; i < nj; i++) {
    sg_job *j = b->jobs[i];
    if (j->sp.pt_every > 0 && j->K > 1 && j->K <= PT_FUSED_KMAX) {
      T.pt_first[i] = (int)T.pt.size();
      make_pt_works(j, T.pt);
      T.pt_count[i] = (int)T.pt.size() - T.pt_first[i];
    }
  }
  const uint64_t off_done = al(nitems * sizeof(Work));
  const uint64_t off_cap = al(off_done + nj * sizeof(uint64_t *));
  const uint64_t off_pt = al(off_cap + nj * sizeof(int32_t));
  const uint64_t total = off_pt + T.pt.size() * sizeof(PtWork);
  if (total > sg::STATIC_SCRATCH_BYTES)
    return fail(SG_E_NOMEM, "the batch's launch tables need %llu bytes, the static scratch holds %llu "
                "(split the batch, or use sg_batch_run)", (unsigned long long)total,
                (unsigned long long)sg::STATIC_SCRATCH_BYTES);
  uint8_t *base = (uint8_t *)b->ctx->scratch;
  Work *d_items = (Work *)base;
  uint64_t **d_done = (uint64_t **)(base + off_done);
  int32_t *d_cap = (int32_t *)(base + off_cap);
  PtWork *d_pt = (PtWork *)(base + off_pt);
  T.done.clear();
  for (sg_job *j : b->jobs) T.done.push_back(j->done_ptr());
  HIPCHK(hipMemcpyAsync(d_done, T.done.data(), nj * sizeof(uint64_t *), hipMemcpyHostToDevice, st));
  if (!T.pt.empty())
    HIPCHK(hipMemcpyAsync(d_pt, T.pt.data(), T.pt.size() * sizeof(PtWork), hipMemcpyHostToDevice, st));
  T.cap.clear();
  uint64_t left = n_sweeps;
  while (left > 0) {
    uint64_t chunk = std::min<uint64_t>(left, 1u << 20);
    for (sg_job *j : b->jobs)
      if (j->sp.pt_every > 0 && j->K > 1)
        chunk = std::min<uint64_t>(chunk, j->sp.pt_every - j->sweeps_done % j->sp.pt_every);
    // per-job sweep caps of this period; the item table is (re)written when
    // they change, after the periods reading it have finished
    std::vector<int32_t> cap(nj);
    for (size_t i = 0; i < nj; i++)
      cap[i] = limit(b, i) == UINT64_MAX ? 0x7FFFFFFF : (int32_t)std::min<uint64_t>(chunk, limit(b, i));
    if (cap != T.cap) {
      if (!T.cap.empty()) HIPCHK(hipStreamSynchronize(st));
      T.cap = cap;
      std::map<const uint64_t *, int32_t> by_counter;
      for (size_t i = 0; i < nj; i++) by_counter[b->jobs[i]->done_ptr()] = cap[i];
      size_t off = 0;
      for (auto &l : T.launches) {
        for (Work &w : l.items) w.nsweeps_cap = by_counter[w.done];
        if (!l.items.empty())
          HIPCHK(hipMemcpyAsync(d_items + off, l.items.data(), l.items.size() * sizeof(Work),
                                hipMemcpyHostToDevice, st));
        off += l.items.size();
      }
      HIPCHK(hipMemcpyAsync(d_cap, T.cap.data(), nj * sizeof(int32_t), hipMemcpyHostToDevice, st));
    }
    const int nsw = (int)chunk;
    size_t off = 0;
    for (const Launch &l : T.launches) {
      HIPCHK(sg::launch_sweep(l.group, l.algo, d_items + off, (int)l.items.size(), l.tpb, l.lds, nsw, st));
      off += l.items.size();
    }
    HIPCHK(sg::launch_advance(d_done, d_cap, (int)nj, nsw, st));
    // parallel tempering of the jobs due after this period: fused launches
    // over runs of consecutive due jobs, the unfused kernel for K > 64
    size_t i = 0;
    while (i < nj) {
      sg_job *j = b->jobs[i];
      const bool due = j->sp.pt_every > 0 && j->K > 1 && (j->sweeps_done + chunk) % j->sp.pt_every == 0;
      if (!due) {
        i++;
        continue;
      }
      if (T.pt_count[i] == 0) {
        rc = run_pt(j, st);
        if (rc) return rc;
        i++;
        continue;
      }
      size_t e = i;
      int kmax = 2, n = 0;
      while (e < nj && T.pt_count[e] > 0 &&
             (b->jobs[e]->sweeps_done + chunk) % b->jobs[e]->sp.pt_every == 0) {
        kmax = std::max(kmax, b->jobs[e]->K);
        n += T.pt_count[e];
        e++;
      }
      HIPCHK(sg::launch_pt_fused(d_pt + T.pt_first[i], n, kmax, st));
      i = e;
    }
    account(b, chunk);
    left -= chunk;
  }
  return SG_OK;
  GUARD_END
}

int sg_batch_set_timing(sg_batch *b, int32_t enable) {
  GUARD_BEGIN
  if (!b) return fail(SG_E_INVALID, "batch is NULL");
  if (enable && !b->ev0) {
    HIPCHK(hipEventCreate(&b->ev0));
    HIPCHK(hipEventCreate(&b->ev1));
  }
  b->timing = enable != 0;
  b->dirty = true;
  return SG_OK;
  GUARD_END
}

int sg_batch_sweep_ms(sg_batch *b, float *ms) {
  if (!b || !ms) return fail(SG_E_INVALID, "NULL argument");
  if (!b->timing) return fail(SG_E_STATE, "timing is off");
  HIPCHK(hipEventSynchronize(b->ev1));
  HIPCHK(hipEventElapsedTime(ms, b->ev0, b->ev1));
  return SG_OK;
}

int sg_batch_destroy(sg_batch *b) {
  if (!b) return SG_OK;
  drop_graphs(b);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_done) (void)hipFree(b->d_done);
  if (b->d_cap) (void)hipFree(b->d_cap);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (hipStream_t sst : b->side) (void)hipStreamDestroy(sst);
  for (hipEvent_t ev : b->join) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
  return SG_OK;
}

}  // extern "C"
