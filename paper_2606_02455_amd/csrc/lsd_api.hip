// lsd_api.hip -- host implementation of the C ABI in include/lsd.h.
//
// Owns no device memory: every device array lives in the caller's workspace
// (laid out here) or in the caller's state/output buffers.  Enforces the
// call order draft -> verify -> accept of one synchronous window (Alg. 1
// with lookahead K, per-step maps of Alg. 2).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "lsd.h"
#include "fit.h"
#include "lsd_launch.h"
#include "mpnn.h"
#include "net.h"

namespace {

thread_local std::string g_err;

lsd_status fail(lsd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(LSD_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LSD_TRY(expr)                 \
  do {                                \
    lsd_status s_ = (expr);           \
    if (s_ != LSD_OK) return s_;      \
  } while (0)

enum State { ST_READY = 0, ST_DRAFTED = 1, ST_VERIFIED = 2, ST_COMMITTED = 3 };

constexpr size_t kAlign = 256;
constexpr int kTimingRing = 512;

struct Layout {
  size_t total = 0;
  // static tables
  size_t atom_rep, species, rep_off, box, rep_nc, rep_cell_off;
  size_t tile_start, tile_count, tile_rep, rep_tile_off;
  // cells and lists
  size_t cell_rep, cell_count, cell_start, cell_cursor, cell_unsorted, cell_atoms, atom_cell;
  size_t nbr_t, cnt_t, nbr_d, cnt_d, qref, qwrap, rebuild;
  // window
  size_t qmid, p, fd, ft, invalid, nvalid, rej, partial, commit_frame, reflected, coef, counters, status;
  size_t tail_bar;
  size_t ec = 0, ec_prev = 0, ec_samples = 0;  // error-correction caches (0: off)
  size_t mpnn = 0, mpnn_bytes = 0;
  size_t net_v = 0;  // learned draft: edge coefficients [N][LSD_NET_MAX_BASIS]
  bool has_mpnn = false;
  int mt = 0, md = 0, n_cells = 0, n_tiles = 0, cell_cap = 0;
  double rl_t = 0, rl_d = 0;
  std::vector<int> atom_rep_h, rep_nc_h, rep_cell_off_h, tile_start_h, tile_count_h, tile_rep_h,
      rep_tile_off_h, cell_rep_h;
};

size_t bump(size_t* off, size_t bytes) {
  size_t o = (*off + kAlign - 1) / kAlign * kAlign;
  *off = o + bytes;
  return o;
}

bool is_binary32(double v) { return (double)(float)v == v; }

int round_up(int v, int m) { return (v + m - 1) / m * m; }

double pot_reach(const lsd_potential& P) {
  return (P.kind == LSD_POT_LJ || P.kind == LSD_POT_MPNN || P.kind == LSD_POT_PAIR ||
          P.kind == LSD_POT_NET)
             ? P.cutoff
             : 0.0;
}


lsd_status check_potential(const lsd_potential& P, const char* what) {
  if (P.kind == LSD_POT_LJ) {
    if (!(P.cutoff > 0.0) || !(P.sigma > 0.0) || !std::isfinite(P.epsilon))
      return fail(LSD_ERR_INVALID_ARG, "%s: Lennard-Jones needs cutoff > 0, sigma > 0", what);
  } else if (P.kind == LSD_POT_HARMONIC) {
    if (!P.anchor || !(P.k_spring >= 0.0))
      return fail(LSD_ERR_INVALID_ARG, "%s: tether needs anchors and k >= 0", what);
  } else if (P.kind == LSD_POT_MPNN) {
    if (!(P.cutoff > 0.0) || !P.weights || P.n_model_species < 1 || !std::isfinite(P.energy_scale))
      return fail(LSD_ERR_INVALID_ARG, "%s: network needs cutoff > 0, weights, species", what);
  } else if (P.kind == LSD_POT_PAIR) {
    if (!(P.cutoff > 0.0) || !P.weights || P.n_model_species < 1 ||
        P.n_model_species > LSD_MAX_SPECIES || P.n_basis < 1 || P.n_basis > LSD_PAIR_MAX_BASIS)
      return fail(LSD_ERR_INVALID_ARG, "%s: pair draft needs cutoff > 0, weights, 1..%d species "
                  "and 1..%d basis functions", what, LSD_MAX_SPECIES, LSD_PAIR_MAX_BASIS);
  } else if (P.kind == LSD_POT_NET) {
    if (!(P.cutoff > 0.0) || !P.weights || P.n_model_species < 1 ||
        P.n_model_species > LSD_NET_MAX_SPECIES || P.n_basis < 1 ||
        P.n_basis > LSD_NET_MAX_BASIS || P.n_model_species * P.n_basis > LSD_NET_MAX_DESC)
      return fail(LSD_ERR_INVALID_ARG, "%s: learned draft needs cutoff > 0, weights, 1..%d "
                  "species, 1..%d radial functions and species x functions <= %d", what,
                  LSD_NET_MAX_SPECIES, LSD_NET_MAX_BASIS, LSD_NET_MAX_DESC);
    if (P.precision != LSD_PREC_FP32 && P.precision != LSD_PREC_BF16 &&
        P.precision != LSD_PREC_FP8)
      return fail(LSD_ERR_INVALID_ARG, "%s: precision %d invalid", what, P.precision);
    if (P.precision == LSD_PREC_FP8 &&
        !(P.act_amax[0] > 0.0 && P.act_amax[1] > 0.0 && std::isfinite(P.act_amax[0]) &&
          std::isfinite(P.act_amax[1])))
      return fail(LSD_ERR_INVALID_ARG, "%s: FP8 needs calibrated activation maxima > 0", what);
  } else {
    return fail(LSD_ERR_UNSUPPORTED, "%s: potential kind %d not supported", what, P.kind);
  }
  return LSD_OK;
}

// Validates the configuration and computes the workspace layout.
lsd_status plan(const lsd_config* c, Layout* L) {
  if (!c) return fail(LSD_ERR_INVALID_ARG, "null config");
  const int N = c->n_atoms, R = c->n_replicas;
  if (N < 1 || N > (1 << 27)) return fail(LSD_ERR_INVALID_ARG, "n_atoms %d outside 1..2^27", N);
  if (R < 1 || R > (1 << 23)) return fail(LSD_ERR_INVALID_ARG, "n_replicas %d invalid", R);
  if (!c->atom_offsets || !c->box || !c->species_mass)
    return fail(LSD_ERR_INVALID_ARG, "atom_offsets, box and species_mass are required");
  if (c->atom_offsets[0] != 0 || c->atom_offsets[R] != N)
    return fail(LSD_ERR_INVALID_ARG, "atom_offsets must start at 0 and end at n_atoms");
  if (c->n_species < 1 || c->n_species > LSD_MAX_SPECIES)
    return fail(LSD_ERR_INVALID_ARG, "n_species must be 1..%d", LSD_MAX_SPECIES);
  for (int s = 0; s < c->n_species; ++s)
    if (!(c->species_mass[s] > 0.0)) return fail(LSD_ERR_INVALID_ARG, "mass of species %d <= 0", s);
  if (c->species)
    for (int i = 0; i < N; ++i)
      if (c->species[i] < 0 || c->species[i] >= c->n_species)
        return fail(LSD_ERR_INVALID_ARG, "species[%d] out of range", i);
  if (!(c->dt > 0.0) || !(c->gamma > 0.0) || !(c->kT > 0.0) || !(c->force_unit > 0.0))
    return fail(LSD_ERR_INVALID_ARG, "dt, gamma, kT and force_unit must be > 0");
  if (!(c->skin > 0.0)) return fail(LSD_ERR_INVALID_ARG, "skin must be > 0");
  if (c->k_max < 1 || c->k_max > LSD_MAX_K)
    return fail(LSD_ERR_INVALID_ARG, "k_max %d outside 1..%d", c->k_max, LSD_MAX_K);
  if (c->mode != LSD_MODE_LSD && c->mode != LSD_MODE_PLAIN)
    return fail(LSD_ERR_INVALID_ARG, "mode %d invalid", c->mode);
  if (c->error_correction < 0 || c->error_correction > 2)
    return fail(LSD_ERR_INVALID_ARG, "error_correction %d outside 0..2", c->error_correction);
  if (c->integrator != LSD_INTEGRATOR_ABOBA && c->integrator != LSD_INTEGRATOR_OBABO)
    return fail(LSD_ERR_INVALID_ARG, "integrator %d invalid", c->integrator);
  LSD_TRY(check_potential(c->target, "target"));
  if (c->mode == LSD_MODE_LSD) LSD_TRY(check_potential(c->draft, "draft"));
  if (c->mode == LSD_MODE_LSD && c->draft.kind == LSD_POT_MPNN)
    return fail(LSD_ERR_UNSUPPORTED, "the message-passing network is supported as target only");
  if (c->target.kind == LSD_POT_PAIR || c->target.kind == LSD_POT_NET)
    return fail(LSD_ERR_UNSUPPORTED, "the pair and learned drafts are supported as drafts only");
  if (c->mode == LSD_MODE_LSD && c->draft.kind == LSD_POT_NET &&
      c->draft.n_model_species < c->n_species)
    return fail(LSD_ERR_INVALID_ARG, "learned draft has %d species, system has %d",
                c->draft.n_model_species, c->n_species);
  if (c->mode == LSD_MODE_LSD && c->draft.kind == LSD_POT_PAIR &&
      c->draft.n_model_species < c->n_species)
    return fail(LSD_ERR_INVALID_ARG, "pair draft has %d species, system has %d",
                c->draft.n_model_species, c->n_species);
  if (c->target.kind == LSD_POT_MPNN && c->target.n_model_species < c->n_species)
    return fail(LSD_ERR_INVALID_ARG, "network embeds %d species, system has %d",
                c->target.n_model_species, c->n_species);

  L->rl_t = pot_reach(c->target) + c->skin;
  L->rl_d = (c->mode == LSD_MODE_LSD ? pot_reach(c->draft) : 0.0) + c->skin;
  const double r_cell = std::max(L->rl_t, L->rl_d);

  L->atom_rep_h.resize(N);
  L->rep_nc_h.resize(R);
  L->rep_cell_off_h.resize(R);
  L->rep_tile_off_h.assign(R + 1, 0);
  L->tile_start_h.clear();
  L->tile_count_h.clear();
  L->tile_rep_h.clear();
  L->cell_rep_h.clear();
  L->cell_cap = 1;
  double rho_max = 0.0;
  long long cells = 0;
  for (int r = 0; r < R; ++r) {
    const int a0 = c->atom_offsets[r], a1 = c->atom_offsets[r + 1];
    if (a1 <= a0) return fail(LSD_ERR_INVALID_ARG, "replica %d has no atoms", r);
    const double Lr = c->box[r];
    if (!(Lr > 0.0) || !is_binary32(Lr))
      return fail(LSD_ERR_INVALID_ARG, "box[%d] = %.17g must be > 0 and binary32", r, Lr);
    if (!(Lr > r_cell))
      return fail(LSD_ERR_INVALID_ARG, "box[%d] = %g must exceed cutoff + skin = %g", r, Lr, r_cell);
    const int n_r = a1 - a0;
    rho_max = std::max(rho_max, n_r / (Lr * Lr * Lr));
    int nc = (int)std::floor(Lr / (r_cell * (1.0 + 1e-6)));
    nc = std::min(nc, std::max(1, (int)std::cbrt((double)n_r)));
    if (nc < 3) nc = 1;
    L->rep_nc_h[r] = nc;
    L->rep_cell_off_h[r] = (int)cells;
    cells += (long long)nc * nc * nc;
    if (cells > (1ll << 30)) return fail(LSD_ERR_INVALID_ARG, "too many cells");
    L->cell_rep_h.insert(L->cell_rep_h.end(), (size_t)nc * nc * nc, r);
    // occupancy the list builder covers: the whole replica for a single
    // cell, else 2.5x the mean occupancy plus 32 (exceeding it is reported)
    const int cap = nc == 1 ? n_r : (int)std::ceil(2.5 * n_r / ((double)nc * nc * nc) + 32.0);
    L->cell_cap = std::max(L->cell_cap, cap);
    for (int i = a0; i < a1; ++i) L->atom_rep_h[i] = r;
    L->rep_tile_off_h[r] = (int)L->tile_start_h.size();
    for (int t = a0; t < a1; t += LSD_TILE) {
      L->tile_start_h.push_back(t);
      L->tile_count_h.push_back(std::min(LSD_TILE, a1 - t));
      L->tile_rep_h.push_back(r);
    }
  }
  L->rep_tile_off_h[R] = (int)L->tile_start_h.size();
  L->n_cells = (int)cells;
  L->n_tiles = (int)L->tile_start_h.size();

  auto auto_width = [&](double rl) {
    const double expect = rho_max * 4.0 / 3.0 * M_PI * rl * rl * rl;
    return round_up((int)std::ceil(1.3 * expect + 32.0), 32);
  };
  L->mt = c->max_neighbors_target > 0 ? c->max_neighbors_target : auto_width(L->rl_t);
  L->md = c->max_neighbors_draft > 0 ? c->max_neighbors_draft : auto_width(L->rl_d);
  if (L->mt > 600) return fail(LSD_ERR_CAPACITY, "target neighbour width %d > 600", L->mt);
  if (L->md > 4096) return fail(LSD_ERR_CAPACITY, "draft neighbour width %d > 4096", L->md);

  const size_t n = (size_t)N, K = (size_t)c->k_max, T = (size_t)L->n_tiles;
  size_t off = 0;
  L->atom_rep = bump(&off, n * 4);
  L->species = bump(&off, n * 4);
  L->rep_off = bump(&off, (R + 1) * 4);
  L->box = bump(&off, R * 8);
  L->rep_nc = bump(&off, R * 4);
  L->rep_cell_off = bump(&off, R * 4);
  L->tile_start = bump(&off, T * 4);
  L->tile_count = bump(&off, T * 4);
  L->tile_rep = bump(&off, T * 4);
  L->rep_tile_off = bump(&off, (R + 1) * 4);
  L->cell_rep = bump(&off, (size_t)L->n_cells * 4);
  L->cell_count = bump(&off, (size_t)L->n_cells * 4);
  L->cell_start = bump(&off, ((size_t)L->n_cells + 1) * 4);
  L->cell_cursor = bump(&off, (size_t)L->n_cells * 4);
  L->cell_unsorted = bump(&off, n * 4);
  L->cell_atoms = bump(&off, n * 4);
  L->atom_cell = bump(&off, n * 4);
  L->nbr_t = bump(&off, (size_t)L->mt * n * 4);
  L->cnt_t = bump(&off, n * 4);
  L->nbr_d = bump(&off, (size_t)L->md * n * 4);
  L->cnt_d = bump(&off, n * 4);
  L->qref = bump(&off, n * 16);
  L->qwrap = bump(&off, n * 16);
  L->rebuild = bump(&off, (size_t)R * 4);
  L->qmid = bump(&off, K * n * 16);
  L->p = bump(&off, (K + 1) * 3 * n * 4);
  L->fd = bump(&off, K * 3 * n * 4);
  L->ft = bump(&off, K * 3 * n * 4);
  L->invalid = bump(&off, (size_t)R * K * 4);
  L->nvalid = bump(&off, 4);
  L->rej = bump(&off, (size_t)R * 4);
  L->partial = bump(&off, K * T * 4 * 8);
  L->commit_frame = bump(&off, R * 4);
  L->reflected = bump(&off, R * 4);
  L->coef = bump(&off, R * 8);
  L->counters = bump(&off, (size_t)R * LSD_NCOUNT * 8);
  L->status = bump(&off, 4 * 4);
  L->tail_bar = bump(&off, 4);
  if (c->error_correction && c->mode == LSD_MODE_LSD) {
    L->ec = bump(&off, 3 * n * 4);
    L->ec_samples = bump(&off, (size_t)R * 4);
    if (c->error_correction == 2) L->ec_prev = bump(&off, 3 * n * 4);
  }
  if (c->mode == LSD_MODE_LSD && c->draft.kind == LSD_POT_NET)
    L->net_v = bump(&off, n * LSD_NET_MAX_BASIS * 4);
  L->has_mpnn = c->target.kind == LSD_POT_MPNN;
  if (L->has_mpnn) {
    L->mpnn_bytes = mpnn_buffer_bytes(c->k_max, N, L->mt);
    L->mpnn = bump(&off, L->mpnn_bytes);
  }
  L->total = (off + kAlign - 1) / kAlign * kAlign;
  return LSD_OK;
}

PotDev make_pot(const lsd_potential& P, const Layout& L) {
  PotDev d;
  memset(&d, 0, sizeof(d));
  d.kind = P.kind;
  d.offset = P.force_offset;
  if (P.kind == LSD_POT_LJ) {
    const double rc = P.cutoff, rc2 = rc * rc;
    // the binary32 separation has relative error <= 4u per component, so
    // |r2_binary32 - r2| <= 12u r2 to first order (u = 2^-24); the band
    // rc2 (1 -+ 32u) hands every closer call to the binary64 predicate
    const double u = std::ldexp(1.0, -24);
    d.rc2_d = rc2;
    d.rc2 = (float)rc2;
    d.rc2_lo = (float)(rc2 * (1.0 - 32.0 * u));
    d.rc2_hi = (float)(rc2 * (1.0 + 32.0 * u));
    d.eps4 = (float)(4.0 * P.epsilon);
    d.eps24 = (float)(24.0 * P.epsilon);
    d.sig2 = (float)(P.sigma * P.sigma);
    const double src = P.sigma / rc;
    const double src6 = src * src * src * src * src * src;
    d.eshift = (float)(4.0 * P.epsilon * (src6 * src6 - src6));
  } else if (P.kind == LSD_POT_HARMONIC) {
    d.kspring = (float)P.k_spring;
    d.anchor = P.anchor;
  } else if (P.kind == LSD_POT_PAIR || P.kind == LSD_POT_NET) {
    d.rc2 = (float)(P.cutoff * P.cutoff);
    d.pi_rc = (float)(M_PI / P.cutoff);
    d.nb = P.n_basis;
    d.ns = P.n_model_species;
    d.w = P.weights;
    d.prec = P.kind == LSD_POT_NET ? P.precision : 0;
    if (P.kind == LSD_POT_NET && P.precision == LSD_PREC_FP8) {
      d.fp8_sD = (float)(P.act_amax[0] / 448.0);
      d.fp8_sh = (float)(P.act_amax[1] / 448.0);
    }
  }
  return d;
}

struct TimingRing {
  hipEvent_t start[kTimingRing], stop[kTimingRing];
  int head = 0, used = 0;
  bool created = false;
};

}  // namespace

// Error text for the host-only parts of the library in other files.
lsd_status lsd_record_error(lsd_status s, const char* msg) { return fail(s, "%s", msg); }

// Executable graphs of one window, per window length K: the whole window,
// or (when the verification launch is timed) the parts before and after it.
struct WindowGraphs {
  // full: a whole window; with verification timing, the kernels before the
  // verification (pre), after it (post), and post of one window followed
  // by pre of the next (mid), so that one graph launch sits between two
  // timed verifications
  hipGraphExec_t full = nullptr, pre = nullptr, post = nullptr, mid = nullptr;
};

struct lsd_system {
  lsd_config cfg;
  lsd_buffers buf;
  Layout lay;
  SysDev S;
  ListDev Lst;
  WinDev W;
  TileDev T;
  OutDev O;
  PotDev Pt, Pd;
  int state = ST_READY;

  bool timing = false;
  int timing_every = 1;      // time every n-th verification launch
  int64_t timing_seq = 0;    // verification launches since timing was set
  TimingRing ring;
  double t_sum = 0.0;
  int64_t t_count = 0;
  bool use_graphs = true;
  MpnnCtx mp;
  bool has_mpnn = false;
  hipStream_t cap_stream = nullptr;
  std::map<int, WindowGraphs> graphs;
  hipEvent_t graphs_done = nullptr;  // recorded after the last graph replay
  std::map<int, int> tuned_fw;  // frames per wave of the verification kernel, by K
  // pipelined windows: frames per verification group (0: synchronous
  // windows), the second stream and the fork/join events
  int pipe_group = 0;
  int draft_tail = 3;  // first draft step of the one-launch chain (0: one launch per step)
  hipStream_t side_stream = nullptr;
  hipEvent_t pipe_ev[LSD_MAX_K + 1] = {};
  std::map<int, hipGraphExec_t> pipe_graphs;
};

namespace {

// frames per wave of the verification kernel for windows of K frames: the
// autotuned (or fixed) choice if any, else 2 (1 for single frames)
int verify_fw(const lsd_system* s, int K) {
  auto it = s->tuned_fw.find(K);
  if (it != s->tuned_fw.end()) return it->second;
  return K >= 2 ? 2 : 1;
}

template <typename T>
T* ws(const lsd_system* s, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(s->buf.workspace) + off);
}

lsd_status upload_ints(const std::vector<int>& v, int* dst, hipStream_t st) {
  if (v.empty()) return LSD_OK;
  HIP_TRY(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, st));
  return LSD_OK;
}

lsd_status timing_drain_one(lsd_system* s) {
  TimingRing& R = s->ring;
  HIP_TRY(hipEventSynchronize(R.stop[R.head]));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, R.start[R.head], R.stop[R.head]));
  s->t_sum += ms;
  s->t_count += 1;
  R.head = (R.head + 1) % kTimingRing;
  R.used -= 1;
  return LSD_OK;
}

// Waits for the last replay to finish before the executable graphs go.
void destroy_graphs(lsd_system* s) {
  if (s->graphs_done && (!s->graphs.empty() || !s->pipe_graphs.empty()))
    (void)hipEventSynchronize(s->graphs_done);
  for (auto& kv : s->graphs) {
    if (kv.second.full) (void)hipGraphExecDestroy(kv.second.full);
    if (kv.second.pre) (void)hipGraphExecDestroy(kv.second.pre);
    if (kv.second.post) (void)hipGraphExecDestroy(kv.second.post);
    if (kv.second.mid) (void)hipGraphExecDestroy(kv.second.mid);
  }
  s->graphs.clear();
  for (auto& kv : s->pipe_graphs)
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  s->pipe_graphs.clear();
}

enum Part { PART_FULL = 0, PART_PRE = 1, PART_POST = 2, PART_MID = 3 };

// Network-target forces of frame k of a plain window into the draft force
// slot (k_draft then steps with them).
lsd_status enqueue_plain_mpnn(lsd_system* s, int k, hipStream_t st) {
  char err[256];
  if (!mpnn_eval(s->mp, s->S, s->Lst, s->W, k, 1, nullptr, s->W.fd, st, err, sizeof(err)))
    return fail(LSD_ERR_HIP, "network forces: %s", err);
  return LSD_OK;
}

// The verification launch(es) of frames [fb, fe) of a drafted window: the
// pair kernel with its fused transport-map epilogue, or the batched network
// evaluation of those frames (the valid ones) followed by the transport-map
// sums.
lsd_status enqueue_verify_range(lsd_system* s, int K, int fb, int fe, hipStream_t st) {
  if (s->has_mpnn) {
    char err[256];
    if (!mpnn_eval(s->mp, s->S, s->Lst, s->W, fb, fe - fb, s->W.nvalid, s->W.ft, st, err,
                   sizeof(err)))
      return fail(LSD_ERR_HIP, "network forces: %s", err);
    HIP_TRY(launch_transport(s->S, s->W, s->T, s->mp.b.Erow, fb, fe, st));
  } else {
    HIP_TRY(launch_verify(s->S, s->Lst, s->W, s->T, s->Pt, verify_fw(s, K), fb, fe, st));
  }
  return LSD_OK;
}

lsd_status enqueue_verify(lsd_system* s, int K, hipStream_t st) {
  return enqueue_verify_range(s, K, 0, K, st);
}

// One pipelined window (Alg. 2 on one GPU): the draft chain runs on `a`;
// each group of pipe_group drafted frames is verified on `b` as soon as its
// last frame is drafted, and its decisions record the first rejection, after
// which the remaining draft and verification launches of the window find no
// frame to work on.  The window ends on `a` with the decision over all kept
// frames and the commit (fused with the next window's start).  With
// `timed`, HIP events bracket every verification launch on `b`.
lsd_status enqueue_pipelined(lsd_system* s, int K, hipStream_t a, hipStream_t b, bool timed) {
  const int G = s->pipe_group;
  s->W.K = K;
  HIP_TRY(launch_build_lists(s->S, s->Lst, s->W, false, a));
  int fb = 0, g = 0;
  for (int k = 0; k < K; ++k) {
    if (s->Pd.kind == LSD_POT_NET) HIP_TRY(launch_net_nodes(s->S, s->Lst, s->W, s->Pd, k, a));
    HIP_TRY(launch_draft(s->S, s->Lst, s->W, s->T, s->Pd, k, 0, a));
    if (k + 1 - fb < G && k + 1 < K) continue;
    HIP_TRY(hipEventRecord(s->pipe_ev[g], a));
    HIP_TRY(hipStreamWaitEvent(b, s->pipe_ev[g], 0));
    int slot = -1;
    if (timed) {
      TimingRing& R = s->ring;
      if (R.used == kTimingRing) LSD_TRY(timing_drain_one(s));
      slot = (R.head + R.used) % kTimingRing;
      HIP_TRY(hipEventRecord(R.start[slot], b));
    }
    LSD_TRY(enqueue_verify_range(s, K, fb, k + 1, b));
    if (timed) {
      HIP_TRY(hipEventRecord(s->ring.stop[slot], b));
      s->ring.used += 1;
    }
    HIP_TRY(launch_decide_group(s->S, s->W, s->T, fb, k + 1, b));
    fb = k + 1;
    ++g;
  }
  HIP_TRY(hipEventRecord(s->pipe_ev[LSD_MAX_K], b));
  HIP_TRY(hipStreamWaitEvent(a, s->pipe_ev[LSD_MAX_K], 0));
  HIP_TRY(launch_decide_commit_start(s->S, s->Lst, s->W, s->T, s->O, s->buf.q, s->buf.p,
                                     s->buf.img, 0, a));
  return LSD_OK;
}

lsd_status pipeline_resources(lsd_system* s) {
  if (!s->side_stream) HIP_TRY(hipStreamCreateWithFlags(&s->side_stream, hipStreamNonBlocking));
  for (int i = 0; i <= LSD_MAX_K; ++i)
    if (!s->pipe_ev[i]) HIP_TRY(hipEventCreateWithFlags(&s->pipe_ev[i], hipEventDisableTiming));
  return LSD_OK;
}

lsd_status capture_pipelined(lsd_system* s, int K, hipGraphExec_t* out) {
  if (!s->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  LSD_TRY(pipeline_resources(s));
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
  const lsd_status e = enqueue_pipelined(s, K, s->cap_stream, s->side_stream, false);
  const std::string enqueue_err = e != LSD_OK ? g_err : std::string();
  hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
  if (e != LSD_OK || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (e != LSD_OK) return fail(e, "pipelined window capture: %s", enqueue_err.c_str());
    return fail(LSD_ERR_HIP, "pipelined window capture: %s", hipGetErrorString(e2));
  }
  hipError_t e3 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(LSD_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e3));
  return LSD_OK;
}

// The window's draft steps on `st`: one launch per step (two with the
// learned draft's node pass), or, where draft_tail_fits and windows are
// synchronous, steps draft_tail .. K-1 in one launch.  Plain stepping (every
// step drafted) takes the one-launch chain only where it needs no grid
// barrier (one block).
lsd_status enqueue_drafts(lsd_system* s, int K, hipStream_t st) {
  const bool plain = s->cfg.mode == LSD_MODE_PLAIN;
  const bool tail = s->draft_tail > 0 && s->pipe_group == 0 && !(plain && s->has_mpnn) &&
                    draft_tail_fits(s->S, plain ? s->Pt : s->Pd) && (!plain || s->S.n_tiles == 1);
  const int k0 = tail ? s->draft_tail : K;
  for (int k = 0; k < K; ++k) {
    if (plain && s->has_mpnn) {
      // plain stepping with the network: its forces on frame k, then the step
      LSD_TRY(enqueue_plain_mpnn(s, k, st));
      HIP_TRY(launch_draft(s->S, s->Lst, s->W, s->T, s->Pt, k, 1, st, 1));
      continue;
    }
    if (k == k0) {
      HIP_TRY(launch_draft_tail(s->S, s->Lst, s->W, s->T, plain ? s->Pt : s->Pd, k0, plain ? 1 : 0,
                                st));
      break;
    }
    if (!plain && s->Pd.kind == LSD_POT_NET)
      HIP_TRY(launch_net_nodes(s->S, s->Lst, s->W, s->Pd, k, st));
    HIP_TRY(launch_draft(s->S, s->Lst, s->W, s->T, plain ? s->Pt : s->Pd, k, plain ? 1 : 0, st));
  }
  return LSD_OK;
}

// Enqueues the kernels of one window part of lsd_run_windows on `st` (no
// state checks).  A part begins at the list kernels: the window's start
// (k_window_start) is fused into the previous window's commit, and the first
// window of a call is started by a separate launch before the replays.
lsd_status enqueue_part(lsd_system* s, int K, int part, hipStream_t st) {
  const bool plain = s->cfg.mode == LSD_MODE_PLAIN;
  s->W.K = K;
  if (part == PART_MID) {
    LSD_TRY(enqueue_part(s, K, PART_POST, st));
    return enqueue_part(s, K, PART_PRE, st);
  }
  if (part == PART_FULL || part == PART_PRE) {
    HIP_TRY(launch_build_lists(s->S, s->Lst, s->W, false, st));
    LSD_TRY(enqueue_drafts(s, K, st));
  }
  if (part == PART_FULL && !plain) LSD_TRY(enqueue_verify(s, K, st));
  if (part == PART_FULL || part == PART_POST) {
    HIP_TRY(launch_decide_commit_start(s->S, s->Lst, s->W, s->T, s->O, s->buf.q, s->buf.p,
                                       s->buf.img, plain ? 1 : 0, st));
  }
  return LSD_OK;
}

lsd_status capture(lsd_system* s, int K, int part, hipGraphExec_t* out) {
  if (!s->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
  const lsd_status e = enqueue_part(s, K, part, s->cap_stream);
  const std::string enqueue_err = e != LSD_OK ? g_err : std::string();
  hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
  if (e != LSD_OK || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (e != LSD_OK) return fail(e, "window capture: %s", enqueue_err.c_str());
    return fail(LSD_ERR_HIP, "window capture: %s", hipGetErrorString(e2));
  }
  hipError_t e3 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(LSD_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e3));
  return LSD_OK;
}

}  // namespace

extern "C" {

const char* lsd_last_error(void) { return g_err.c_str(); }

lsd_status lsd_workspace_size(const lsd_config* cfg, size_t* bytes) {
  if (!bytes) return fail(LSD_ERR_INVALID_ARG, "null bytes");
  Layout L;
  LSD_TRY(plan(cfg, &L));
  *bytes = L.total;
  return LSD_OK;
}

lsd_status lsd_init_system(const lsd_config* cfg, const lsd_buffers* buf, lsd_stream stream,
                           lsd_system** out) {
  if (!out || !buf) return fail(LSD_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  Layout L;
  LSD_TRY(plan(cfg, &L));
  if (!buf->q || !buf->p || !buf->img || !buf->step || !buf->workspace || !buf->log_ratio ||
      !buf->energy || !buf->accepted || !buf->n_committed)
    return fail(LSD_ERR_INVALID_ARG, "all state, output and workspace pointers are required");
  if (cfg->integrator == LSD_INTEGRATOR_OBABO && (!buf->obabo_q || !buf->obabo_p))
    return fail(LSD_ERR_INVALID_ARG, "the OBABO integrator needs obabo_q and obabo_p");
  if (reinterpret_cast<uintptr_t>(buf->workspace) % kAlign)
    return fail(LSD_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
  if (buf->workspace_bytes < L.total)
    return fail(LSD_ERR_CAPACITY, "workspace %zu bytes < required %zu", buf->workspace_bytes, L.total);
  hipStream_t st = static_cast<hipStream_t>(stream);

  lsd_system* s = new lsd_system();
  s->cfg = *cfg;
  s->cfg.atom_offsets = nullptr;  // host arrays are not kept
  s->cfg.box = nullptr;
  s->cfg.species = nullptr;
  s->cfg.species_mass = nullptr;
  s->buf = *buf;
  s->lay = L;
  const int N = cfg->n_atoms, R = cfg->n_replicas;

  // --- static tables
  std::vector<int> species_h(N, 0), rep_off_h(R + 1);
  if (cfg->species)
    for (int i = 0; i < N; ++i) species_h[i] = cfg->species[i];
  for (int r = 0; r <= R; ++r) rep_off_h[r] = cfg->atom_offsets[r];
  std::vector<double> box_h(cfg->box, cfg->box + R);
  lsd_status st_ok = LSD_OK;
  auto up = [&](const std::vector<int>& v, size_t off) {
    if (st_ok == LSD_OK) st_ok = upload_ints(v, ws<int>(s, off), st);
  };
  up(L.atom_rep_h, L.atom_rep);
  up(species_h, L.species);
  up(rep_off_h, L.rep_off);
  up(L.rep_nc_h, L.rep_nc);
  up(L.rep_cell_off_h, L.rep_cell_off);
  up(L.tile_start_h, L.tile_start);
  up(L.tile_count_h, L.tile_count);
  up(L.tile_rep_h, L.tile_rep);
  up(L.rep_tile_off_h, L.rep_tile_off);
  up(L.cell_rep_h, L.cell_rep);
  if (st_ok != LSD_OK) { delete s; return st_ok; }
  hipError_t e = hipMemcpyAsync(ws<double>(s, L.box), box_h.data(), R * sizeof(double),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.cell_count), 0, L.n_cells, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.cell_cursor), 0, L.n_cells, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.status), 0, 4, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.invalid), 0, R * cfg->k_max, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.nvalid), 0, 1, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.tail_bar), 0, 1, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.rej), LSD_MAX_K, R, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.cnt_t), 0, N, st);
  if (e == hipSuccess) e = launch_zero_i64(ws<long long>(s, L.counters), LSD_NCOUNT * R, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.cnt_d), 0, N, st);
  if (e == hipSuccess && L.ec) e = launch_fill_int(ws<int>(s, L.ec), 0, 3 * N, st);  // +0.0f
  if (e == hipSuccess && L.ec) e = launch_fill_int(ws<int>(s, L.ec_samples), 0, R, st);
  if (e == hipSuccess && L.ec_prev) e = launch_fill_int(ws<int>(s, L.ec_prev), 0, 3 * N, st);
  if (e == hipSuccess) e = launch_fill_int(ws<int>(s, L.rebuild), 1, R, st);  // first window builds
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete s;
    return fail(LSD_ERR_HIP, "init upload: %s", hipGetErrorString(e));
  }

  // --- device descriptors
  SysDev& S = s->S;
  memset(&S, 0, sizeof(S));
  S.n = N;
  S.R = R;
  S.n_tiles = L.n_tiles;
  S.kmax = cfg->k_max;
  S.atom_rep = ws<int>(s, L.atom_rep);
  S.species = cfg->n_species > 1 ? ws<int>(s, L.species) : nullptr;
  S.rep_off = ws<int>(s, L.rep_off);
  S.box = ws<double>(s, L.box);
  S.a = std::exp(-cfg->gamma * cfg->dt);
  S.c1fu = (1.0 + S.a) * (0.5 * cfg->dt) * cfg->force_unit;
  for (int sp = 0; sp < LSD_MAX_SPECIES; ++sp) {
    const double m = cfg->species_mass[sp < cfg->n_species ? sp : 0];
    S.hdt_m[sp] = (0.5 * cfg->dt) / m;
    S.sig[sp] = std::sqrt(m * cfg->kT * cfg->force_unit * (1.0 - std::exp(-2.0 * cfg->gamma * cfg->dt)));
  }
  const double hs = 0.5 * cfg->skin * (1.0 - 1e-4);
  S.half_skin2 = (float)(hs * hs);
  S.seed = cfg->seed;
  S.replay_u = buf->replay_u;
  S.replay_xi = buf->replay_xi;
  S.step = buf->step;
  S.step_limit = INT64_MAX;
  if (cfg->integrator == LSD_INTEGRATOR_OBABO) {
    const double a = std::exp(-cfg->gamma * cfg->dt);
    S.obabo = 1;
    S.ah = std::exp(-0.5 * cfg->gamma * cfg->dt);
    S.hfu = 0.5 * cfg->dt * cfg->force_unit;
    S.cw = S.ah / (1.0 + a);
    S.cs = 1.0 / std::sqrt(1.0 + a);
    for (int sp = 0; sp < LSD_MAX_SPECIES; ++sp) {
      const double m = cfg->species_mass[sp < cfg->n_species ? sp : 0];
      S.sh[sp] = std::sqrt(m * cfg->kT * cfg->force_unit * (1.0 - a));
    }
    S.obabo_q = buf->obabo_q;
    S.obabo_p = buf->obabo_p;
  }

  ListDev& Ls = s->Lst;
  memset(&Ls, 0, sizeof(Ls));
  Ls.rep_nc = ws<int>(s, L.rep_nc);
  Ls.rep_cell_off = ws<int>(s, L.rep_cell_off);
  Ls.cell_rep = ws<int>(s, L.cell_rep);
  Ls.cell_count = ws<int>(s, L.cell_count);
  Ls.cell_start = ws<int>(s, L.cell_start);
  Ls.cell_cursor = ws<int>(s, L.cell_cursor);
  Ls.cell_unsorted = ws<int>(s, L.cell_unsorted);
  Ls.cell_atoms = ws<int>(s, L.cell_atoms);
  Ls.cell_cap = L.cell_cap;
  Ls.atom_cell = ws<int>(s, L.atom_cell);
  Ls.n_cells = L.n_cells;
  Ls.nbr_t = ws<uint32_t>(s, L.nbr_t);
  Ls.cnt_t = ws<int>(s, L.cnt_t);
  Ls.mt = L.mt;
  Ls.nbr_d = ws<uint32_t>(s, L.nbr_d);
  Ls.cnt_d = ws<int>(s, L.cnt_d);
  Ls.md = L.md;
  Ls.rl2_t = L.rl_t * L.rl_t;
  Ls.rl2_d = L.rl_d * L.rl_d;
  {
    // outside these bands the binary32 distance decides the list predicate
    const double u = std::ldexp(1.0, -24);
    Ls.rl2_t_lo = (float)(Ls.rl2_t * (1.0 - 32.0 * u));
    Ls.rl2_t_hi = (float)(Ls.rl2_t * (1.0 + 32.0 * u));
    Ls.rl2_d_lo = (float)(Ls.rl2_d * (1.0 - 32.0 * u));
    Ls.rl2_d_hi = (float)(Ls.rl2_d * (1.0 + 32.0 * u));
  }
  Ls.status = ws<int>(s, L.status);
  Ls.qref = ws<float4>(s, L.qref);
  Ls.qwrap = ws<float4>(s, L.qwrap);
  Ls.rebuild = ws<int>(s, L.rebuild);
  const double qs = 0.25 * cfg->skin * (1.0 - 1e-4);
  Ls.reuse2 = (float)(qs * qs);
  Ls.always_rebuild = cfg->no_list_reuse ? 1 : 0;

  WinDev& W = s->W;
  memset(&W, 0, sizeof(W));
  W.qmid = ws<float4>(s, L.qmid);
  W.p = ws<float>(s, L.p);
  W.fd = ws<float>(s, L.fd);
  W.ft = ws<float>(s, L.ft);
  W.invalid = ws<int>(s, L.invalid);
  W.nvalid = ws<int>(s, L.nvalid);
  W.rej = ws<int>(s, L.rej);
  W.partial = ws<double>(s, L.partial);
  W.commit_frame = ws<int>(s, L.commit_frame);
  W.reflected = ws<int>(s, L.reflected);
  W.coef = ws<double>(s, L.coef);
  W.counters = ws<long long>(s, L.counters);
  W.tail_bar = ws<int>(s, L.tail_bar);
  W.ec = L.ec ? ws<float>(s, L.ec) : nullptr;
  W.ec_prev = L.ec_prev ? ws<float>(s, L.ec_prev) : nullptr;
  W.ec_samples = L.ec ? ws<int>(s, L.ec_samples) : nullptr;
  W.K = 0;

  TileDev& T = s->T;
  T.start = ws<int>(s, L.tile_start);
  T.count = ws<int>(s, L.tile_count);
  T.rep = ws<int>(s, L.tile_rep);
  T.rep_tile_off = ws<int>(s, L.rep_tile_off);

  OutDev& O = s->O;
  O.log_ratio = buf->log_ratio;
  O.energy = buf->energy;
  O.accepted = buf->accepted;
  O.n_committed = buf->n_committed;

  s->Pt = make_pot(cfg->target, L);
  s->Pd = cfg->mode == LSD_MODE_LSD ? make_pot(cfg->draft, L) : s->Pt;
  if (L.net_v) s->Pd.v = ws<float>(s, L.net_v);
  if (L.has_mpnn) {
    s->has_mpnn = true;
    MpnnCtx& M = s->mp;
    mpnn_bind(M, ws<char>(s, L.mpnn), cfg->k_max, N, L.mt, cfg->target.weights,
              cfg->target.n_model_species);
    M.rc = (float)cfg->target.cutoff;
    M.scale = (float)cfg->target.energy_scale;
    char err[256];
    if (!mpnn_prepare(M, st, err, sizeof(err))) {
      delete s;
      return fail(LSD_ERR_HIP, "network weight fragments: %s", err);
    }
  }
  if (cfg->integrator == LSD_INTEGRATOR_OBABO) {
    // initial OB half step (App. E): target force at the given positions
    hipError_t eo = launch_obabo_begin(S, s->Lst, s->W, s->Pt, false, buf->q, buf->p, buf->img, st, 0);
    if (eo == hipSuccess) eo = launch_build_lists(S, s->Lst, s->W, true, st);
    bool given = false;
    if (eo == hipSuccess && s->has_mpnn) {
      char err[256];
      if (!mpnn_eval(s->mp, S, s->Lst, s->W, 0, 1, nullptr, s->W.ft, st, err, sizeof(err))) {
        lsd_destroy(s);
        return fail(LSD_ERR_HIP, "network forces at the initial state: %s", err);
      }
      given = true;
    }
    if (eo == hipSuccess)
      eo = launch_obabo_begin(S, s->Lst, s->W, s->Pt, given, buf->q, buf->p, buf->img, st, 1);
    if (eo == hipSuccess) eo = hipStreamSynchronize(st);
    if (eo != hipSuccess) {
      lsd_destroy(s);
      return fail(LSD_ERR_HIP, "initial OB half step: %s", hipGetErrorString(eo));
    }
  }
  s->state = ST_READY;
  *out = s;
  return LSD_OK;
}

lsd_status lsd_draft_steps(lsd_system* s, int32_t K, lsd_stream stream) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (s->state != ST_READY && s->state != ST_COMMITTED)
    return fail(LSD_ERR_BAD_STATE, "draft_steps needs a committed state (state %d)", s->state);
  if (K < 1 || K > s->cfg.k_max) return fail(LSD_ERR_INVALID_ARG, "K = %d outside 1..k_max", K);
  hipStream_t st = static_cast<hipStream_t>(stream);
  s->W.K = K;
  HIP_TRY(launch_window_start(s->S, s->Lst, s->W, s->buf.q, s->buf.p, st));
  HIP_TRY(launch_build_lists(s->S, s->Lst, s->W, false, st));
  LSD_TRY(enqueue_drafts(s, K, st));
  s->state = ST_DRAFTED;
  return LSD_OK;
}

lsd_status lsd_mark_drafted(lsd_system* s, int32_t K, lsd_stream stream) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (s->state != ST_READY && s->state != ST_COMMITTED)
    return fail(LSD_ERR_BAD_STATE, "mark_drafted needs a committed state (state %d)", s->state);
  if (K < 1 || K > s->cfg.k_max) return fail(LSD_ERR_INVALID_ARG, "K = %d outside 1..k_max", K);
  hipStream_t st = static_cast<hipStream_t>(stream);
  s->W.K = K;
  HIP_TRY(launch_fill_int(s->W.invalid, 0, s->S.R * s->S.kmax, st));
  HIP_TRY(launch_fill_int(s->W.nvalid, K, 1, st));  // bound: every frame
  HIP_TRY(launch_fill_int(s->W.rej, LSD_MAX_K, s->S.R, st));
  HIP_TRY(launch_fill_int(s->Lst.rebuild, 1, s->S.R, st));  // lists from the caller's frame 0
  HIP_TRY(launch_build_lists(s->S, s->Lst, s->W, true, st));
  HIP_TRY(launch_frame_validity(s->S, s->Lst, s->W, st));
  s->state = ST_DRAFTED;
  return LSD_OK;
}

lsd_status lsd_verify_window(lsd_system* s, lsd_stream stream) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (s->state != ST_DRAFTED) return fail(LSD_ERR_BAD_STATE, "verify_window needs a drafted window");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->cfg.mode == LSD_MODE_LSD) {
    TimingRing& R = s->ring;
    int slot = -1;
    const bool timed = s->timing && (s->timing_seq++ % s->timing_every) == s->timing_every - 1;
    if (timed) {
      if (R.used == kTimingRing) LSD_TRY(timing_drain_one(s));
      slot = (R.head + R.used) % kTimingRing;
      HIP_TRY(hipEventRecord(R.start[slot], st));
    }
    LSD_TRY(enqueue_verify(s, s->W.K, st));
    if (timed) {
      HIP_TRY(hipEventRecord(R.stop[slot], st));
      R.used += 1;
    }
  }
  s->state = ST_VERIFIED;
  return LSD_OK;
}

lsd_status lsd_accept_rollback(lsd_system* s, int32_t* n_host, lsd_stream stream) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  const bool plain = s->cfg.mode == LSD_MODE_PLAIN;
  if (!(s->state == ST_VERIFIED || (plain && s->state == ST_DRAFTED)))
    return fail(LSD_ERR_BAD_STATE, "accept_rollback needs a verified window");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_decide(s->S, s->Lst, s->W, s->T, s->O, plain ? 1 : 0, st));
  HIP_TRY(launch_commit(s->S, s->W, s->buf.q, s->buf.p, s->buf.img, plain ? 1 : 0, st));
  s->state = ST_COMMITTED;
  if (n_host) {
    HIP_TRY(hipMemcpyAsync(n_host, s->buf.n_committed, sizeof(int32_t) * s->S.R,
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return LSD_OK;
}

lsd_status lsd_run_windows(lsd_system* s, int32_t n_windows, int32_t K, lsd_stream stream) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (n_windows < 0) return fail(LSD_ERR_INVALID_ARG, "n_windows < 0");
  if (K < 1 || K > s->cfg.k_max) return fail(LSD_ERR_INVALID_ARG, "K = %d outside 1..k_max", K);
  if (s->state != ST_READY && s->state != ST_COMMITTED)
    return fail(LSD_ERR_BAD_STATE, "run_windows needs a committed state (state %d)", s->state);
  if (!s->use_graphs) {
    for (int w = 0; w < n_windows; ++w) {
      LSD_TRY(lsd_draft_steps(s, K, stream));
      LSD_TRY(lsd_verify_window(s, stream));
      LSD_TRY(lsd_accept_rollback(s, nullptr, stream));
    }
    return LSD_OK;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool timed = s->timing && s->cfg.mode == LSD_MODE_LSD;
  if (s->pipe_group > 0 && s->cfg.mode == LSD_MODE_LSD) {
    // pipelined windows: an untimed window is one launch of its two-stream
    // graph; a timed one is issued eagerly with its verification launches
    // bracketed by events
    LSD_TRY(pipeline_resources(s));
    hipGraphExec_t& PG = s->pipe_graphs[K];
    if ((!timed || s->timing_every > 1) && !PG) LSD_TRY(capture_pipelined(s, K, &PG));
    s->W.K = K;
    if (n_windows > 0) HIP_TRY(launch_window_start(s->S, s->Lst, s->W, s->buf.q, s->buf.p, st));
    for (int w = 0; w < n_windows; ++w) {
      const bool t = timed && (s->timing_seq++ % s->timing_every) == s->timing_every - 1;
      if (t) {
        LSD_TRY(enqueue_pipelined(s, K, st, s->side_stream, true));
      } else {
        HIP_TRY(hipGraphLaunch(PG, st));
      }
    }
    if (!s->graphs_done) HIP_TRY(hipEventCreateWithFlags(&s->graphs_done, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(s->graphs_done, st));
    s->state = ST_COMMITTED;
    return LSD_OK;
  }
  WindowGraphs& G = s->graphs[K];
  if ((!timed || s->timing_every > 1) && !G.full) LSD_TRY(capture(s, K, PART_FULL, &G.full));
  if (timed && !G.pre) LSD_TRY(capture(s, K, PART_PRE, &G.pre));
  if (timed && !G.post) LSD_TRY(capture(s, K, PART_POST, &G.post));
  if (timed && !G.mid) LSD_TRY(capture(s, K, PART_MID, &G.mid));
  s->W.K = K;
  // the first window's start; every later one is fused into a commit (the
  // start that the last commit leaves behind is redone by the next call)
  if (n_windows > 0) HIP_TRY(launch_window_start(s->S, s->Lst, s->W, s->buf.q, s->buf.p, st));
  // a timed window runs as pre, the event-bracketed verification, and post
  // (merged with the next window's pre into mid when that one is timed
  // too); an untimed window is one launch of the whole-window graph
  bool open = false;  // a timed window's post is still to be launched
  for (int w = 0; w < n_windows; ++w) {
    const bool t = timed && (s->timing_seq++ % s->timing_every) == s->timing_every - 1;
    if (!t) {
      if (open) HIP_TRY(hipGraphLaunch(G.post, st));
      open = false;
      HIP_TRY(hipGraphLaunch(G.full, st));
      continue;
    }
    HIP_TRY(hipGraphLaunch(open ? G.mid : G.pre, st));
    TimingRing& R = s->ring;
    if (R.used == kTimingRing) LSD_TRY(timing_drain_one(s));
    const int slot = (R.head + R.used) % kTimingRing;
    HIP_TRY(hipEventRecord(R.start[slot], st));
    LSD_TRY(enqueue_verify(s, K, st));
    HIP_TRY(hipEventRecord(R.stop[slot], st));
    R.used += 1;
    open = true;
  }
  if (open) HIP_TRY(hipGraphLaunch(G.post, st));
  if (!s->graphs_done) HIP_TRY(hipEventCreateWithFlags(&s->graphs_done, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(s->graphs_done, st));
  s->state = ST_COMMITTED;
  return LSD_OK;
}

lsd_status lsd_autotune_verify(lsd_system* s, int32_t K, int32_t repeats, int32_t* chosen,
                               double* us, lsd_stream stream) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (K < 1 || K > s->cfg.k_max) return fail(LSD_ERR_INVALID_ARG, "K = %d outside 1..k_max", K);
  if (repeats < 1) return fail(LSD_ERR_INVALID_ARG, "repeats must be >= 1");
  if (s->cfg.mode != LSD_MODE_LSD)
    return fail(LSD_ERR_UNSUPPORTED, "the verification is tuned in LSD mode");
  hipStream_t st = static_cast<hipStream_t>(stream);
  LSD_TRY(lsd_draft_steps(s, K, stream));  // leaves the window drafted
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  if (s->has_mpnn) {
    // the network evaluation's launch shapes, timed on the drafted frames
    // (evaluation and transport sums only write the window's target forces,
    // the per-tile sums and the network's own buffers: repeatable)
    int best = 0;
    float best_ms = 0.0f;
    for (int c = 0; c < MP_TUNE_CANDIDATES; ++c) {
      mpnn_set_shape(s->mp, c);
      lsd_status ls = enqueue_verify(s, K, st);
      hipError_t e = ls == LSD_OK ? hipEventRecord(e0, st) : hipSuccess;
      for (int r = 0; r < repeats && ls == LSD_OK && e == hipSuccess; ++r)
        ls = enqueue_verify(s, K, st);
      if (ls == LSD_OK && e == hipSuccess) e = hipEventRecord(e1, st);
      if (ls == LSD_OK && e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (ls == LSD_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (ls != LSD_OK || e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (ls != LSD_OK) return ls;
        return fail(LSD_ERR_HIP, "autotune: %s", hipGetErrorString(e));
      }
      if (us) us[c] = 1e3 * ms / repeats;
      if (c == 0 || ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    mpnn_set_shape(s->mp, best);
    s->tuned_fw[K] = best;
    destroy_graphs(s);
    if (chosen) *chosen = best;
    return LSD_OK;
  }
  static const int kCandidates[4] = {1, 2, 4, 8};
  int best = verify_fw(s, K);
  float best_ms = 0.0f;
  for (int c = 0; c < 4; ++c) {
    const int fw = kCandidates[c];
    // one untimed launch, then `repeats` timed ones on the same drafted frames
    // (verification only writes f_target and the per-tile sums: repeatable)
    hipError_t e = launch_verify(s->S, s->Lst, s->W, s->T, s->Pt, fw, 0, K, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < repeats && e == hipSuccess; ++r)
      e = launch_verify(s->S, s->Lst, s->W, s->T, s->Pt, fw, 0, K, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(LSD_ERR_HIP, "autotune: %s", hipGetErrorString(e));
    }
    if (us) us[c] = 1e3 * ms / repeats;
    if (c == 0 || ms < best_ms) {
      best_ms = ms;
      best = fw;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->tuned_fw[K] = best;
  destroy_graphs(s);  // captured windows used the previous choice
  if (chosen) *chosen = best;
  return LSD_OK;
}

lsd_status lsd_set_verify_variant(lsd_system* s, int32_t K, int32_t frames_per_wave) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (K < 1 || K > s->cfg.k_max) return fail(LSD_ERR_INVALID_ARG, "K = %d outside 1..k_max", K);
  const int fw = frames_per_wave;
  if (s->has_mpnn) {
    if (fw < 0 || fw >= MP_TUNE_CANDIDATES)
      return fail(LSD_ERR_INVALID_ARG, "network launch shape %d outside 0..%d", fw,
                  MP_TUNE_CANDIDATES - 1);
    mpnn_set_shape(s->mp, fw);
    s->tuned_fw[K] = fw;
    destroy_graphs(s);
    return LSD_OK;
  }
  if (fw != 1 && fw != 2 && fw != 4 && fw != 8)
    return fail(LSD_ERR_INVALID_ARG, "frames per wave %d not in {1, 2, 4, 8}", fw);
  s->tuned_fw[K] = fw;
  destroy_graphs(s);
  return LSD_OK;
}

lsd_status lsd_set_pipeline(lsd_system* s, int32_t group_frames) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (group_frames < 0 || group_frames > LSD_MAX_K)
    return fail(LSD_ERR_INVALID_ARG, "group_frames %d outside 0..%d", group_frames, LSD_MAX_K);
  if (group_frames > 0 && !s->use_graphs)
    return fail(LSD_ERR_UNSUPPORTED, "pipelined windows run through lsd_run_windows with graphs on");
  if (s->pipe_group != group_frames) destroy_graphs(s);
  s->pipe_group = group_frames;
  return LSD_OK;
}

lsd_status lsd_set_draft_tail(lsd_system* s, int32_t first_step) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (first_step < 0 || first_step > LSD_MAX_K)
    return fail(LSD_ERR_INVALID_ARG, "first_step %d outside 0..%d", first_step, LSD_MAX_K);
  if (s->draft_tail != first_step) destroy_graphs(s);  // captured windows hold the old choice
  s->draft_tail = first_step;
  return LSD_OK;
}

lsd_status lsd_set_graphs(lsd_system* s, int32_t enable) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  s->use_graphs = enable != 0;
  return LSD_OK;
}

lsd_status lsd_get_window_layout(const lsd_system* s, lsd_window_layout* out) {
  if (!s || !out) return fail(LSD_ERR_INVALID_ARG, "null argument");
  out->q_mid = s->lay.qmid;
  out->p_draft = s->lay.p;
  out->f_draft = s->lay.fd;
  out->f_target = s->lay.ft;
  out->frame_invalid = s->lay.invalid;
  out->nbr_target = s->lay.nbr_t;
  out->cnt_target = s->lay.cnt_t;
  out->nbr_draft = s->lay.nbr_d;
  out->cnt_draft = s->lay.cnt_d;
  out->error_cache = s->lay.ec;
  out->error_cache_prev = s->lay.ec_prev;
  out->max_neighbors_target = s->lay.mt;
  out->max_neighbors_draft = s->lay.md;
  out->n_atoms = s->S.n;
  out->k_max = s->S.kmax;
  return LSD_OK;
}

lsd_status lsd_get_status(lsd_system* s, int32_t* flags, lsd_stream stream) {
  if (!s || !flags) return fail(LSD_ERR_INVALID_ARG, "null argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(flags, s->Lst.status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return LSD_OK;
}

lsd_status lsd_set_step_limit(lsd_system* s, int64_t limit) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (limit < 0) return fail(LSD_ERR_INVALID_ARG, "step limit < 0");
  s->S.step_limit = limit;
  destroy_graphs(s);  // captured kernels hold the old limit
  return LSD_OK;
}

lsd_status lsd_get_counters(lsd_system* s, int64_t* out, lsd_stream stream) {
  if (!s || !out) return fail(LSD_ERR_INVALID_ARG, "null argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(out, s->W.counters, sizeof(int64_t) * LSD_NCOUNT * s->S.R,
                          hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return LSD_OK;
}

lsd_status lsd_reset_counters(lsd_system* s, lsd_stream stream) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  HIP_TRY(launch_zero_i64(s->W.counters, LSD_NCOUNT * s->S.R, static_cast<hipStream_t>(stream)));
  return LSD_OK;
}

lsd_status lsd_set_verify_timing(lsd_system* s, int32_t enable) {
  if (!s) return fail(LSD_ERR_INVALID_ARG, "null system");
  if (enable < 0) return fail(LSD_ERR_INVALID_ARG, "timing period %d < 0", enable);
  TimingRing& R = s->ring;
  if (enable && !R.created) {
    for (int i = 0; i < kTimingRing; ++i) {
      HIP_TRY(hipEventCreate(&R.start[i]));
      HIP_TRY(hipEventCreate(&R.stop[i]));
    }
    R.created = true;
  }
  while (R.used > 0) LSD_TRY(timing_drain_one(s));
  s->timing = enable != 0;
  s->timing_every = enable > 1 ? enable : 1;
  s->timing_seq = 0;
  s->t_sum = 0.0;
  s->t_count = 0;
  return LSD_OK;
}

lsd_status lsd_get_verify_timing(lsd_system* s, double* total_ms, int64_t* launches) {
  if (!s || !total_ms || !launches) return fail(LSD_ERR_INVALID_ARG, "null argument");
  while (s->ring.used > 0) LSD_TRY(timing_drain_one(s));
  *total_ms = s->t_sum;
  *launches = s->t_count;
  return LSD_OK;
}

lsd_status lsd_rng_normals(uint64_t seed, int32_t replica, int64_t step, int32_t n, double* out,
                           lsd_stream stream) {
  if (!out || n < 0 || replica < 0) return fail(LSD_ERR_INVALID_ARG, "bad rng arguments");
  HIP_TRY(launch_rng_normals(seed, replica, step, n, out, static_cast<hipStream_t>(stream)));
  return LSD_OK;
}

lsd_status lsd_rng_uniforms(uint64_t seed, int32_t replica, int64_t step0, int32_t count,
                            double* out, lsd_stream stream) {
  if (!out || count < 0 || replica < 0) return fail(LSD_ERR_INVALID_ARG, "bad rng arguments");
  HIP_TRY(launch_rng_uniforms(seed, replica, step0, count, out, static_cast<hipStream_t>(stream)));
  return LSD_OK;
}

lsd_status lsd_fit_pair_scratch_size(const lsd_system* s, int32_t n_basis, size_t* bytes) {
  if (!s || !bytes) return fail(LSD_ERR_INVALID_ARG, "null argument");
  if (n_basis < 1 || n_basis > LSD_PAIR_MAX_BASIS)
    return fail(LSD_ERR_INVALID_ARG, "n_basis %d outside 1..%d", n_basis, LSD_PAIR_MAX_BASIS);
  FitDev F;
  F.ns = s->cfg.n_species;
  F.nb = n_basis;
  F.LP = F.ns * n_basis;
  if (F.LP > FIT_MAX_LP)
    return fail(LSD_ERR_UNSUPPORTED, "species x basis = %d > %d", F.LP, FIT_MAX_LP);
  *bytes = (size_t)s->S.n_tiles * fit_partial_entries(F) * sizeof(double);
  return LSD_OK;
}

lsd_status lsd_fit_pair_accumulate(lsd_system* s, int32_t n_basis, double cutoff,
                                   int32_t use_target_forces, int32_t differences, void* scratch,
                                   size_t scratch_bytes, double* gram, lsd_stream stream) {
  if (!s || !scratch || !gram) return fail(LSD_ERR_INVALID_ARG, "null argument");
  size_t need = 0;
  LSD_TRY(lsd_fit_pair_scratch_size(s, n_basis, &need));
  if (scratch_bytes < need)
    return fail(LSD_ERR_CAPACITY, "fit scratch %zu bytes < required %zu", scratch_bytes, need);
  if (s->state == ST_READY || s->W.K < 1)
    return fail(LSD_ERR_BAD_STATE, "fit needs a drafted window");
  if (use_target_forces &&
      !(s->cfg.mode == LSD_MODE_LSD && (s->state == ST_VERIFIED || s->state == ST_COMMITTED)))
    return fail(LSD_ERR_BAD_STATE, "target forces exist only for a verified window (LSD mode)");
  if (!(cutoff > 0.0) || cutoff > pot_reach(s->cfg.target))
    return fail(LSD_ERR_INVALID_ARG, "fit cutoff %g must be in (0, target cutoff %g]", cutoff,
                pot_reach(s->cfg.target));
  FitDev F;
  F.rc2 = (float)(cutoff * cutoff);
  F.pi_rc = (float)(M_PI / cutoff);
  F.nb = n_basis;
  F.ns = s->cfg.n_species;
  F.LP = F.ns * n_basis;
  HIP_TRY(launch_fit(s->S, s->Lst, s->W, s->T, F, use_target_forces ? 1 : 0, differences ? 1 : 0,
                     static_cast<double*>(scratch), gram, static_cast<hipStream_t>(stream)));
  return LSD_OK;
}

int32_t lsd_net_param_count(int32_t n_species, int32_t n_basis) {
  if (n_species < 1 || n_species > LSD_NET_MAX_SPECIES || n_basis < 1 ||
      n_basis > LSD_NET_MAX_BASIS || n_species * n_basis > LSD_NET_MAX_DESC)
    return 0;
  return net_params(n_species, n_basis);
}

lsd_status lsd_net_train_scratch_size(const lsd_system* s, size_t* bytes) {
  if (!s || !bytes) return fail(LSD_ERR_INVALID_ARG, "null argument");
  *bytes = net_train_bytes(s->cfg.k_max, s->cfg.n_atoms);
  return LSD_OK;
}

lsd_status lsd_net_train_accumulate(lsd_system* s, const lsd_potential* net,
                                    int32_t use_target_forces, int32_t differences, void* scratch,
                                    size_t scratch_bytes, double* grad, lsd_stream stream) {
  if (!s || !net || !scratch || !grad) return fail(LSD_ERR_INVALID_ARG, "null argument");
  if (net->kind != LSD_POT_NET) return fail(LSD_ERR_INVALID_ARG, "not a learned draft");
  lsd_potential copy = *net;
  copy.precision = LSD_PREC_FP32;  // training evaluates in binary32
  LSD_TRY(check_potential(copy, "learned draft"));
  if (net->n_model_species < s->cfg.n_species)
    return fail(LSD_ERR_INVALID_ARG, "learned draft has %d species, system has %d",
                net->n_model_species, s->cfg.n_species);
  if (net->cutoff > pot_reach(s->cfg.target))
    return fail(LSD_ERR_INVALID_ARG, "learned draft cutoff %g exceeds the target cutoff %g",
                net->cutoff, pot_reach(s->cfg.target));
  const size_t need = net_train_bytes(s->cfg.k_max, s->cfg.n_atoms);
  if (scratch_bytes < need)
    return fail(LSD_ERR_CAPACITY, "training scratch %zu bytes < required %zu", scratch_bytes, need);
  if (s->state == ST_READY || s->W.K < 1)
    return fail(LSD_ERR_BAD_STATE, "training needs a drafted window");
  if (use_target_forces &&
      !(s->cfg.mode == LSD_MODE_LSD && (s->state == ST_VERIFIED || s->state == ST_COMMITTED)))
    return fail(LSD_ERR_BAD_STATE, "target forces exist only for a verified window (LSD mode)");
  PotDev P = make_pot(copy, s->lay);
  const NetTrainDev T = net_train_bind(static_cast<char*>(scratch), s->cfg.k_max, s->cfg.n_atoms);
  HIP_TRY(launch_net_train(s->S, s->Lst, s->W, P, T, use_target_forces ? 1 : 0,
                           differences ? 1 : 0, grad, static_cast<hipStream_t>(stream)));
  return LSD_OK;
}

lsd_status lsd_net_activation_amax(lsd_system* s, const lsd_potential* net, void* scratch,
                                   size_t scratch_bytes, double* amax, lsd_stream stream) {
  if (!s || !net || !scratch || !amax) return fail(LSD_ERR_INVALID_ARG, "null argument");
  if (net->kind != LSD_POT_NET) return fail(LSD_ERR_INVALID_ARG, "not a learned draft");
  lsd_potential copy = *net;
  copy.precision = LSD_PREC_FP32;
  LSD_TRY(check_potential(copy, "learned draft"));
  if (copy.n_model_species < s->cfg.n_species)
    return fail(LSD_ERR_INVALID_ARG, "learned draft has %d species, system has %d",
                copy.n_model_species, s->cfg.n_species);
  if (copy.cutoff > pot_reach(s->cfg.target))
    return fail(LSD_ERR_INVALID_ARG, "learned draft cutoff %g exceeds the target cutoff %g",
                copy.cutoff, pot_reach(s->cfg.target));
  const size_t need = net_train_bytes(s->cfg.k_max, s->cfg.n_atoms);
  if (scratch_bytes < need)
    return fail(LSD_ERR_CAPACITY, "scratch %zu bytes < required %zu", scratch_bytes, need);
  if (s->state == ST_READY || s->W.K < 1)
    return fail(LSD_ERR_BAD_STATE, "calibration needs a drafted window");
  PotDev P = make_pot(copy, s->lay);
  const NetTrainDev T = net_train_bind(static_cast<char*>(scratch), s->cfg.k_max, s->cfg.n_atoms);
  HIP_TRY(launch_net_amax(s->S, s->Lst, s->W, P, T, amax, static_cast<hipStream_t>(stream)));
  return LSD_OK;
}

lsd_status lsd_net_adam_step(float* params, double* m, double* v, double* grad, int32_t n_params,
                             double lr, double beta1, double beta2, double eps, int64_t t,
                             lsd_stream stream) {
  if (!params || !m || !v || !grad) return fail(LSD_ERR_INVALID_ARG, "null argument");
  if (n_params < 1 || t < 1) return fail(LSD_ERR_INVALID_ARG, "n_params and t must be >= 1");
  if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return fail(LSD_ERR_INVALID_ARG, "Adam needs lr >= 0, beta1, beta2 in [0, 1), eps > 0");
  HIP_TRY(launch_net_adam(params, m, v, grad, n_params, lr, beta1, beta2, eps, (long long)t,
                          static_cast<hipStream_t>(stream)));
  return LSD_OK;
}

lsd_status lsd_fit_pair_solve(const double* gram, int32_t n_params, double ridge, double* weights) {
  if (!gram || !weights || n_params < 1) return fail(LSD_ERR_INVALID_ARG, "bad argument");
  if (!(ridge >= 0.0)) return fail(LSD_ERR_INVALID_ARG, "ridge must be >= 0");
  const int P = n_params, Pe = P + 1;
  double tr = 0.0;
  for (int c = 0; c < P; ++c) tr += gram[(size_t)c * Pe + c];
  const double lam = ridge * (tr > 0.0 ? tr / P : 1.0);
  std::vector<double> A((size_t)P * P), b(P);
  for (int r = 0; r < P; ++r) {
    for (int c = 0; c < P; ++c)
      A[(size_t)r * P + c] = 0.5 * (gram[(size_t)r * Pe + c] + gram[(size_t)c * Pe + r]);
    A[(size_t)r * P + r] += lam;
    b[r] = 0.5 * (gram[(size_t)r * Pe + P] + gram[(size_t)P * Pe + r]);
  }
  // Cholesky A = L L^T (lower triangle in place), then two triangular solves
  for (int j = 0; j < P; ++j) {
    double d = A[(size_t)j * P + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * P + k] * A[(size_t)j * P + k];
    if (!(d > 0.0))
      return fail(LSD_ERR_INVALID_ARG, "normal equations not positive definite (pivot %d); "
                  "raise the ridge", j);
    const double ljj = std::sqrt(d);
    A[(size_t)j * P + j] = ljj;
    for (int i = j + 1; i < P; ++i) {
      double v = A[(size_t)i * P + j];
      for (int k = 0; k < j; ++k) v -= A[(size_t)i * P + k] * A[(size_t)j * P + k];
      A[(size_t)i * P + j] = v / ljj;
    }
  }
  for (int i = 0; i < P; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= A[(size_t)i * P + k] * b[k];
    b[i] = v / A[(size_t)i * P + i];
  }
  for (int i = P - 1; i >= 0; --i) {
    double v = b[i];
    for (int k = i + 1; k < P; ++k) v -= A[(size_t)k * P + i] * b[k];
    b[i] = v / A[(size_t)i * P + i];
  }
  for (int i = 0; i < P; ++i) weights[i] = b[i];
  return LSD_OK;
}

lsd_status lsd_destroy(lsd_system* s) {
  if (!s) return LSD_OK;
  destroy_graphs(s);
  if (s->graphs_done) (void)hipEventDestroy(s->graphs_done);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->side_stream) {
    (void)hipStreamSynchronize(s->side_stream);
    (void)hipStreamDestroy(s->side_stream);
  }
  for (int i = 0; i <= LSD_MAX_K; ++i)
    if (s->pipe_ev[i]) (void)hipEventDestroy(s->pipe_ev[i]);
  if (s->ring.created) {
    for (int i = 0; i < kTimingRing; ++i) {
      (void)hipEventDestroy(s->ring.start[i]);
      (void)hipEventDestroy(s->ring.stop[i]);
    }
  }
  delete s;
  return LSD_OK;
}

}  // extern "C"
