// lsd_device.h -- device-side data structures and inline helpers shared by
// the HIP kernels of the LSD library (gfx950, wave64).
//
// Everything here is written for CDNA4: 64-lane wavefronts, binary64 vector
// ALU for the transport-map reductions, binary32 for the pair forces.  The
// translation unit is compiled with -ffp-contract=off so that every product
// and sum is rounded as written; fused multiply-adds appear only where the
// code says fma().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define LSD_MAX_SPECIES 8
#define LSD_TILE 64           // atoms per verification tile
#ifndef LSD_LPA
#define LSD_LPA 4             // lanes per atom in the force loops (power of 2, <= 64)
#endif
#define LSD_VTHREADS (LSD_TILE * LSD_LPA)  // threads of a verification block
#define LSD_VWAVES (LSD_VTHREADS / 64)
#define LSD_MAX_K 64
#define LSD_NCOUNT 5          // per-replica counters (see WinDev::counters)
#define LSD_POT_LJ 1
#define LSD_POT_HARMONIC 2
#define LSD_POT_MPNN 3
#define LSD_POT_PAIR 4
#define LSD_POT_NET 5
#define LSD_NET_HIDDEN 32     // hidden units of the learned draft
#define LSD_NET_MAX_BASIS 16  // radial functions (edge coefficients per atom, v stride)
#define LSD_NET_MAX_DESC 64   // species x radial functions of the descriptor
#define LSD_NET_MAX_SPECIES 4
#define LSD_NET_MAX_TYPES (LSD_NET_MAX_SPECIES * (LSD_NET_MAX_SPECIES + 1) / 2)
// drafting with the learned draft: lanes per atom and blocks per tile of the
// force loop (a block holds LSD_TILE / LSD_NET_SUB atoms), so that the
// latency-bound loop of a small system spreads over many compute units
#ifndef LSD_NET_LPA
#define LSD_NET_LPA 16
#endif
#ifndef LSD_NET_SUB
#define LSD_NET_SUB 16
#endif

// status word bits
#define LSD_STATUS_NBR_TARGET 1
#define LSD_STATUS_NBR_DRAFT 2
#define LSD_STATUS_CELL 4
#define LSD_STATUS_PAIRS 8    // network target: more pairs than its buffers hold
#define LSD_STATUS_EDGES 16   // network target: the two directions of a pair differ
#define LSD_STATUS_TAIL 32    // the one-launch draft chain's grid barrier timed out

struct PotDev {
  int kind;
  float rc2;              // cutoff^2 in binary32
  float rc2_lo, rc2_hi;   // binary32 band around rc2; inside it the binary64 test decides
  double rc2_d;           // cutoff^2 in binary64
  float eps4, eps24, sig2, eshift;  // 4 eps, 24 eps, sigma^2, 4 eps((s/rc)^12 - (s/rc)^6)
  float kspring;
  const float* anchor;    // [3][N]
  const float* offset;    // [3][N] or null
  // pair draft: rc2 above, pi / rc, basis size, species, weights [T][nb]
  // learned draft: the same, w = flat parameters, and the edge coefficients
  // v [N][LSD_NET_MAX_BASIS] of the frame being drafted
  float pi_rc;
  int nb, ns;
  const float* w;
  float* v;
  int prec;
  float fp8_sD, fp8_sh;  // FP8 node pass: static scales max|D| / 448, max|h| / 448
};

// offsets of the learned draft's parameter blocks W1 [H][S B], b1 [S][H],
// W2 [B][H], c [T][B]
__host__ __device__ __forceinline__ int net_off_b1(int S, int B) { return LSD_NET_HIDDEN * S * B; }
__host__ __device__ __forceinline__ int net_off_w2(int S, int B) {
  return net_off_b1(S, B) + S * LSD_NET_HIDDEN;
}
__host__ __device__ __forceinline__ int net_off_c(int S, int B) {
  return net_off_w2(S, B) + B * LSD_NET_HIDDEN;
}
__host__ __device__ __forceinline__ int net_params(int S, int B) {
  return net_off_c(S, B) + S * (S + 1) / 2 * B;
}

// index of the unordered species pair {a, b} among S(S+1)/2 types
__host__ __device__ __forceinline__ int pair_type(int a, int b, int S) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return lo * S - lo * (lo - 1) / 2 + (hi - lo);
}

struct SysDev {
  int n, R, n_tiles, kmax;
  const int* atom_rep;    // [N] replica of each atom
  const int* species;     // [N] or null (single species)
  const int* rep_off;     // [R+1]
  const double* box;      // [R] box edge (binary32 value held in binary64)
  double a;               // e^{-gamma dt}
  double c1fu;            // (1 + a) dt / 2 * force_unit
  double hdt_m[LSD_MAX_SPECIES];  // (dt / 2) / m_s
  double sig[LSD_MAX_SPECIES];    // sqrt(m_s kT force_unit (1 - a^2))
  float half_skin2;       // (skin / 2)^2, slightly reduced
  uint64_t seed;
  const double* replay_u;   // [R][kmax] or null
  const double* replay_xi;  // [kmax][N][3] or null
  int64_t* step;            // [R] committed step
  int64_t step_limit;       // frames producing steps beyond this are not verified
  // (OBABO) outputs (App. E): half-step friction and noise, recovery weights
  int obabo;
  double ah, hfu, cw, cs;   // e^{-gamma dt/2}, dt/2 force_unit, ah/(1+a), (1+a)^{-1/2}
  double sh[LSD_MAX_SPECIES];  // sqrt(m_s kT force_unit (1 - e^{-gamma dt}))
  float* obabo_q;           // [3][N]
  float* obabo_p;           // [3][N]
};

struct ListDev {
  const int* rep_nc;        // [R] cells per edge (1 = whole replica, 27 images)
  const int* rep_cell_off;  // [R] first cell of the replica
  const int* cell_rep;      // [C] replica of each cell
  int* cell_count;          // [C]
  int* cell_start;          // [C + 1]
  int* cell_cursor;         // [C]
  int* cell_unsorted;       // [N] atoms binned by cell, arbitrary order inside a cell
  int* cell_atoms;          // [N] atoms binned by cell, ascending inside a cell
  int* atom_cell;           // [N]
  int n_cells;
  int cell_cap;             // largest cell occupancy the list builder covers
  uint32_t* nbr_t; int* cnt_t; int mt;   // target list, atom-major [N][mt]
  uint32_t* nbr_d; int* cnt_d; int md;   // draft list, atom-major [N][md]
  double rl2_t, rl2_d;      // list radii squared (binary64)
  float rl2_t_lo, rl2_t_hi, rl2_d_lo, rl2_d_hi;  // binary32 bands rl2 (1 -+ 32u)
  int* status;
  // reuse across windows: the lists hold for positions within skin/2 of the
  // positions they were built at; window frames are kept continuous with
  // those positions, and a replica rebuilds when an atom's first midpoint is
  // more than skin/4 away from them
  float4* qref;             // [N] list positions (wrapped), image deltas unused
  float4* qwrap;            // [N] wrapped first midpoints of the current window
  int* rebuild;             // [R] 1: rebuild this replica's lists in this window
  float reuse2;             // (skin/4)^2, slightly reduced
  int always_rebuild;       // 1: rebuild every window
};

struct WinDev {
  float4* qmid;       // [kmax][N]
  float* p;           // [kmax+1][3][N]
  float* fd;          // [kmax][3][N]
  float* ft;          // [kmax][3][N]
  int* invalid;       // [R][kmax]
  int* nvalid;        // [1]: bound on the valid frames of any replica in this window
  int* rej;           // [R]: first rejected frame found while the window is still being
                      //      drafted (pipelined windows), LSD_MAX_K while none is known
  double* partial;    // [kmax][n_tiles][4]: S1, S2, E, unused
  int* commit_frame;  // [R]
  int* reflected;     // [R]
  double* coef;       // [R] 2 S1 / S2 of the rejected frame
  float* ec;          // [3][N] error-correction cache dF, or null (off)
  float* ec_prev;     // [3][N] dF of the committed step before, or null (constant EC)
  int* ec_samples;    // [R] committed error samples held (0, 1, 2 = both caches valid)
  long long* counters;  // [R][5]: windows, committed steps, rejections, frames verified,
                        // neighbour-list builds
  int* tail_bar;      // [1]: arrivals at the grid barriers of the one-launch draft chain,
                      //      cleared at every window start
  int K;              // frames in the current window
};

struct OutDev {
  double* log_ratio;  // [R][kmax]
  double* energy;     // [R][kmax]
  uint8_t* accepted;  // [R][kmax]
  int32_t* n_committed;  // [R]
};

struct TileDev {
  const int* start;   // [T] first atom
  const int* count;   // [T] atoms (<= 64)
  const int* rep;     // [T] replica
  const int* rep_tile_off;  // [R+1]
};

// Tile t: first atom, atoms, replica, and whether it is its replica's first
// tile.  A single system's tiles are consecutive runs of LSD_TILE atoms and
// need no loads (their table holds the same values).
struct TileInfo {
  int start, count, rep;
  bool first;
};
__device__ __forceinline__ TileInfo tile_info(int n, int R, const TileDev& Tl, int t) {
  TileInfo T;
  if (R == 1) {
    T.start = t * LSD_TILE;
    T.count = min(LSD_TILE, n - T.start);
    T.rep = 0;
    T.first = t == 0;
  } else {
    T.start = Tl.start[t];
    T.count = Tl.count[t];
    T.rep = Tl.rep[t];
    T.first = t == Tl.rep_tile_off[T.rep];
  }
  return T;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the step-keyed stream
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t hi0 = __umulhi(m0, c[0]), lo0 = m0 * c[0];
    uint32_t hi1 = __umulhi(m1, c[2]), lo1 = m1 * c[2];
    uint32_t y0 = hi1 ^ c[1] ^ k0;
    uint32_t y2 = hi0 ^ c[3] ^ k1;
    c[0] = y0; c[1] = lo1; c[2] = y2; c[3] = lo0;
  }
}

#define LSD_TAG_XI 1u
#define LSD_TAG_U 2u
#define LSD_TAG_OB 3u  // (OBABO) output noise

__device__ __forceinline__ double u53(uint32_t lo, uint32_t hi) {
  uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
  return (double)((x >> 11) + 1ull) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void stream_block(uint64_t seed, uint32_t replica, uint64_t step,
                                             uint32_t index, uint32_t tag, uint32_t block,
                                             uint32_t w[4]) {
  w[0] = index; w[1] = (uint32_t)step; w[2] = (uint32_t)(step >> 32);
  w[3] = (replica << 8) | (tag << 4) | block;
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ double stream_uniform(uint64_t seed, uint32_t replica, uint64_t step) {
  uint32_t w[4];
  stream_block(seed, replica, step, 0u, LSD_TAG_U, 0u, w);
  return u53(w[0], w[1]);
}

// three normals of local atom `index` at step `step` (Box-Muller, binary64)
__device__ __forceinline__ void stream_normals3(uint64_t seed, uint32_t replica, uint64_t step,
                                                uint32_t index, double xi[3],
                                                uint32_t tag = LSD_TAG_XI) {
  const double two_pi = 6.283185307179586476925286766559;
  uint32_t w[4];
  stream_block(seed, replica, step, index, tag, 0u, w);
  double r = sqrt(-2.0 * log(u53(w[0], w[1])));
  double s, c;
  sincos(two_pi * u53(w[2], w[3]), &s, &c);
  xi[0] = r * c;
  xi[1] = r * s;
  stream_block(seed, replica, step, index, tag, 1u, w);
  r = sqrt(-2.0 * log(u53(w[0], w[1])));
  xi[2] = r * cos(two_pi * u53(w[2], w[3]));
}

// ---------------------------------------------------------------------------
// Integrator pieces (Eq. aboba, Eq. bob)
// ---------------------------------------------------------------------------
// (A): x + (dt/2)/m p evaluated in binary64, wrapped into [0, L) and rounded
// to binary32; the applied image shift is added to *dimg.
__device__ __forceinline__ float a_half(float x, float p, double hdt_m, double L, int* dimg) {
  double v = (double)x + hdt_m * (double)p;
  int s = 0;
  if (v >= L || v < 0.0) {
    double f = floor(v / L);
    v = v - f * L;
    s = (int)f;
    if (v >= L) { v -= L; s += 1; }
    if (v < 0.0) { v += L; s -= 1; }
  }
  float r = (float)v;
  if ((double)r >= L) { r = 0.0f; s += 1; }
  *dimg += s;
  return r;
}

// (A) without wrapping: positions inside a window stay continuous with the
// wrapped frame-0 positions the neighbour lists (and their image codes) were
// built from; the commit wraps them.
__device__ __forceinline__ float a_half_cont(float x, float p, double hdt_m) {
  return (float)((double)x + hdt_m * (double)p);
}

// Draft force that enters the draft mean of frame k of replica r: F~ itself,
// or F~ + dF with error correction on (App. D), dF being the error of the
// last committed step; with the linear variant and two samples held, the
// error is extrapolated to the frame: dF + (k + 1) (dF - dF_prev).  Binary32,
// the same expression wherever the draft mean is formed.
__device__ __forceinline__ float draft_mean_force(const WinDev& W, int r, size_t c, int k, float Fd) {
  if (!W.ec) return Fd;
  float corr = W.ec[c];
  if (W.ec_prev && W.ec_samples[r] >= 2) corr = corr + (float)(k + 1) * (W.ec[c] - W.ec_prev[c]);
  return Fd + corr;
}

// Mean of the (BOB) Gaussian: e^{-gamma dt} p + (1 + e^{-gamma dt}) dt/2 F.
__device__ __forceinline__ double bob_mean(double a, double c1fu, float p, float F) {
  return fma(a, (double)p, c1fu * (double)F);
}

// image deltas (relative to the committed counters) packed in 3 x 10 bits
__device__ __forceinline__ float pack_img(int dx, int dy, int dz) {
  uint32_t v = ((uint32_t)dx & 0x3FFu) | (((uint32_t)dy & 0x3FFu) << 10) |
               (((uint32_t)dz & 0x3FFu) << 20);
  return __uint_as_float(v);
}
__device__ __forceinline__ void unpack_img(float w, int d[3]) {
  int v = (int)__float_as_uint(w);
  d[0] = (v << 22) >> 22;
  d[1] = (v << 12) >> 22;
  d[2] = (v << 2) >> 22;
}

// ---------------------------------------------------------------------------
// Pair geometry and the Lennard-Jones pair force
// ---------------------------------------------------------------------------
// neighbour entry: j << 5 | image code, code = (nx+1) + 3 (ny+1) + 9 (nz+1)
__device__ __forceinline__ int code_nx(int c) { return c % 3 - 1; }
__device__ __forceinline__ int code_ny(int c) { return (c / 3) % 3 - 1; }
__device__ __forceinline__ int code_nz(int c) { return c / 9 - 1; }

// Exact binary64 cutoff predicate: d = (x_j - x_i) + n L, d2 = (dx dx + dy dy)
// + dz dz, d2 < rc2.  Same expression and rounding as the reference
// definition of the pair set.
__device__ __forceinline__ bool inside_exact(float4 xi, float4 xj, int code, double L,
                                             double rc2) {
  double dx = ((double)xj.x - (double)xi.x) + (double)code_nx(code) * L;
  double dy = ((double)xj.y - (double)xi.y) + (double)code_ny(code) * L;
  double dz = ((double)xj.z - (double)xi.z) + (double)code_nz(code) * L;
  double d2 = dx * dx + dy * dy + dz * dz;
  return d2 < rc2;
}

// Separation of the image n of j from i in binary32 without cancellation
// across the box boundary: the box edge is subtracted from whichever
// coordinate lies in the far half of the box (that subtraction is exact), so
// dx = (x_j + min(n,0) L) - (x_i - max(n,0) L) has relative error <= 4u.
// sj = min(n,0) L and si = max(n,0) L per component.
__device__ __forceinline__ float sep(float xj, float sj, float xi, float si) {
  return (xj + sj) - (xi - si);
}

// Lennard-Jones force on i from image n of j; returns whether the pair is
// inside the cutoff.  The binary32 distance decides unless it falls in the
// relative band rc2 (1 -+ 32u) around the cutoff, where the exact binary64
// predicate decides.  The squared distance and the accumulations are fused
// multiply-adds (one rounding each, so the squared distance stays inside the
// error the band allows for); the pair energy is added as
// (eps4/2) s6 (s6 - 1) - eshift/2.
__device__ __forceinline__ bool lj_pair(const PotDev& P, float4 xi, float4 xj, const float* sj,
                                        const float* si, int code, double L, float& fx, float& fy,
                                        float& fz, float& e) {
  float dx = sep(xj.x, sj[0], xi.x, si[0]);
  float dy = sep(xj.y, sj[1], xi.y, si[1]);
  float dz = sep(xj.z, sj[2], xi.z, si[2]);
  float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
  if (r2 >= P.rc2_lo) {
    if (r2 >= P.rc2_hi) return false;
    if (!inside_exact(xi, xj, code, L, P.rc2_d)) return false;
  }
  float inv = __builtin_amdgcn_rcpf(r2);
  float s2 = P.sig2 * inv;
  float s6 = s2 * s2 * s2;
  float fs = P.eps24 * inv * s6 * (2.0f * s6 - 1.0f);
  fx = __builtin_fmaf(-fs, dx, fx);
  fy = __builtin_fmaf(-fs, dy, fy);
  fz = __builtin_fmaf(-fs, dz, fz);
  e = __builtin_fmaf(0.5f * P.eps4 * s6, s6 - 1.0f, e) - 0.5f * P.eshift;
  return true;
}

// Basis values sin(b pi r / rc), b = 1..nb, by the Chebyshev recurrence
// sin((b+1) t) = 2 cos(t) sin(b t) - sin((b-1) t); returns cos(pi r / rc).
__device__ __forceinline__ float pair_basis(float pi_rc, float r, int nb, float* sb) {
  float s, c;
  sincosf(pi_rc * r, &s, &c);
  float prev = 0.0f, cur = s;
  const float two_c = 2.0f * c;
  sb[0] = s;
  for (int b = 1; b < nb; ++b) {
    const float nx = two_c * cur - prev;
    prev = cur;
    cur = nx;
    sb[b] = cur;
  }
  return c;
}

// Pair-draft force on i from image n of j (species spi, spj):
// -f_t(r) d / r with f_t(r) = f_c(r) sum_b w[t][b] sin(b pi r / rc) / r.
__device__ __forceinline__ void pair_draft_force(const PotDev& P, float4 xi, float4 xj,
                                                 const float* sj, const float* si, int spi,
                                                 int spj, float& fx, float& fy, float& fz) {
  const float dx = sep(xj.x, sj[0], xi.x, si[0]);
  const float dy = sep(xj.y, sj[1], xi.y, si[1]);
  const float dz = sep(xj.z, sj[2], xi.z, si[2]);
  const float r2 = dx * dx + dy * dy + dz * dz;
  if (r2 >= P.rc2) return;
  const float r = sqrtf(r2);
  const float inv_r = 1.0f / r;
  const float* w = P.w + pair_type(spi, spj, P.ns) * P.nb;
  float s, c;
  sincosf(P.pi_rc * r, &s, &c);
  float prev = 0.0f, cur = s, acc = w[0] * s;
  const float two_c = 2.0f * c;
  for (int b = 1; b < P.nb; ++b) {
    const float nx = two_c * cur - prev;
    prev = cur;
    cur = nx;
    acc += w[b] * cur;
  }
  const float g = 0.5f * (c + 1.0f) * acc * inv_r * inv_r;  // f_t(r) / r
  fx -= g * dx;
  fy -= g * dy;
  fz -= g * dz;
}

// Radial functions of the learned draft, e_b(r) = f_c(r) sin(b pi r/rc)/r
// for b = 1..B, by the same recurrence; entries from B on are 0.
__device__ __forceinline__ void net_radial(float pi_rc, float r, float inv_r, int B,
                                           float e[LSD_NET_MAX_BASIS]) {
  float s, c;
  sincosf(pi_rc * r, &s, &c);
  const float g0 = 0.5f * (c + 1.0f) * inv_r;
  float prev = 0.0f, cur = s;
  const float two_c = 2.0f * c;
#pragma unroll
  for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) {
    if (b < B) {
      if (b > 0) {
        const float nx = two_c * cur - prev;
        prev = cur;
        cur = nx;
      }
      e[b] = g0 * cur;
    } else {
      e[b] = 0.0f;
    }
  }
}

// Edge coefficients of one atom (first B of its LSD_NET_MAX_BASIS slots).
__device__ __forceinline__ void net_load_v(const float* __restrict__ v, int B,
                                           float out[LSD_NET_MAX_BASIS]) {
  const float4* v4 = reinterpret_cast<const float4*>(v);
#pragma unroll
  for (int q = 0; q < LSD_NET_MAX_BASIS / 4; ++q) {
    float4 t = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (4 * q < B) t = v4[q];
    out[4 * q] = t.x;
    out[4 * q + 1] = t.y;
    out[4 * q + 2] = t.z;
    out[4 * q + 3] = t.w;
  }
}

// Learned-draft pair coefficient f_ij = sum_b e_b (c_t[b] + v_i[b] + v_j[b]).
__device__ __forceinline__ float net_pair_coef(const float e[LSD_NET_MAX_BASIS],
                                               const float* __restrict__ ct,
                                               const float vi[LSD_NET_MAX_BASIS],
                                               const float vj[LSD_NET_MAX_BASIS], int B) {
  float f = 0.0f;
#pragma unroll
  for (int b = 0; b < LSD_NET_MAX_BASIS; ++b)
    if (b < B) f += e[b] * ((ct[b] + vi[b]) + vj[b]);
  return f;
}

// per image code: sj = min(n,0) L, si = max(n,0) L for x, y, z
__device__ __forceinline__ void image_shifts(int code, float Lf, float sj[3], float si[3]) {
  const int n[3] = {code_nx(code), code_ny(code), code_nz(code)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sj[a] = n[a] < 0 ? -Lf : 0.0f;
    si[a] = n[a] > 0 ? Lf : 0.0f;
  }
}

// List entries of one lane whose loads are issued together in the draft-side
// force loops: the row entries, then the neighbour positions and species,
// so that the gathers of several entries are in flight at once.  Entries are
// still added in the lane's order; NL lanes share a row (lane `sub` takes
// entries sub, sub + NL, ...).
#ifndef LSD_GATHER
#define LSD_GATHER 4
#endif
struct Gathered {
  float4 x[LSD_GATHER];
  int code[LSD_GATHER], j[LSD_GATHER], sp[LSD_GATHER];
  bool ok[LSD_GATHER];
};
// The entry words are read for every slot below the row width (words past
// the count are read but not used), so the first group's loads need not wait
// for the count; an unused slot gathers atom 0.
template <int NL = LSD_LPA>
__device__ __forceinline__ void gather_entries(const uint32_t* __restrict__ row, int width,
                                               int cnt, int m0, const float4* __restrict__ X,
                                               const int* __restrict__ species, Gathered& g) {
  uint32_t ent[LSD_GATHER];
#pragma unroll
  for (int u = 0; u < LSD_GATHER; ++u) {
    const int m = m0 + u * NL;
    g.ok[u] = m < cnt;
    ent[u] = row[m < width ? m : 0];
  }
#pragma unroll
  for (int u = 0; u < LSD_GATHER; ++u) {
    g.j[u] = g.ok[u] ? (int)(ent[u] >> 5) : 0;
    g.code[u] = (int)(ent[u] & 31u);
    g.x[u] = X[g.j[u]];
    g.sp[u] = species ? species[g.j[u]] : 0;
  }
}

// sum over the NL lanes of an atom (aligned groups of NL lanes) by a fixed
// butterfly
template <int NL>
__device__ __forceinline__ float lanes_sum(float v) {
#pragma unroll
  for (int o = 1; o < NL; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float lpa_sum(float v) { return lanes_sum<LSD_LPA>(v); }

// Learned-draft force on atom i (replica r) at frame positions X from its
// list row: F_i = - sum_j f_ij d / r with the edge coefficients P.v of this
// frame and the pair-type coefficients ctab [T][B] (the parameters' c
// block, or a copy of it in LDS); the NL lanes of the atom split the row as
// in every force loop and the result is their fixed butterfly sum.
template <int NL = LSD_LPA>
__device__ __forceinline__ void net_force(const PotDev& P, const SysDev& S,
                                          const float4* __restrict__ X,
                                          const uint32_t* __restrict__ row, int width, int cnt,
                                          int i, int r, int sub, const float* __restrict__ ctab,
                                          float& fx, float& fy, float& fz) {
  fx = fy = fz = 0.0f;
  const float Lf = (float)S.box[r];
  const float4 xi = X[i];
  const int spi = S.species ? S.species[i] : 0;
  const int B = P.nb;
  float vi[LSD_NET_MAX_BASIS];
  net_load_v(P.v + (size_t)i * LSD_NET_MAX_BASIS, B, vi);
  // the first group of entries is gathered whatever the count (its loads
  // overlap those of the count), the rest while entries remain
  for (int m0 = sub, first = 1; first || m0 < cnt; m0 += LSD_GATHER * NL, first = 0) {
    Gathered gt;
    gather_entries<NL>(row, width, cnt, m0, X, S.species, gt);
#pragma unroll
    for (int u = 0; u < LSD_GATHER; ++u) {
      if (!gt.ok[u]) break;
      float sj[3], si[3];
      image_shifts(gt.code[u], Lf, sj, si);
      const float dx = sep(gt.x[u].x, sj[0], xi.x, si[0]);
      const float dy = sep(gt.x[u].y, sj[1], xi.y, si[1]);
      const float dz = sep(gt.x[u].z, sj[2], xi.z, si[2]);
      const float r2 = dx * dx + dy * dy + dz * dz;
      if (r2 >= P.rc2) continue;
      const float rr = sqrtf(r2);
      const float inv_r = 1.0f / rr;
      float eb[LSD_NET_MAX_BASIS], vj[LSD_NET_MAX_BASIS];
      net_radial(P.pi_rc, rr, inv_r, B, eb);
      net_load_v(P.v + (size_t)gt.j[u] * LSD_NET_MAX_BASIS, B, vj);
      const float* ct = ctab + pair_type(spi, gt.sp[u], P.ns) * B;
      const float g = net_pair_coef(eb, ct, vi, vj, B) * inv_r;
      fx -= g * dx;
      fy -= g * dy;
      fz -= g * dz;
    }
  }
  fx = lanes_sum<NL>(fx);
  fy = lanes_sum<NL>(fy);
  fz = lanes_sum<NL>(fz);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
