// mpnn.hip -- the message-passing target evaluated on a batch of frames.
//
// Edges: the in-cutoff entries of every atom's list in every frame, compacted
// per (frame, atom) row in list order (count, scan, write).  The filters
// depend only on the distance, so they (and dE/dr) are evaluated once per
// unordered pair: the directed edge from the lower row (or, for an atom and
// its own image, the one with the positive image code) owns the pair, and the
// reverse edge refers to it.  The dense filter contractions thus run over
// the pairs that contribute, once each.
// Forward (per layer t): filters W_t(r) = f_c(r) (A2 silu(A1 e(r) + a1) + a2)
// for every edge, X_t = B_t h, m = sum over edges W_t (.) X_t[neighbour],
// h += C2 silu(C1 m + c1) + c2; readout E = s_E sum (w2 . silu(W1 h + b1) + b2).
// Reverse pass to the forces F = -dE/dq: gh = dE/dh from the readout, then per
// layer gM = dE/dm, gX = dE/dX (gathered over each atom's own list, using
// W_ij = W_ji), and per pair dE/dr accumulated for both directions of the
// pair; finally F_a = sum over a's edges of dE/dr * (q_b - q_a) / r.
//
// Dense contractions on the matrix cores (v_mfma_f32_16x16x32_bf16, binary32
// accumulation).  Every binary32 operand x is split into bfloat16 parts
// hi = bf16(x), lo = bf16(x - hi) (|x - hi - lo| <= 2^-18 |x|), and a product
// is formed as hi.hi + hi.lo + lo.hi: per product a relative error of at most
// about 3 x 2^-18 before the binary32 accumulation, with the range of
// binary32.  The weight matrices are split once (mpnn_prepare), the
// activations as they are loaded.  Operand layout of the instruction: lane l
// holds A[l % 16][8 (l / 16) + 0..7] and B[8 (l / 16) + 0..7][l % 16]; the
// result D[4 (l / 16) + 0..3][l % 16].  The weights are the A operand (rows =
// output channels), the activations of 16 rows (or pairs) the B operand, so
// a lane ends with four consecutive channels of one row.
//
// Nothing here reads a count on the host: the edge and pair totals stay in
// device memory and every kernel bounds itself by them, so an evaluation can
// be captured in a graph.  More pairs than the buffers hold, or edge lists
// whose two directions differ, are latched in the system's status word.
#include <climits>
#include <cstdio>

#include "mpnn.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNoPair = INT_MAX;  // uid of an edge whose pair is past the capacity

// Frames of an evaluation of frames f0 .. f0 + nf - 1 that can be valid:
// below the device bound on the window's valid frames (all nf without one).
// Rows are frame-major, so the rows to evaluate are a prefix.
__device__ __forceinline__ int eff_frames(const int* nvalid, int f0, int nf) {
  if (!nvalid) return nf;
  const int v = nvalid[0] - f0;
  return v < 0 ? 0 : (v < nf ? v : nf);
}

// logistic function from the hardware exponential and reciprocal (each
// within about one ulp; far below the binary32 rounding of the products
// around them)
__device__ __forceinline__ float sigmoidf(float x) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-x));
}
__device__ __forceinline__ float siluf(float x) { return x * sigmoidf(x); }
__device__ __forceinline__ float dsiluf(float x) {
  const float s = sigmoidf(x);
  return s * (1.0f + x * (1.0f - s));
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// bfloat16 hi/lo parts of eight binary32 values (round to nearest even)
__device__ __forceinline__ void split8(const float x[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

// acc += a . b with both operands split (the lo.lo term is dropped)
__device__ __forceinline__ f32x4 mfma3(bf16x8 ahi, bf16x8 alo, bf16x8 bhi, bf16x8 blo, f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc, 0, 0, 0);
}

// Separation of list entry m of atom i in local frame fl; true when the pair
// is inside the cutoff (0 < r < rc).
__device__ __forceinline__ bool edge_geometry(const SysDev& S, const ListDev& L, const WinDev& W,
                                              int f0, int fl, int i, int m, float rc, int* j_out,
                                              float d[3], float* r_out) {
  const long N = S.n;
  const uint32_t ent = L.nbr_t[(size_t)i * L.mt + m];
  const int j = (int)(ent >> 5), code = (int)(ent & 31u);
  const float Lf = (float)S.box[S.atom_rep[i]];
  const float4* X = W.qmid + (size_t)(f0 + fl) * N;
  const float4 xi = X[i], xj = X[j];
  float sj[3], si[3];
  image_shifts(code, Lf, sj, si);
  d[0] = sep(xj.x, sj[0], xi.x, si[0]);
  d[1] = sep(xj.y, sj[1], xi.y, si[1]);
  d[2] = sep(xj.z, sj[2], xi.z, si[2]);
  const float r = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  *j_out = j;
  *r_out = r;
  return r < rc && r > 0.f;
}

// Per (frame, atom) row, one block of kRowThreads threads over the list
// entries (entry m handled by thread m % kRowThreads in pass m / kRowThreads):
// in-cutoff flags and, from ballots, each entry's rank among the row's
// in-cutoff entries and owner entries (list order).
constexpr int kRowThreads = 128;

struct RowScan {
  int edges, owners;  // totals of the row
};

template <bool WRITE>
__device__ __forceinline__ RowScan row_pass(MpnnBuffers& b, const SysDev& S, const ListDev& L,
                                            const WinDev& W, int f0, long row, float rc,
                                            long pair_cap) {
  __shared__ int s_e[kRowThreads / 64], s_o[kRowThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int fl = (int)(row / S.n), i = (int)(row - (long)fl * S.n);
  // frames that are not verified (past the skin or the step limit, or after
  // a rejection already found in a pipelined window) contribute no edges
  const int rep = S.atom_rep[i];
  const bool live = W.invalid[(size_t)rep * S.kmax + f0 + fl] == 0 && f0 + fl <= W.rej[rep];
  const int cnt = live ? L.cnt_t[i] : 0;
  int base_e = WRITE ? b.off[row] : 0, base_o = WRITE ? b.poff[row] : 0;
  int tot_e = 0, tot_o = 0;
  for (int m0 = 0; m0 < cnt; m0 += kRowThreads) {
    const int m = m0 + t;
    int j = 0, code = 0;
    float d[3] = {0.f, 0.f, 0.f}, r = 0.f;
    bool in = false, own = false;
    if (m < cnt) {
      in = edge_geometry(S, L, W, f0, fl, i, m, rc, &j, d, &r);
      code = (int)(L.nbr_t[(size_t)i * L.mt + m] & 31u);
      own = in && (i < j || (i == j && code > 13));
    }
    const unsigned long long be = __ballot(in), bo = __ballot(own);
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) {
      s_e[wave] = __popcll(be);
      s_o[wave] = __popcll(bo);
    }
    __syncthreads();
    int pe = 0, po = 0;
    for (int q = 0; q < wave; ++q) {
      pe += s_e[q];
      po += s_o[q];
    }
    int ce = 0, co = 0;
    for (int q = 0; q < kRowThreads / 64; ++q) {
      ce += s_e[q];
      co += s_o[q];
    }
    if (WRITE && in) {
      const long e = base_e + tot_e + pe + __popcll(be & below);
      b.erow[e] = (int)row;
      b.enbr[e] = (int)((long)fl * S.n + j);
      b.ecode[e] = code;
      if (own) {
        const int pp = base_o + tot_o + po + __popcll(bo & below);
        if (pp < pair_cap) {
          b.uid[e] = pp;
          b.ua[pp] = (int)row;
          b.ub[pp] = (int)((long)fl * S.n + j);
          b.uv[4 * pp] = d[0] / r;
          b.uv[4 * pp + 1] = d[1] / r;
          b.uv[4 * pp + 2] = d[2] / r;
          b.uv[4 * pp + 3] = r;
        } else {
          // more pairs than the buffers hold: latched, never written
          b.uid[e] = kNoPair;
          atomicOr(L.status, LSD_STATUS_PAIRS);
        }
      } else {
        b.uid[e] = -1;  // reverse edge: resolved by k_mp_reverse
      }
    }
    tot_e += ce;
    tot_o += co;
    __syncthreads();
  }
  return RowScan{tot_e, tot_o};
}

// in-cutoff entries and owned pairs per row
__global__ __launch_bounds__(kRowThreads) void k_mp_count(MpnnBuffers b, SysDev S, ListDev L,
                                                          WinDev W, int f0, int nf,
                                                          const int* nvalid, float rc) {
  const long row = blockIdx.x;
  if (row >= (long)eff_frames(nvalid, f0, nf) * S.n) {  // uniform
    if (threadIdx.x == 0) {
      b.off[row] = 0;
      b.poff[row] = 0;
    }
    return;
  }
  const RowScan c = row_pass<false>(b, S, L, W, f0, row, rc, 0);
  if (threadIdx.x == 0) {
    b.off[row] = c.edges;
    b.poff[row] = c.owners;
  }
}

// Exclusive scans of the row counts of edges (off) and pairs (poff) in place;
// off[rows], poff[rows] = totals, also copied to counts[0..1].
// Small evaluations (up to kScanSingleMax rows): one block, thread t scanning
// the contiguous rows [t chunk, (t+1) chunk) of the rows that can hold edges
// (the valid-frame prefix); the rows after it get the totals.  Large ones:
// blocks of kScanTile rows scan their tile (coalesced, wave scans) and record
// its totals, one block scans the totals, and a last pass adds each tile's
// offset.
constexpr int kScanTile = 1024;
constexpr int kScanChunk = 16;                          // rows per thread of the single-block form
constexpr long kScanSingleMax = 1024L * kScanChunk;     // rows scanned by the single-block form

__device__ __forceinline__ int block_scan_incl(int v, int* s_w, int* total);

__global__ __launch_bounds__(1024) void k_mp_scan(MpnnBuffers b, long rows, long n_atoms, int f0,
                                                  int nf, const int* nvalid) {
  __shared__ int s_w[32];
  const int t = threadIdx.x;
  const long live = (long)eff_frames(nvalid, f0, nf) * n_atoms;  // <= rows
  const long chunk = (live + 1023) / 1024;
  const long lo = min(live, (long)t * chunk), hi = min(live, lo + chunk);
  int c1[kScanChunk], c2[kScanChunk];
  int sum = 0, sum2 = 0;
#pragma unroll
  for (int u = 0; u < kScanChunk; ++u) {
    const long r = lo + u;
    c1[u] = r < hi ? b.off[r] : 0;
    c2[u] = r < hi ? b.poff[r] : 0;
  }
#pragma unroll
  for (int u = 0; u < kScanChunk; ++u) {
    sum += c1[u];
    sum2 += c2[u];
  }
  int tot, tot2;
  int run = block_scan_incl(sum, s_w, &tot) - sum;
  int run2 = block_scan_incl(sum2, s_w, &tot2) - sum2;
#pragma unroll
  for (int u = 0; u < kScanChunk; ++u) {
    const long r = lo + u;
    if (r < hi) {
      b.off[r] = run;
      b.poff[r] = run2;
    }
    run += c1[u];
    run2 += c2[u];
  }
  for (long r = live + t; r <= rows; r += 1024) {
    b.off[r] = tot;
    b.poff[r] = tot2;
  }
  if (t == 0) {
    b.counts[0] = tot;
    b.counts[1] = tot2;
  }
}

// inclusive scan of one int over a 1024-thread block (wave scans, then the
// sixteen wave totals); returns the inclusive prefix, *total the block sum
__device__ __forceinline__ int block_scan_incl(int v, int* s_w, int* total) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  if (lane == 63) s_w[wave] = v;
  __syncthreads();
  if (t < 64) {
    int w = t < 16 ? s_w[t] : 0;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const int u = __shfl_up(w, o, 64);
      if (t >= o) w += u;
    }
    if (t < 16) s_w[16 + t] = w;  // inclusive prefix of the wave totals
  }
  __syncthreads();
  const int incl = v + (wave > 0 ? s_w[16 + wave - 1] : 0);
  *total = s_w[16 + 15];
  __syncthreads();
  return incl;
}

// pass 1: each tile's exclusive prefixes and totals
__global__ __launch_bounds__(1024) void k_mp_scan_tiles(MpnnBuffers b, long rows, int* tile_sums) {
  __shared__ int s_w[32];
  const long r = (long)blockIdx.x * kScanTile + threadIdx.x;
  const int v1 = r < rows ? b.off[r] : 0, v2 = r < rows ? b.poff[r] : 0;
  int t1, t2;
  const int i1 = block_scan_incl(v1, s_w, &t1);
  const int i2 = block_scan_incl(v2, s_w, &t2);
  if (r < rows) {
    b.off[r] = i1 - v1;
    b.poff[r] = i2 - v2;
  }
  if (threadIdx.x == 0) {
    tile_sums[2 * blockIdx.x] = t1;
    tile_sums[2 * blockIdx.x + 1] = t2;
  }
}

// pass 2: exclusive prefixes of the tile totals (one block, up to 1024
// tiles per round; rounds carried)
__global__ __launch_bounds__(1024) void k_mp_scan_top(MpnnBuffers b, long rows, int* tile_sums,
                                                      int tiles) {
  __shared__ int s_w[32];
  int carry1 = 0, carry2 = 0;
  for (int base = 0; base < tiles; base += 1024) {
    const int i = base + threadIdx.x;
    const int v1 = i < tiles ? tile_sums[2 * i] : 0, v2 = i < tiles ? tile_sums[2 * i + 1] : 0;
    int t1, t2;
    const int i1 = block_scan_incl(v1, s_w, &t1);
    const int i2 = block_scan_incl(v2, s_w, &t2);
    if (i < tiles) {
      tile_sums[2 * i] = carry1 + i1 - v1;
      tile_sums[2 * i + 1] = carry2 + i2 - v2;
    }
    carry1 += t1;
    carry2 += t2;
  }
  if (threadIdx.x == 0) {
    b.off[rows] = carry1;
    b.poff[rows] = carry2;
    b.counts[0] = carry1;
    b.counts[1] = carry2;
  }
}

// pass 3: add each tile's offset
__global__ __launch_bounds__(1024) void k_mp_scan_add(MpnnBuffers b, long rows,
                                                      const int* __restrict__ tile_sums) {
  const long r = (long)blockIdx.x * kScanTile + threadIdx.x;
  if (r >= rows) return;
  b.off[r] += tile_sums[2 * blockIdx.x];
  b.poff[r] += tile_sums[2 * blockIdx.x + 1];
}

// directed edge records of every row in list order, and the pair records of
// the edges the row owns
__global__ __launch_bounds__(kRowThreads) void k_mp_edges(MpnnBuffers b, SysDev S, ListDev L,
                                                          WinDev W, int f0, int nf,
                                                          const int* nvalid, float rc,
                                                          long pair_cap) {
  if ((long)blockIdx.x >= (long)eff_frames(nvalid, f0, nf) * S.n) return;  // no edges
  row_pass<true>(b, S, L, W, f0, blockIdx.x, rc, pair_cap);
}

// Fixed grids over a list of n items (edges or pairs, ordered by row): the
// blocks are dealt to the eight XCDs in turn (block b to XCD b mod 8), so XCD
// x takes the contiguous eighth [x c, (x + 1) c), c = ceil(n / 8), of the
// items, its gridDim / 8 blocks striding through it.  The rows an item reads
// (its own and its neighbour's, close in the ordering) then come through one
// L2.  The grid is a multiple of eight.
struct XcdSpan {
  long base, end, first, stride;
  __device__ __forceinline__ XcdSpan(long n, int per_block, int local) {
    const long c = (n + 7) / 8;
    const int x = blockIdx.x % 8;
    base = (long)x * c;
    end = base + c < n ? base + c : n;
    first = base + (long)(blockIdx.x / 8) * per_block + local;
    stride = (long)(gridDim.x / 8) * per_block;
  }
};

// every reverse edge refers to its owner: the neighbour row's edge back to
// this row with the opposite image; uid = ~pair (kNoPair if the owner's pair
// is past the capacity).  Sixteen lanes per edge test sixteen of the
// neighbour row's edges at a time; the first match in row order wins.
constexpr int kRevLanes = 16;
constexpr unsigned kRevBlocks = 2048;  // fixed grid; edges taken in strides

__global__ __launch_bounds__(256) void k_mp_reverse(MpnnBuffers b, long rows, long cap,
                                                    int* __restrict__ status) {
  const int sub = threadIdx.x % kRevLanes;
  const int lane = threadIdx.x & 63, g0 = lane & ~(kRevLanes - 1);
  const long n_edges = min((long)b.off[rows], cap);
  const XcdSpan xs(n_edges, blockDim.x / kRevLanes, threadIdx.x / kRevLanes);
  for (long e = xs.first; e < xs.end; e += xs.stride) {
    if (b.uid[e] >= 0) continue;  // an owner edge (or a capped one): uniform over the lanes
    const int rj = b.enbr[e], ri = b.erow[e], back = 26 - b.ecode[e];
    const int q0 = b.off[rj], q1 = b.off[rj + 1];
    int found = -1;
    for (int q = q0; q < q1; q += kRevLanes) {
      const int qq = q + sub;
      const bool hit = qq < q1 && b.enbr[qq] == ri && b.ecode[qq] == back;
      const unsigned long long m = (__ballot(hit) >> g0) & ((1ull << kRevLanes) - 1);
      if (m) {
        found = b.uid[q + __ffsll((long long)m) - 1];
        break;
      }
    }
    if (sub == 0) {
      if (found < 0) {
        atomicOr(status, LSD_STATUS_EDGES);  // the edge sets of the two directions differ
        found = kNoPair;
      }
      b.uid[e] = found == kNoPair ? kNoPair : ~found;
    }
  }
}

// pairs the buffers hold
__device__ __forceinline__ long held_pairs(const MpnnBuffers& b, long cap) {
  const long n = b.counts[1];
  return n < cap ? n : cap;
}

// Filters of every pair and layer (Sec. 8 target, layer t):
//   z = A1 e(r) + a1, S = silu(z), DS = silu'(z) (A1 de/dr)   (binary32)
//   W = f_c (A2 S + a2),  dW/dr = f_c' (A2 S + a2) + f_c A2 DS (matrix cores)
// Block: 4 waves, tiles of 32 pairs; wave w holds the A2 fragments of the
// output channels 32 w .. 32 w + 31 of the current layer in registers, and
// the layers are the outer loop, so A2 is read once per block and layer.
constexpr int kFiltPairs = 32;
constexpr int kFiltLd = MP_H + 8;  // bfloat16 row stride of the staged S, DS (no bank conflicts)

__global__ __launch_bounds__(256) void k_mp_filter(MpnnWeights w, MpnnBuffers b, float rc,
                                                   long cap) {
  __shared__ float s_e[kFiltPairs][MP_R], s_de[kFiltPairs][MP_R];
  __shared__ float s_fc[kFiltPairs], s_dfc[kFiltPairs];
  __shared__ __align__(16) __bf16 s_sh[kFiltPairs][kFiltLd], s_sl[kFiltPairs][kFiltLd];
  __shared__ __align__(16) __bf16 s_dh[kFiltPairs][kFiltLd], s_dl[kFiltPairs][kFiltLd];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const long np = held_pairs(b, cap);
  const long ntiles = (np + kFiltPairs - 1) / kFiltPairs;
  if ((long)blockIdx.x >= ntiles) return;  // uniform
  const float pre = sqrtf(2.0f / rc), pi_rc = 3.14159265358979f / rc;
  for (int l = 0; l < MP_T; ++l) {
    bf16x8 ah[2][4], al[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const long fi = ((long)(2 * wave + mt) * 4 + ks) * 64 + lane;
        ah[mt][ks] = as_bf16x8(w.A2f[l].hi[fi]);
        al[mt][ks] = as_bf16x8(w.A2f[l].lo[fi]);
      }
    bf16x8 a1h[2], a1l[2];
    float a1v[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const long fi = (long)(2 * wave + mt) * 64 + lane;
      a1h[mt] = as_bf16x8(w.A1f[l].hi[fi]);
      a1l[mt] = as_bf16x8(w.A1f[l].lo[fi]);
#pragma unroll
      for (int q = 0; q < 4; ++q) a1v[mt][q] = w.a1[l][32 * wave + 16 * mt + 4 * (lane >> 4) + q];
    }
    float a2v[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) a2v[mt][q] = w.a2[l][32 * wave + 16 * mt + 4 * (lane >> 4) + q];
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      const long p0 = tile * kFiltPairs;
      // radial basis e_b(r) = sqrt(2/rc) sin(b pi r/rc)/r, de_b/dr, cutoff;
      // eight threads per pair, two functions each: sin and cos of the
      // first one's angle, the second one's by a rotation by pi r/rc
      {
        const int q = t >> 3, b0 = 2 * (t & 7);
        const long p = p0 + q;
        const float r = p < np ? b.uv[4 * p + 3] : 0.5f * rc;
        const float inv_r = 1.0f / r;
        float s1, c1, sn, cs;
        sincosf(pi_rc * r, &s1, &c1);
        sincosf((float)(b0 + 1) * pi_rc * r, &sn, &cs);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int bb = b0 + u;
          const float k = (float)(bb + 1) * pi_rc;
          s_e[q][bb] = pre * sn * inv_r;
          s_de[q][bb] = pre * (k * cs - sn * inv_r) * inv_r;
          const float sn2 = sn * c1 + cs * s1, cs2 = cs * c1 - sn * s1;
          sn = sn2;
          cs = cs2;
        }
        if ((t & 7) == 0) {
          s_fc[q] = 0.5f * (c1 + 1.0f);
          s_dfc[q] = -0.5f * pi_rc * s1;
        }
      }
      __syncthreads();
      // first layer of the filter MLP on the matrix cores (16 inputs padded
      // to 32): z = A1 e + a1 and A1 de/dr per channel and pair; then
      // S = silu(z), DS = silu'(z) (A1 de/dr), staged as bfloat16 parts
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int q = 16 * nt + (lane & 15), kk = 8 * (lane >> 4);
        float xe[8], xd[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          xe[e] = kk < MP_R ? s_e[q][kk + e] : 0.0f;
          xd[e] = kk < MP_R ? s_de[q][kk + e] : 0.0f;
        }
        bf16x8 beh, bel, bdh, bdl;
        split8(xe, beh, bel);
        split8(xd, bdh, bdl);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
          const f32x4 z = mfma3(a1h[mt], a1l[mt], beh, bel, zero);
          const f32x4 dz = mfma3(a1h[mt], a1l[mt], bdh, bdl, zero);
          __bf16 sh[4], sl[4], dh[4], dl[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float zz = z[e] + a1v[mt][e];
            const float sg = sigmoidf(zz);
            const float S = zz * sg, DS = sg * (1.0f + zz * (1.0f - sg)) * dz[e];
            sh[e] = (__bf16)S;
            sl[e] = (__bf16)(S - (float)sh[e]);
            dh[e] = (__bf16)DS;
            dl[e] = (__bf16)(DS - (float)dh[e]);
          }
          const int c0 = 32 * wave + 16 * mt + 4 * (lane >> 4);
          *reinterpret_cast<uint2*>(&s_sh[q][c0]) = __builtin_bit_cast(uint2, sh);
          *reinterpret_cast<uint2*>(&s_sl[q][c0]) = __builtin_bit_cast(uint2, sl);
          *reinterpret_cast<uint2*>(&s_dh[q][c0]) = __builtin_bit_cast(uint2, dh);
          *reinterpret_cast<uint2*>(&s_dl[q][c0]) = __builtin_bit_cast(uint2, dl);
        }
      }
      __syncthreads();
      // A2 S and A2 DS for 16 pairs at a time
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int q = 16 * nt + (lane & 15), kk = 8 * (lane >> 4);
        f32x4 z[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        f32x4 dz[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const bf16x8 bsh = *reinterpret_cast<const bf16x8*>(&s_sh[q][32 * ks + kk]);
          const bf16x8 bsl = *reinterpret_cast<const bf16x8*>(&s_sl[q][32 * ks + kk]);
          const bf16x8 bdh = *reinterpret_cast<const bf16x8*>(&s_dh[q][32 * ks + kk]);
          const bf16x8 bdl = *reinterpret_cast<const bf16x8*>(&s_dl[q][32 * ks + kk]);
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            z[mt] = mfma3(ah[mt][ks], al[mt][ks], bsh, bsl, z[mt]);
            dz[mt] = mfma3(ah[mt][ks], al[mt][ks], bdh, bdl, dz[mt]);
          }
        }
        const long p = p0 + q;
        if (p < np) {
          const float fc = s_fc[q], dfc = s_dfc[q];
#pragma unroll
          for (int mt = 0; mt < 2; ++mt) {
            float4 wv, vv;
            float* wp = &wv.x;
            float* vp = &vv.x;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float y = z[mt][e] + a2v[mt][e];
              wp[e] = fc * y;
              vp[e] = dfc * y + fc * dz[mt][e];
            }
            const long o = p * MP_HT + l * MP_H + 32 * wave + 16 * mt + 4 * (lane >> 4);
            *reinterpret_cast<float4*>(b.Wf + o) = wv;
            *reinterpret_cast<float4*>(b.Vf + o) = vv;
          }
        }
      }
      __syncthreads();  // the next tile rewrites the staged values
    }
  }
}

// rows of an evaluation that are computed: the frames below the device bound
struct RowSpan {
  const int* nvalid;
  int f0, nf;
  long n;
  const int* atom_rep;   // [N]
  const int* invalid;    // [R][kmax]
  const int* rej;        // [R]
  int kmax;
  __device__ __forceinline__ long rows() const { return (long)eff_frames(nvalid, f0, nf) * n; }
  // the row's frame is one the window verifies (the same test as the edges')
  __device__ __forceinline__ bool live(long row) const {
    const int fl = (int)(row / n), i = (int)(row - (long)fl * n);
    const int r = atom_rep[i];
    return invalid[(size_t)r * kmax + f0 + fl] == 0 && f0 + fl <= rej[r];
  }
};

// Row chains: the node MLPs between two gathers, fused.  A block owns 16 NT
// consecutive rows (NT tiles of 16) and runs a fixed sequence of stages on
// them; each stage is one product out = in . op on the matrix cores (the
// weights' fragments of the stage in registers, wave w computing the output
// channels [w ND/4, (w+1) ND/4) of every tile) with its epilogue, the input
// and output tiles staying in LDS between stages.
//   CH_EMBED     h0 = W_emb[s]            -> H0; X0 = h0 B0^T         -> X0
//   CH_FWD(t)    U = m C1^T + c1           -> U_t; Sn = silu(U)
//                h' = h + Sn C2^T + c2     -> H_{t+1}; X = h' B_{t+1}^T -> X_{t+1}
//   CH_LAST      the same up to h' = h_T, then the readout and the row part
//                of the reverse pass of the last layer:
//                y = h_T W1^T + b1, e = s_E (w2 . silu(y) + b2) -> energy per row,
//                gY = s_E w2 (.) silu'(y), gH = gY W1                -> gH
//                gS = (gH C2) (.) silu'(U_t), gM = gS C1              -> gM
//   CH_BWD(t)    gH' = gH + gX B_{t+1}     -> gH (other buffer)
//                gS = (gH' C2_t) (.) silu'(U_t), gM = gS C1_t          -> gM
enum ChainMode { CH_EMBED = 0, CH_FWD = 1, CH_LAST = 2, CH_BWD = 3 };

constexpr int kChainLd = MP_H + 4;        // fp32 row stride of the LDS tiles

struct ChainArgs {
  int t;                                  // layer
  const float* in;                        // m (CH_FWD, CH_LAST) or gX (CH_BWD), [rows][128]
  const float* h;                         // h_t (CH_FWD, CH_LAST)
  float* u_out;                           // U_t (CH_FWD, CH_LAST)
  float* h_out;                           // h_{t+1} (CH_EMBED: h0; CH_FWD)
  float* x_out;                           // X_{t+1} (CH_EMBED: X0; CH_FWD)
  const float* gh;                        // gH (CH_BWD)
  float* gh_out;                          // gH' (CH_BWD) or gH (CH_LAST)
  const float* u_in;                      // U_t (CH_BWD)
  float* gm_out;                          // gM (CH_LAST, CH_BWD)
  double* e_row;                          // energy of every row (CH_LAST)
  float scale;
};

// out = tile . op for the 64 rows staged in `in` (LDS); the epilogue gets
// (row in block, channel c0, four values) for four consecutive channels.
template <int NT, int KD, int ND, typename Epi>
__device__ __forceinline__ void chain_stage(const MpnnFrag& op, const float (*in)[kChainLd],
                                            Epi epi) {
  constexpr int KS = KD / 32, MT = ND / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bf16x8 ah[MT][KS], al[MT][KS];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const long fi = ((long)(MT * wave + mt) * KS + ks) * 64 + lane;
      ah[mt][ks] = as_bf16x8(op.hi[fi]);
      al[mt][ks] = as_bf16x8(op.lo[fi]);
    }
  const int kk = 8 * (lane >> 4);
#pragma unroll 1
  for (int nt = 0; nt < NT; ++nt) {
    const int rr = 16 * nt + (lane & 15);
    f32x4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float4 u0 = *reinterpret_cast<const float4*>(&in[rr][32 * ks + kk]);
      const float4 u1 = *reinterpret_cast<const float4*>(&in[rr][32 * ks + kk + 4]);
      const float x[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
      bf16x8 bh, bl;
      split8(x, bh, bl);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma3(ah[mt][ks], al[mt][ks], bh, bl, acc[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      epi(rr, (ND / 4) * wave + 16 * mt + 4 * (lane >> 4), acc[mt]);
  }
}

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

// The row part of the reverse pass of layer t from gH (staged in `g`):
// gS = (gH C2_t) (.) silu'(U_t) into `scratch`, gM = gS C1_t to global.
template <int NT>
__device__ __forceinline__ void chain_tail(const MpnnWeights& w, const ChainArgs& a,
                                           float (*g)[kChainLd], float (*scratch)[kChainLd],
                                           const float (*su)[kChainLd], long r0, long rows) {
  const int l = a.t;
  chain_stage<NT, MP_H, MP_H>(w.C2b[l], g, [&](int rr, int c0, f32x4 v) {
    const float4 u = ld4(&su[rr][c0]);
    const float uv[4] = {u.x, u.y, u.z, u.w};
    float o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = v[e] * dsiluf(uv[e]);
    st4(&scratch[rr][c0], make_float4(o[0], o[1], o[2], o[3]));
  });
  __syncthreads();
  chain_stage<NT, MP_H, MP_H>(w.C1b[l], scratch, [&](int rr, int c0, f32x4 v) {
    const long row = r0 + rr;
    if (row < rows) st4(a.gm_out + row * MP_H + c0, make_float4(v[0], v[1], v[2], v[3]));
  });
  __syncthreads();
}

template <int MODE, int NT>
__global__ __launch_bounds__(256) void k_mp_chain(MpnnWeights w, MpnnBuffers b, SysDev S,
                                                  RowSpan span, ChainArgs a) {
  constexpr int kChainRows = 16 * NT;
  __shared__ __align__(16) float s_a[kChainRows][kChainLd];
  __shared__ __align__(16) float s_b[kChainRows][kChainLd];
  __shared__ __align__(16) float s_u[MODE == CH_EMBED ? 1 : kChainRows][kChainLd];
  __shared__ float s_e[4][kChainRows];
  const long rows = span.rows();
  const int t = threadIdx.x;
  for (long r0 = (long)blockIdx.x * kChainRows; r0 < rows; r0 += (long)gridDim.x * kChainRows) {
    // rows of frames the window does not verify (another replica's
    // truncated window, past the skin) are skipped block by block: no
    // gather or force of a verified frame reads them
    const bool lv = t < kChainRows && r0 + t < rows && span.live(r0 + t);
    if (!__syncthreads_or(lv ? 1 : 0)) continue;
    // stage the block's input rows (zeros past the end)
    for (int idx = t; idx < kChainRows * (MP_H / 4); idx += 256) {
      const int rr = idx / (MP_H / 4), c = 4 * (idx % (MP_H / 4));
      const long row = r0 + rr;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row < rows) {
        if constexpr (MODE == CH_EMBED) {
          const int i = (int)(row % S.n);
          const int sp = S.species ? S.species[i] : 0;
          v = ld4(w.W_emb + sp * MP_H + c);
          st4(a.h_out + row * MP_H + c, v);
        } else {
          v = ld4(a.in + row * MP_H + c);
        }
      }
      st4(&s_a[rr][c], v);
    }
    __syncthreads();
    if constexpr (MODE == CH_EMBED) {
      chain_stage<NT, MP_H, MP_H>(w.Bf[0], s_a, [&](int rr, int c0, f32x4 v) {
        const long row = r0 + rr;
        if (row < rows) st4(a.x_out + row * MP_H + c0, make_float4(v[0], v[1], v[2], v[3]));
      });
      __syncthreads();
      continue;
    }
    if constexpr (MODE == CH_FWD || MODE == CH_LAST) {
      const int l = a.t;
      // U = m C1^T + c1 (kept), Sn = silu(U)
      chain_stage<NT, MP_H, MP_H>(w.C1f[l], s_a, [&](int rr, int c0, f32x4 v) {
        const long row = r0 + rr;
        float u[4], sn[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          u[e] = v[e] + w.c1[l][c0 + e];
          sn[e] = siluf(u[e]);
        }
        st4(&s_u[rr][c0], make_float4(u[0], u[1], u[2], u[3]));
        st4(&s_b[rr][c0], make_float4(sn[0], sn[1], sn[2], sn[3]));
        if (row < rows) st4(a.u_out + row * MP_H + c0, make_float4(u[0], u[1], u[2], u[3]));
      });
      __syncthreads();
      // h' = h + Sn C2^T + c2
      chain_stage<NT, MP_H, MP_H>(w.C2f[l], s_b, [&](int rr, int c0, f32x4 v) {
        const long row = r0 + rr;
        float4 hp = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < rows) hp = ld4(a.h + row * MP_H + c0);
        const float hv[4] = {hp.x, hp.y, hp.z, hp.w};
        float o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = (v[e] + hv[e]) + w.c2[l][c0 + e];
        const float4 ov = make_float4(o[0], o[1], o[2], o[3]);
        st4(&s_a[rr][c0], ov);
        if (MODE == CH_FWD && row < rows) st4(a.h_out + row * MP_H + c0, ov);
      });
      __syncthreads();
      if constexpr (MODE == CH_FWD) {
        // X_{t+1} = h' B_{t+1}^T
        chain_stage<NT, MP_H, MP_H>(w.Bf[l + 1], s_a, [&](int rr, int c0, f32x4 v) {
          const long row = r0 + rr;
          if (row < rows) st4(a.x_out + row * MP_H + c0, make_float4(v[0], v[1], v[2], v[3]));
        });
        __syncthreads();
        continue;
      }
      // readout: y = h_T W1^T + b1; per row e = w2 . silu(y) + b2 and
      // gY = s_E w2 (.) silu'(y) (into s_b, 64 columns)
      chain_stage<NT, MP_H, MP_RH>(w.W1f, s_a, [&](int rr, int c0, f32x4 v) {
        float gy[4], ep = 0.f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float y = v[e] + w.b1[c0 + e];
          const float sg = sigmoidf(y);
          ep = fmaf(w.w2[c0 + e], y * sg, ep);
          gy[e] = a.scale * w.w2[c0 + e] * (sg * (1.0f + y * (1.0f - sg)));
        }
        st4(&s_b[rr][c0], make_float4(gy[0], gy[1], gy[2], gy[3]));
        // the four lane groups of the wave hold consecutive channel quads of
        // the same row: a fixed butterfly, then one value per wave and row
        ep += __shfl_xor(ep, 16, 64);
        ep += __shfl_xor(ep, 32, 64);
        if ((threadIdx.x & 63) < 16) s_e[threadIdx.x >> 6][rr] = ep;
      });
      __syncthreads();
      if (t < kChainRows && r0 + t < rows) {
        const float ei = ((s_e[0][t] + s_e[1][t]) + (s_e[2][t] + s_e[3][t])) + w.b2[0];
        a.e_row[r0 + t] = (double)a.scale * (double)ei;
      }
      // gH = gY W1 (into s_a)
      chain_stage<NT, MP_RH, MP_H>(w.W1b, s_b, [&](int rr, int c0, f32x4 v) {
        const long row = r0 + rr;
        const float4 ov = make_float4(v[0], v[1], v[2], v[3]);
        st4(&s_a[rr][c0], ov);
        if (row < rows) st4(a.gh_out + row * MP_H + c0, ov);
      });
      __syncthreads();
      chain_tail<NT>(w, a, s_a, s_b, s_u, r0, rows);
    } else {  // CH_BWD: gH' = gH + gX B_{t+1} (into s_b)
      chain_stage<NT, MP_H, MP_H>(w.Bb[a.t + 1], s_a, [&](int rr, int c0, f32x4 v) {
        const long row = r0 + rr;
        float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < rows) g = ld4(a.gh + row * MP_H + c0);
        const float4 ov = make_float4(g.x + v[0], g.y + v[1], g.z + v[2], g.w + v[3]);
        st4(&s_b[rr][c0], ov);
        if (row < rows) st4(a.gh_out + row * MP_H + c0, ov);
      });
      // U_t of the block's rows for silu'
      for (int idx = t; idx < kChainRows * (MP_H / 4); idx += 256) {
        const int rr = idx / (MP_H / 4), c = 4 * (idx % (MP_H / 4));
        const long row = r0 + rr;
        st4(&s_u[rr][c], row < rows ? ld4(a.u_in + row * MP_H + c) : make_float4(0.f, 0.f, 0.f, 0.f));
      }
      __syncthreads();
      chain_tail<NT>(w, a, s_b, s_a, s_u, r0, rows);
    }
  }
}

// Fragments of G(i, k) (i: output channel, k: contraction index) for the A
// operand: element [(it KS + ks) 64 + lane][e] = G(16 it + lane % 16,
// 32 ks + 8 (lane / 16) + e), split into bfloat16 hi and lo.  G(i, k) =
// src[i ld + k], or src[k ld + i] when transposed; 0 for k >= Ksrc.
__global__ void k_mp_frag(const float* __restrict__ src, int ld, int trans, int I, int K,
                          int Ksrc, uint4* __restrict__ hi, uint4* __restrict__ lo) {
  const int KS = K / 32;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)(I / 16) * KS * 64) return;
  const int lane = (int)(idx % 64), ks = (int)((idx / 64) % KS), it = (int)(idx / 64 / KS);
  const int i = 16 * it + lane % 16, k0 = 32 * ks + 8 * (lane / 16);
  float x[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = k0 + e;  // contraction indices from Ksrc on are zero padding
    x[e] = k >= Ksrc ? 0.0f : (trans ? src[(long)k * ld + i] : src[(long)i * ld + k]);
  }
  bf16x8 h, l;
  split8(x, h, l);
  hi[idx] = __builtin_bit_cast(uint4, h);
  lo[idx] = __builtin_bit_cast(uint4, l);
}


// out[row][c] = sum over the row's edges e of W_t[pair(e)][c] * V[neighbour row][c]
// (messages with V = X_t; dE/dX with V = gM: W is symmetric in the pair).
// One block of 128 threads (channels) per row; eight edges' loads issued
// together, terms added in edge order.  Blocks are dealt to the eight XCDs in
// turn (block b to XCD b mod 8), so the rows are handed out in pieces of G
// consecutive rows, piece s of XCD x being rows [(8 s + x) G, (8 s + x + 1) G),
// with G = ceil(rows / 8) up to kGatherPiece: the two rows of a pair (atoms
// close in the ordering) then read its filters and each other's features
// through the same L2, and long evaluations (whose later frames hold fewer
// live rows) still spread every frame over all eight XCDs.
constexpr int kGatherDepth = 8;
constexpr long kGatherPiece = 1024;

// grid of the gather: enough blocks for every row count up to rows
static unsigned gather_grid(long rows) {
  const long q = rows <= 8 * kGatherPiece ? 8 : 8 * kGatherPiece;
  return (unsigned)((rows + q - 1) / q * q);
}

__device__ __forceinline__ float pair_filter(const MpnnBuffers& b, int u, int t, int c) {
  if (u == kNoPair) return 0.f;  // only after a latched capacity overflow
  const long p = u >= 0 ? u : ~u;
  return b.Wf[p * MP_HT + t * MP_H + c];
}

__global__ __launch_bounds__(128) void k_mp_gather(MpnnBuffers b, int t, const float* __restrict__ V,
                                                   float* __restrict__ out, RowSpan span) {
  const long nrow = span.rows();
  if (nrow == 0) return;
  const long cch = (nrow + 7) / 8, G = cch < kGatherPiece ? cch : kGatherPiece;
  const long l = blockIdx.x / 8;
  const long row = (l / G) * 8 * G + (long)(blockIdx.x % 8) * G + l % G;
  if (row >= nrow) return;
  const int c = threadIdx.x;
  const int e1 = b.off[row + 1];
  float acc = 0.f;
  int e = b.off[row];
  // the pair and neighbour indices of the next group of edges are requested
  // while this group's filter and feature values load
  int un[kGatherDepth], jn[kGatherDepth];
  if (e + kGatherDepth <= e1) {
#pragma unroll
    for (int q = 0; q < kGatherDepth; ++q) {
      un[q] = b.uid[e + q];
      jn[q] = b.enbr[e + q];
    }
  }
  for (; e + kGatherDepth <= e1; e += kGatherDepth) {
    float wv[kGatherDepth], vv[kGatherDepth];
#pragma unroll
    for (int q = 0; q < kGatherDepth; ++q) {
      wv[q] = pair_filter(b, un[q], t, c);
      vv[q] = V[(long)jn[q] * MP_H + c];
    }
    const int en = e + kGatherDepth;
    if (en + kGatherDepth <= e1) {
#pragma unroll
      for (int q = 0; q < kGatherDepth; ++q) {
        un[q] = b.uid[en + q];
        jn[q] = b.enbr[en + q];
      }
    }
#pragma unroll
    for (int q = 0; q < kGatherDepth; ++q) acc = fmaf(wv[q], vv[q], acc);
  }
  for (; e < e1; ++e) acc = fmaf(pair_filter(b, b.uid[e], t, c), V[(long)b.enbr[e] * MP_H + c], acc);
  out[row * MP_H + c] = acc;
}

// dE/dr of one pair (both directions), layer t:
// sum_c (gM[a] X[b] + gM[b] X[a])_c dW_c/dr.  Thirty-two lanes per pair (four
// channels each, 16-byte loads), two pairs per wave, pairs taken by a fixed
// grid up to the device pair count (in XCD pieces); a fixed butterfly over
// the 32 lanes.  The first layer of the reverse pass stores, the others add.
__global__ __launch_bounds__(256) void k_mp_dedr(MpnnBuffers b, int t, int first,
                                                 const float* __restrict__ X, long cap) {
  const int l32 = threadIdx.x & 31, c = 4 * l32;
  const long np = held_pairs(b, cap);
  const XcdSpan xs(np, 8, threadIdx.x >> 5);
  // the next pair's row indices are requested while this pair's rows load
  int ua = 0, ub = 0;
  if (xs.first < xs.end) {
    ua = b.ua[xs.first];
    ub = b.ub[xs.first];
  }
  for (long p = xs.first; p < xs.end; p += xs.stride) {
    const long ra = (long)ua * MP_H + c, rb = (long)ub * MP_H + c;
    const float4 ga = *reinterpret_cast<const float4*>(b.gM + ra);
    const float4 gb = *reinterpret_cast<const float4*>(b.gM + rb);
    const float4 xa = *reinterpret_cast<const float4*>(X + ra);
    const float4 xb = *reinterpret_cast<const float4*>(X + rb);
    const float4 v = *reinterpret_cast<const float4*>(b.Vf + p * MP_HT + t * MP_H + c);
    const long pn = p + xs.stride;
    if (pn < xs.end) {
      ua = b.ua[pn];
      ub = b.ub[pn];
    }
    float acc = (ga.x * xb.x + gb.x * xa.x) * v.x;
    acc = fmaf(ga.y * xb.y + gb.y * xa.y, v.y, acc);
    acc = fmaf(ga.z * xb.z + gb.z * xa.z, v.z, acc);
    acc = fmaf(ga.w * xb.w + gb.w * xa.w, v.w, acc);
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 32);
    if (l32 == 0) b.gr[p] = first ? acc : b.gr[p] + acc;
  }
}

// F_a = sum over a's edges of dE/dr (q_b - q_a)/r, frame-major [f][3][N].
// Sixteen lanes per row: lane sub sums the edges sub, sub + 16, ... in
// order, then a fixed butterfly over the sixteen lanes.
constexpr int kForceLanes = 16;

__global__ __launch_bounds__(256) void k_mp_forces(MpnnBuffers b, SysDev S, RowSpan span,
                                                   float* Fout) {
  const long row = ((long)blockIdx.x * blockDim.x + threadIdx.x) / kForceLanes;
  const int sub = threadIdx.x % kForceLanes;
  const bool in = row < span.rows();
  const long N = S.n;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  if (in) {
    const int e1 = b.off[row + 1];
    for (int e = b.off[row] + sub; e < e1; e += kForceLanes) {
      // the pair's unit vector points from its owner row; the reverse edge
      // sees it negated
      const int u = b.uid[e];
      if (u == kNoPair) continue;  // only after a latched capacity overflow
      const long p = u >= 0 ? u : ~u;
      const float g = u >= 0 ? b.gr[p] : -b.gr[p];
      const float4 v = *reinterpret_cast<const float4*>(b.uv + 4 * p);
      fx = fmaf(g, v.x, fx);
      fy = fmaf(g, v.y, fy);
      fz = fmaf(g, v.z, fz);
    }
  }
#pragma unroll
  for (int o = 1; o < kForceLanes; o <<= 1) {
    fx += __shfl_xor(fx, o, 64);
    fy += __shfl_xor(fy, o, 64);
    fz += __shfl_xor(fz, o, 64);
  }
  if (!in || sub != 0) return;
  const int f0 = span.f0;
  const long fl = row / N;
  const int i = (int)(row - fl * N);
  float* F = Fout + (size_t)(f0 + fl) * 3 * N;
  F[i] = fx;
  F[N + i] = fy;
  F[2 * N + i] = fz;
}

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// fragment elements (uint4) of an I x K operand: I/16 tiles x K/32 steps x 64 lanes
size_t frag_elems(int I, int K) { return (size_t)(I / 16) * (K / 32) * 64; }

// all fragment arrays: per layer A2 and six node matrices (128 x 128), plus
// W1 forward (64 x 128) and reverse (128 x 64), each hi and lo
size_t frag_total() {
  return 2 * ((size_t)MP_T * (7 * frag_elems(MP_H, MP_H) + frag_elems(MP_H, 32)) +
              frag_elems(MP_RH, MP_H) + frag_elems(MP_H, MP_RH));
}

// blocks of the fixed grids over pairs: two per compute unit
constexpr unsigned kPairBlocks = 512;

}  // namespace

// capacities: directed edges <= rows x list width; unordered pairs <= a
// quarter of that.  A pair is about half of the row's in-cutoff entries,
// and with the automatic list width (1.3 x the expected entries within
// cutoff + skin, plus 32, rounded up to 32) that is about 0.17 of the width
// on the 1536-atom liquid (two thirds of the quarter); a narrower caller-set
// width can exceed it, which k_mp_edges latches in the status word instead
// of writing past the buffers
static size_t pair_capacity(size_t slots) { return slots / 4 + 1; }

size_t mpnn_buffer_bytes(int frames, int n, int mt) {
  const size_t rows = (size_t)frames * n, slots = rows * mt, pairs = pair_capacity(slots);
  size_t b = 0;
  b += 2 * al(pairs * MP_HT * 4);            // Wf, Vf
  b += al(pairs * 4 * 4) + al(pairs * 4) + 2 * al(pairs * 4);
  b += 2 * al((rows + 1) * 4) + 4 * al(slots * 4);
  b += al(4 * 4) + al(((rows + kScanTile - 1) / kScanTile) * 2 * 4);
  b += al((MP_T + 1) * rows * MP_H * 4) + 2 * al(MP_T * rows * MP_H * 4);
  b += al(rows * MP_H * 4) + al(rows * 8) + 4 * al(rows * MP_H * 4);
  b += al(frag_total() * 16);
  return b;
}

void mpnn_bind(MpnnCtx& M, char* base, int frames, int n, int mt, const float* weights,
               int n_model_species) {
  const size_t rows = (size_t)frames * n, slots = rows * mt, pairs = pair_capacity(slots);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    float* p = reinterpret_cast<float*>(base + off);
    off += al(bytes);
    return p;
  };
  MpnnBuffers& b = M.b;
  b.Wf = take(pairs * MP_HT * 4);
  b.Vf = take(pairs * MP_HT * 4);
  b.uv = take(pairs * 4 * 4);
  b.gr = take(pairs * 4);
  b.ua = reinterpret_cast<int*>(take(pairs * 4));
  b.ub = reinterpret_cast<int*>(take(pairs * 4));
  b.off = reinterpret_cast<int*>(take((rows + 1) * 4));
  b.poff = reinterpret_cast<int*>(take((rows + 1) * 4));
  b.erow = reinterpret_cast<int*>(take(slots * 4));
  b.enbr = reinterpret_cast<int*>(take(slots * 4));
  b.ecode = reinterpret_cast<int*>(take(slots * 4));
  b.uid = reinterpret_cast<int*>(take(slots * 4));
  b.counts = reinterpret_cast<int*>(take(4 * 4));
  b.tile_sums = reinterpret_cast<int*>(take(((rows + kScanTile - 1) / kScanTile) * 2 * 4));
  b.H = take((MP_T + 1) * rows * MP_H * 4);
  b.X = take(MP_T * rows * MP_H * 4);
  b.U = take(MP_T * rows * MP_H * 4);
  b.Mm = take(rows * MP_H * 4);
  b.Erow = reinterpret_cast<double*>(take(rows * 8));
  b.gH = take(rows * MP_H * 4);
  b.gP = take(rows * MP_H * 4);
  b.gM = take(rows * MP_H * 4);
  b.gX = take(rows * MP_H * 4);
  b.frag = reinterpret_cast<uint4*>(take(frag_total() * 16));
  M.frames = frames;
  M.pair_cap = (long)pairs;
  MpnnWeights& w = M.w;
  const float* p = weights;
  w.W_emb = p;
  p += (size_t)n_model_species * MP_H;
  w.layer_stride = (long)MP_H * MP_R + MP_H + 4L * MP_H * MP_H + 3L * MP_H;
  for (int t = 0; t < MP_T; ++t) {
    w.A1[t] = p; p += MP_H * MP_R;
    w.a1[t] = p; p += MP_H;
    w.A2[t] = p; p += MP_H * MP_H;
    w.a2[t] = p; p += MP_H;
    w.B[t] = p; p += MP_H * MP_H;
    w.C1[t] = p; p += MP_H * MP_H;
    w.c1[t] = p; p += MP_H;
    w.C2[t] = p; p += MP_H * MP_H;
    w.c2[t] = p; p += MP_H;
  }
  w.W1 = p; p += MP_RH * MP_H;
  w.b1 = p; p += MP_RH;
  w.w2 = p; p += MP_RH;
  w.b2 = p;
  // fragment arrays, hi then lo of each matrix
  uint4* f = b.frag;
  auto frag = [&](int I, int K) {
    const size_t n_el = frag_elems(I, K);
    MpnnFrag r{f, f + n_el};
    f += 2 * n_el;
    return r;
  };
  for (int t = 0; t < MP_T; ++t) {
    w.A1f[t] = frag(MP_H, 32);
    w.A2f[t] = frag(MP_H, MP_H);
    w.Bf[t] = frag(MP_H, MP_H);
    w.C1f[t] = frag(MP_H, MP_H);
    w.C2f[t] = frag(MP_H, MP_H);
    w.Bb[t] = frag(MP_H, MP_H);
    w.C1b[t] = frag(MP_H, MP_H);
    w.C2b[t] = frag(MP_H, MP_H);
  }
  w.W1f = frag(MP_RH, MP_H);
  w.W1b = frag(MP_H, MP_RH);
}

#define MP_HIP(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      snprintf(err, errlen, "%s: %s", #x, hipGetErrorString(e_));                       \
      return false;                                                                     \
    }                                                                                   \
  } while (0)

void mpnn_set_shape(MpnnCtx& M, int c) {
  static const unsigned kFilt[3] = {256, 512, 1024};
  static const int kNt[3] = {1, 2, 4};
  M.filt_blocks = kFilt[(c / 3) % 3];
  M.chain_nt = kNt[c % 3];
}

bool mpnn_prepare(MpnnCtx& M, hipStream_t st, char* err, size_t errlen) {
  const MpnnWeights& w = M.w;
  auto launch = [&](const float* src, int ld, int trans, int I, int K, const MpnnFrag& d,
                    int Ksrc = 0) {
    const long n = (long)frag_elems(I, K);
    hipLaunchKernelGGL(k_mp_frag, dim3(nblk(n, 256)), dim3(256), 0, st, src, ld, trans, I, K,
                       Ksrc ? Ksrc : K, const_cast<uint4*>(d.hi), const_cast<uint4*>(d.lo));
    return hipGetLastError();
  };
  for (int t = 0; t < MP_T; ++t) {
    // first filter layer: A1 [128][16], contraction padded to 32
    MP_HIP(launch(w.A1[t], MP_R, 0, MP_H, 32, w.A1f[t], MP_R));
    // filter: A2 [out][in] as stored; forward node products use W^T, i.e.
    // G(out, in) = W[out][in]; reverse products use W, G(i, k) = W[k][i]
    MP_HIP(launch(w.A2[t], MP_H, 0, MP_H, MP_H, w.A2f[t]));
    MP_HIP(launch(w.B[t], MP_H, 0, MP_H, MP_H, w.Bf[t]));
    MP_HIP(launch(w.C1[t], MP_H, 0, MP_H, MP_H, w.C1f[t]));
    MP_HIP(launch(w.C2[t], MP_H, 0, MP_H, MP_H, w.C2f[t]));
    MP_HIP(launch(w.B[t], MP_H, 1, MP_H, MP_H, w.Bb[t]));
    MP_HIP(launch(w.C1[t], MP_H, 1, MP_H, MP_H, w.C1b[t]));
    MP_HIP(launch(w.C2[t], MP_H, 1, MP_H, MP_H, w.C2b[t]));
  }
  MP_HIP(launch(w.W1, MP_H, 0, MP_RH, MP_H, w.W1f));   // Y = H W1^T: G(o, k) = W1[o][k]
  MP_HIP(launch(w.W1, MP_H, 1, MP_H, MP_RH, w.W1b));   // gH = gY W1: G(i, o) = W1[o][i]
  return true;
}

bool mpnn_eval(MpnnCtx& M, const SysDev& S, const ListDev& L, const WinDev& W, int f0, int nf,
               const int* nvalid, float* Fout, hipStream_t st, char* err, size_t errlen) {
  const MpnnWeights& w = M.w;
  MpnnBuffers& b = M.b;
  const long N = S.n, mt = L.mt;
  const long rows = (long)nf * N;
  const long cap = M.pair_cap;
  const RowSpan span{nvalid, f0, nf, N, S.atom_rep, W.invalid, W.rej, S.kmax};
  // compact the in-cutoff pairs of every row into edges (list order), then
  // into unordered pairs; the totals stay on the device
  hipLaunchKernelGGL(k_mp_count, dim3((unsigned)rows), dim3(kRowThreads), 0, st, b, S, L, W, f0,
                     nf, nvalid, M.rc);
  MP_HIP(hipGetLastError());
  if (rows <= kScanSingleMax) {
    hipLaunchKernelGGL(k_mp_scan, dim3(1), dim3(1024), 0, st, b, rows, N, f0, nf, nvalid);
    MP_HIP(hipGetLastError());
  } else {
    const int tiles = (int)((rows + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_mp_scan_tiles, dim3(tiles), dim3(1024), 0, st, b, rows, b.tile_sums);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mp_scan_top, dim3(1), dim3(1024), 0, st, b, rows, b.tile_sums, tiles);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mp_scan_add, dim3(tiles), dim3(1024), 0, st, b, rows, b.tile_sums);
    MP_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_mp_edges, dim3((unsigned)rows), dim3(kRowThreads), 0, st, b, S, L, W, f0,
                     nf, nvalid, M.rc, cap);
  MP_HIP(hipGetLastError());
  {
    const unsigned need = nblk(rows * mt * kRevLanes, 256);
    const unsigned nb = ((need < kRevBlocks ? need : kRevBlocks) + 7) / 8 * 8;
    hipLaunchKernelGGL(k_mp_reverse, dim3(nb), dim3(256), 0, st,
                       b, rows, rows * mt, L.status);
  }
  MP_HIP(hipGetLastError());
  // filters W and dW/dr of every pair and layer
  hipLaunchKernelGGL(k_mp_filter, dim3(M.filt_blocks), dim3(256), 0, st, w, b, M.rc, cap);
  MP_HIP(hipGetLastError());
  // forward through the layers: gathers and fused row chains
  const long rh = rows * MP_H;
  // rows per chain block: 16, 32 or 64, so that a small evaluation still
  // spreads over a few hundred blocks
  const long tiles16 = (rows + 15) / 16;
  const int nt = M.chain_nt ? M.chain_nt : (tiles16 >= 4L * 512 ? 4 : (tiles16 >= 2L * 256 ? 2 : 1));
  const dim3 cg((unsigned)((tiles16 + nt - 1) / nt)), cb(256);
  auto chain = [&](int mode, const ChainArgs& c) {
#define MP_CHAIN(MODE_)                                                                    \
  if (nt == 4) hipLaunchKernelGGL((k_mp_chain<MODE_, 4>), cg, cb, 0, st, w, b, S, span, c); \
  else if (nt == 2) hipLaunchKernelGGL((k_mp_chain<MODE_, 2>), cg, cb, 0, st, w, b, S, span, c); \
  else hipLaunchKernelGGL((k_mp_chain<MODE_, 1>), cg, cb, 0, st, w, b, S, span, c);
    if (mode == CH_EMBED) { MP_CHAIN(CH_EMBED) }
    else if (mode == CH_FWD) { MP_CHAIN(CH_FWD) }
    else if (mode == CH_LAST) { MP_CHAIN(CH_LAST) }
    else { MP_CHAIN(CH_BWD) }
#undef MP_CHAIN
    return hipGetLastError();
  };
  ChainArgs ca{};
  ca.scale = M.scale;
  ca.h_out = b.H;
  ca.x_out = b.X;
  MP_HIP(chain(CH_EMBED, ca));
  for (int t = 0; t < MP_T; ++t) {
    float* Xt = b.X + t * rh;
    hipLaunchKernelGGL(k_mp_gather, dim3(gather_grid(rows)), dim3(MP_H), 0, st, b, t, Xt, b.Mm,
                       span);
    MP_HIP(hipGetLastError());
    ChainArgs c{};
    c.scale = M.scale;
    c.t = t;
    c.in = b.Mm;
    c.h = b.H + t * rh;
    c.u_out = b.U + t * rh;
    if (t + 1 < MP_T) {
      c.h_out = b.H + (t + 1) * rh;
      c.x_out = b.X + (t + 1) * rh;
      MP_HIP(chain(CH_FWD, c));
    } else {
      // readout, energies per row, and the row part of the last layer's
      // reverse pass
      c.gh_out = b.gH;
      c.gm_out = b.gM;
      c.e_row = b.Erow;
      MP_HIP(chain(CH_LAST, c));
    }
    MP_HIP(hipGetLastError());
  }
  // reverse pass through the layers
  for (int t = MP_T - 1; t >= 0; --t) {
    hipLaunchKernelGGL(k_mp_dedr, dim3(kPairBlocks * 2), dim3(256), 0, st, b, t,
                       t == MP_T - 1 ? 1 : 0, b.X + t * rh, cap);
    MP_HIP(hipGetLastError());
    if (t == 0) break;
    hipLaunchKernelGGL(k_mp_gather, dim3(gather_grid(rows)), dim3(MP_H), 0, st, b, t, b.gM, b.gX,
                       span);
    MP_HIP(hipGetLastError());
    ChainArgs c{};
    c.scale = M.scale;
    c.t = t - 1;
    c.in = b.gX;
    c.gh = b.gH;
    c.gh_out = b.gP;
    c.u_in = b.U + (t - 1) * rh;
    c.gm_out = b.gM;
    MP_HIP(chain(CH_BWD, c));
    float* tmp = b.gH;
    b.gH = b.gP;
    b.gP = tmp;
  }
  hipLaunchKernelGGL(k_mp_forces, dim3(nblk(rows * kForceLanes, 256)), dim3(256), 0, st, b, S,
                     span, Fout);
  MP_HIP(hipGetLastError());
  return true;
}
