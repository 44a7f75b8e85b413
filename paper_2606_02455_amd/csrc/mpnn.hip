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
// W_ij = W_ji), and per slot dE/dr accumulated for both directions of the
// pair; finally F_a = sum over a's edges of dE/dr * (q_b - q_a) / r.
#include <cstdio>

#include "mpnn.h"

namespace {

constexpr int kSlotsPerBlock = 8;  // 8 edges x 16 basis functions = 128 threads

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }
__device__ __forceinline__ float siluf(float x) { return x * sigmoidf(x); }
__device__ __forceinline__ float dsiluf(float x) {
  const float s = sigmoidf(x);
  return s * (1.0f + x * (1.0f - s));
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
  const int cnt = L.cnt_t[i];
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
        const float a = 3.14159265358979f / rc;
        b.uid[e] = pp;
        if (pp < pair_cap) {
          b.ua[pp] = (int)row;
          b.ub[pp] = (int)((long)fl * S.n + j);
          b.fcd[2 * pp] = 0.5f * (cosf(a * r) + 1.0f);
          b.fcd[2 * pp + 1] = -0.5f * a * sinf(a * r);
          b.uv[4 * pp] = d[0] / r;
          b.uv[4 * pp + 1] = d[1] / r;
          b.uv[4 * pp + 2] = d[2] / r;
          b.uv[4 * pp + 3] = r;
        } else {
          b.counts[3] = 1;  // more pairs than the buffers hold: reported, not written
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
                                                          WinDev W, int f0, float rc) {
  const long row = blockIdx.x;
  const RowScan c = row_pass<false>(b, S, L, W, f0, row, rc, 0);
  if (threadIdx.x == 0) {
    b.off[row] = c.edges;
    b.poff[row] = c.owners;
  }
}

// exclusive scans of the row counts of edges and pairs in place (one block);
// off[rows], poff[rows] = totals, also copied to counts[0..1]
__global__ __launch_bounds__(1024) void k_mp_scan(MpnnBuffers b, long rows) {
  __shared__ long s[1024], s2[1024];
  const int t = threadIdx.x;
  const long chunk = (rows + 1023) / 1024;
  const long lo = min(rows, (long)t * chunk), hi = min(rows, lo + chunk);
  long sum = 0, sum2 = 0;
  for (long r = lo; r < hi; ++r) {
    sum += b.off[r];
    sum2 += b.poff[r];
  }
  s[t] = sum;
  s2[t] = sum2;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const long v = t >= o ? s[t - o] : 0, v2 = t >= o ? s2[t - o] : 0;
    __syncthreads();
    s[t] += v;
    s2[t] += v2;
    __syncthreads();
  }
  long run = s[t] - sum, run2 = s2[t] - sum2;
  for (long r = lo; r < hi; ++r) {
    const long c = b.off[r], c2 = b.poff[r];
    b.off[r] = (int)run;
    b.poff[r] = (int)run2;
    run += c;
    run2 += c2;
  }
  if (t == 1023) {
    b.off[rows] = (int)s[1023];
    b.poff[rows] = (int)s2[1023];
    b.counts[0] = (int)s[1023];
    b.counts[1] = (int)s2[1023];
    b.counts[2] = 0;  // set by k_mp_reverse if a reverse edge has no owner
    b.counts[3] = 0;  // set by k_mp_edges if the pairs exceed the capacity
  }
}

// directed edge records of every row in list order, and the pair records of
// the edges the row owns
__global__ __launch_bounds__(kRowThreads) void k_mp_edges(MpnnBuffers b, SysDev S, ListDev L,
                                                          WinDev W, int f0, float rc,
                                                          long pair_cap) {
  row_pass<true>(b, S, L, W, f0, blockIdx.x, rc, pair_cap);
}

// every reverse edge refers to its owner: the neighbour row's edge back to
// this row with the opposite image; uid = ~pair
__global__ __launch_bounds__(256) void k_mp_reverse(MpnnBuffers b, long rows, long cap) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cap || e >= b.off[rows]) return;
  if (b.uid[e] >= 0) return;
  const int rj = b.enbr[e], ri = b.erow[e], back = 26 - b.ecode[e];
  int found = -1;
  for (int q = b.off[rj]; q < b.off[rj + 1]; ++q)
    if (b.enbr[q] == ri && b.ecode[q] == back) { found = b.uid[q]; break; }
  if (found < 0) {
    b.counts[2] = 1;  // the edge sets of the two directions differ (not expected)
    found = 0;
  }
  b.uid[e] = ~found;
}

// Radial basis and the first filter layer of all three layers per edge:
// S = silu(A1 e + a1), DS = silu'(A1 e + a1) (.) (A1 de/dr).  Block: 128
// threads (channels), kSlotsPerBlock edges.
__global__ __launch_bounds__(128) void k_mp_radial(MpnnWeights w, MpnnBuffers b, long edges,
                                                   float rc) {
  __shared__ float s_e[kSlotsPerBlock][MP_R], s_de[kSlotsPerBlock][MP_R];
  const int c = threadIdx.x;
  const long e0 = (long)blockIdx.x * kSlotsPerBlock;
  // radial basis e_b(r) = sqrt(2/rc) sin(b pi r/rc)/r and de_b/dr
  {
    const int q = c / MP_R, bb = c % MP_R;  // kSlotsPerBlock * MP_R == blockDim
    float e = 0.f, de = 0.f;
    if (e0 + q < edges) {
      const float r = b.uv[4 * (e0 + q) + 3];
      const float pre = sqrtf(2.0f / rc);
      const float k = (float)(bb + 1) * 3.14159265358979f / rc;
      const float sn = sinf(k * r), cs = cosf(k * r);
      e = pre * sn / r;
      de = pre * (k * cs / r - sn / (r * r));
    }
    s_e[q][bb] = e;
    s_de[q][bb] = de;
  }
  __syncthreads();
  float A[MP_T][MP_R], a1v[MP_T];
#pragma unroll
  for (int t = 0; t < MP_T; ++t) {
#pragma unroll
    for (int q = 0; q < MP_R; ++q) A[t][q] = w.A1[t][c * MP_R + q];
    a1v[t] = w.a1[t][c];
  }
  for (int q = 0; q < kSlotsPerBlock; ++q) {
    const long e = e0 + q;
    if (e >= edges) break;
#pragma unroll
    for (int t = 0; t < MP_T; ++t) {
      float z = a1v[t], dz = 0.f;
#pragma unroll
      for (int k = 0; k < MP_R; ++k) {
        z = fmaf(A[t][k], s_e[q][k], z);
        dz = fmaf(A[t][k], s_de[q][k], dz);
      }
      b.S[e * MP_HT + t * MP_H + c] = siluf(z);
      b.DS[e * MP_HT + t * MP_H + c] = dsiluf(z) * dz;
    }
  }
}

// Filters from the GEMM outputs of a pair (Z = S A2^T, DZ = DS A2^T):
// W = f_c (Z + a2) and dW/dr = f_c' (Z + a2) + f_c DZ, formed where used.
__device__ __forceinline__ float filter_w(const MpnnWeights& w, const MpnnBuffers& b, long p, int t,
                                          int c) {
  return b.fcd[2 * p] * (b.Z[p * MP_HT + t * MP_H + c] + w.a2[t][c]);
}

__global__ __launch_bounds__(128) void k_mp_embed(MpnnWeights w, MpnnBuffers b, SysDev S, long rows) {
  const long row = blockIdx.x;
  if (row >= rows) return;
  const int i = (int)(row % S.n);
  const int sp = S.species ? S.species[i] : 0;
  b.H[row * MP_H + threadIdx.x] = w.W_emb[sp * MP_H + threadIdx.x];
}

// out[row][c] = sum over the row's edges e of W_t[pair(e)][c] * V[neighbour row][c]
// (messages with V = X_t; dE/dX with V = gM: W is symmetric in the pair)
__global__ __launch_bounds__(128) void k_mp_gather(MpnnWeights w, MpnnBuffers b, int t,
                                                   const float* __restrict__ V,
                                                   float* __restrict__ out, long rows) {
  const long row = blockIdx.x;
  if (row >= rows) return;
  const int c = threadIdx.x;
  const int e1 = b.off[row + 1];
  float acc = 0.f;
  int e = b.off[row];
  // four edges' loads issued together, terms added in edge order
  for (; e + 4 <= e1; e += 4) {
    float wv[4], vv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = b.uid[e + q];
      const long p = u >= 0 ? u : ~u;
      wv[q] = filter_w(w, b, p, t, c);
      vv[q] = V[(long)b.enbr[e + q] * MP_H + c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = fmaf(wv[q], vv[q], acc);
  }
  for (; e < e1; ++e) {
    const int u = b.uid[e];
    const long p = u >= 0 ? u : ~u;
    acc = fmaf(filter_w(w, b, p, t, c), V[(long)b.enbr[e] * MP_H + c], acc);
  }
  out[row * MP_H + c] = acc;
}

// U += c1 (kept for the reverse pass); Sn = silu(U)
__global__ __launch_bounds__(256) void k_mp_act(const float* __restrict__ c1, float* U, float* Sn,
                                                long n) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const float u = U[id] + c1[id % MP_H];
  U[id] = u;
  Sn[id] = siluf(u);
}

// Hn += Hp + c2 (residual update)
__global__ __launch_bounds__(256) void k_mp_residual(const float* __restrict__ c2,
                                                     const float* __restrict__ Hp, float* Hn, long n) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  Hn[id] = Hn[id] + Hp[id] + c2[id % MP_H];
}

// Readout of one tile of one frame (64 rows, one lane each): energy summed
// in binary64 by a wave butterfly; gY = s_E w2 (.) silu'(Y + b1).
__global__ __launch_bounds__(64) void k_mp_readout(MpnnWeights w, MpnnBuffers b, SysDev S,
                                                   TileDev T, int f0, float scale, double* epart) {
  const int tile = blockIdx.x, fl = blockIdx.y;
  const int lane = threadIdx.x;
  const int start = T.start[tile], count = T.count[tile];
  const long row = (long)fl * S.n + start + lane;
  double e = 0.0;
  if (lane < count) {
    float ei = w.b2[0];
    for (int o = 0; o < MP_RH; ++o) {
      const float y = b.Y[row * MP_RH + o] + w.b1[o];
      ei = fmaf(w.w2[o], siluf(y), ei);
      b.gY[row * MP_RH + o] = scale * w.w2[o] * dsiluf(y);
    }
    e = (double)scale * (double)ei;
  }
  e = wave_sum(e);
  if (lane == 0) epart[(size_t)(f0 + fl) * S.n_tiles + tile] = e;
}

__global__ __launch_bounds__(256) void k_mp_mul_dsilu(const float* __restrict__ U, float* g, long n) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  g[id] *= dsiluf(U[id]);
}

// dE/dr of one pair (both directions), layer t:
// sum_c (gM[a] X[b] + gM[b] X[a])_c dW_c/dr.  One wave per pair.
__global__ __launch_bounds__(256) void k_mp_dedr(MpnnWeights w, MpnnBuffers b, int t,
                                                 const float* __restrict__ X, long pairs) {
  const long p = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= pairs) return;  // uniform per wave
  const long ra = (long)b.ua[p] * MP_H, rb = (long)b.ub[p] * MP_H;
  const float fc = b.fcd[2 * p], dfc = b.fcd[2 * p + 1];
  const float* Z = b.Z + p * MP_HT + t * MP_H;
  const float* DZ = b.DZ + p * MP_HT + t * MP_H;
  float acc = 0.f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = lane + 64 * h;
    const float g = b.gM[ra + c] * X[rb + c] + b.gM[rb + c] * X[ra + c];
    const float dW = dfc * (Z[c] + w.a2[t][c]) + fc * DZ[c];
    acc = fmaf(g, dW, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) b.gr[p] += acc;
}

// F_a = sum over a's edges of dE/dr (q_b - q_a)/r, frame-major [f][3][N]
__global__ __launch_bounds__(256) void k_mp_forces(MpnnBuffers b, SysDev S, int f0, float* Fout,
                                                   long rows) {
  const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  const long N = S.n;
  const long fl = row / N;
  const int i = (int)(row - fl * N);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int e1 = b.off[row + 1];
  for (int e = b.off[row]; e < e1; ++e) {
    // the pair's unit vector points from its owner row; the reverse edge
    // sees it negated
    const int u = b.uid[e];
    const long p = u >= 0 ? u : ~u;
    const float g = u >= 0 ? b.gr[p] : -b.gr[p];
    fx = fmaf(g, b.uv[4 * p], fx);
    fy = fmaf(g, b.uv[4 * p + 1], fy);
    fz = fmaf(g, b.uv[4 * p + 2], fz);
  }
  float* F = Fout + (size_t)(f0 + fl) * 3 * N;
  F[i] = fx;
  F[N + i] = fy;
  F[2 * N + i] = fz;
}

__global__ void k_mp_zero(float* p, long n) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) p[id] = 0.f;
}

__global__ void k_mp_copy(const float* __restrict__ a, float* __restrict__ b, long n) {
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) b[id] = a[id];
}

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// row-major C[M][Nc] = A[M][K] . op(B), with op(B) = B^T for B stored
// [Nc][K] (trans) or op(B) = B for B stored [K][Nc]; column-major view for
// rocBLAS: C^c = op(B)^c . A^c.
rocblas_status gemm_rm(rocblas_handle h, const float* A, const float* B, float* C, int M, int Nc,
                       int K, bool transB, float beta, int lda, int ldc) {
  const float one = 1.0f;
  return rocblas_sgemm(h, transB ? rocblas_operation_transpose : rocblas_operation_none,
                       rocblas_operation_none, Nc, M, K, &one, B, transB ? K : Nc, A, lda, &beta,
                       C, ldc);
}

}  // namespace

// capacities: directed edges <= rows x list width; unordered pairs <= a
// quarter of that.  A pair is about half of the row's in-cutoff entries,
// and with the automatic list width (1.3 x the expected entries within
// cutoff + skin, plus 32, rounded up to 32) that is 0.17 of the width on the
// 1536-atom liquid; a narrower caller-set width can exceed a quarter, which
// k_mp_edges reports (counts[3]) instead of writing past the buffers
static size_t pair_capacity(size_t slots) { return slots / 4 + 1; }

size_t mpnn_buffer_bytes(int frames, int n, int mt) {
  const size_t rows = (size_t)frames * n, slots = rows * mt, pairs = pair_capacity(slots);
  size_t b = 0;
  b += 4 * al(pairs * MP_HT * 4);            // S, DS, Z, DZ
  b += al(pairs * 2 * 4) + al(pairs * 4 * 4) + al(pairs * 4) + 2 * al(pairs * 4);
  b += 2 * al((rows + 1) * 4) + 4 * al(slots * 4);
  b += al(4 * 4);
  b += al((MP_T + 1) * rows * MP_H * 4) + 2 * al(MP_T * rows * MP_H * 4);
  b += 2 * al(rows * MP_H * 4) + 2 * al(rows * MP_RH * 4) + 5 * al(rows * MP_H * 4);
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
  b.S = take(pairs * MP_HT * 4);
  b.DS = take(pairs * MP_HT * 4);
  b.Z = take(pairs * MP_HT * 4);
  b.DZ = take(pairs * MP_HT * 4);
  b.fcd = take(pairs * 2 * 4);
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
  b.H = take((MP_T + 1) * rows * MP_H * 4);
  b.X = take(MP_T * rows * MP_H * 4);
  b.U = take(MP_T * rows * MP_H * 4);
  b.Mm = take(rows * MP_H * 4);
  b.Sn = take(rows * MP_H * 4);
  b.Y = take(rows * MP_RH * 4);
  b.gY = take(rows * MP_RH * 4);
  b.gH = take(rows * MP_H * 4);
  b.gP = take(rows * MP_H * 4);
  b.gS = take(rows * MP_H * 4);
  b.gM = take(rows * MP_H * 4);
  b.gX = take(rows * MP_H * 4);
  M.frames = frames;
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
}

#define MP_HIP(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      snprintf(err, errlen, "%s: %s", #x, hipGetErrorString(e_));                       \
      return false;                                                                     \
    }                                                                                   \
  } while (0)
#define MP_BLAS(x)                                                                      \
  do {                                                                                  \
    rocblas_status s_ = (x);                                                            \
    if (s_ != rocblas_status_success) {                                                 \
      snprintf(err, errlen, "%s: rocblas status %d", #x, (int)s_);                      \
      return false;                                                                     \
    }                                                                                   \
  } while (0)

bool mpnn_eval(MpnnCtx& M, const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
               int f0, int nf, float* Fout, double* epart, hipStream_t st, char* err,
               size_t errlen) {
  const MpnnWeights& w = M.w;
  MpnnBuffers& b = M.b;
  const long N = S.n, mt = L.mt;
  const long rows = (long)nf * N;
  MP_BLAS(rocblas_set_stream(M.blas, st));
  // compact the in-cutoff pairs of every row into edges (list order), then
  // into unordered pairs
  hipLaunchKernelGGL(k_mp_count, dim3((unsigned)rows), dim3(kRowThreads), 0, st, b, S, L, W, f0,
                     M.rc);
  MP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mp_scan, dim3(1), dim3(1024), 0, st, b, rows);
  MP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mp_edges, dim3((unsigned)rows), dim3(kRowThreads), 0, st, b, S, L, W, f0,
                     M.rc, (long)pair_capacity((size_t)rows * mt));
  MP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mp_reverse, dim3(nblk(rows * mt, 256)), dim3(256), 0, st, b, rows, rows * mt);
  MP_HIP(hipGetLastError());
  // the pair count sizes the contractions below
  int counts[4] = {0, 0, 0, 0};
  MP_HIP(hipMemcpyAsync(counts, b.counts, sizeof(counts), hipMemcpyDeviceToHost, st));
  MP_HIP(hipStreamSynchronize(st));
  if (counts[3]) {
    snprintf(err, errlen, "pair count exceeds the capacity %zu", pair_capacity((size_t)rows * mt));
    return false;
  }
  if (counts[2]) {
    snprintf(err, errlen, "edge lists of the two directions of a pair differ");
    return false;
  }
  const long slots = counts[1];  // unordered pairs
  if ((size_t)slots > pair_capacity((size_t)rows * mt)) {
    snprintf(err, errlen, "pair count %ld exceeds capacity %zu", slots,
             pair_capacity((size_t)rows * mt));
    return false;
  }
  if (slots > 0) {
    hipLaunchKernelGGL(k_mp_radial, dim3(nblk(slots, kSlotsPerBlock)), dim3(128), 0, st, w, b, slots,
                       M.rc);
    MP_HIP(hipGetLastError());
  }
  const float one = 1.0f, zero = 0.0f;
  // Z_t = S_t A2_t^T and DZ_t = DS_t A2_t^T for the three layers at once
  if (slots > 0) {
  MP_BLAS(rocblas_sgemm_strided_batched(M.blas, rocblas_operation_transpose,
                                        rocblas_operation_none, MP_H, (int)slots, MP_H, &one,
                                        w.A2[0], MP_H, w.layer_stride, b.S, MP_HT, MP_H, &zero,
                                        b.Z, MP_HT, MP_H, MP_T));
  MP_BLAS(rocblas_sgemm_strided_batched(M.blas, rocblas_operation_transpose,
                                        rocblas_operation_none, MP_H, (int)slots, MP_H, &one,
                                        w.A2[0], MP_H, w.layer_stride, b.DS, MP_HT, MP_H, &zero,
                                        b.DZ, MP_HT, MP_H, MP_T));
  }
  // forward through the layers
  hipLaunchKernelGGL(k_mp_embed, dim3((unsigned)rows), dim3(MP_H), 0, st, w, b, S, rows);
  MP_HIP(hipGetLastError());
  const long rh = rows * MP_H;
  for (int t = 0; t < MP_T; ++t) {
    float* Ht = b.H + t * rh;
    float* Hn = b.H + (t + 1) * rh;
    float* Xt = b.X + t * rh;
    float* Ut = b.U + t * rh;
    MP_BLAS(gemm_rm(M.blas, Ht, w.B[t], Xt, (int)rows, MP_H, MP_H, true, 0.f, MP_H, MP_H));
    hipLaunchKernelGGL(k_mp_gather, dim3((unsigned)rows), dim3(MP_H), 0, st, w, b, t, Xt, b.Mm,
                       rows);
    MP_HIP(hipGetLastError());
    MP_BLAS(gemm_rm(M.blas, b.Mm, w.C1[t], Ut, (int)rows, MP_H, MP_H, true, 0.f, MP_H, MP_H));
    hipLaunchKernelGGL(k_mp_act, dim3(nblk(rh, 256)), dim3(256), 0, st, w.c1[t], Ut, b.Sn, rh);
    MP_HIP(hipGetLastError());
    MP_BLAS(gemm_rm(M.blas, b.Sn, w.C2[t], Hn, (int)rows, MP_H, MP_H, true, 0.f, MP_H, MP_H));
    hipLaunchKernelGGL(k_mp_residual, dim3(nblk(rh, 256)), dim3(256), 0, st, w.c2[t], Ht, Hn, rh);
    MP_HIP(hipGetLastError());
  }
  // readout and its gradient
  MP_BLAS(gemm_rm(M.blas, b.H + MP_T * rh, w.W1, b.Y, (int)rows, MP_RH, MP_H, true, 0.f, MP_H,
                  MP_RH));
  hipLaunchKernelGGL(k_mp_readout, dim3(S.n_tiles, nf), dim3(64), 0, st, w, b, S, T, f0, M.scale,
                     epart);
  MP_HIP(hipGetLastError());
  MP_BLAS(gemm_rm(M.blas, b.gY, w.W1, b.gH, (int)rows, MP_H, MP_RH, false, 0.f, MP_RH, MP_H));
  if (slots > 0) {
    hipLaunchKernelGGL(k_mp_zero, dim3(nblk(slots, 256)), dim3(256), 0, st, b.gr, slots);
    MP_HIP(hipGetLastError());
  }
  // reverse pass through the layers
  for (int t = MP_T - 1; t >= 0; --t) {
    float* Xt = b.X + t * rh;
    float* Ut = b.U + t * rh;
    MP_BLAS(gemm_rm(M.blas, b.gH, w.C2[t], b.gS, (int)rows, MP_H, MP_H, false, 0.f, MP_H, MP_H));
    hipLaunchKernelGGL(k_mp_mul_dsilu, dim3(nblk(rh, 256)), dim3(256), 0, st, Ut, b.gS, rh);
    MP_HIP(hipGetLastError());
    MP_BLAS(gemm_rm(M.blas, b.gS, w.C1[t], b.gM, (int)rows, MP_H, MP_H, false, 0.f, MP_H, MP_H));
    if (slots > 0) {
      hipLaunchKernelGGL(k_mp_dedr, dim3(nblk(slots, 4)), dim3(256), 0, st, w, b, t, Xt, slots);
      MP_HIP(hipGetLastError());
    }
    if (t > 0) {
      hipLaunchKernelGGL(k_mp_gather, dim3((unsigned)rows), dim3(MP_H), 0, st, w, b, t, b.gM, b.gX,
                         rows);
      MP_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_mp_copy, dim3(nblk(rh, 256)), dim3(256), 0, st, b.gH, b.gP, rh);
      MP_HIP(hipGetLastError());
      MP_BLAS(gemm_rm(M.blas, b.gX, w.B[t], b.gP, (int)rows, MP_H, MP_H, false, 1.f, MP_H, MP_H));
      float* tmp = b.gH;
      b.gH = b.gP;
      b.gP = tmp;
    }
  }
  hipLaunchKernelGGL(k_mp_forces, dim3(nblk(rows, 256)), dim3(256), 0, st, b, S, f0, Fout, rows);
  MP_HIP(hipGetLastError());
  return true;
}
