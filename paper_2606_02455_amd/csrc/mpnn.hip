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

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }
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
  // frames that are not verified (past the skin, or past the step limit)
  // contribute no edges
  const bool live = W.invalid[(size_t)S.atom_rep[i] * S.kmax + f0 + fl] == 0;
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
  }
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

// every reverse edge refers to its owner: the neighbour row's edge back to
// this row with the opposite image; uid = ~pair (kNoPair if the owner's pair
// is past the capacity)
__global__ __launch_bounds__(256) void k_mp_reverse(MpnnBuffers b, long rows, long cap,
                                                    int* __restrict__ status) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cap || e >= b.off[rows]) return;
  if (b.uid[e] >= 0) return;
  const int rj = b.enbr[e], ri = b.erow[e], back = 26 - b.ecode[e];
  int found = -1;
  for (int q = b.off[rj]; q < b.off[rj + 1]; ++q)
    if (b.enbr[q] == ri && b.ecode[q] == back) { found = b.uid[q]; break; }
  if (found < 0) {
    atomicOr(status, LSD_STATUS_EDGES);  // the edge sets of the two directions differ
    found = kNoPair;
  }
  b.uid[e] = found == kNoPair ? kNoPair : ~found;
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
  const int c = t & (MP_H - 1), ph = t >> 7;  // channel and pair half of the S stage
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
    float a1r[MP_R];
#pragma unroll
    for (int k = 0; k < MP_R; ++k) a1r[k] = w.A1[l][c * MP_R + k];
    const float a1c = w.a1[l][c];
    float a2v[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) a2v[mt][q] = w.a2[l][32 * wave + 16 * mt + 4 * (lane >> 4) + q];
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      const long p0 = tile * kFiltPairs;
      // radial basis e_b(r) = sqrt(2/rc) sin(b pi r/rc)/r, de_b/dr, cutoff
      {
        const int q = t >> 3, b0 = 2 * (t & 7);
        const long p = p0 + q;
        const float r = p < np ? b.uv[4 * p + 3] : 0.5f * rc;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int bb = b0 + u;
          const float k = (float)(bb + 1) * pi_rc;
          const float sn = sinf(k * r), cs = cosf(k * r);
          s_e[q][bb] = pre * sn / r;
          s_de[q][bb] = pre * (k * cs / r - sn / (r * r));
        }
        if ((t & 7) == 0) {
          s_fc[q] = 0.5f * (cosf(pi_rc * r) + 1.0f);
          s_dfc[q] = -0.5f * pi_rc * sinf(pi_rc * r);
        }
      }
      __syncthreads();
      // first layer of the filter MLP (binary32), staged as bfloat16 parts
      for (int q = 16 * ph; q < 16 * ph + 16; ++q) {
        float z = a1c, dz = 0.f;
#pragma unroll
        for (int k = 0; k < MP_R; ++k) {
          z = fmaf(a1r[k], s_e[q][k], z);
          dz = fmaf(a1r[k], s_de[q][k], dz);
        }
        const float S = siluf(z), DS = dsiluf(z) * dz;
        const __bf16 sh = (__bf16)S, dh = (__bf16)DS;
        s_sh[q][c] = sh;
        s_sl[q][c] = (__bf16)(S - (float)sh);
        s_dh[q][c] = dh;
        s_dl[q][c] = (__bf16)(DS - (float)dh);
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

// Dense row products out[row][n] = sum_k in[row][k] op[k][n] (+ epilogue) on
// the matrix cores, rows in tiles of 16; wave w computes the output channels
// [w ND/4, (w+1) ND/4) from fragments of op held in registers.
// rows of an evaluation that are computed: the frames below the device bound
struct RowSpan {
  const int* nvalid;
  int f0, nf;
  long n;
  __device__ __forceinline__ long rows() const { return (long)eff_frames(nvalid, f0, nf) * n; }
};

enum RowEpilogue {
  EP_STORE = 0,      // out = x
  EP_BIAS_SILU = 1,  // out = u = x + bias (kept), out2 = silu(u)
  EP_RESID = 2,      // out = in2 + x + bias
  EP_DSILU = 3,      // out = x * silu'(in2)
  EP_ACCUM = 4,      // out = in2 + x
};

template <int KD, int ND, int EP>
__global__ __launch_bounds__(256) void k_mp_rows(MpnnFrag op, const float* __restrict__ in,
                                                 RowSpan span, float* __restrict__ out,
                                                 float* __restrict__ out2,
                                                 const float* __restrict__ in2,
                                                 const float* __restrict__ bias) {
  constexpr int KS = KD / 32, MT = ND / 64;
  const long rows = span.rows();
  if ((long)blockIdx.x * 16 >= rows) return;  // uniform
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  bf16x8 ah[MT][KS], al[MT][KS];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const long fi = ((long)(MT * wave + mt) * KS + ks) * 64 + lane;
      ah[mt][ks] = as_bf16x8(op.hi[fi]);
      al[mt][ks] = as_bf16x8(op.lo[fi]);
    }
  const long ntiles = (rows + 15) / 16;
  const int kk = 8 * (lane >> 4);
  for (long rt = blockIdx.x; rt < ntiles; rt += gridDim.x) {
    const long row = rt * 16 + (lane & 15);
    const bool ok = row < rows;
    f32x4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      float x[8];
      if (ok) {
        const float4 u0 = *reinterpret_cast<const float4*>(in + row * KD + 32 * ks + kk);
        const float4 u1 = *reinterpret_cast<const float4*>(in + row * KD + 32 * ks + kk + 4);
        x[0] = u0.x; x[1] = u0.y; x[2] = u0.z; x[3] = u0.w;
        x[4] = u1.x; x[5] = u1.y; x[6] = u1.z; x[7] = u1.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = 0.f;
      }
      bf16x8 bh, bl;
      split8(x, bh, bl);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = mfma3(ah[mt][ks], al[mt][ks], bh, bl, acc[mt]);
    }
    if (!ok) continue;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int c0 = (ND / 4) * wave + 16 * mt + 4 * (lane >> 4);
      const long o = row * ND + c0;
      float4 y;
      float* yp = &y.x;
      if (EP == EP_STORE) {
#pragma unroll
        for (int e = 0; e < 4; ++e) yp[e] = acc[mt][e];
      } else if (EP == EP_BIAS_SILU) {
        float4 s;
        float* sp = &s.x;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          yp[e] = acc[mt][e] + bias[c0 + e];
          sp[e] = siluf(yp[e]);
        }
        *reinterpret_cast<float4*>(out2 + o) = s;
      } else if (EP == EP_RESID) {
        const float4 h = *reinterpret_cast<const float4*>(in2 + o);
        const float* hp = &h.x;
#pragma unroll
        for (int e = 0; e < 4; ++e) yp[e] = (acc[mt][e] + hp[e]) + bias[c0 + e];
      } else if (EP == EP_DSILU) {
        const float4 u = *reinterpret_cast<const float4*>(in2 + o);
        const float* up = &u.x;
#pragma unroll
        for (int e = 0; e < 4; ++e) yp[e] = acc[mt][e] * dsiluf(up[e]);
      } else {  // EP_ACCUM
        const float4 h = *reinterpret_cast<const float4*>(in2 + o);
        const float* hp = &h.x;
#pragma unroll
        for (int e = 0; e < 4; ++e) yp[e] = hp[e] + acc[mt][e];
      }
      *reinterpret_cast<float4*>(out + o) = y;
    }
  }
}

// Fragments of G(i, k) (i: output channel, k: contraction index) for the A
// operand: element [(it KS + ks) 64 + lane][e] = G(16 it + lane % 16,
// 32 ks + 8 (lane / 16) + e), split into bfloat16 hi and lo.  G(i, k) =
// src[i ld + k], or src[k ld + i] when transposed.
__global__ void k_mp_frag(const float* __restrict__ src, int ld, int trans, int I, int K,
                          uint4* __restrict__ hi, uint4* __restrict__ lo) {
  const int KS = K / 32;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)(I / 16) * KS * 64) return;
  const int lane = (int)(idx % 64), ks = (int)((idx / 64) % KS), it = (int)(idx / 64 / KS);
  const int i = 16 * it + lane % 16, k0 = 32 * ks + 8 * (lane / 16);
  float x[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) x[e] = trans ? src[(long)(k0 + e) * ld + i] : src[(long)i * ld + k0 + e];
  bf16x8 h, l;
  split8(x, h, l);
  hi[idx] = __builtin_bit_cast(uint4, h);
  lo[idx] = __builtin_bit_cast(uint4, l);
}

__global__ __launch_bounds__(128) void k_mp_embed(MpnnWeights w, MpnnBuffers b, SysDev S,
                                                  RowSpan span) {
  const long row = blockIdx.x;
  if (row >= span.rows()) return;
  const int i = (int)(row % S.n);
  const int sp = S.species ? S.species[i] : 0;
  b.H[row * MP_H + threadIdx.x] = w.W_emb[sp * MP_H + threadIdx.x];
}

// out[row][c] = sum over the row's edges e of W_t[pair(e)][c] * V[neighbour row][c]
// (messages with V = X_t; dE/dX with V = gM: W is symmetric in the pair)
__device__ __forceinline__ float pair_filter(const MpnnBuffers& b, int u, int t, int c) {
  if (u == kNoPair) return 0.f;  // only after a latched capacity overflow
  const long p = u >= 0 ? u : ~u;
  return b.Wf[p * MP_HT + t * MP_H + c];
}

__global__ __launch_bounds__(128) void k_mp_gather(MpnnBuffers b, int t, const float* __restrict__ V,
                                                   float* __restrict__ out, RowSpan span) {
  const long row = blockIdx.x;
  if (row >= span.rows()) return;
  const int c = threadIdx.x;
  const int e1 = b.off[row + 1];
  float acc = 0.f;
  int e = b.off[row];
  // four edges' loads issued together, terms added in edge order
  for (; e + 4 <= e1; e += 4) {
    float wv[4], vv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wv[q] = pair_filter(b, b.uid[e + q], t, c);
      vv[q] = V[(long)b.enbr[e + q] * MP_H + c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = fmaf(wv[q], vv[q], acc);
  }
  for (; e < e1; ++e) acc = fmaf(pair_filter(b, b.uid[e], t, c), V[(long)b.enbr[e] * MP_H + c], acc);
  out[row * MP_H + c] = acc;
}

// Readout of one tile of one frame (64 rows, one lane each): energy summed
// in binary64 by a wave butterfly; gY = s_E w2 (.) silu'(Y + b1).
__global__ __launch_bounds__(64) void k_mp_readout(MpnnWeights w, MpnnBuffers b, SysDev S,
                                                   TileDev T, RowSpan span, float scale,
                                                   double* epart) {
  const int tile = blockIdx.x, fl = blockIdx.y;
  const int f0 = span.f0;
  if (fl >= eff_frames(span.nvalid, f0, span.nf)) return;  // energy not needed
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

// dE/dr of one pair (both directions), layer t:
// sum_c (gM[a] X[b] + gM[b] X[a])_c dW_c/dr.  One wave per pair, pairs
// taken by a fixed grid up to the device pair count; the first layer of the
// reverse pass stores, the others add.
__global__ __launch_bounds__(256) void k_mp_dedr(MpnnBuffers b, int t, int first,
                                                 const float* __restrict__ X, long cap) {
  const int lane = threadIdx.x & 63;
  const long np = held_pairs(b, cap);
  for (long p = (long)blockIdx.x * 4 + (threadIdx.x >> 6); p < np; p += (long)gridDim.x * 4) {
    const long ra = (long)b.ua[p] * MP_H, rb = (long)b.ub[p] * MP_H;
    const float* V = b.Vf + p * MP_HT + t * MP_H;
    float acc = 0.f;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h;
      const float g = b.gM[ra + c] * X[rb + c] + b.gM[rb + c] * X[ra + c];
      acc = fmaf(g, V[c], acc);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) b.gr[p] = first ? acc : b.gr[p] + acc;
  }
}

// F_a = sum over a's edges of dE/dr (q_b - q_a)/r, frame-major [f][3][N]
__global__ __launch_bounds__(256) void k_mp_forces(MpnnBuffers b, SysDev S, RowSpan span,
                                                   float* Fout) {
  const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= span.rows()) return;
  const int f0 = span.f0;
  const long N = S.n;
  const long fl = row / N;
  const int i = (int)(row - fl * N);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int e1 = b.off[row + 1];
  for (int e = b.off[row]; e < e1; ++e) {
    // the pair's unit vector points from its owner row; the reverse edge
    // sees it negated
    const int u = b.uid[e];
    if (u == kNoPair) continue;  // only after a latched capacity overflow
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

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// fragment elements (uint4) of an I x K operand: I/16 tiles x K/32 steps x 64 lanes
size_t frag_elems(int I, int K) { return (size_t)(I / 16) * (K / 32) * 64; }

// all fragment arrays: per layer A2 and six node matrices (128 x 128), plus
// W1 forward (64 x 128) and reverse (128 x 64), each hi and lo
size_t frag_total() {
  return 2 * ((size_t)MP_T * 7 * frag_elems(MP_H, MP_H) + frag_elems(MP_RH, MP_H) +
              frag_elems(MP_H, MP_RH));
}

// blocks of the fixed grids over pairs: two per compute unit
constexpr unsigned kPairBlocks = 512;
// row tiles per block of the dense row products: up to one tile per block
constexpr unsigned kRowBlocksMax = 1024;

unsigned row_blocks(long rows) {
  const long tiles = (rows + 15) / 16;
  return (unsigned)(tiles < (long)kRowBlocksMax ? tiles : (long)kRowBlocksMax);
}

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
  b += al(4 * 4);
  b += al((MP_T + 1) * rows * MP_H * 4) + 2 * al(MP_T * rows * MP_H * 4);
  b += 2 * al(rows * MP_H * 4) + 2 * al(rows * MP_RH * 4) + 5 * al(rows * MP_H * 4);
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

bool mpnn_prepare(MpnnCtx& M, hipStream_t st, char* err, size_t errlen) {
  const MpnnWeights& w = M.w;
  auto launch = [&](const float* src, int ld, int trans, int I, int K, const MpnnFrag& d) {
    const long n = (long)frag_elems(I, K);
    hipLaunchKernelGGL(k_mp_frag, dim3(nblk(n, 256)), dim3(256), 0, st, src, ld, trans, I, K,
                       const_cast<uint4*>(d.hi), const_cast<uint4*>(d.lo));
    return hipGetLastError();
  };
  for (int t = 0; t < MP_T; ++t) {
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

bool mpnn_eval(MpnnCtx& M, const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
               int f0, int nf, const int* nvalid, float* Fout, double* epart, hipStream_t st,
               char* err, size_t errlen) {
  const MpnnWeights& w = M.w;
  MpnnBuffers& b = M.b;
  const long N = S.n, mt = L.mt;
  const long rows = (long)nf * N;
  const long cap = M.pair_cap;
  const RowSpan span{nvalid, f0, nf, N};
  // compact the in-cutoff pairs of every row into edges (list order), then
  // into unordered pairs; the totals stay on the device
  hipLaunchKernelGGL(k_mp_count, dim3((unsigned)rows), dim3(kRowThreads), 0, st, b, S, L, W, f0,
                     nf, nvalid, M.rc);
  MP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mp_scan, dim3(1), dim3(1024), 0, st, b, rows);
  MP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mp_edges, dim3((unsigned)rows), dim3(kRowThreads), 0, st, b, S, L, W, f0,
                     nf, nvalid, M.rc, cap);
  MP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mp_reverse, dim3(nblk(rows * mt, 256)), dim3(256), 0, st, b, rows,
                     rows * mt, L.status);
  MP_HIP(hipGetLastError());
  // filters W and dW/dr of every pair and layer
  hipLaunchKernelGGL(k_mp_filter, dim3(kPairBlocks), dim3(256), 0, st, w, b, M.rc, cap);
  MP_HIP(hipGetLastError());
  // forward through the layers
  hipLaunchKernelGGL(k_mp_embed, dim3((unsigned)rows), dim3(MP_H), 0, st, w, b, S, span);
  MP_HIP(hipGetLastError());
  const long rh = rows * MP_H;
  const dim3 rg(row_blocks(rows)), rb(256);
  for (int t = 0; t < MP_T; ++t) {
    float* Ht = b.H + t * rh;
    float* Hn = b.H + (t + 1) * rh;
    float* Xt = b.X + t * rh;
    float* Ut = b.U + t * rh;
    hipLaunchKernelGGL((k_mp_rows<MP_H, MP_H, EP_STORE>), rg, rb, 0, st, w.Bf[t], Ht, span, Xt,
                       nullptr, nullptr, nullptr);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mp_gather, dim3((unsigned)rows), dim3(MP_H), 0, st, b, t, Xt, b.Mm, span);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_mp_rows<MP_H, MP_H, EP_BIAS_SILU>), rg, rb, 0, st, w.C1f[t], b.Mm, span,
                       Ut, b.Sn, nullptr, w.c1[t]);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_mp_rows<MP_H, MP_H, EP_RESID>), rg, rb, 0, st, w.C2f[t], b.Sn, span, Hn,
                       nullptr, Ht, w.c2[t]);
    MP_HIP(hipGetLastError());
  }
  // readout and its gradient
  hipLaunchKernelGGL((k_mp_rows<MP_H, MP_RH, EP_STORE>), rg, rb, 0, st, w.W1f, b.H + MP_T * rh,
                     span, b.Y, nullptr, nullptr, nullptr);
  MP_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mp_readout, dim3(S.n_tiles, nf), dim3(64), 0, st, w, b, S, T, span, M.scale,
                     epart);
  MP_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_mp_rows<MP_RH, MP_H, EP_STORE>), rg, rb, 0, st, w.W1b, b.gY, span, b.gH,
                     nullptr, nullptr, nullptr);
  MP_HIP(hipGetLastError());
  // reverse pass through the layers
  for (int t = MP_T - 1; t >= 0; --t) {
    float* Xt = b.X + t * rh;
    float* Ut = b.U + t * rh;
    hipLaunchKernelGGL((k_mp_rows<MP_H, MP_H, EP_DSILU>), rg, rb, 0, st, w.C2b[t], b.gH, span,
                       b.gS, nullptr, Ut, nullptr);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_mp_rows<MP_H, MP_H, EP_STORE>), rg, rb, 0, st, w.C1b[t], b.gS, span,
                       b.gM, nullptr, nullptr, nullptr);
    MP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mp_dedr, dim3(kPairBlocks * 2), dim3(256), 0, st, b, t,
                       t == MP_T - 1 ? 1 : 0, Xt, cap);
    MP_HIP(hipGetLastError());
    if (t > 0) {
      hipLaunchKernelGGL(k_mp_gather, dim3((unsigned)rows), dim3(MP_H), 0, st, b, t, b.gM, b.gX,
                         span);
      MP_HIP(hipGetLastError());
      hipLaunchKernelGGL((k_mp_rows<MP_H, MP_H, EP_ACCUM>), rg, rb, 0, st, w.Bb[t], b.gX, span,
                         b.gP, nullptr, b.gH, nullptr);
      MP_HIP(hipGetLastError());
      float* tmp = b.gH;
      b.gH = b.gP;
      b.gP = tmp;
    }
  }
  hipLaunchKernelGGL(k_mp_forces, dim3(nblk(rows, 256)), dim3(256), 0, st, b, S, span, Fout);
  MP_HIP(hipGetLastError());
  return true;
}
