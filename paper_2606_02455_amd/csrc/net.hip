// net.hip -- the learned many-body draft on the GPU.
//
// Drafting evaluates, per frame, a node pass (this file) and then the pair
// force loop of the draft kernel (net_force in lsd_device.h):
//   node pass: D_i = species-resolved radial descriptor over the draft list,
//              h_i = silu(W1 D_i + b1[s_i]), v_i = W2 h_i;
//   force:     F_i = - sum_j sum_b e_b(r) (c_t[b] + v_i[b] + v_j[b]) d / r.
// The two dense layers are a [16 atoms x S B] x [S B x 32] and a
// [16 x 32] x [32 x B] product per block: in bfloat16 they run on the
// matrix cores (v_mfma_f32_16x16x16_bf16, binary32 accumulation), in
// binary32 on the vector ALUs.
//
// Training (force matching) runs in binary32 with binary64 reductions in a
// fixed order, so gradients are deterministic:
//   k_nt_nodes  descriptor, pre-activations z and v of every atom frame;
//   k_nt_resid  forces and G = dSSE/dF = 2 (F - y), squared error per block;
//               for the loss of force changes the forces are kept and
//   k_nt_diff   forms delta_k = (F_k+1 - F_k) - (y_k+1 - y_k) and
//               G_k = 2 (delta_k-1 - delta_k);
//   k_nt_back   gamma_ij = (G_j - G_i) . d / r per list entry, the
//               species-resolved sums Pc_i[s][b] = sum_{j in s} gamma_ij e_b,
//               dv_i = sum_s Pc_i[s], dz_i = (W2^T dv_i) silu'(z_i), and per
//               block the parameter partials dW1 = sum dz D^T, db1, dW2 =
//               sum dv h^T, dc_t = 1/2 sum Pc over the entries of type t;
//   k_nt_reduce blocks summed in order into the caller's gradient.
#include "net.h"
#include "net_node.h"

static_assert(LSD_LPA >= 4 && LSD_NET_HIDDEN % LSD_LPA == 0,
              "the node pass splits the hidden units over the lanes of an atom");
#define NET_THREADS (NET_ROWS * LSD_LPA)
#define NET_HPL (LSD_NET_HIDDEN / LSD_LPA)   // hidden units per lane
#define NET_DPL (LSD_NET_MAX_DESC / LSD_LPA) // descriptor slots per lane
#define NET_ITHREADS (NET_IROWS * LSD_LPA)

namespace {


struct NetLds {
  float W1[LSD_NET_HIDDEN][LSD_NET_MAX_DESC + 1];   // [h][d], zero beyond S B
  float W2[LSD_NET_MAX_BASIS][LSD_NET_HIDDEN + 1];  // [b][h], zero rows beyond B
  float b1[LSD_NET_MAX_SPECIES][LSD_NET_HIDDEN];
};

__device__ __forceinline__ void load_weights(const PotDev& P, NetLds& L, int t, int nt) {
  const int S = P.ns, B = P.nb, Din = S * B;
  const float* w2 = P.w + net_off_w2(S, B);
  const float* b1 = P.w + net_off_b1(S, B);
  for (int idx = t; idx < LSD_NET_HIDDEN * LSD_NET_MAX_DESC; idx += nt) {
    const int h = idx / LSD_NET_MAX_DESC, d = idx % LSD_NET_MAX_DESC;
    L.W1[h][d] = d < Din ? P.w[h * Din + d] : 0.0f;
  }
  for (int idx = t; idx < LSD_NET_MAX_BASIS * LSD_NET_HIDDEN; idx += nt) {
    const int b = idx / LSD_NET_HIDDEN, h = idx % LSD_NET_HIDDEN;
    L.W2[b][h] = b < B ? w2[b * LSD_NET_HIDDEN + h] : 0.0f;
  }
  for (int idx = t; idx < LSD_NET_MAX_SPECIES * LSD_NET_HIDDEN; idx += nt) {
    const int s = idx / LSD_NET_HIDDEN, h = idx % LSD_NET_HIDDEN;
    L.b1[s][h] = s < S ? b1[s * LSD_NET_HIDDEN + h] : 0.0f;
  }
}

// D[s][b] = sum over the row's entries j of species s within the cutoff of
// e_b(r_ij), summed over the NL lanes of the atom (all lanes hold it).
template <int NL = LSD_LPA>
__device__ __forceinline__ void net_descriptor(const PotDev& P, const SysDev& S,
                                               const float4* __restrict__ X,
                                               const uint32_t* __restrict__ row, int width,
                                               int cnt, int i, int r, int sub,
                                               float D[LSD_NET_MAX_SPECIES][LSD_NET_MAX_BASIS]) {
#pragma unroll
  for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
#pragma unroll
    for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) D[s][b] = 0.0f;
  const float Lf = (float)S.box[r];
  const float4 xi = X[i];
  const int B = P.nb;
  // the first group of entries is gathered whatever the count
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
      float e[LSD_NET_MAX_BASIS];
      net_radial(P.pi_rc, rr, 1.0f / rr, B, e);
      const int spj = gt.sp[u];
#pragma unroll
      for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
#pragma unroll
        for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) D[s][b] += s == spj ? e[b] : 0.0f;
    }
  }
#pragma unroll
  for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
#pragma unroll
    for (int b = 0; b < LSD_NET_MAX_BASIS; ++b)
      if (s < P.ns && b < B) D[s][b] = lanes_sum<NL>(D[s][b]);
}

// Binary32 dense layers for the hidden units sub*HPL .. of one atom: z of
// those units and this lane's share vp of v (summed over the lanes later).
__device__ __forceinline__ void mlp_fp32(const NetLds& L, const float* __restrict__ Drow, int sp,
                                         int sub, float z[NET_HPL],
                                         float vp[LSD_NET_MAX_BASIS]) {
#pragma unroll
  for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) vp[b] = 0.0f;
#pragma unroll
  for (int u = 0; u < NET_HPL; ++u) {
    const int h = sub * NET_HPL + u;
    float acc = L.b1[sp][h];
#pragma unroll
    for (int d = 0; d < LSD_NET_MAX_DESC; ++d) acc += L.W1[h][d] * Drow[d];
    z[u] = acc;
    const float hv = silu(acc);
#pragma unroll
    for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) vp[b] += L.W2[b][h] * hv;
  }
}

__device__ __forceinline__ void store_v(float* __restrict__ dst, const float v[LSD_NET_MAX_BASIS],
                                        int B) {
  float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
  for (int q = 0; q < LSD_NET_MAX_BASIS / 4; ++q)
    d4[q] = make_float4(4 * q < B ? v[4 * q] : 0.0f, 4 * q + 1 < B ? v[4 * q + 1] : 0.0f,
                        4 * q + 2 < B ? v[4 * q + 2] : 0.0f, 4 * q + 3 < B ? v[4 * q + 3] : 0.0f);
}

// Node pass of frame k for drafting: P.v[i] for every atom of a valid frame.
// Small blocks (NET_IROWS atoms, one wave) spread a frame of a small system
// over many compute units; the pass is latency bound.
__global__ __launch_bounds__(NET_ITHREADS) void k_net_nodes_f32(SysDev S, ListDev Lst, WinDev W,
                                                                PotDev P, int k) {
  __shared__ NetLds L;
  __shared__ float s_D[NET_IROWS][LSD_NET_MAX_DESC + 1];
  const int t = threadIdx.x, a = t / LSD_LPA, sub = t % LSD_LPA;
  const int i0 = blockIdx.x * NET_IROWS + a;
  const bool in = i0 < S.n;
  const int i = in ? i0 : S.n - 1;
  const int r = S.R == 1 ? 0 : S.atom_rep[i];
  // frames past the skin or after a rejection already found are not
  // drafted: a block none of whose atoms has a valid frame does nothing
  // (the atom's entry count is requested together with that test)
  const bool ok = in && W.invalid[(size_t)r * S.kmax + k] == 0 && k <= W.rej[r];
  const int cnt = Lst.cnt_d[i];
  if (!__syncthreads_or(ok ? 1 : 0)) return;
  const int B = P.nb, Din = P.ns * B;
  const size_t N = (size_t)S.n;
  load_weights(P, L, t, NET_ITHREADS);
  float D[LSD_NET_MAX_SPECIES][LSD_NET_MAX_BASIS];
  net_descriptor(P, S, W.qmid + (size_t)k * N, Lst.nbr_d + (size_t)i * Lst.md, Lst.md,
                 ok ? cnt : 0, i, r, sub, D);
  const int sp = S.species ? S.species[i] : 0;
  if (sub == 0) {
#pragma unroll
    for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
#pragma unroll
      for (int b = 0; b < LSD_NET_MAX_BASIS; ++b)
        if (s < P.ns && b < B) s_D[a][s * B + b] = D[s][b];
    for (int d = Din; d < LSD_NET_MAX_DESC; ++d) s_D[a][d] = 0.0f;
  }
  __syncthreads();
  float z[NET_HPL], vp[LSD_NET_MAX_BASIS];
  mlp_fp32(L, s_D[a], sp, sub, z, vp);
#pragma unroll
  for (int b = 0; b < LSD_NET_MAX_BASIS; ++b)
    if (b < B) vp[b] = lpa_sum(vp[b]);
  if (sub == 0 && ok) store_v(P.v + (size_t)i * LSD_NET_MAX_BASIS, vp, B);
}

// The bfloat16 node pass (net_node.h), one block per 16 atoms.
template <int NL>
__global__ __launch_bounds__(NET_IROWS * NL) void k_net_nodes_bf16(SysDev S, ListDev Lst, WinDev W,
                                                                  PotDev P, int k) {
  net_nodes_bf16_block<NL>(S, Lst, W, P, k, blockIdx.x);
}

// OCP e4m3 (largest finite 448), 8 values of x / s packed for one operand
// of v_mfma_f32_16x16x32_fp8_fp8 (element e in byte e), round to nearest
// even after saturation to +-448.
__device__ __forceinline__ long pack_fp8(const float x[8], float inv_s) {
  float y[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) y[e] = fminf(fmaxf(x[e] * inv_s, -448.0f), 448.0f);
  int w0 = __builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
  w0 = __builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], w0, true);
  int w1 = __builtin_amdgcn_cvt_pk_fp8_f32(y[4], y[5], 0, false);
  w1 = __builtin_amdgcn_cvt_pk_fp8_f32(y[6], y[7], w1, true);
  return (long)(((unsigned long)(unsigned)w1 << 32) | (unsigned)w0);
}

__device__ __forceinline__ unsigned char to_fp8(float x, float inv_s) {
  const float y = fminf(fmaxf(x * inv_s, -448.0f), 448.0f);
  return (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(y, 0.0f, 0, false) & 0xFF);
}

__device__ __forceinline__ float wave_absmax(float v) {
  v = fabsf(v);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// FP8 (OCP e4m3) on the matrix cores, one scale per tensor: W1, W2 by their
// max |.| / 448 (every block reduces the same values, so all blocks agree),
// D and h by the calibrated static scales.  16x16x32 operands: lane l holds
// A[l % 16][8 (l / 16) + 0..7] and B[8 (l / 16) + 0..7][l % 16]; the result
// D[4 (l / 16) + 0..3][l % 16].
template <int NL>
__global__ __launch_bounds__(NET_IROWS * NL) void k_net_nodes_fp8(SysDev S, ListDev Lst, WinDev W,
                                                                 PotDev P, int k) {
  __shared__ float s_b1[LSD_NET_MAX_SPECIES][LSD_NET_HIDDEN];
  __shared__ __align__(8) unsigned char s_Dq[NET_IROWS][LSD_NET_MAX_DESC];
  __shared__ __align__(8) unsigned char s_hq[NET_IROWS][LSD_NET_HIDDEN];
  __shared__ int s_sp[NET_IROWS], s_ok[NET_IROWS];
  __shared__ NetStage stage;
  static_assert(NL == LSD_NET_MAX_BASIS, "one lane per radial function");
  const int t = threadIdx.x, a = t / NL, sub = t % NL;
  const int i0 = blockIdx.x * NET_IROWS + a;
  const bool in = i0 < S.n;
  const int i = in ? i0 : S.n - 1;
  const int r = S.R == 1 ? 0 : S.atom_rep[i];
  // frames past the skin or after a rejection already found are not
  // drafted: a block none of whose atoms has a valid frame does nothing
  // (the atom's entry count is requested together with that test)
  const bool ok = in && W.invalid[(size_t)r * S.kmax + k] == 0 && k <= W.rej[r];
  const int cnt = Lst.cnt_d[i];
  if (!__syncthreads_or(ok ? 1 : 0)) return;
  const int B = P.nb, Din = P.ns * B;
  const size_t N = (size_t)S.n;
  const int li = t % 16, kq = (t % 64) / 16;
  const bool mw = t < 64;
  constexpr int KS1 = LSD_NET_MAX_DESC / 32;
  const int ks1 = (Din + 31) / 32;
  long bw1[2][KS1], bw2 = 0;
  float s_w1 = 1.0f, s_w2 = 1.0f;
  if (mw) {
    const float* w2 = P.w + net_off_w2(P.ns, B);
    float f1[2][KS1][8], f2[8];
    float m1 = 0.0f, m2 = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int d = 32 * ks + 8 * kq + e, h = 16 * nt + li;
          f1[nt][ks][e] = d < Din ? P.w[h * Din + d] : 0.0f;
          m1 = fmaxf(m1, fabsf(f1[nt][ks][e]));
        }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      f2[e] = li < B ? w2[li * LSD_NET_HIDDEN + 8 * kq + e] : 0.0f;
      m2 = fmaxf(m2, fabsf(f2[e]));
    }
    m1 = wave_absmax(m1);
    m2 = wave_absmax(m2);
    s_w1 = m1 > 0.0f ? m1 / 448.0f : 1.0f;
    s_w2 = m2 > 0.0f ? m2 / 448.0f : 1.0f;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) bw1[nt][ks] = pack_fp8(f1[nt][ks], 1.0f / s_w1);
    bw2 = pack_fp8(f2, 1.0f / s_w2);
  }
  {
    const float* b1 = P.w + net_off_b1(P.ns, B);
    for (int idx = t; idx < LSD_NET_MAX_SPECIES * LSD_NET_HIDDEN; idx += NET_IROWS * NL) {
      const int s = idx / LSD_NET_HIDDEN, h = idx % LSD_NET_HIDDEN;
      s_b1[s][h] = s < P.ns ? b1[s * LSD_NET_HIDDEN + h] : 0.0f;
    }
  }
  float acc[LSD_NET_MAX_SPECIES];
  net_descriptor_lanes(P, S, W.qmid + (size_t)k * N, Lst.nbr_d + (size_t)i * Lst.md, Lst.md,
                       ok ? cnt : 0, i, r, a, sub, stage, acc);
  const float inv_sD = 1.0f / P.fp8_sD, inv_sh = 1.0f / P.fp8_sh;
  if (sub == 0) {
    s_sp[a] = S.species ? S.species[i] : 0;
    s_ok[a] = ok ? 1 : 0;
  }
  if (sub < B) {
#pragma unroll
    for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
      if (s < P.ns) s_Dq[a][s * B + sub] = to_fp8(acc[s], inv_sD);
  }
  for (int d = Din + sub; d < LSD_NET_MAX_DESC; d += NL) s_Dq[a][d] = 0;
  __syncthreads();
  if (mw) {
    f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KS1; ++ks) {
      if (ks >= ks1) break;  // zero descriptor slots
      const long av = *reinterpret_cast<const long*>(&s_Dq[li][32 * ks + 8 * kq]);
      acc0 = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bw1[0][ks], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bw1[1][ks], acc1, 0, 0, 0);
    }
    const float sc1 = P.fp8_sD * s_w1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ar = 4 * kq + q;
      const int spa = s_sp[ar];
      s_hq[ar][li] = to_fp8(silu(acc0[q] * sc1 + s_b1[spa][li]), inv_sh);
      s_hq[ar][16 + li] = to_fp8(silu(acc1[q] * sc1 + s_b1[spa][16 + li]), inv_sh);
    }
  }
  __syncthreads();
  if (mw) {
    f32x4 acc2 = {0.0f, 0.0f, 0.0f, 0.0f};
    const long av = *reinterpret_cast<const long*>(&s_hq[li][8 * kq]);
    acc2 = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bw2, acc2, 0, 0, 0);
    const float sc2 = P.fp8_sh * s_w2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ar = 4 * kq + q;
      const int ia = blockIdx.x * NET_IROWS + ar;
      if (ia < S.n && s_ok[ar])
        P.v[(size_t)ia * LSD_NET_MAX_BASIS + li] = li < B ? acc2[q] * sc2 : 0.0f;
    }
  }
}

// ---------------------------------------------------------------------------
// Training: block (atom tile, frame f)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NET_THREADS) void k_nt_nodes(SysDev S, ListDev Lst, WinDev W,
                                                          PotDev P, NetTrainDev T) {
  __shared__ NetLds L;
  __shared__ float s_D[NET_ROWS][LSD_NET_MAX_DESC + 1];
  const int t = threadIdx.x, a = t / LSD_LPA, sub = t % LSD_LPA, f = blockIdx.y;
  const int i0 = blockIdx.x * NET_ROWS + a;
  const bool in = i0 < S.n;
  const int i = in ? i0 : S.n - 1;
  const int r = S.atom_rep[i];
  const bool ok = in && W.invalid[(size_t)r * S.kmax + f] == 0;
  const int B = P.nb, Din = P.ns * B;
  const size_t N = (size_t)S.n, fi = (size_t)f * N + i;
  load_weights(P, L, t, NET_THREADS);
  float D[LSD_NET_MAX_SPECIES][LSD_NET_MAX_BASIS];
  net_descriptor(P, S, W.qmid + (size_t)f * N, Lst.nbr_t + (size_t)i * Lst.mt, Lst.mt,
                 ok ? Lst.cnt_t[i] : 0, i, r, sub, D);
  const int sp = S.species ? S.species[i] : 0;
  if (sub == 0) {
#pragma unroll
    for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
#pragma unroll
      for (int b = 0; b < LSD_NET_MAX_BASIS; ++b)
        if (s < P.ns && b < B) s_D[a][s * B + b] = D[s][b];
    for (int d = Din; d < LSD_NET_MAX_DESC; ++d) s_D[a][d] = 0.0f;
  }
  __syncthreads();
  if (in) {
#pragma unroll
    for (int u = 0; u < NET_DPL; ++u)
      T.D[fi * LSD_NET_MAX_DESC + sub * NET_DPL + u] = s_D[a][sub * NET_DPL + u];
  }
  float z[NET_HPL], vp[LSD_NET_MAX_BASIS];
  mlp_fp32(L, s_D[a], sp, sub, z, vp);
  if (in) {
#pragma unroll
    for (int u = 0; u < NET_HPL; ++u) T.z[fi * LSD_NET_HIDDEN + sub * NET_HPL + u] = z[u];
  }
#pragma unroll
  for (int b = 0; b < LSD_NET_MAX_BASIS; ++b)
    if (b < B) vp[b] = lpa_sum(vp[b]);
  if (sub == 0 && in) store_v(T.v + fi * LSD_NET_MAX_BASIS, vp, B);
}

__global__ __launch_bounds__(NET_THREADS) void k_nt_resid(SysDev S, ListDev Lst, WinDev W,
                                                          PotDev P, NetTrainDev T,
                                                          int use_target, int diff) {
  __shared__ double s_e[NET_ROWS];
  __shared__ int s_c[NET_ROWS];
  const int t = threadIdx.x, a = t / LSD_LPA, sub = t % LSD_LPA, f = blockIdx.y;
  const int i0 = blockIdx.x * NET_ROWS + a;
  const bool in = i0 < S.n;
  const int i = in ? i0 : S.n - 1;
  const int r = S.atom_rep[i];
  const bool ok = in && W.invalid[(size_t)r * S.kmax + f] == 0;
  const size_t N = (size_t)S.n;
  PotDev Q = P;
  Q.v = T.v + (size_t)f * N * LSD_NET_MAX_BASIS;
  float F[3];
  net_force(Q, S, W.qmid + (size_t)f * N, Lst.nbr_t + (size_t)i * Lst.mt, Lst.mt,
            ok ? Lst.cnt_t[i] : 0, i, r, sub, P.w + net_off_c(P.ns, P.nb), F[0], F[1], F[2]);
  if (diff) {
    if (sub == 0 && in) {
#pragma unroll
      for (int d = 0; d < 3; ++d) T.F[((size_t)f * 3 + d) * N + i] = ok ? F[d] : 0.0f;
    }
    return;
  }
  if (sub == 0) {
    const float* Y = (use_target ? W.ft : W.fd) + (size_t)f * 3 * N;
    double e = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float res = ok ? F[d] - Y[d * N + i] : 0.0f;
      if (in) T.G[((size_t)f * 3 + d) * N + i] = 2.0f * res;
      e += (double)res * (double)res;
    }
    s_e[a] = e;
    s_c[a] = ok ? 1 : 0;
  }
  __syncthreads();
  if (t == 0) {
    double se = 0.0;
    int c = 0;
    for (int q = 0; q < NET_ROWS; ++q) {
      se += s_e[q];
      c += s_c[q];
    }
    double* row = T.partial + ((size_t)f * T.nblk + blockIdx.x) * NET_PROW;
    row[NET_PMAX] = se;
    row[NET_PMAX + 1] = (double)c;
  }
}

// Loss of force changes: one thread per atom of frame f.  Frames are valid
// up to K_eff, so a valid frame f + 1 implies a valid frame f.
__global__ __launch_bounds__(NET_ROWS) void k_nt_diff(SysDev S, WinDev W, NetTrainDev T,
                                                      int use_target) {
  __shared__ double s_e[NET_ROWS];
  __shared__ int s_c[NET_ROWS];
  const int a = threadIdx.x, f = blockIdx.y;
  const int i0 = blockIdx.x * NET_ROWS + a;
  const bool in = i0 < S.n;
  const int i = in ? i0 : S.n - 1;
  const int* inv = W.invalid + (size_t)S.atom_rep[i] * S.kmax;
  const size_t N = (size_t)S.n;
  const float* Y = use_target ? W.ft : W.fd;
  // delta_k of this atom, for k = f - 1 (before) and k = f (after)
  const bool has_before = in && f >= 1 && inv[f] == 0;
  const bool has_after = in && f + 1 < W.K && inv[f + 1] == 0;
  double e = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const size_t c0 = ((size_t)f * 3 + d) * N + i;
    float before = 0.0f, after = 0.0f;
    if (has_before) {
      const size_t cm = c0 - 3 * N;
      before = (T.F[c0] - T.F[cm]) - (Y[c0] - Y[cm]);
    }
    if (has_after) {
      const size_t cp = c0 + 3 * N;
      after = (T.F[cp] - T.F[c0]) - (Y[cp] - Y[c0]);
      e += (double)after * (double)after;
    }
    if (in) T.G[c0] = 2.0f * before - 2.0f * after;
  }
  s_e[a] = e;
  s_c[a] = has_after ? 1 : 0;
  __syncthreads();
  if (a == 0) {
    double se = 0.0;
    int c = 0;
    for (int q = 0; q < NET_ROWS; ++q) {
      se += s_e[q];
      c += s_c[q];
    }
    double* row = T.partial + ((size_t)f * T.nblk + blockIdx.x) * NET_PROW;
    row[NET_PMAX] = se;
    row[NET_PMAX + 1] = (double)c;
  }
}

__global__ __launch_bounds__(NET_THREADS) void k_nt_back(SysDev S, ListDev Lst, WinDev W,
                                                         PotDev P, NetTrainDev T) {
  __shared__ float s_D[NET_ROWS][LSD_NET_MAX_DESC + 1];
  __shared__ float s_dz[NET_ROWS][LSD_NET_HIDDEN + 1];
  __shared__ float s_h[NET_ROWS][LSD_NET_HIDDEN + 1];
  __shared__ float s_Pc[NET_ROWS][LSD_NET_MAX_DESC + 1];
  __shared__ float s_dv[NET_ROWS][LSD_NET_MAX_BASIS + 1];
  __shared__ float s_W2[LSD_NET_MAX_BASIS][LSD_NET_HIDDEN + 1];
  __shared__ int s_sp[NET_ROWS];
  const int t = threadIdx.x, a = t / LSD_LPA, sub = t % LSD_LPA, f = blockIdx.y;
  const int i0 = blockIdx.x * NET_ROWS + a;
  const bool in = i0 < S.n;
  const int i = in ? i0 : S.n - 1;
  const int r = S.atom_rep[i];
  const bool ok = in && W.invalid[(size_t)r * S.kmax + f] == 0;
  const int Sn = P.ns, B = P.nb, Din = Sn * B;
  const size_t N = (size_t)S.n, fi = (size_t)f * N + i;
  {
    const float* w2 = P.w + net_off_w2(Sn, B);
    for (int idx = t; idx < LSD_NET_MAX_BASIS * LSD_NET_HIDDEN; idx += NET_THREADS) {
      const int b = idx / LSD_NET_HIDDEN, h = idx % LSD_NET_HIDDEN;
      s_W2[b][h] = b < B ? w2[b * LSD_NET_HIDDEN + h] : 0.0f;
    }
  }
  // gamma_ij e_b(r_ij) summed by the species of j
  float Pc[LSD_NET_MAX_SPECIES][LSD_NET_MAX_BASIS];
#pragma unroll
  for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
#pragma unroll
    for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) Pc[s][b] = 0.0f;
  {
    const float4* X = W.qmid + (size_t)f * N;
    const float* G = T.G + (size_t)f * 3 * N;
    const float Lf = (float)S.box[r];
    const float4 xi = X[i];
    const float gx = G[i], gy = G[N + i], gz = G[2 * N + i];
    const uint32_t* row = Lst.nbr_t + (size_t)i * Lst.mt;
    const int cnt = ok ? Lst.cnt_t[i] : 0;
    for (int m = sub; m < cnt; m += LSD_LPA) {
      const uint32_t ent = row[m];
      const int j = (int)(ent >> 5), code = (int)(ent & 31u);
      const float4 xj = X[j];
      float sj[3], si[3];
      image_shifts(code, Lf, sj, si);
      const float dx = sep(xj.x, sj[0], xi.x, si[0]);
      const float dy = sep(xj.y, sj[1], xi.y, si[1]);
      const float dz = sep(xj.z, sj[2], xi.z, si[2]);
      const float r2 = dx * dx + dy * dy + dz * dz;
      if (r2 >= P.rc2) continue;
      const float rr = sqrtf(r2);
      const float inv_r = 1.0f / rr;
      float e[LSD_NET_MAX_BASIS];
      net_radial(P.pi_rc, rr, inv_r, B, e);
      const float gam = ((G[j] - gx) * dx + (G[N + j] - gy) * dy + (G[2 * N + j] - gz) * dz) * inv_r;
      const int spj = S.species ? S.species[j] : 0;
#pragma unroll
      for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
#pragma unroll
        for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) Pc[s][b] += s == spj ? gam * e[b] : 0.0f;
    }
  }
#pragma unroll
  for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
#pragma unroll
    for (int b = 0; b < LSD_NET_MAX_BASIS; ++b)
      if (s < Sn && b < B) Pc[s][b] = lpa_sum(Pc[s][b]);
  if (sub == 0) {
    s_sp[a] = ok ? (S.species ? S.species[i] : 0) : -1;
#pragma unroll
    for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) {
      float dv = 0.0f;
#pragma unroll
      for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
        if (s < Sn && b < B) {
          s_Pc[a][s * B + b] = Pc[s][b];
          dv += Pc[s][b];
        }
      s_dv[a][b] = dv;
    }
  }
  __syncthreads();
  // node backward for this lane's hidden units and descriptor slots
#pragma unroll
  for (int u = 0; u < NET_HPL; ++u) {
    const int h = sub * NET_HPL + u;
    const float z = ok ? T.z[fi * LSD_NET_HIDDEN + h] : 0.0f;
    float dh = 0.0f;
#pragma unroll
    for (int b = 0; b < LSD_NET_MAX_BASIS; ++b) dh += s_W2[b][h] * s_dv[a][b];
    s_dz[a][h] = ok ? dh * silu_grad(z) : 0.0f;
    s_h[a][h] = ok ? silu(z) : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < NET_DPL; ++u) {
    const int d = sub * NET_DPL + u;
    s_D[a][d] = ok ? T.D[fi * LSD_NET_MAX_DESC + d] : 0.0f;
  }
  __syncthreads();
  // parameter partials of this block, atoms summed in order
  const int ob1 = net_off_b1(Sn, B), ow2 = net_off_w2(Sn, B), oc = net_off_c(Sn, B);
  const int np = net_params(Sn, B);
  double* out = T.partial + ((size_t)f * T.nblk + blockIdx.x) * NET_PROW;
  for (int p = t; p < np; p += NET_THREADS) {
    double acc = 0.0;
    if (p < ob1) {
      const int h = p / Din, d = p % Din;
      for (int q = 0; q < NET_ROWS; ++q) acc += (double)s_dz[q][h] * (double)s_D[q][d];
    } else if (p < ow2) {
      const int s = (p - ob1) / LSD_NET_HIDDEN, h = (p - ob1) % LSD_NET_HIDDEN;
      for (int q = 0; q < NET_ROWS; ++q)
        if (s_sp[q] == s) acc += (double)s_dz[q][h];
    } else if (p < oc) {
      const int b = (p - ow2) / LSD_NET_HIDDEN, h = (p - ow2) % LSD_NET_HIDDEN;
      for (int q = 0; q < NET_ROWS; ++q) acc += (double)s_dv[q][b] * (double)s_h[q][h];
    } else {
      const int ty = (p - oc) / B, b = (p - oc) % B;
      for (int q = 0; q < NET_ROWS; ++q) {
        if (s_sp[q] < 0) continue;
        for (int s = 0; s < Sn; ++s)
          if (pair_type(s_sp[q], s, Sn) == ty) acc += 0.5 * (double)s_Pc[q][s * B + b];
      }
    }
    out[p] = acc;
  }
}

// Calibration of the FP8 activation scales: per block the largest |D| and
// |silu(z)| of its valid atom frames, then one block takes the maximum.
__global__ __launch_bounds__(NET_ROWS) void k_nt_amax(SysDev S, WinDev W, NetTrainDev T, int Din) {
  __shared__ float s_m[2][NET_ROWS];
  const int a = threadIdx.x, f = blockIdx.y;
  const int i0 = blockIdx.x * NET_ROWS + a;
  const bool in = i0 < S.n;
  const int i = in ? i0 : S.n - 1;
  const bool ok = in && W.invalid[(size_t)S.atom_rep[i] * S.kmax + f] == 0;
  const size_t fi = (size_t)f * S.n + i;
  float mD = 0.0f, mh = 0.0f;
  if (ok) {
    for (int d = 0; d < Din; ++d) mD = fmaxf(mD, fabsf(T.D[fi * LSD_NET_MAX_DESC + d]));
    for (int h = 0; h < LSD_NET_HIDDEN; ++h)
      mh = fmaxf(mh, fabsf(silu(T.z[fi * LSD_NET_HIDDEN + h])));
  }
  s_m[0][a] = mD;
  s_m[1][a] = mh;
  __syncthreads();
  if (a < 2) {
    float m = 0.0f;
    for (int q = 0; q < NET_ROWS; ++q) m = fmaxf(m, s_m[a][q]);
    T.partial[((size_t)f * T.nblk + blockIdx.x) * 2 + a] = (double)m;
  }
}

__global__ __launch_bounds__(256) void k_nt_amax_final(const double* __restrict__ part, int rows,
                                                       double* __restrict__ out) {
  __shared__ double s_m[2][256];
  const int t = threadIdx.x;
  double m0 = 0.0, m1 = 0.0;
  for (int b = t; b < rows; b += 256) {
    m0 = fmax(m0, part[(size_t)b * 2]);
    m1 = fmax(m1, part[(size_t)b * 2 + 1]);
  }
  s_m[0][t] = m0;
  s_m[1][t] = m1;
  __syncthreads();
  if (t < 2) {
    double m = 0.0;
    for (int q = 0; q < 256; ++q) m = fmax(m, s_m[t][q]);
    out[t] = m;
  }
}

__global__ __launch_bounds__(256) void k_nt_reduce(const double* __restrict__ partial, int rows,
                                                   int np, double* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np + 2) return;
  const int idx = p < np ? p : NET_PMAX + (p - np);
  double acc = 0.0;
  for (int b = 0; b < rows; ++b) acc += partial[(size_t)b * NET_PROW + idx];
  grad[p] += acc;
}

__global__ __launch_bounds__(1024) void k_net_adam(float* __restrict__ params, double* __restrict__ m,
                                                   double* __restrict__ v, double* __restrict__ grad,
                                                   int np, double lr, double beta1, double beta2,
                                                   double eps, double c1, double c2) {
  const double rows = grad[np + 1];
  __syncthreads();  // every thread has read the count before it is cleared
  if (!(rows > 0.0)) return;
  const double sc = 1.0 / (3.0 * rows);
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const double g = grad[p] * sc;
    const double mp = beta1 * m[p] + (1.0 - beta1) * g;
    const double vp = beta2 * v[p] + (1.0 - beta2) * g * g;
    m[p] = mp;
    v[p] = vp;
    const double mh = mp / c1, vh = vp / c2;
    params[p] = (float)((double)params[p] - lr * mh / (sqrt(vh) + eps));
    grad[p] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    grad[np] = 0.0;
    grad[np + 1] = 0.0;
  }
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t net_train_bytes(int K, int N) {
  const size_t kn = (size_t)K * N, nblk = ((size_t)N + NET_ROWS - 1) / NET_ROWS;
  return align256(kn * LSD_NET_MAX_DESC * 4) + align256(kn * LSD_NET_HIDDEN * 4) +
         align256(kn * LSD_NET_MAX_BASIS * 4) + 2 * align256(kn * 3 * 4) +
         align256((size_t)K * nblk * NET_PROW * 8);
}

NetTrainDev net_train_bind(char* base, int K, int N) {
  const size_t kn = (size_t)K * N;
  NetTrainDev T;
  T.nblk = (N + NET_ROWS - 1) / NET_ROWS;
  size_t off = 0;
  T.D = reinterpret_cast<float*>(base + off);
  off += align256(kn * LSD_NET_MAX_DESC * 4);
  T.z = reinterpret_cast<float*>(base + off);
  off += align256(kn * LSD_NET_HIDDEN * 4);
  T.v = reinterpret_cast<float*>(base + off);
  off += align256(kn * LSD_NET_MAX_BASIS * 4);
  T.G = reinterpret_cast<float*>(base + off);
  off += align256(kn * 3 * 4);
  T.F = reinterpret_cast<float*>(base + off);
  off += align256(kn * 3 * 4);
  T.partial = reinterpret_cast<double*>(base + off);
  return T;
}

hipError_t launch_net_nodes(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P,
                            int k, hipStream_t st) {
  const dim3 grid((S.n + NET_IROWS - 1) / NET_IROWS), wide(NET_IROWS * NET_NODE_LPA);
  if (P.prec == 2)
    hipLaunchKernelGGL(k_net_nodes_fp8<NET_NODE_LPA>, grid, wide, 0, st, S, L, W, P, k);
  else if (P.prec == 1)
    hipLaunchKernelGGL(k_net_nodes_bf16<NET_NODE_LPA>, grid, wide, 0, st, S, L, W, P, k);
  else
    hipLaunchKernelGGL(k_net_nodes_f32, grid, dim3(NET_ITHREADS), 0, st, S, L, W, P, k);
  return hipGetLastError();
}

hipError_t launch_net_train(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P,
                            const NetTrainDev& T, int use_target, int diff, double* grad,
                            hipStream_t st) {
  const dim3 grid(T.nblk, W.K), block(NET_THREADS);
  hipLaunchKernelGGL(k_nt_nodes, grid, block, 0, st, S, L, W, P, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nt_resid, grid, block, 0, st, S, L, W, P, T, use_target, diff);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (diff) {
    hipLaunchKernelGGL(k_nt_diff, grid, dim3(NET_ROWS), 0, st, S, W, T, use_target);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_nt_back, grid, block, 0, st, S, L, W, P, T);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int np = net_params(P.ns, P.nb);
  hipLaunchKernelGGL(k_nt_reduce, dim3((np + 2 + 255) / 256), dim3(256), 0, st, T.partial,
                     W.K * T.nblk, np, grad);
  return hipGetLastError();
}

hipError_t launch_net_amax(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P,
                           const NetTrainDev& T, double* amax, hipStream_t st) {
  hipLaunchKernelGGL(k_nt_nodes, dim3(T.nblk, W.K), dim3(NET_THREADS), 0, st, S, L, W, P, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nt_amax, dim3(T.nblk, W.K), dim3(NET_ROWS), 0, st, S, W, T, P.ns * P.nb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nt_amax_final, dim3(1), dim3(256), 0, st, T.partial, W.K * T.nblk, amax);
  return hipGetLastError();
}

hipError_t launch_net_adam(float* params, double* m, double* v, double* grad, int n_params,
                           double lr, double beta1, double beta2, double eps, long long t,
                           hipStream_t st) {
  const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  hipLaunchKernelGGL(k_net_adam, dim3(1), dim3(1024), 0, st, params, m, v, grad, n_params, lr,
                     beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}
