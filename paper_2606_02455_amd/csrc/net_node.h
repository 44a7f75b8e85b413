// net_node.h -- the learned draft's node pass on the matrix cores in
// bfloat16, as a function of one block of 16 atoms (block index `blk`), so
// that the per-frame node-pass kernel and the one-launch tail of a short
// system's draft chain run the same code.
//   D_i = species-resolved radial descriptor over the draft list,
//   h_i = silu(W1 D_i + b1[s_i]),  v_i = W2 h_i.
#pragma once
#include <hip/hip_runtime.h>

#include "lsd_device.h"

#define NET_IROWS 16  // atoms per block of the drafting node pass
// lanes per atom of the matrix-core node passes: one per radial function
#define NET_NODE_LPA LSD_NET_MAX_BASIS

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// binary32 -> bfloat16, round to nearest even (finite values)
__device__ __forceinline__ unsigned short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

// Descriptor of the 16 atoms of a node-pass block with one lane per radial
// function (16 lanes per atom).  The atom's lanes first stage the distance
// and species of its list entries in LDS, 64 entries at a time (entry m on
// lane m mod 16); then lane b sums e_{b+1}(r) = f_c(r) sin((b+1) pi r / r_c) / r
// over the staged entries of each species, in entry order, so no lanes are
// summed across.  sin and cos come from the vector unit's own instructions
// (arguments in turns, at most 8 here): their error is far below the
// bfloat16 or FP8 rounding of D that follows.  Every thread of the block
// calls it (it holds barriers); acc[s] is D[s][b] of the lane's atom.
#define NET_STAGE 64
struct NetStage {
  float r[NET_IROWS][NET_STAGE];
  int sp[NET_IROWS][NET_STAGE];
  int maxcnt;
};
__device__ __forceinline__ void net_descriptor_lanes(const PotDev& P, const SysDev& S,
                                                     const float4* __restrict__ X,
                                                     const uint32_t* __restrict__ row,
                                                     int width, int cnt, int i, int r, int a,
                                                     int sub, NetStage& st,
                                                     float acc[LSD_NET_MAX_SPECIES]) {
#pragma unroll
  for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s) acc[s] = 0.0f;
  if (threadIdx.x == 0) st.maxcnt = 0;
  __syncthreads();
  if (sub == 0 && cnt > 0) atomicMax(&st.maxcnt, cnt);
  __syncthreads();
  const int maxcnt = st.maxcnt;
  const float Lf = (float)S.box[r];
  const float4 xi = X[i];
  const float turn_rc = P.pi_rc * 0.15915494309189535f;  // 1 / (2 r_c): turns per unit r
  const float kb = (float)(sub + 1) * turn_rc;
  for (int c0 = 0; c0 < maxcnt; c0 += NET_STAGE) {
    // stage: four entries per lane
    uint32_t ent[NET_STAGE / 16];
#pragma unroll
    for (int u = 0; u < NET_STAGE / 16; ++u) {
      const int m = c0 + sub + 16 * u;
      ent[u] = row[m < width ? m : 0];
    }
#pragma unroll
    for (int u = 0; u < NET_STAGE / 16; ++u) {
      const int m = c0 + sub + 16 * u;
      const bool ok = m < cnt;
      const int j = ok ? (int)(ent[u] >> 5) : 0;
      const float4 xj = X[j];
      const int spj = S.species ? S.species[j] : 0;
      float sj[3], si[3];
      image_shifts((int)(ent[u] & 31u), Lf, sj, si);
      const float dx = sep(xj.x, sj[0], xi.x, si[0]);
      const float dy = sep(xj.y, sj[1], xi.y, si[1]);
      const float dz = sep(xj.z, sj[2], xi.z, si[2]);
      const float r2 = dx * dx + dy * dy + dz * dz;
      st.r[a][sub + 16 * u] = (ok && r2 < P.rc2) ? sqrtf(r2) : -1.0f;
      st.sp[a][sub + 16 * u] = spj;
    }
    __syncthreads();
    const int n = min(NET_STAGE, cnt - c0);
    if (sub < P.nb) {
#pragma unroll 4
      for (int m = 0; m < n; ++m) {
        const float rr = st.r[a][m];
        if (rr > 0.0f) {
          const int spj = st.sp[a][m];
          const float fc = 0.5f * (__builtin_amdgcn_cosf(rr * turn_rc) + 1.0f);
          const float e = fc * __builtin_amdgcn_sinf(rr * kb) * __builtin_amdgcn_rcpf(rr);
#pragma unroll
          for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s) acc[s] += s == spj ? e : 0.0f;
        }
      }
    }
    __syncthreads();  // the next chunk rewrites the stage
  }
}

// bfloat16 on the matrix cores: the first wave multiplies the block's 16
// descriptors by W1 and the hidden activations by W2 with
// v_mfma_f32_16x16x16_bf16.  16x16x16 operands: lane l holds
// A[l % 16][4 (l / 16) + 0..3] and B[4 (l / 16) + 0..3][l % 16]; the result
// D[4 (l / 16) + 0..3][l % 16].  Each lane loads its own B fragments of W1
// and W2 from the parameters before the descriptor loop.
template <int NL>
__device__ __forceinline__ void net_nodes_bf16_block(const SysDev& S, const ListDev& Lst,
                                                     const WinDev& W, const PotDev& P, int k,
                                                     int blk) {
  __shared__ float s_b1[LSD_NET_MAX_SPECIES][LSD_NET_HIDDEN];
  __shared__ unsigned short s_Db[NET_IROWS][LSD_NET_MAX_DESC];
  __shared__ unsigned short s_hb[NET_IROWS][LSD_NET_HIDDEN];
  __shared__ int s_sp[NET_IROWS], s_ok[NET_IROWS];
  __shared__ NetStage stage;
  static_assert(NL == LSD_NET_MAX_BASIS, "one lane per radial function");
  const int t = threadIdx.x, a = t / NL, sub = t % NL;
  const int i0 = blk * NET_IROWS + a;
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
  const bool mw = t < 64;  // the wave on the matrix cores
  constexpr int KS1 = LSD_NET_MAX_DESC / 16, KS2 = LSD_NET_HIDDEN / 16;
  const int ks1 = (Din + 15) / 16;
  bf16x4 bw1[2][KS1], bw2[KS2];
  if (mw) {
    const float* w2 = P.w + net_off_w2(P.ns, B);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int d = 16 * ks + 4 * kq + q, h = 16 * nt + li;
          bw1[nt][ks][q] = (short)to_bf16(d < Din ? P.w[h * Din + d] : 0.0f);
        }
#pragma unroll
    for (int ks = 0; ks < KS2; ++ks)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        bw2[ks][q] = (short)to_bf16(li < B ? w2[li * LSD_NET_HIDDEN + 16 * ks + 4 * kq + q] : 0.0f);
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
  if (sub == 0) {
    s_sp[a] = S.species ? S.species[i] : 0;
    s_ok[a] = ok ? 1 : 0;
  }
  if (sub < B) {
#pragma unroll
    for (int s = 0; s < LSD_NET_MAX_SPECIES; ++s)
      if (s < P.ns) s_Db[a][s * B + sub] = to_bf16(acc[s]);
  }
  for (int d = Din + sub; d < LSD_NET_MAX_DESC; d += NL) s_Db[a][d] = 0;
  __syncthreads();
  if (mw) {
    f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KS1; ++ks) {
      if (ks >= ks1) break;  // zero descriptor slots
      bf16x4 av;
#pragma unroll
      for (int q = 0; q < 4; ++q) av[q] = (short)s_Db[li][16 * ks + 4 * kq + q];
      acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bw1[0][ks], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bw1[1][ks], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ar = 4 * kq + q;
      const int spa = s_sp[ar];
      s_hb[ar][li] = to_bf16(silu(acc0[q] + s_b1[spa][li]));
      s_hb[ar][16 + li] = to_bf16(silu(acc1[q] + s_b1[spa][16 + li]));
    }
  }
  __syncthreads();
  if (mw) {
    f32x4 acc2 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < KS2; ++ks) {
      bf16x4 av;
#pragma unroll
      for (int q = 0; q < 4; ++q) av[q] = (short)s_hb[li][16 * ks + 4 * kq + q];
      acc2 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bw2[ks], acc2, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ar = 4 * kq + q;
      const int ia = blk * NET_IROWS + ar;
      if (ia < S.n && s_ok[ar]) P.v[(size_t)ia * LSD_NET_MAX_BASIS + li] = li < B ? acc2[q] : 0.0f;
    }
  }
}

}  // namespace
