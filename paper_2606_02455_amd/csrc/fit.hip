// fit.hip -- force matching of the pair draft on the GPU.
//
// The pair-draft forces are linear in the weights, F_i = A_i w, so fitting
// them to target forces is linear least squares.  Only the columns of the
// types {s_i, s'} (s' = 0..S-1) are non-zero in atom i's design rows, so each
// tile accumulates per-species normal equations over its atoms in the local
// column space (s', b) and a second kernel maps them onto the global
// (type, basis) columns, summing tiles in a fixed order.
#include "fit.h"

#define FIT_EPT 16  // partial-sum entries per thread

// One block per (tile, entry chunk): for every valid frame of the window the
// design rows of the tile's atoms are built in LDS (one thread per atom, list
// entries in order), then each thread adds its entries
//   G_s[l1][l2] += sum_{atoms a of species s} sum_d A_a[d][l1] A_a[d][l2]
//   h_s[l]      += sum_{atoms a of species s} sum_d A_a[d][l] F_a[d]
// in binary64.
__global__ __launch_bounds__(256) void k_fit_tile(SysDev S, ListDev Lst, WinDev W, TileDev Tl,
                                                  FitDev F, int use_target, int diff,
                                                  double* __restrict__ partial) {
  extern __shared__ float s_a[];  // [64][3][LP]
  const int tile = blockIdx.x, t = threadIdx.x;
  const int start = Tl.start[tile], count = Tl.count[tile], r = Tl.rep[tile];
  const int* inv = W.invalid + (size_t)r * S.kmax;
  const int LP = F.LP, nb = F.nb;
  const int GE = F.ns * LP * LP, E = GE + F.ns * LP;
  const int e0 = blockIdx.y * 256 * FIT_EPT;
  const float Lf = (float)S.box[r];
  const size_t N = (size_t)S.n;
  double acc[FIT_EPT];
#pragma unroll
  for (int q = 0; q < FIT_EPT; ++q) acc[q] = 0.0;
  for (int f = 0; f < W.K; ++f) {
    // frames from K_eff on are not valid; a difference needs frame f + 1
    if (inv[f] || (diff && (f + 1 >= W.K || inv[f + 1]))) break;  // uniform over the block
    for (int k = t; k < 64 * 3 * LP; k += 256) s_a[k] = 0.0f;
    __syncthreads();
    // rows of frame f, or of frame f + 1 minus those of frame f
    for (int side = 0; side < (diff ? 2 : 1) && t < count; ++side) {
      const int fr = diff ? f + 1 - side : f;
      const float sgn = side ? -1.0f : 1.0f;
      const int i = start + t;
      const float4* X = W.qmid + (size_t)fr * N;
      const float4 xi = X[i];
      const int cnt = Lst.cnt_t[i];
      const uint32_t* row = Lst.nbr_t + (size_t)i * Lst.mt;
      float* a = s_a + t * 3 * LP;
      for (int m = 0; m < cnt; ++m) {
        const uint32_t ent = row[m];
        const int j = (int)(ent >> 5), code = (int)(ent & 31u);
        const float4 xj = X[j];
        float sj[3], si[3];
        image_shifts(code, Lf, sj, si);
        const float dx = sep(xj.x, sj[0], xi.x, si[0]);
        const float dy = sep(xj.y, sj[1], xi.y, si[1]);
        const float dz = sep(xj.z, sj[2], xi.z, si[2]);
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= F.rc2) continue;
        const float rr = sqrtf(r2);
        const float inv_r = 1.0f / rr;
        float sn, cs;
        sincosf(F.pi_rc * rr, &sn, &cs);
        const float g0 = 0.5f * (cs + 1.0f) * inv_r * inv_r;
        const int col0 = (S.species ? S.species[j] : 0) * nb;
        float prev = 0.0f, cur = sn;
        const float two_c = 2.0f * cs;
        for (int b = 0; b < nb; ++b) {
          if (b > 0) {
            const float nx = two_c * cur - prev;
            prev = cur;
            cur = nx;
          }
          const float v = sgn * (g0 * cur);
          a[col0 + b] -= v * dx;
          a[LP + col0 + b] -= v * dy;
          a[2 * LP + col0 + b] -= v * dz;
        }
      }
    }
    __syncthreads();
    const float* Fsrc = use_target ? W.ft : W.fd;
    const float* Ff = Fsrc + (size_t)f * 3 * N;
    const float* Fn = Fsrc + (size_t)(diff ? f + 1 : f) * 3 * N;
#pragma unroll
    for (int q = 0; q < FIT_EPT; ++q) {
      const int e = e0 + t + 256 * q;
      if (e >= E) break;
      double sum = 0.0;
      if (e < GE) {
        const int s = e / (LP * LP), l1 = (e / LP) % LP, l2 = e % LP;
        for (int aa = 0; aa < count; ++aa) {
          if ((S.species ? S.species[start + aa] : 0) != s) continue;
          const float* a = s_a + aa * 3 * LP;
#pragma unroll
          for (int d = 0; d < 3; ++d) sum += (double)a[d * LP + l1] * (double)a[d * LP + l2];
        }
      } else {
        const int s = (e - GE) / LP, l = (e - GE) % LP;
        for (int aa = 0; aa < count; ++aa) {
          const int i = start + aa;
          if ((S.species ? S.species[i] : 0) != s) continue;
          const float* a = s_a + aa * 3 * LP;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const double y = diff ? (double)Fn[d * N + i] - (double)Ff[d * N + i] : (double)Ff[d * N + i];
            sum += (double)a[d * LP + l] * y;
          }
        }
      }
      acc[q] += sum;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < FIT_EPT; ++q) {
    const int e = e0 + t + 256 * q;
    if (e < E) partial[(size_t)tile * E + e] = acc[q];
  }
}

// species s' with pair_type(s, s') == type, or -1
__device__ __forceinline__ int other_species(int type, int s, int ns) {
  for (int o = 0; o < ns; ++o)
    if (pair_type(s, o, ns) == type) return o;
  return -1;
}

// gram[(P+1)][(P+1)] (row-major, column P = right-hand side) += the tile
// partials mapped to the global (type, basis) columns, tiles in order.
__global__ __launch_bounds__(256) void k_fit_reduce(const double* __restrict__ partial, int n_tiles,
                                                    FitDev F, int P, double* __restrict__ gram) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int Pe = P + 1;
  if (g >= Pe * Pe) return;
  const int c1 = g / Pe, c2 = g % Pe;
  if (c1 == P && c2 == P) return;
  const int LP = F.LP, nb = F.nb;
  const int GE = F.ns * LP * LP, E = GE + F.ns * LP;
  double total = 0.0;
  for (int s = 0; s < F.ns; ++s) {
    int idx;
    if (c1 < P && c2 < P) {
      const int o1 = other_species(c1 / nb, s, F.ns), o2 = other_species(c2 / nb, s, F.ns);
      if (o1 < 0 || o2 < 0) continue;
      idx = s * LP * LP + (o1 * nb + c1 % nb) * LP + (o2 * nb + c2 % nb);
    } else {
      const int c = c1 < P ? c1 : c2;
      const int o = other_species(c / nb, s, F.ns);
      if (o < 0) continue;
      idx = GE + s * LP + o * nb + c % nb;
    }
    for (int tl = 0; tl < n_tiles; ++tl) total += partial[(size_t)tl * E + idx];
  }
  gram[g] += total;
}

size_t fit_partial_entries(const FitDev& F) {
  return (size_t)F.ns * F.LP * F.LP + (size_t)F.ns * F.LP;
}

hipError_t launch_fit(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                      const FitDev& F, int use_target, int diff, double* partial, double* gram,
                      hipStream_t st) {
  const int E = (int)fit_partial_entries(F);
  const size_t lds = (size_t)64 * 3 * F.LP * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)k_fit_tile,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  dim3 grid(S.n_tiles, (E + 256 * FIT_EPT - 1) / (256 * FIT_EPT));
  hipLaunchKernelGGL(k_fit_tile, grid, dim3(256), lds, st, S, L, W, T, F, use_target, diff,
                     partial);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int P = (F.ns * (F.ns + 1) / 2) * F.nb;
  const int Pe2 = (P + 1) * (P + 1);
  hipLaunchKernelGGL(k_fit_reduce, dim3((Pe2 + 255) / 256), dim3(256), 0, st, partial, S.n_tiles,
                     F, P, gram);
  return hipGetLastError();
}
