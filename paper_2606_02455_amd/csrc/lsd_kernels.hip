// lsd_kernels.hip -- HIP kernels of the LSD window for gfx950.
//
// One window of one or many replicas:
//   k_window_start  first midpoint (map f of Thm. 1 / the A half step of
//                   draft_step, Alg. 2) and cell assignment
//   k_cell_scan / k_cell_fill / k_cell_sort
//                   counting sort of atoms into cells (deterministic order)
//   k_nl_build      Verlet lists (cutoff + skin) for the target and the draft,
//                   ELL layout [m][N], exact binary64 predicate
//   k_draft         one draft_step of Alg. 2 for every atom (Eq. bob draw)
//   k_verify        target forces for ALL K frames in one launch with the
//                   neighbour tile staged in LDS once and reused by every
//                   frame, fused with the binary64 transport-map sums of
//                   Eq. reflectionVerify
//   k_decide        accept / first rejection per replica (Alg. 1)
//   k_commit        reflection of the rejected momentum and map g (Thm. 1)
#include "lsd_device.h"
#include "lsd_launch.h"

// ---------------------------------------------------------------------------
__global__ void k_fill_int(int* p, int v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Midpoint of the first draft step from the committed state, copy of the
// committed momenta into the window, and cell binning of the midpoints.
__global__ __launch_bounds__(256) void k_window_start(SysDev S, ListDev Lst, WinDev W,
                                                      const float* __restrict__ q,
                                                      const float* __restrict__ p) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S.R * S.kmax) W.invalid[i] = 0;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  const int sp = S.species ? S.species[i] : 0;
  const double L = S.box[r];
  const double hm = S.hdt_m[sp];
  int dimg[3] = {0, 0, 0};
  float x[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float pd = p[d * S.n + i];
    W.p[d * S.n + i] = pd;
    x[d] = a_half(q[d * S.n + i], pd, hm, L, &dimg[d]);
  }
  W.qmid[i] = make_float4(x[0], x[1], x[2], pack_img(dimg[0], dimg[1], dimg[2]));
  // cell of the midpoint
  const int nc = Lst.rep_nc[r];
  int c[3];
  const float inv_w = (float)((double)nc / L);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int v = (int)(x[d] * inv_w);
    c[d] = v < 0 ? 0 : (v >= nc ? nc - 1 : v);
  }
  const int cell = Lst.rep_cell_off[r] + c[0] + nc * (c[1] + nc * c[2]);
  Lst.atom_cell[i] = cell;
  atomicAdd(&Lst.cell_count[cell], 1);
}

// Cell binning only (lists rebuilt from caller-written frame 0).
__global__ __launch_bounds__(256) void k_bin_frame0(SysDev S, ListDev Lst, WinDev W) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  const double L = S.box[r];
  float4 xq = W.qmid[i];
  float x[3] = {xq.x, xq.y, xq.z};
  const int nc = Lst.rep_nc[r];
  const float inv_w = (float)((double)nc / L);
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int v = (int)(x[d] * inv_w);
    c[d] = v < 0 ? 0 : (v >= nc ? nc - 1 : v);
  }
  const int cell = Lst.rep_cell_off[r] + c[0] + nc * (c[1] + nc * c[2]);
  Lst.atom_cell[i] = cell;
  atomicAdd(&Lst.cell_count[cell], 1);
}

// Exclusive scan of the cell counts (one block), then clear the counters
// for the next binning.
__global__ __launch_bounds__(1024) void k_cell_scan(ListDev Lst) {
  __shared__ int s[1024];
  const int C = Lst.n_cells;
  const int t = threadIdx.x;
  const int chunk = (C + 1023) / 1024;
  const int lo = min(C, t * chunk), hi = min(C, lo + chunk);
  int sum = 0;
  for (int c = lo; c < hi; ++c) sum += Lst.cell_count[c];
  s[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int v = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  int run = s[t] - sum;  // exclusive prefix of this chunk
  for (int c = lo; c < hi; ++c) {
    Lst.cell_start[c] = run;
    run += Lst.cell_count[c];
    Lst.cell_count[c] = 0;
    Lst.cell_cursor[c] = 0;
  }
  if (t == 1023) Lst.cell_start[C] = s[1023];
}

__global__ __launch_bounds__(256) void k_cell_fill(int n, ListDev Lst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = Lst.atom_cell[i];
  int pos = Lst.cell_start[c] + atomicAdd(&Lst.cell_cursor[c], 1);
  Lst.cell_atoms[pos] = i;
}

// ascending atom order inside each cell: the list order then depends only on
// the positions, not on the order the atomics were served in
__global__ __launch_bounds__(256) void k_cell_sort(ListDev Lst) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Lst.n_cells) return;
  int lo = Lst.cell_start[c], hi = Lst.cell_start[c + 1];
  for (int a = lo + 1; a < hi; ++a) {
    int v = Lst.cell_atoms[a];
    int b = a - 1;
    while (b >= lo && Lst.cell_atoms[b] > v) {
      Lst.cell_atoms[b + 1] = Lst.cell_atoms[b];
      --b;
    }
    Lst.cell_atoms[b + 1] = v;
  }
}

// Verlet lists at the frame-0 midpoints: every (j, image) with
// |x_j + n L - x_i| < r_list, scanned over the 27 neighbouring cells.
__global__ __launch_bounds__(256) void k_nl_build(SysDev S, ListDev Lst, WinDev W) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  const double L = S.box[r];
  const int nc = Lst.rep_nc[r];
  const int coff = Lst.rep_cell_off[r];
  const float4 xi = W.qmid[i];
  int c = Lst.atom_cell[i] - coff;
  const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
  int nt = 0, nd = 0;
  for (int oz = -1; oz <= 1; ++oz) {
    int tz = cz + oz, nz = 0;
    if (tz < 0) { tz += nc; nz = -1; } else if (tz >= nc) { tz -= nc; nz = 1; }
    for (int oy = -1; oy <= 1; ++oy) {
      int ty = cy + oy, ny = 0;
      if (ty < 0) { ty += nc; ny = -1; } else if (ty >= nc) { ty -= nc; ny = 1; }
      for (int ox = -1; ox <= 1; ++ox) {
        int tx = cx + ox, nx = 0;
        if (tx < 0) { tx += nc; nx = -1; } else if (tx >= nc) { tx -= nc; nx = 1; }
        const int code = (nx + 1) + 3 * (ny + 1) + 9 * (nz + 1);
        const int cell = coff + tx + nc * (ty + nc * tz);
        const int lo = Lst.cell_start[cell], hi = Lst.cell_start[cell + 1];
        for (int a = lo; a < hi; ++a) {
          const int j = Lst.cell_atoms[a];
          if (j == i && code == 13) continue;
          const float4 xj = W.qmid[j];
          double dx = ((double)xj.x - (double)xi.x) + (double)nx * L;
          double dy = ((double)xj.y - (double)xi.y) + (double)ny * L;
          double dz = ((double)xj.z - (double)xi.z) + (double)nz * L;
          double d2 = dx * dx + dy * dy + dz * dz;
          const uint32_t e = ((uint32_t)j << 5) | (uint32_t)code;
          if (d2 < Lst.rl2_t) {
            if (nt < Lst.mt) Lst.nbr_t[(size_t)nt * S.n + i] = e;
            ++nt;
          }
          if (d2 < Lst.rl2_d) {
            if (nd < Lst.md) Lst.nbr_d[(size_t)nd * S.n + i] = e;
            ++nd;
          }
        }
      }
    }
  }
  if (nt > Lst.mt) { atomicOr(Lst.status, LSD_STATUS_NBR_TARGET); nt = Lst.mt; }
  if (nd > Lst.md) { atomicOr(Lst.status, LSD_STATUS_NBR_DRAFT); nd = Lst.md; }
  Lst.cnt_t[i] = nt;
  Lst.cnt_d[i] = nd;
}

// Force of potential P on atom i at frame positions X using list (nbr, cnt).
__device__ __forceinline__ void pot_force(const PotDev& P, const SysDev& S, const float4* __restrict__ X,
                                          const uint32_t* __restrict__ nbr, int cnt, int i, int r,
                                          float& fx, float& fy, float& fz, float& e) {
  fx = fy = fz = e = 0.0f;
  const double L = S.box[r];
  const float Lf = (float)L;
  const float4 xi = X[i];
  if (P.kind == LSD_POT_LJ) {
    for (int m = 0; m < cnt; ++m) {
      const uint32_t ent = nbr[(size_t)m * S.n + i];
      const int j = (int)(ent >> 5), code = (int)(ent & 31u);
      const float4 xj = X[j];
      lj_pair(P, xi, xj, (float)code_nx(code) * Lf, (float)code_ny(code) * Lf,
              (float)code_nz(code) * Lf, code, L, fx, fy, fz, e);
    }
  } else if (P.kind == LSD_POT_HARMONIC) {
    float d[3] = {xi.x - P.anchor[i], xi.y - P.anchor[S.n + i], xi.z - P.anchor[2 * S.n + i]};
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] -= Lf * rintf(d[a] / Lf);
    fx = -P.kspring * d[0];
    fy = -P.kspring * d[1];
    fz = -P.kspring * d[2];
    e = 0.5f * P.kspring * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  }
  if (P.offset) {
    fx += P.offset[i];
    fy += P.offset[S.n + i];
    fz += P.offset[2 * S.n + i];
  }
}

// One draft_step (Alg. 2) for frame k: draft forces at the midpoint, the
// (BOB) Gaussian draw of Eq. bob, then the two position half steps that end
// this step and start the next one; flags the next frame invalid when an
// atom left the skin of the lists.
__global__ __launch_bounds__(256) void k_draft(SysDev S, ListDev Lst, WinDev W, PotDev P, int k,
                                               int use_target_list) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  const int sp = S.species ? S.species[i] : 0;
  const size_t N = (size_t)S.n;
  const float4* X = W.qmid + (size_t)k * N;
  float F[3], e;
  if (use_target_list)
    pot_force(P, S, X, Lst.nbr_t, Lst.cnt_t[i], i, r, F[0], F[1], F[2], e);
  else
    pot_force(P, S, X, Lst.nbr_d, Lst.cnt_d[i], i, r, F[0], F[1], F[2], e);

  double xi[3];
  if (S.replay_xi) {
    const double* rx = S.replay_xi + ((size_t)k * N + i) * 3;
    xi[0] = rx[0]; xi[1] = rx[1]; xi[2] = rx[2];
  } else {
    stream_normals3(S.seed, (uint32_t)r, (uint64_t)(S.step[r] + k + 1),
                    (uint32_t)(i - S.rep_off[r]), xi);
  }
  const float* pk = W.p + (size_t)k * 3 * N;
  float* pk1 = W.p + (size_t)(k + 1) * 3 * N;
  float* fk = W.fd + (size_t)k * 3 * N;
  const double sg = S.sig[sp];
  float pn[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double mu = bob_mean(S.a, S.c1fu, pk[d * N + i], F[d]);
    pn[d] = (float)fma(sg, xi[d], mu);
    fk[d * N + i] = F[d];
    pk1[d * N + i] = pn[d];
  }
  if (k + 1 < W.K) {
    const double L = S.box[r];
    const double hm = S.hdt_m[sp];
    const float4 x = X[i];
    int dimg[3];
    unpack_img(x.w, dimg);
    float xs[3] = {x.x, x.y, x.z}, xn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float qend = a_half(xs[d], pn[d], hm, L, &dimg[d]);   // q~_k
      xn[d] = a_half(qend, pn[d], hm, L, &dimg[d]);         // next midpoint
    }
    W.qmid[(size_t)(k + 1) * N + i] = make_float4(xn[0], xn[1], xn[2], pack_img(dimg[0], dimg[1], dimg[2]));
    // displacement from the list positions (frame 0), minimum image
    const float4 x0 = W.qmid[i];
    const float Lf = (float)L;
    float dd[3] = {xn[0] - x0.x, xn[1] - x0.y, xn[2] - x0.z};
    float d2 = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      dd[d] -= Lf * rintf(dd[d] / Lf);
      d2 += dd[d] * dd[d];
    }
    int* inv = W.invalid + (size_t)r * S.kmax;
    if (d2 > S.half_skin2 || inv[k] != 0) atomicOr(&inv[k + 1], 1);
  }
}

// Validity of caller-written frames against the frame-0 lists.
__global__ __launch_bounds__(256) void k_frame_validity(SysDev S, WinDev W) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  const float Lf = (float)S.box[r];
  const float4 x0 = W.qmid[i];
  int* inv = W.invalid + (size_t)r * S.kmax;
  for (int k = 1; k < W.K; ++k) {
    const float4 x = W.qmid[(size_t)k * S.n + i];
    float dd[3] = {x.x - x0.x, x.y - x0.y, x.z - x0.z};
    float d2 = 0.0f;
    for (int d = 0; d < 3; ++d) {
      dd[d] -= Lf * rintf(dd[d] / Lf);
      d2 += dd[d] * dd[d];
    }
    if (d2 > S.half_skin2) {
      for (int kk = k; kk < W.K; ++kk) atomicOr(&inv[kk], 1);
      break;
    }
  }
}

// verify_step (Alg. 2) for every valid frame of the window.  Block = one
// tile of up to 64 atoms of one replica x `fpb` frames; wave w of the block
// handles frames f0 + w, f0 + w + 4, ...  The tile's neighbour entries are
// read from HBM once into LDS and reused by all frames of the block.
// Epilogue per atom and frame (binary64):
//   z = (p~_k - <p~_k>) / sigma,  delta = c1 (F~_k - F_k) / sigma
// summed over the tile with a wavefront butterfly: S1 = delta.z,
// S2 = delta.delta, plus the potential energy.
__global__ __launch_bounds__(256) void k_verify(SysDev S, ListDev Lst, WinDev W, TileDev Tl,
                                                PotDev P, int fpb) {
  extern __shared__ uint32_t s_nbr[];  // [mt][64]
  __shared__ float s_shift[27][3];
  const int tile = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int start = Tl.start[tile], count = Tl.count[tile], r = Tl.rep[tile];
  const double L = S.box[r];
  const float Lf = (float)L;
  const size_t N = (size_t)S.n;
  const int i = start + lane;
  const bool active = lane < count;
  if (threadIdx.x < 27) {
    int c = threadIdx.x;
    s_shift[c][0] = (float)code_nx(c) * Lf;
    s_shift[c][1] = (float)code_ny(c) * Lf;
    s_shift[c][2] = (float)code_nz(c) * Lf;
  }
  const int cnt = active ? Lst.cnt_t[i] : 0;
  const int maxcnt = wave_max(cnt);
  for (int m = wave; m < maxcnt; m += 4)
    s_nbr[m * 64 + lane] = active ? Lst.nbr_t[(size_t)m * N + i] : 0u;
  __syncthreads();

  const int f0 = blockIdx.y * fpb;
  const int f1 = min(f0 + fpb, W.K);
  const int* inv = W.invalid + (size_t)r * S.kmax;
  const int sp = (active && S.species) ? S.species[i] : 0;
  for (int f = f0 + wave; f < f1; f += 4) {
    if (inv[f]) continue;  // frame beyond the valid prefix: not verified
    const float4* X = W.qmid + (size_t)f * N;
    float fx = 0.0f, fy = 0.0f, fz = 0.0f, e = 0.0f;
    if (active) {
      const float4 xi = X[i];
      if (P.kind == LSD_POT_LJ) {
        for (int m = 0; m < cnt; ++m) {
          const uint32_t ent = s_nbr[m * 64 + lane];
          const int j = (int)(ent >> 5), code = (int)(ent & 31u);
          const float4 xj = X[j];
          lj_pair(P, xi, xj, s_shift[code][0], s_shift[code][1], s_shift[code][2], code, L, fx,
                  fy, fz, e);
        }
        if (P.offset) {
          fx += P.offset[i];
          fy += P.offset[N + i];
          fz += P.offset[2 * N + i];
        }
      } else {
        pot_force(P, S, X, Lst.nbr_t, cnt, i, r, fx, fy, fz, e);
      }
    }
    double s1 = 0.0, s2 = 0.0;
    if (active) {
      const float Ft[3] = {fx, fy, fz};
      const float* pk = W.p + (size_t)f * 3 * N;
      const float* pk1 = W.p + (size_t)(f + 1) * 3 * N;
      const float* fdk = W.fd + (size_t)f * 3 * N;
      float* ftk = W.ft + (size_t)f * 3 * N;
      const double isg = 1.0 / S.sig[sp];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float Fd = fdk[d * N + i];
        ftk[d * N + i] = Ft[d];
        const double mud = bob_mean(S.a, S.c1fu, pk[d * N + i], Fd);
        const double z = ((double)pk1[d * N + i] - mud) * isg;
        const double dl = S.c1fu * ((double)Fd - (double)Ft[d]) * isg;
        s1 = fma(dl, z, s1);
        s2 = fma(dl, dl, s2);
      }
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    const double es = wave_sum((double)e);
    if (lane == 0) {
      double* out = W.partial + ((size_t)f * S.n_tiles + tile) * 4;
      out[0] = s1;
      out[1] = s2;
      out[2] = es;
    }
  }
}

// Per replica: frame sums over its tiles (fixed order), log ratio, decision
// with u_{s+k}, first rejection (Alg. 1), outputs and the commit record.
__global__ __launch_bounds__(64) void k_decide(SysDev S, WinDev W, TileDev Tl, OutDev O, int plain) {
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  const int K = W.K;
  const int* inv = W.invalid + (size_t)r * S.kmax;
  int keff = K;
  for (int f = 1; f < K; ++f)
    if (inv[f]) { keff = f; break; }
  const int t0 = Tl.rep_tile_off[r], t1 = Tl.rep_tile_off[r + 1];
  int j = keff, reflected = 0;
  double coef = 0.0;
  const uint64_t s0 = (uint64_t)S.step[r];
  bool rejected = false;
  for (int f = 0; f < K; ++f) {
    const size_t o = (size_t)r * S.kmax + f;
    if (plain || f >= keff) {
      if (lane == 0) {
        O.accepted[o] = 2;
        O.log_ratio[o] = 0.0;
        O.energy[o] = 0.0;
      }
      continue;
    }
    double s1 = 0.0, s2 = 0.0, es = 0.0;
    for (int t = t0 + lane; t < t1; t += 64) {
      const double* pp = W.partial + ((size_t)f * S.n_tiles + t) * 4;
      s1 += pp[0];
      s2 += pp[1];
      es += pp[2];
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    es = wave_sum(es);
    const double logr = -s1 - 0.5 * s2;
    const double u = S.replay_u ? S.replay_u[o] : stream_uniform(S.seed, (uint32_t)r, s0 + f + 1);
    const bool acc = log(u) <= logr;
    if (lane == 0) {
      O.accepted[o] = acc ? 1 : 0;
      O.log_ratio[o] = logr;
      O.energy[o] = es;
    }
    if (!acc && !rejected) {
      rejected = true;
      j = f + 1;
      reflected = 1;
      coef = 2.0 * s1 / s2;
    }
  }
  if (lane == 0) {
    O.n_committed[r] = j;
    W.commit_frame[r] = j - 1;
    W.reflected[r] = reflected;
    W.coef[r] = coef;
    S.step[r] = (int64_t)(s0 + (uint64_t)j);
  }
}

// Commit: the last kept frame's state; a rejected frame takes the reflected
// momentum <p> + Sigma^{1/2} (z - (2 delta.z / delta.delta) delta) and map g.
__global__ __launch_bounds__(256) void k_commit(SysDev S, WinDev W, float* __restrict__ q,
                                                float* __restrict__ p, int* __restrict__ img) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  const int sp = S.species ? S.species[i] : 0;
  const size_t N = (size_t)S.n;
  const int f = W.commit_frame[r];
  const float4 x = W.qmid[(size_t)f * N + i];
  int dimg[3];
  unpack_img(x.w, dimg);
  const float xs[3] = {x.x, x.y, x.z};
  const float* pk = W.p + (size_t)f * 3 * N;
  const float* pk1 = W.p + (size_t)(f + 1) * 3 * N;
  const double L = S.box[r];
  const double hm = S.hdt_m[sp];
  const bool refl = W.reflected[r] != 0;
  const double coef = W.coef[r];
  const double sg = S.sig[sp], isg = 1.0 / sg;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float pn = pk1[d * N + i];
    if (refl) {
      const float Fd = W.fd[(size_t)f * 3 * N + d * N + i];
      const float Ft = W.ft[(size_t)f * 3 * N + d * N + i];
      const double mut = bob_mean(S.a, S.c1fu, pk[d * N + i], Ft);
      const double mud = bob_mean(S.a, S.c1fu, pk[d * N + i], Fd);
      const double z = ((double)pn - mud) * isg;
      const double dl = S.c1fu * ((double)Fd - (double)Ft) * isg;
      pn = (float)fma(sg, z - coef * dl, mut);
    }
    const float qn = a_half(xs[d], pn, hm, L, &dimg[d]);
    q[d * N + i] = qn;
    p[d * N + i] = pn;
    img[d * N + i] += dimg[d];
  }
}

// ---------------------------------------------------------------------------
__global__ void k_rng_normals(uint64_t seed, int replica, int64_t step, int n, double* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xi[3];
  stream_normals3(seed, (uint32_t)replica, (uint64_t)step, (uint32_t)i, xi);
  out[3 * i] = xi[0];
  out[3 * i + 1] = xi[1];
  out[3 * i + 2] = xi[2];
}

__global__ void k_rng_uniforms(uint64_t seed, int replica, int64_t step0, int count, double* out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  out[k] = stream_uniform(seed, (uint32_t)replica, (uint64_t)(step0 + k + 1));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int blocks_for(int n, int b) { return (n + b - 1) / b; }

hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_window_start(const SysDev& S, const ListDev& L, const WinDev& W, const float* q,
                               const float* p, hipStream_t st) {
  int n = S.n > S.R * S.kmax ? S.n : S.R * S.kmax;
  hipLaunchKernelGGL(k_window_start, dim3(blocks_for(n, 256)), dim3(256), 0, st, S, L, W, q, p);
  return hipGetLastError();
}

hipError_t launch_build_lists(const SysDev& S, const ListDev& L, const WinDev& W, bool bin_frame0,
                              hipStream_t st) {
  if (bin_frame0)
    hipLaunchKernelGGL(k_bin_frame0, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S, L, W);
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, st, L);
  hipLaunchKernelGGL(k_cell_fill, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S.n, L);
  hipLaunchKernelGGL(k_cell_sort, dim3(blocks_for(L.n_cells, 256)), dim3(256), 0, st, L);
  hipLaunchKernelGGL(k_nl_build, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S, L, W);
  return hipGetLastError();
}

hipError_t launch_draft(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P, int k,
                        int use_target_list, hipStream_t st) {
  hipLaunchKernelGGL(k_draft, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S, L, W, P, k,
                     use_target_list);
  return hipGetLastError();
}

hipError_t launch_frame_validity(const SysDev& S, const WinDev& W, hipStream_t st) {
  hipLaunchKernelGGL(k_frame_validity, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S, W);
  return hipGetLastError();
}

hipError_t prepare_verify(int mt) {
  size_t lds = (size_t)mt * 64 * sizeof(uint32_t);
  return hipFuncSetAttribute((const void*)k_verify, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

hipError_t launch_verify(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                         const PotDev& P, int fpb, hipStream_t st) {
  size_t lds = (size_t)L.mt * 64 * sizeof(uint32_t);
  dim3 grid(S.n_tiles, (W.K + fpb - 1) / fpb);
  hipLaunchKernelGGL(k_verify, grid, dim3(256), lds, st, S, L, W, T, P, fpb);
  return hipGetLastError();
}

hipError_t launch_decide(const SysDev& S, const WinDev& W, const TileDev& T, const OutDev& O,
                         int plain, hipStream_t st) {
  hipLaunchKernelGGL(k_decide, dim3(S.R), dim3(64), 0, st, S, W, T, O, plain);
  return hipGetLastError();
}

hipError_t launch_commit(const SysDev& S, const WinDev& W, float* q, float* p, int* img,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_commit, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S, W, q, p, img);
  return hipGetLastError();
}

hipError_t launch_rng_normals(uint64_t seed, int replica, int64_t step, int n, double* out,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rng_normals, dim3(blocks_for(n, 256)), dim3(256), 0, st, seed, replica, step,
                     n, out);
  return hipGetLastError();
}

hipError_t launch_rng_uniforms(uint64_t seed, int replica, int64_t step0, int count, double* out,
                               hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rng_uniforms, dim3(blocks_for(count, 256)), dim3(256), 0, st, seed, replica,
                     step0, count, out);
  return hipGetLastError();
}
