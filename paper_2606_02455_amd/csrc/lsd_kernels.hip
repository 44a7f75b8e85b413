// lsd_kernels.hip -- HIP kernels of the LSD window for gfx950.
//
// One window of one or many replicas:
//   k_window_start  first midpoint (map f of Thm. 1 / the A half step of
//                   draft_step, Alg. 2) and cell assignment
//   k_cell_scan / k_cell_fill / k_cell_sort
//                   counting sort of atoms into cells (deterministic order)
//   k_nl_build      Verlet lists (cutoff + skin) for the target and the draft,
//                   atom-major rows [N][m], exact binary64 predicate
//   k_draft         one draft_step of Alg. 2 for every atom (Eq. bob draw)
//   k_verify        target forces for ALL K frames in one launch, each
//                   neighbour entry decoded once for all frames of a wave,
//                   fused with the binary64 transport-map sums of
//                   Eq. reflectionVerify
//   k_decide        accept / first rejection per replica (Alg. 1)
//   k_commit        reflection of the rejected momentum and map g (Thm. 1)
#include "lsd_device.h"
#include "lsd_launch.h"
#include "net_node.h"

// ---------------------------------------------------------------------------
__global__ void k_fill_int(int* p, int v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Sets flags[r] = 1 for every replica r of a lane with `need`, with one
// atomic per distinct replica in the wave (lanes that left early take no
// part).
__device__ __forceinline__ void flag_replicas(bool need, int r, int* flags) {
  unsigned long long m = __ballot(need);
  const int lane = threadIdx.x & 63;
  while (m) {
    const int leader = __ffsll((long long)m) - 1;
    const int rl = __shfl(r, leader, 64);
    if (lane == leader) atomicOr(&flags[rl], 1);
    m &= ~__ballot(need && r == rl);
  }
}

// Midpoint of the first draft step from the committed state and copy of the
// committed momenta into the window.  Frame 0 is written continuous with the
// list positions (so the image codes of the lists stay valid); a replica
// whose atoms moved too far from them is flagged for a rebuild.
// Item i: the validity flag i (i < R kmax) and atom i (i < N).
// qc, pc: the atom's committed position and momentum when the caller holds
// them (null: read from q and p).
__device__ __forceinline__ void window_start_item(const SysDev& S, const ListDev& Lst,
                                                  const WinDev& W, const float* q, const float* p,
                                                  int i, const float* qc = nullptr,
                                                  const float* pc = nullptr) {
  if (i < S.R * S.kmax) {
    // frames that would produce steps past the step limit are never verified
    const int rr = i / S.kmax, f = i % S.kmax;
    W.invalid[i] = (S.step[rr] + f + 1 > S.step_limit) ? 1 : 0;
  }
  if (i == 0) {
    W.nvalid[0] = 0;  // raised by the drafting of each valid frame
    W.tail_bar[0] = 0;
  }
  if (i < S.R) W.rej[i] = LSD_MAX_K;  // no rejection known yet
  if (i >= S.n) return;
  const int r = S.R == 1 ? 0 : S.atom_rep[i];
  const int sp = S.species ? S.species[i] : 0;
  const double L = S.box[r];
  const double hm = S.hdt_m[sp];
  int dimg[3] = {0, 0, 0};
  float x[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float pd = pc ? pc[d] : p[d * S.n + i];
    W.p[d * S.n + i] = pd;
    x[d] = a_half(qc ? qc[d] : q[d * S.n + i], pd, hm, L, &dimg[d]);
  }
  const float4 xw = make_float4(x[0], x[1], x[2], pack_img(dimg[0], dimg[1], dimg[2]));
  Lst.qwrap[i] = xw;
  if (Lst.always_rebuild) {
    W.qmid[i] = xw;
    return;
  }
  // continuous with the list positions: both lie in [0, L), so at most one
  // box edge separates the nearest images
  const float4 xr = Lst.qref[i];
  const float xrs[3] = {xr.x, xr.y, xr.z};
  const float half = (float)(0.5 * L);
  float d2 = 0.0f;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float dd0 = x[d] - xrs[d];
    const int n = dd0 > half ? 1 : (dd0 < -half ? -1 : 0);
    if (n != 0) {
      x[d] = (float)((double)x[d] - (double)n * L);
      dimg[d] += n;
    }
    const float dd = x[d] - xrs[d];
    d2 += dd * dd;
  }
  W.qmid[i] = make_float4(x[0], x[1], x[2], pack_img(dimg[0], dimg[1], dimg[2]));
  flag_replicas(d2 > Lst.reuse2 && Lst.rebuild[r] == 0, r, Lst.rebuild);
}

__global__ __launch_bounds__(256) void k_window_start(SysDev S, ListDev Lst, WinDev W,
                                                      const float* __restrict__ q,
                                                      const float* __restrict__ p) {
  window_start_item(S, Lst, W, q, p, blockIdx.x * blockDim.x + threadIdx.x);
}

// For replicas flagged for a rebuild: frame 0 becomes the wrapped midpoints
// (or stays the caller's frame 0), the list positions are reset to them, and
// they are binned into cells.
__global__ __launch_bounds__(256) void k_rebuild_bin(SysDev S, ListDev Lst, WinDev W,
                                                     int caller_frame0) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  if (!Lst.rebuild[r]) return;
  const double L = S.box[r];
  const float4 xq = caller_frame0 ? W.qmid[i] : Lst.qwrap[i];
  W.qmid[i] = xq;
  Lst.qref[i] = xq;
  const float x[3] = {xq.x, xq.y, xq.z};
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

// Cell offsets (one block): an exclusive scan of the cell counts restarted
// at every replica's first atom, so each replica's cells index its own range
// [rep_off[r], rep_off[r+1]) of the cell-sorted atom list (replicas that keep
// their lists have zero counts and keep their entries); then the counters
// are cleared for the next binning.
__global__ __launch_bounds__(1024) void k_cell_scan(ListDev Lst, const int* __restrict__ rep_off,
                                                    int R) {
  __shared__ int s[1024];
  const int C = Lst.n_cells;
  const int t = threadIdx.x;
  // nothing to do when no replica rebuilds its lists: the counts are all
  // zero (only rebuilt replicas are binned), every scan rewrites the cursors
  // before the next fill, and the offsets of kept lists are not read
  int any = 0;
  for (int r = t; r < R; r += 1024) any |= Lst.rebuild[r];
  if (!__syncthreads_or(any)) return;
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
  // global exclusive prefix, held in the cursors for the moment
  int run = s[t] - sum;
  for (int c = lo; c < hi; ++c) {
    Lst.cell_cursor[c] = run;
    run += Lst.cell_count[c];
    Lst.cell_count[c] = 0;
  }
  __syncthreads();
  for (int c = lo; c < hi; ++c) {
    const int r = Lst.cell_rep[c];
    Lst.cell_start[c] = rep_off[r] + Lst.cell_cursor[c] - Lst.cell_cursor[Lst.rep_cell_off[r]];
  }
  __syncthreads();
  for (int c = lo; c < hi; ++c) Lst.cell_cursor[c] = 0;
  if (t == 0) Lst.cell_start[C] = rep_off[Lst.cell_rep[C - 1] + 1];
}

__global__ __launch_bounds__(256) void k_cell_fill(int n, const int* __restrict__ atom_rep,
                                                   ListDev Lst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!Lst.rebuild[atom_rep[i]]) return;
  int c = Lst.atom_cell[i];
  int pos = Lst.cell_start[c] + atomicAdd(&Lst.cell_cursor[c], 1);
  Lst.cell_unsorted[pos] = i;
}

// ascending atom order inside each cell (rank sort, one block per cell): the
// list order then depends only on the positions, not on the order in which
// the binning atomics were served
__global__ __launch_bounds__(64) void k_cell_sort(ListDev Lst) {
  const int c = blockIdx.x;
  if (!Lst.rebuild[Lst.cell_rep[c]]) return;
  const int lo = Lst.cell_start[c], hi = Lst.cell_start[c + 1];
  for (int e = lo + (int)threadIdx.x; e < hi; e += 64) {
    const int v = Lst.cell_unsorted[e];
    int rank = 0;
    for (int a = lo; a < hi; ++a) rank += Lst.cell_unsorted[a] < v;
    Lst.cell_atoms[lo + rank] = v;
  }
}

// One list candidate (j at image code, position xj, image shift sh) of
// atom i at xi: in the target list (ht) and in the draft list (hd).  The
// binary32 separation has relative error <= 4u per component, as in the
// force kernels; the exact binary64 predicate decides inside the band
// rl2 (1 -+ 32u) around either list radius.
__device__ __forceinline__ void nl_pair_test(const ListDev& Lst, double L, float4 xi, int i,
                                             float4 xj, int j, int code, const float* sh,
                                             bool& ht, bool& hd) {
  ht = false;
  hd = false;
  if (j == i && code == 13) return;
  const float fdx = sep(xj.x, sh[0], xi.x, sh[3]);
  const float fdy = sep(xj.y, sh[1], xi.y, sh[4]);
  const float fdz = sep(xj.z, sh[2], xi.z, sh[5]);
  const float r2 = fdx * fdx + fdy * fdy + fdz * fdz;
  const bool bt = r2 >= Lst.rl2_t_lo && r2 < Lst.rl2_t_hi;
  const bool bd = r2 >= Lst.rl2_d_lo && r2 < Lst.rl2_d_hi;
  ht = r2 < Lst.rl2_t_lo;
  hd = r2 < Lst.rl2_d_lo;
  if (bt || bd) {
    double dx = ((double)xj.x - (double)xi.x) + (double)code_nx(code) * L;
    double dy = ((double)xj.y - (double)xi.y) + (double)code_ny(code) * L;
    double dz = ((double)xj.z - (double)xi.z) + (double)code_nz(code) * L;
    double d2 = dx * dx + dy * dy + dz * dz;
    if (bt) ht = d2 < Lst.rl2_t;
    if (bd) hd = d2 < Lst.rl2_d;
  }
}

// Appends the wave's hits in lane (candidate) order to a list row holding n
// entries so far (ballot compaction; entries past the row's width m are
// counted, not written).
__device__ __forceinline__ void nl_append(bool hit, uint32_t ent, unsigned long long below, int& n,
                                          uint32_t* row, int m) {
  const unsigned long long b = __ballot(hit);
  if (hit) {
    const int pos = n + __popcll(b & below);
    if (pos < m) row[pos] = ent;
  }
  n += __popcll(b);
}

// Verlet lists at the frame-0 midpoints: every (j, image) with
// |x_j + n L - x_i| < r_list.  One block per (cell, group of NL_IPB atoms of
// that cell): the candidates of the 27 neighbouring cells (ascending atom
// order per cell, fixed cell order) are staged in LDS in chunks; each wave
// tests one i-atom against 64 candidates at a time with the exact binary64
// predicate and appends the hits in candidate order by ballot compaction, so
// list rows are written contiguously (atom-major layout [i][m]).
#define NL_IPB 32
#define NL_CH 1024
#define NL_NT 256
__global__ __launch_bounds__(NL_NT) void k_nl_build(SysDev S, ListDev Lst, WinDev W) {
  constexpr int NT = NL_NT, NW = NT / 64, IPB = NL_IPB;
  __shared__ float4 s_x[NL_CH];
  __shared__ uint32_t s_e[NL_CH];
  __shared__ int s_pre[28];
  __shared__ int s_cstart[27];
  __shared__ int s_code[27];
  __shared__ float s_sh[27][6];
  const int c = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int r = Lst.cell_rep[c];
  if (!Lst.rebuild[r]) return;  // uniform over the block
  const int nc = Lst.rep_nc[r];
  const int coff = Lst.rep_cell_off[r];
  const int lo = Lst.cell_start[c], hi = Lst.cell_start[c + 1];
  const int occ = hi - lo;
  const int ib = blockIdx.y * IPB;
  if (blockIdx.y == 0 && t == 0 && occ > Lst.cell_cap) atomicOr(Lst.status, LSD_STATUS_CELL);
  if (ib >= occ) return;
  const int ie = min(occ, ib + IPB);
  const int nib = ie - ib;
  const double L = S.box[r];
  // the block's i-atoms and their positions, requested together with the
  // neighbour cells' offsets so that no wave waits on them per atom
  __shared__ int s_i[IPB];
  __shared__ float4 s_xi[IPB];
  for (int u = t; u < nib; u += NT) {
    const int i = Lst.cell_atoms[lo + ib + u];
    s_i[u] = i;
    s_xi[u] = W.qmid[i];
  }
  if (t < 27) {
    const int cl = c - coff;
    const int cx = cl % nc, cy = (cl / nc) % nc, cz = cl / (nc * nc);
    const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = t / 9 - 1;
    int tx = cx + ox, ty = cy + oy, tz = cz + oz, nx = 0, ny = 0, nz = 0;
    if (tx < 0) { tx += nc; nx = -1; } else if (tx >= nc) { tx -= nc; nx = 1; }
    if (ty < 0) { ty += nc; ny = -1; } else if (ty >= nc) { ty -= nc; ny = 1; }
    if (tz < 0) { tz += nc; nz = -1; } else if (tz >= nc) { tz -= nc; nz = 1; }
    const int cell = coff + tx + nc * (ty + nc * tz);
    s_cstart[t] = Lst.cell_start[cell];
    s_pre[t + 1] = Lst.cell_start[cell + 1] - Lst.cell_start[cell];
    s_code[t] = (nx + 1) + 3 * (ny + 1) + 9 * (nz + 1);
    image_shifts(t, (float)L, &s_sh[t][0], &s_sh[t][3]);  // by image code
  }
  __syncthreads();
  if (t == 0) {
    s_pre[0] = 0;
    for (int q = 0; q < 27; ++q) s_pre[q + 1] += s_pre[q];
  }
  __syncthreads();
  const int total = s_pre[27];
  // list lengths of the block's i-atoms so far (atom u of the block is
  // handled by wave u % NW in every chunk)
  __shared__ int s_nt[IPB], s_nd[IPB];
  for (int u = t; u < nib; u += NT) {
    s_nt[u] = 0;
    s_nd[u] = 0;
  }
  for (int cb = 0; cb < total; cb += NL_CH) {
    const int cn = min(NL_CH, total - cb);
    __syncthreads();
    // a thread's candidates: all their atom indices are requested before
    // any position, so the staging costs two dependent loads, not two per
    // candidate
    int jv[NL_CH / NT], cv[NL_CH / NT];
#pragma unroll
    for (int a = 0; a < NL_CH / NT; ++a) {
      const int k = t + NT * a;
      jv[a] = 0;
      cv[a] = 0;
      if (k < cn) {
        const int idx = cb + k;
        // neighbour cell of candidate idx: s_pre[q] <= idx < s_pre[q + 1]
        int q = 0;
#pragma unroll
        for (int step = 16; step > 0; step >>= 1)
          if (q + step < 27 && s_pre[q + step] <= idx) q += step;
        jv[a] = Lst.cell_atoms[s_cstart[q] + (idx - s_pre[q])];
        cv[a] = s_code[q];
      }
    }
#pragma unroll
    for (int a = 0; a < NL_CH / NT; ++a) {
      const int k = t + NT * a;
      if (k < cn) {
        s_x[k] = W.qmid[jv[a]];
        s_e[k] = ((uint32_t)jv[a] << 5) | (uint32_t)cv[a];
      }
    }
    __syncthreads();
    // each wave takes its atoms two at a time (u and u + NW), so every
    // staged candidate it reads serves both
    for (int u0 = wave; u0 < nib; u0 += 2 * NW) {
      const int u1 = u0 + NW;
      const bool two = u1 < nib;  // uniform per wave
      const int i0 = s_i[u0], i1 = two ? s_i[u1] : -1;
      const float4 x0 = s_xi[u0], x1 = two ? s_xi[u1] : x0;
      int nt0 = s_nt[u0], nd0 = s_nd[u0];
      int nt1 = two ? s_nt[u1] : 0, nd1 = two ? s_nd[u1] : 0;
      uint32_t* rowt0 = Lst.nbr_t + (size_t)i0 * Lst.mt;
      uint32_t* rowd0 = Lst.nbr_d + (size_t)i0 * Lst.md;
      uint32_t* rowt1 = Lst.nbr_t + (size_t)(two ? i1 : i0) * Lst.mt;
      uint32_t* rowd1 = Lst.nbr_d + (size_t)(two ? i1 : i0) * Lst.md;
      for (int k0 = 0; k0 < cn; k0 += 64) {
        const int k = k0 + lane;
        bool ht0 = false, hd0 = false, ht1 = false, hd1 = false;
        uint32_t ent = 0;
        if (k < cn) {
          ent = s_e[k];
          const int j = (int)(ent >> 5), code = (int)(ent & 31u);
          const float4 xj = s_x[k];
          const float* sh = s_sh[code];
          nl_pair_test(Lst, L, x0, i0, xj, j, code, sh, ht0, hd0);
          if (two) nl_pair_test(Lst, L, x1, i1, xj, j, code, sh, ht1, hd1);
        }
        const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        nl_append(ht0, ent, below, nt0, rowt0, Lst.mt);
        nl_append(hd0, ent, below, nd0, rowd0, Lst.md);
        if (two) {
          nl_append(ht1, ent, below, nt1, rowt1, Lst.mt);
          nl_append(hd1, ent, below, nd1, rowd1, Lst.md);
        }
      }
      if (lane == 0) {
        s_nt[u0] = nt0;
        s_nd[u0] = nd0;
        if (two) {
          s_nt[u1] = nt1;
          s_nd[u1] = nd1;
        }
      }
    }
  }
  __syncthreads();
  for (int u = t; u < nib; u += NT) {
    const int i = s_i[u];
    int a = s_nt[u], b = s_nd[u];
    if (a > Lst.mt) { atomicOr(Lst.status, LSD_STATUS_NBR_TARGET); a = Lst.mt; }
    if (b > Lst.md) { atomicOr(Lst.status, LSD_STATUS_NBR_DRAFT); b = Lst.md; }
    Lst.cnt_t[i] = a;
    Lst.cnt_d[i] = b;
  }
}

// Verlet lists of one small system in one launch, without cells: wave u of
// block b takes atom i = 4 b + u and tests every candidate (image, j) in a
// fixed order -- j ascending, each at its nearest image, when the box holds
// no second image of an atom inside the larger list radius (L > 2 r_list),
// else all 27 images of every j, image-major -- with the binary32 test and
// the binary64 band predicate of k_nl_build, appending the hits in candidate
// order by ballot compaction.  The same wave resets its atom's list position
// (and frame 0) as k_rebuild_bin does.  Every candidate is read from the
// positions the lists are built at, which no wave writes here.
#define NL_SMALL_MAX 2048
__global__ __launch_bounds__(256) void k_nl_small(SysDev S, ListDev Lst, WinDev W,
                                                  int caller_frame0) {
  __shared__ float s_sh[27][6];
  if (!Lst.rebuild[0]) return;  // uniform over the grid
  const int t = threadIdx.x, lane = t & 63;
  const double L = S.box[0];
  const float Lf = (float)L;
  if (t < 27) image_shifts(t, Lf, &s_sh[t][0], &s_sh[t][3]);
  __syncthreads();
  const int n = S.n;
  const int i = blockIdx.x * 4 + (t >> 6);
  if (i >= n) return;  // uniform per wave; no barrier follows
  const float4* src = caller_frame0 ? W.qmid : Lst.qwrap;
  const float4 xi = src[i];
  if (lane == 0) {
    if (!caller_frame0) W.qmid[i] = xi;
    Lst.qref[i] = xi;
  }
  // one image per atom at most inside the list radius: L^2 > 4 r^2 with a
  // margin far above the rounding of the binary32 separations below
  const double rl2 = Lst.rl2_t > Lst.rl2_d ? Lst.rl2_t : Lst.rl2_d;
  const bool nearest = L * L > 4.0 * rl2 * (1.0 + 1e-5);
  const int total = nearest ? n : 27 * n;
  const float half = 0.5f * Lf;
  uint32_t* rowt = Lst.nbr_t + (size_t)i * Lst.mt;
  uint32_t* rowd = Lst.nbr_d + (size_t)i * Lst.md;
  int nt = 0, nd = 0;
  for (int k0 = 0; k0 < total; k0 += 64) {
    const int k = k0 + lane;
    bool ht = false, hd = false;
    uint32_t ent = 0;
    if (k < total) {
      int j, code;
      if (nearest) {
        j = k;
      } else {
        code = k / n;
        j = k - code * n;
      }
      const float4 xj = src[j];
      if (nearest) {
        const float ex = xj.x - xi.x, ey = xj.y - xi.y, ez = xj.z - xi.z;
        const int nx = ex > half ? -1 : (ex < -half ? 1 : 0);
        const int ny = ey > half ? -1 : (ey < -half ? 1 : 0);
        const int nz = ez > half ? -1 : (ez < -half ? 1 : 0);
        code = (nx + 1) + 3 * (ny + 1) + 9 * (nz + 1);
      }
      ent = ((uint32_t)j << 5) | (uint32_t)code;
      if (!(j == i && code == 13)) {
        const float* sh = s_sh[code];
        const float fdx = sep(xj.x, sh[0], xi.x, sh[3]);
        const float fdy = sep(xj.y, sh[1], xi.y, sh[4]);
        const float fdz = sep(xj.z, sh[2], xi.z, sh[5]);
        const float r2 = fdx * fdx + fdy * fdy + fdz * fdz;
        const bool bt = r2 >= Lst.rl2_t_lo && r2 < Lst.rl2_t_hi;
        const bool bd = r2 >= Lst.rl2_d_lo && r2 < Lst.rl2_d_hi;
        ht = r2 < Lst.rl2_t_lo;
        hd = r2 < Lst.rl2_d_lo;
        if (bt || bd) {
          double dx = ((double)xj.x - (double)xi.x) + (double)code_nx(code) * L;
          double dy = ((double)xj.y - (double)xi.y) + (double)code_ny(code) * L;
          double dz = ((double)xj.z - (double)xi.z) + (double)code_nz(code) * L;
          double d2 = dx * dx + dy * dy + dz * dz;
          if (bt) ht = d2 < Lst.rl2_t;
          if (bd) hd = d2 < Lst.rl2_d;
        }
      }
    }
    const unsigned long long bt = __ballot(ht), bd = __ballot(hd);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (ht) {
      const int pos = nt + __popcll(bt & below);
      if (pos < Lst.mt) rowt[pos] = ent;
    }
    if (hd) {
      const int pos = nd + __popcll(bd & below);
      if (pos < Lst.md) rowd[pos] = ent;
    }
    nt += __popcll(bt);
    nd += __popcll(bd);
  }
  if (lane == 0) {
    if (nt > Lst.mt) { atomicOr(Lst.status, LSD_STATUS_NBR_TARGET); nt = Lst.mt; }
    if (nd > Lst.md) { atomicOr(Lst.status, LSD_STATUS_NBR_DRAFT); nd = Lst.md; }
    Lst.cnt_t[i] = nt;
    Lst.cnt_d[i] = nd;
  }
}

// Tether force and energy of atom i at position xi (minimum image).
__device__ __forceinline__ void tether_force(const PotDev& P, const SysDev& S, float4 xi, int i,
                                             float Lf, float& fx, float& fy, float& fz, float& e) {
  float d[3] = {xi.x - P.anchor[i], xi.y - P.anchor[S.n + i], xi.z - P.anchor[2 * S.n + i]};
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a] -= Lf * rintf(d[a] / Lf);
  fx = -P.kspring * d[0];
  fy = -P.kspring * d[1];
  fz = -P.kspring * d[2];
  e = 0.5f * P.kspring * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

// Force of potential P on atom i at frame positions X.  The NL lanes of an
// atom share the list row: lane `sub` sums the entries m = sub, sub + NL, ...
// in order, and the partial sums are combined by a fixed butterfly, so every
// kernel that uses this pattern with the same NL obtains bit-identical forces
// for identical positions and lists.  NL is LSD_LPA everywhere but in the
// drafting kernel of the learned draft; ctab: that draft's pair-type
// coefficients (null: read from its parameters).
// width: the list's row width (the first group of entries is read before
// the count is known).
// KIND: the potential kind when the launch fixes it (the other kinds' code is
// then left out of the kernel), 0 to read it from P.
template <int NL = LSD_LPA, int KIND = 0>
__device__ __forceinline__ void pot_force(const PotDev& P, const SysDev& S,
                                          const float4* __restrict__ X,
                                          const uint32_t* __restrict__ row, int width, int cnt,
                                          int i, int r, int sub, float& fx, float& fy, float& fz,
                                          float& e, const float* __restrict__ ctab = nullptr) {
  fx = fy = fz = e = 0.0f;
  const double L = S.box[r];
  const float Lf = (float)L;
  const float4 xi = X[i];
  const int kind = KIND > 0 ? KIND : P.kind;
  if (kind == LSD_POT_LJ) {
    // LSD_GATHER entries per iteration (gathers issued together), added in
    // order
    for (int m0 = sub, first = 1; first || m0 < cnt; m0 += LSD_GATHER * NL, first = 0) {
      Gathered gt;
      gather_entries<NL>(row, width, cnt, m0, X, nullptr, gt);
#pragma unroll
      for (int u = 0; u < LSD_GATHER; ++u) {
        if (!gt.ok[u]) break;
        float sj[3], si[3];
        image_shifts(gt.code[u], Lf, sj, si);
        lj_pair(P, xi, gt.x[u], sj, si, gt.code[u], L, fx, fy, fz, e);
      }
    }
    fx = lanes_sum<NL>(fx);
    fy = lanes_sum<NL>(fy);
    fz = lanes_sum<NL>(fz);
    e = lanes_sum<NL>(e);
  } else if (kind == LSD_POT_PAIR) {
    const int spi = S.species ? S.species[i] : 0;
    for (int m0 = sub, first = 1; first || m0 < cnt; m0 += LSD_GATHER * NL, first = 0) {
      Gathered gt;
      gather_entries<NL>(row, width, cnt, m0, X, S.species, gt);
#pragma unroll
      for (int u = 0; u < LSD_GATHER; ++u) {
        if (!gt.ok[u]) break;
        float sj[3], si[3];
        image_shifts(gt.code[u], Lf, sj, si);
        pair_draft_force(P, xi, gt.x[u], sj, si, spi, gt.sp[u], fx, fy, fz);
      }
    }
    fx = lanes_sum<NL>(fx);
    fy = lanes_sum<NL>(fy);
    fz = lanes_sum<NL>(fz);
  } else if (kind == LSD_POT_NET) {
    net_force<NL>(P, S, X, row, width, cnt, i, r, sub,
                  ctab ? ctab : P.w + net_off_c(P.ns, P.nb), fx, fy, fz);
  } else if (kind == LSD_POT_HARMONIC) {
    tether_force(P, S, xi, i, Lf, fx, fy, fz, e);
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
// atom left the skin of the lists.  SUB blocks share one tile of up to 64
// atoms of one replica (NL lanes per atom), so the validity test of the
// frame is uniform over each block.
static_assert(LSD_TILE % LSD_NET_SUB == 0 && LSD_NET_LPA <= 64 &&
                  (LSD_NET_LPA & (LSD_NET_LPA - 1)) == 0 &&
                  LSD_TILE / LSD_NET_SUB * LSD_NET_LPA <= 1024,
              "learned-draft launch: whole atoms per block, power-of-two lanes per atom");
// KIND: the draft's potential kind fixed by the launch (0: read from P), or
// LSD_KIND_GIVEN for forces already in the window.
#define LSD_KIND_GIVEN (-1)
// One block of the draft step (block index blk, thread tid of LSD_TILE / SUB
// * NL).  STAGE: the block stages the learned draft's pair-type coefficients
// in s_ct itself (one launch per step); otherwise they are in s_ct already.
template <int NL, int SUB, int KIND, bool STAGE>
__device__ __forceinline__ void draft_block(const SysDev& S, const ListDev& Lst, const WinDev& W,
                                            const TileDev& Tl, const PotDev& P, int k,
                                            int use_target_list, int blk, int tid, float* s_ct) {
  constexpr bool forces_given = KIND == LSD_KIND_GIVEN;
  constexpr int APB = LSD_TILE / SUB;  // atoms per block
  const int tile = blk / SUB, part = blk % SUB;
  const TileInfo T = tile_info(S.n, S.R, Tl, tile);
  const int r = T.rep;
  int* inv = W.invalid + (size_t)r * S.kmax;
  // a frame after a rejection that the verification of earlier frames has
  // already found (pipelined windows) is discarded like one past the skin;
  // a block that sees it marks the frame, so that no part of it is verified
  const bool after_reject = W.rej[r] < k;
  const int inv_k = inv[k];
  // the atom's list row and position are requested before the test of the
  // frame, so that their latency overlaps it
  const int a = part * APB + tid / NL, sub = tid % NL;
  const bool in = a < T.count;
  const int i = T.start + (in ? a : 0);
  const int width = use_target_list ? Lst.mt : Lst.md;
  const uint32_t* row = (use_target_list ? Lst.nbr_t : Lst.nbr_d) + (size_t)i * width;
  const int cnt = forces_given ? 0 : (use_target_list ? Lst.cnt_t[i] : Lst.cnt_d[i]);
  // the learned draft's pair-type coefficients, read by every entry: staged
  // in LDS (requested here as well)
  constexpr int CT_PER = (LSD_NET_MAX_TYPES * LSD_NET_MAX_BASIS + APB * NL - 1) / (APB * NL);
  const bool net = !forces_given && (KIND > 0 ? KIND : P.kind) == LSD_POT_NET;
  const int nct = net ? P.ns * (P.ns + 1) / 2 * P.nb : 0;
  float ctv[CT_PER];
#pragma unroll
  for (int q = 0; q < CT_PER; ++q) {
    const int t = tid + q * APB * NL;
    ctv[q] = (STAGE && t < nct) ? P.w[net_off_c(P.ns, P.nb) + t] : 0.0f;
  }
  if (after_reject && tid == 0 && inv_k == 0) atomicOr(&inv[k], 1);
  if (after_reject || inv_k) {
    // frames from K_eff on are discarded: no work, and the next frame is
    // invalid as well (one thread per replica records it)
    if (tid == 0 && T.first && part == 0 && k + 1 < W.K) inv[k + 1] = 1;
    return;
  }
  // frame k is valid for this replica: the verification covers it
  if (tid == 0 && T.first && part == 0) atomicMax(W.nvalid, k + 1);
  if (STAGE && net) {
#pragma unroll
    for (int q = 0; q < CT_PER; ++q) {
      const int t = tid + q * APB * NL;
      if (t < nct) s_ct[t] = ctv[q];
    }
    __syncthreads();
  }
  const int sp = S.species ? S.species[i] : 0;
  const size_t N = (size_t)S.n;
  const float4* X = W.qmid + (size_t)k * N;
  // inputs of the step after the force, requested before the force loop
  const bool lead = in && sub == 0;
  float pk[3] = {0.0f, 0.0f, 0.0f}, fmc[3] = {0.0f, 0.0f, 0.0f};
  float4 x0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (lead) {
    const float* pkp = W.p + (size_t)k * 3 * N;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pk[d] = pkp[d * N + i];
      fmc[d] = draft_mean_force(W, r, d * N + i, k, 0.0f);  // error-correction term
    }
    x0 = Lst.qref[i];
  }
  float F[3], e;
  if constexpr (forces_given) {
    // forces of this frame already in the window (batched network pass)
    const float* fk0 = W.fd + (size_t)k * 3 * N;
    F[0] = fk0[i];
    F[1] = fk0[N + i];
    F[2] = fk0[2 * N + i];
  } else {
    pot_force<NL, KIND>(P, S, X, row, width, cnt, i, r, sub, F[0], F[1], F[2], e, s_ct);
  }
  if (!lead) return;

  double xi[3];
  if (S.replay_xi) {
    const double* rx = S.replay_xi + ((size_t)k * N + i) * 3;
    xi[0] = rx[0]; xi[1] = rx[1]; xi[2] = rx[2];
  } else {
    stream_normals3(S.seed, (uint32_t)r, (uint64_t)(S.step[r] + k + 1),
                    (uint32_t)(i - S.rep_off[r]), xi);
  }
  float* pk1 = W.p + (size_t)(k + 1) * 3 * N;
  float* fk = W.fd + (size_t)k * 3 * N;
  const double sg = S.sig[sp];
  float pn[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float Fm = W.ec ? F[d] + fmc[d] : F[d];
    double mu = bob_mean(S.a, S.c1fu, pk[d], Fm);
    pn[d] = (float)fma(sg, xi[d], mu);
    fk[d * N + i] = F[d];
    pk1[d * N + i] = pn[d];
  }
  if (k + 1 < W.K) {
    const double hm = S.hdt_m[sp];
    const float4 x = X[i];
    const float xs[3] = {x.x, x.y, x.z};
    float xn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float qend = a_half_cont(xs[d], pn[d], hm);   // q~_k
      xn[d] = a_half_cont(qend, pn[d], hm);                // next midpoint
    }
    // frames stay continuous with frame 0, so frame 0's image deltas apply
    W.qmid[(size_t)(k + 1) * N + i] = make_float4(xn[0], xn[1], xn[2], x.w);
    // displacement from the list positions
    const float dx = xn[0] - x0.x, dy = xn[1] - x0.y, dz = xn[2] - x0.z;
    const float d2 = dx * dx + dy * dy + dz * dz;
    if (d2 > S.half_skin2 && inv[k + 1] == 0) atomicOr(&inv[k + 1], 1);
  }
}


template <int NL, int SUB, int KIND>
__global__ __launch_bounds__(LSD_TILE / SUB * NL) void k_draft(SysDev S, ListDev Lst, WinDev W,
                                                               TileDev Tl, PotDev P, int k,
                                                               int use_target_list) {
  __shared__ float s_ct[LSD_NET_MAX_TYPES * LSD_NET_MAX_BASIS];
  draft_block<NL, SUB, KIND, true>(S, Lst, W, Tl, P, k, use_target_list, blockIdx.x, threadIdx.x,
                                   s_ct);
}

// Draft steps k0 .. K-1 of a window of one small system with the learned
// draft (bfloat16 node pass) in one launch.  Each step is the node pass and
// the force pass of the per-step kernels, run block by block over the same
// blocks (the node pass's 16-atom blocks, then four of the force pass's
// 64-thread blocks per block, one per wave), with a grid barrier after each
// pass, so the results are those of the per-step launches bit for bit.  The
// chain stops at the first frame that is not drafted (past the skin), and
// flags the later frames as the per-step launches would; launches for those
// frames are what it saves.  Every block of the grid is resident at once
// (at most one per compute unit), and every wait at a barrier is bounded: a
// barrier that times out latches LSD_STATUS_TAIL and ends the chain.
#define LSD_TAIL_SPIN (1 << 16)
__device__ __forceinline__ bool tail_barrier(int* bar, int target, int* status, int* s_fail) {
  // the stores of every wave have completed before the block arrives
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (gridDim.x == 1) return true;  // one block: its waves share the compute unit's caches
  if (threadIdx.x == 0) {
    __threadfence();  // release: this block's writes are visible device-wide
    atomicAdd(bar, 1);
    int spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target &&
           spins < LSD_TAIL_SPIN)
      ++spins;
    if (spins >= LSD_TAIL_SPIN) {
      atomicOr(status, LSD_STATUS_TAIL);
      *s_fail = 1;
    }
    __threadfence();  // acquire: the other blocks' writes are seen from here on
  }
  __syncthreads();
  return *s_fail == 0;
}

__global__ __launch_bounds__(256) void k_draft_tail_net(SysDev S, ListDev Lst, WinDev W,
                                                        TileDev Tl, PotDev P, int k0) {
  __shared__ float s_ct[LSD_NET_MAX_TYPES * LSD_NET_MAX_BASIS];
  __shared__ int s_fail;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int nct = P.ns * (P.ns + 1) / 2 * P.nb;
  for (int q = t; q < nct; q += 256) s_ct[q] = P.w[net_off_c(P.ns, P.nb) + q];
  if (t == 0) s_fail = 0;
  __syncthreads();
  const int G = gridDim.x;
  const int node_blocks = (S.n + NET_IROWS - 1) / NET_IROWS;
  const int force_blocks = S.n_tiles * LSD_NET_SUB;
  int target = 0, k = k0;
  for (; k < W.K; ++k) {
    // frame k is drafted unless the skin (or a rejection already known)
    // ended the window before it; every block reads the same flags, at
    // device scope (the previous pass set them)
    if (__hip_atomic_load(&W.invalid[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
        W.rej[0] < k)
      break;
    for (int b = blockIdx.x; b < node_blocks; b += G)
      net_nodes_bf16_block<NET_NODE_LPA>(S, Lst, W, P, k, b);
    target += G;
    if (!tail_barrier(W.tail_bar, target, Lst.status, &s_fail)) return;
    for (int b = blockIdx.x * 4 + wave; b < force_blocks; b += G * 4)
      draft_block<LSD_NET_LPA, LSD_NET_SUB, LSD_POT_NET, false>(S, Lst, W, Tl, P, k, 0, b, lane,
                                                                s_ct);
    target += G;
    if (!tail_barrier(W.tail_bar, target, Lst.status, &s_fail)) return;
  }
  // frames after the first one not drafted are flagged, as the per-step
  // launches flag them one by one
  if (blockIdx.x == 0 && t == 0)
    for (int kk = k + 1; kk < W.K; ++kk) W.invalid[kk] = 1;
}

// The same for a pair draft (Lennard-Jones or force-matched pair forces), or
// for plain stepping with such a target (use_target_list), on one system:
// steps k0 .. K-1 in one launch of at most LSD_TAIL_PAIR_BLOCKS blocks, each
// running the per-step kernel's 64-atom blocks in turn, one bounded grid
// barrier per step.
#define LSD_TAIL_PAIR_BLOCKS 128
template <int KIND>
__global__ __launch_bounds__(LSD_VTHREADS) void k_draft_tail_pair(SysDev S, ListDev Lst, WinDev W,
                                                                  TileDev Tl, PotDev P, int k0,
                                                                  int use_target_list) {
  __shared__ int s_fail;
  if (threadIdx.x == 0) s_fail = 0;
  __syncthreads();
  const int G = gridDim.x;
  int target = 0, k = k0;
  for (; k < W.K; ++k) {
    if (__hip_atomic_load(&W.invalid[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
        W.rej[0] < k)
      break;
    for (int b = blockIdx.x; b < S.n_tiles; b += G)
      draft_block<LSD_LPA, 1, KIND, false>(S, Lst, W, Tl, P, k, use_target_list, b, threadIdx.x,
                                           nullptr);
    target += G;
    if (!tail_barrier(W.tail_bar, target, Lst.status, &s_fail)) return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int kk = k + 1; kk < W.K; ++kk) W.invalid[kk] = 1;
}

// Validity of caller-written frames against the frame-0 lists.
__global__ __launch_bounds__(256) void k_frame_validity(SysDev S, ListDev Lst, WinDev W) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  const float4 x0 = Lst.qref[i];
  int* inv = W.invalid + (size_t)r * S.kmax;
  if (i == S.rep_off[r])
    for (int k = 0; k < W.K; ++k)
      if (S.step[r] + k + 1 > S.step_limit) inv[k] = 1;
  // caller frames must be continuous with frame 0 (not wrapped): a frame in
  // which an atom jumped by a box edge is reported invalid, never verified
  for (int k = 1; k < W.K; ++k) {
    const float4 x = W.qmid[(size_t)k * S.n + i];
    const float dx = x.x - x0.x, dy = x.y - x0.y, dz = x.z - x0.z;
    const float d2 = dx * dx + dy * dy + dz * dz;
    if (d2 > S.half_skin2) {
      for (int kk = k; kk < W.K; ++kk) atomicOr(&inv[kk], 1);
      break;
    }
  }
}

// verify_step (Alg. 2) for the valid frames of the window.  Work item = one
// tile of up to 64 atoms of one replica x FW frames; the items of the frame
// groups that can hold a valid frame (W.nvalid, raised by the drafting of
// every valid frame) are taken by a fixed grid in order, frame group by
// frame group, so no block is launched for the frames a window never
// reaches.  Each atom uses LSD_LPA lanes (same entry split and butterfly as
// the draft kernel), which read their neighbour entries straight from the
// list (the lanes of an atom read consecutive words; the rows stay in L1 over
// the loop), and each lane advances all FW frames per neighbour entry, so an
// entry is decoded once and its image shift reused.  No LDS staging:
// occupancy is set by the registers alone (staging the rows, in full or in
// chunks, measured 1.4-1.9x slower).
// Epilogue per atom and frame (binary64):
//   z = (p~_k - <p~_k>) / sigma,  delta = c1 (F~_k - F_k) / sigma
// reduced over the tile in a fixed order: S1 = delta.z, S2 = delta.delta,
// and the potential energy.  Which block takes an item does not change any
// result.
#ifndef LSD_VGATHER
#define LSD_VGATHER 2  // neighbour entries per lane per iteration of k_verify
#endif
template <int FW>
__device__ __forceinline__ void verify_item(const SysDev& S, const ListDev& Lst, const WinDev& W,
                                            const TileDev& Tl, const PotDev& P, int tile, int f0,
                                            int fend, float (*s_shift)[6],
                                            double (*s_red)[FW][3]) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int a = t / LSD_LPA, sub = t % LSD_LPA;
  const TileInfo T = tile_info(S.n, S.R, Tl, tile);
  const int start = T.start, count = T.count, r = T.rep;
  const int* inv = W.invalid + (size_t)r * S.kmax;
  const int rej = W.rej[r];
  const double L = S.box[r];
  const size_t N = (size_t)S.n;
  const bool lj = P.kind == LSD_POT_LJ;
  // the atom's positions, entry count and first group of entry words are
  // requested together with the frame flags (for a frame that is not
  // verified they go unused; every slot below the row width is in the list,
  // and a word past the count is not used)
  const bool active = a < count;
  const int i = start + (active ? a : 0);
  const uint32_t* row = Lst.nbr_t + (size_t)i * Lst.mt;
  const int cnt = (active && lj) ? Lst.cnt_t[i] : 0;
  uint32_t e0[LSD_VGATHER];
#pragma unroll
  for (int u = 0; u < LSD_VGATHER; ++u) {
    const int m = sub + u * LSD_LPA;
    e0[u] = row[m < Lst.mt ? m : 0];
  }
  float4 xi[FW];
#pragma unroll
  for (int f = 0; f < FW; ++f)
    xi[f] = W.qmid[(size_t)(f0 + f < fend ? f0 + f : f0) * N + i];
  bool valid[FW];
  bool any = false;
#pragma unroll
  for (int f = 0; f < FW; ++f) {
    // frames after a rejection found earlier in the window are not needed
    valid[f] = (f0 + f < fend) && inv[f0 + f] == 0 && f0 + f <= rej;
    any = any || valid[f];
  }
  if (!any) return;  // uniform over the block
  const float Lf = (float)L;
  if (t < 27) image_shifts(t, Lf, &s_shift[t][0], &s_shift[t][3]);
  __syncthreads();

  float fx[FW], fy[FW], fz[FW], en[FW];
#pragma unroll
  for (int f = 0; f < FW; ++f) fx[f] = fy[f] = fz[f] = en[f] = 0.0f;
  // one frame per wave: the epilogue's inputs are requested before the
  // force loop (error-correction term as in draft_mean_force)
  float pre_p[3] = {0.f, 0.f, 0.f}, pre_p1[3] = {0.f, 0.f, 0.f};
  float pre_fd[3] = {0.f, 0.f, 0.f}, pre_ec[3] = {0.f, 0.f, 0.f};
  if constexpr (FW == 1) {
    if (active && sub == 0 && valid[0]) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        pre_p[d] = W.p[(size_t)f0 * 3 * N + d * N + i];
        pre_p1[d] = W.p[(size_t)(f0 + 1) * 3 * N + d * N + i];
        pre_fd[d] = W.fd[(size_t)f0 * 3 * N + d * N + i];
        pre_ec[d] = draft_mean_force(W, r, d * N + i, f0, 0.0f);
      }
    }
  }
  // LSD_VGATHER entries per iteration (m, m + LSD_LPA, ...): their gathers
  // are issued together; the terms are added in entry order as in the draft
  // kernel
  for (int m0 = sub, first = 1; first || m0 < cnt; m0 += LSD_VGATHER * LSD_LPA, first = 0) {
    int jj[LSD_VGATHER], cc[LSD_VGATHER];
#pragma unroll
    for (int u = 0; u < LSD_VGATHER; ++u) {
      const int m = m0 + u * LSD_LPA;
      const uint32_t e = first ? e0[u] : row[m < Lst.mt ? m : 0];
      jj[u] = m < cnt ? (int)(e >> 5) : 0;
      cc[u] = (int)(e & 31u);
    }
    float4 xj[LSD_VGATHER][FW];
#pragma unroll
    for (int u = 0; u < LSD_VGATHER; ++u)
#pragma unroll
      for (int f = 0; f < FW; ++f) {
        // frame f0 exists in every item; an invalid frame's load is unused
        const size_t fr = (size_t)(valid[f] ? f0 + f : f0) * N;
        xj[u][f] = W.qmid[fr + jj[u]];
      }
#pragma unroll
    for (int u = 0; u < LSD_VGATHER; ++u) {
      if (m0 + u * LSD_LPA >= cnt) break;
      const float* sh = s_shift[cc[u]];
#pragma unroll
      for (int f = 0; f < FW; ++f)
        if (valid[f]) lj_pair(P, xi[f], xj[u][f], sh, sh + 3, cc[u], L, fx[f], fy[f], fz[f], en[f]);
    }
  }
  const int sp = (active && S.species) ? S.species[i] : 0;
  const double isg = 1.0 / S.sig[sp];
#pragma unroll
  for (int f = 0; f < FW; ++f) {
    double s1 = 0.0, s2 = 0.0, es = 0.0;
    if (valid[f]) {
      float Ft[3], e;
      if (lj) {
        Ft[0] = lpa_sum(fx[f]);
        Ft[1] = lpa_sum(fy[f]);
        Ft[2] = lpa_sum(fz[f]);
        e = lpa_sum(en[f]);
      } else {
        // the other target kind here is the tether (network targets take
        // the batched path; the drafts are never targets)
        tether_force(P, S, xi[f], i, Lf, Ft[0], Ft[1], Ft[2], e);
      }
      if (P.offset) {
        Ft[0] += P.offset[i];
        Ft[1] += P.offset[N + i];
        Ft[2] += P.offset[2 * N + i];
      }
      if (active && sub == 0) {
        const int fr = f0 + f;
        const float* pk = W.p + (size_t)fr * 3 * N;
        const float* pk1 = W.p + (size_t)(fr + 1) * 3 * N;
        const float* fdk = W.fd + (size_t)fr * 3 * N;
        float* ftk = W.ft + (size_t)fr * 3 * N;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          float Fd, pkd, pk1d;
          if constexpr (FW == 1) {
            Fd = W.ec ? pre_fd[d] + pre_ec[d] : pre_fd[d];
            pkd = pre_p[d];
            pk1d = pre_p1[d];
          } else {
            Fd = draft_mean_force(W, r, d * N + i, fr, fdk[d * N + i]);
            pkd = pk[d * N + i];
            pk1d = pk1[d * N + i];
          }
          ftk[d * N + i] = Ft[d];
          const double mud = bob_mean(S.a, S.c1fu, pkd, Fd);
          const double z = ((double)pk1d - mud) * isg;
          const double dl = S.c1fu * ((double)Fd - (double)Ft[d]) * isg;
          s1 = fma(dl, z, s1);
          s2 = fma(dl, dl, s2);
        }
        es = (double)e;
      }
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    es = wave_sum(es);
    if (lane == 0) {
      s_red[wave][f][0] = s1;
      s_red[wave][f][1] = s2;
      s_red[wave][f][2] = es;
    }
  }
  __syncthreads();
  if (t < FW && valid[t]) {
    double* out = W.partial + ((size_t)(f0 + t) * S.n_tiles + tile) * 4;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double v = s_red[0][t][q];
      for (int w = 1; w < LSD_VWAVES; ++w) v += s_red[w][t][q];
      out[q] = v;
    }
  }
  __syncthreads();  // the next item rewrites s_shift and s_red
}

// Frames [fbeg, fend) of the window (all of it, or one group of a pipelined
// window).
template <int FW>
__global__ __launch_bounds__(LSD_VTHREADS) void k_verify(SysDev S, ListDev Lst, WinDev W,
                                                         TileDev Tl, PotDev P, int fbeg,
                                                         int fend) {
  __shared__ float s_shift[27][6];
  __shared__ double s_red[LSD_VWAVES][FW][3];
  // the block's first item needs no count: frames from the window's valid
  // count on are flagged invalid, which the item tests itself; the count
  // (requested here) bounds the items the block takes after it
  const int nvalid = W.nvalid[0];
  const int all_items = (fend - fbeg + FW - 1) / FW * S.n_tiles;
  int v = blockIdx.x;
  if (v < all_items) {
    const int g = v / S.n_tiles;
    verify_item<FW>(S, Lst, W, Tl, P, v - g * S.n_tiles, fbeg + g * FW, fend, s_shift, s_red);
  }
  const int nv = min(min(nvalid, W.K), fend);
  const int items = nv > fbeg ? (nv - fbeg + FW - 1) / FW * S.n_tiles : 0;
  for (v += gridDim.x; v < items; v += gridDim.x) {
    const int g = v / S.n_tiles;
    verify_item<FW>(S, Lst, W, Tl, P, v - g * S.n_tiles, fbeg + g * FW, fend, s_shift, s_red);
  }
}

// Transport-map sums for frames whose target forces are already in the
// window (batched network pass): S1, S2 and the energy per (frame, tile), in
// the same binary64 form as the epilogue of k_verify; the energies of the
// tile's rows come from the network pass (e_rows, frames counted from fbeg).
__global__ __launch_bounds__(64) void k_transport(SysDev S, WinDev W, TileDev Tl,
                                                  const double* __restrict__ e_rows, int fbeg) {
  const int tile = blockIdx.x, f = fbeg + blockIdx.y;
  const int lane = threadIdx.x;
  const int start = Tl.start[tile], count = Tl.count[tile], r = Tl.rep[tile];
  if (f >= W.K || W.invalid[(size_t)r * S.kmax + f] || f > W.rej[r]) return;  // uniform
  const size_t N = (size_t)S.n;
  double s1 = 0.0, s2 = 0.0, es = 0.0;
  if (lane < count) {
    es = e_rows[(size_t)(f - fbeg) * N + start + lane];
    const int i = start + lane;
    const int sp = S.species ? S.species[i] : 0;
    const double isg = 1.0 / S.sig[sp];
    const float* pk = W.p + (size_t)f * 3 * N;
    const float* pk1 = W.p + (size_t)(f + 1) * 3 * N;
    const float* fdk = W.fd + (size_t)f * 3 * N;
    const float* ftk = W.ft + (size_t)f * 3 * N;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float Fd = draft_mean_force(W, r, d * N + i, f, fdk[d * N + i]), Ft = ftk[d * N + i];
      const double mud = bob_mean(S.a, S.c1fu, pk[d * N + i], Fd);
      const double z = ((double)pk1[d * N + i] - mud) * isg;
      const double dl = S.c1fu * ((double)Fd - (double)Ft) * isg;
      s1 = fma(dl, z, s1);
      s2 = fma(dl, dl, s2);
    }
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  es = wave_sum(es);
  if (lane == 0) {
    double* out = W.partial + ((size_t)f * S.n_tiles + tile) * 4;
    out[0] = s1;
    out[1] = s2;
    out[2] = es;
  }
}

// Per replica: frame sums over its tiles (fixed order), log ratio, decision
// with u_{s+k}, first rejection (Alg. 1), outputs and the commit record.
// One block per replica; wave w handles frames w, w + nw, ... (the sum over
// a frame's tiles is lane-strided plus the wave butterfly, whatever the
// block size), then one thread scans the decisions for the first rejection.
// Frames after a rejection already found while the window was drafted
// (pipelined windows) are not verified.

// S1, S2 and the energy of frame f of replica r from the per-tile partials,
// in a fixed order (lane-strided over the tiles, then the wave butterfly),
// and the decision log u_{s+f+1} <= log r (Eq. reflectionVerify).
__device__ __forceinline__ bool frame_decision(const SysDev& S, const WinDev& W, const TileDev& Tl,
                                               int r, int f, int lane, double* s1o, double* s2o,
                                               double* eso, double* logro) {
  const int t0 = Tl.rep_tile_off[r], t1 = Tl.rep_tile_off[r + 1];
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
  const size_t o = (size_t)r * S.kmax + f;
  const double u = S.replay_u ? S.replay_u[o]
                              : stream_uniform(S.seed, (uint32_t)r, (uint64_t)S.step[r] + f + 1);
  *s1o = s1;
  *s2o = s2;
  *eso = es;
  *logro = logr;
  return log(u) <= logr;
}

// Decisions of the frames [fbeg, fend) of a pipelined window as soon as they
// are verified: the first rejected frame is recorded (W.rej), so that the
// drafting and verification of later frames stop.  One block per replica,
// one wave per frame of the group.  k_decide later repeats the same
// arithmetic for every kept frame.
__global__ __launch_bounds__(1024) void k_decide_group(SysDev S, WinDev W, TileDev Tl, int fbeg,
                                                       int fend) {
  __shared__ int s_acc[LSD_MAX_K];
  const int r = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int* inv = W.invalid + (size_t)r * S.kmax;
  const int rej = W.rej[r];
  for (int f = fbeg + wave; f < fend; f += nw) {
    int acc = 1;
    if (f <= rej && !inv[f]) {
      double s1, s2, es, logr;
      acc = frame_decision(S, W, Tl, r, f, lane, &s1, &s2, &es, &logr) ? 1 : 0;
    }
    if (lane == 0) s_acc[f] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0 && rej >= fend) {
    for (int f = fbeg; f < fend; ++f) {
      if (inv[f]) break;
      if (!s_acc[f]) {
        W.rej[r] = f;
        break;
      }
    }
  }
}

__device__ __forceinline__ void decide_replica(const SysDev& S, const WinDev& W, const TileDev& Tl,
                                               const OutDev& O, int plain, int* rebuild,
                                               int always_rebuild, int r) {
  __shared__ double s_s1[LSD_MAX_K], s_s2[LSD_MAX_K];
  __shared__ int s_acc[LSD_MAX_K];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int K = W.K;
  const int* inv = W.invalid + (size_t)r * S.kmax;
  int keff = K;
  for (int f = 0; f < K; ++f)
    if (inv[f]) { keff = f; break; }
  // a rejection found while the window was drafted ends the verified frames
  if (!plain && W.rej[r] + 1 < keff) keff = W.rej[r] + 1;
  const uint64_t s0 = (uint64_t)S.step[r];
  for (int f = wave; f < K; f += nw) {
    const size_t o = (size_t)r * S.kmax + f;
    if (plain || f >= keff) {
      if (lane == 0) {
        O.accepted[o] = 2;
        O.log_ratio[o] = 0.0;
        O.energy[o] = 0.0;
        s_acc[f] = 1;
      }
      continue;
    }
    double s1, s2, es, logr;
    const bool acc = frame_decision(S, W, Tl, r, f, lane, &s1, &s2, &es, &logr);
    if (lane == 0) {
      O.accepted[o] = acc ? 1 : 0;
      O.log_ratio[o] = logr;
      O.energy[o] = es;
      s_acc[f] = acc ? 1 : 0;
      s_s1[f] = s1;
      s_s2[f] = s2;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int j = keff, reflected = 0;
    double coef = 0.0;
    if (!plain) {
      for (int f = 0; f < keff; ++f)
        if (!s_acc[f]) {
          j = f + 1;
          reflected = 1;
          coef = 2.0 * s_s1[f] / s_s2[f];
          break;
        }
    }
    long long* cn = W.counters + (size_t)r * LSD_NCOUNT;
    cn[0] += 1;
    cn[1] += j;
    cn[2] += reflected;
    cn[3] += plain ? 0 : keff;
    cn[4] += rebuild[r];
    O.n_committed[r] = j;
    W.commit_frame[r] = j - 1;
    W.reflected[r] = reflected;
    W.coef[r] = coef;
    S.step[r] = (int64_t)(s0 + (uint64_t)j);
    // the next window decides afresh whether this replica's lists are rebuilt
    rebuild[r] = always_rebuild;
    if (W.ec_samples) W.ec_samples[r] = min(2, W.ec_samples[r] + j);
  }
}

__global__ __launch_bounds__(1024) void k_decide(SysDev S, WinDev W, TileDev Tl, OutDev O, int plain,
                                                 int* __restrict__ rebuild, int always_rebuild) {
  decide_replica(S, W, Tl, O, plain, rebuild, always_rebuild, blockIdx.x);
}

// Commit: the last kept frame's state; a rejected frame takes the reflected
// momentum <p> + Sigma^{1/2} (z - (2 delta.z / delta.delta) delta) and map g.
// With error correction the cache becomes F - F~ of the committed frame,
// from the EC-uncorrected draft force (App. D).
// Returns whether the atom was committed; qc, pc (if given) then hold the
// committed position and momentum.
__device__ __forceinline__ bool commit_atom(const SysDev& S, const WinDev& W, float* q, float* p,
                                            int* img, int plain, int i, float* qc = nullptr,
                                            float* pc = nullptr) {
  if (i >= S.n) return false;
  const int r = S.R == 1 ? 0 : S.atom_rep[i];
  const int sp = S.species ? S.species[i] : 0;
  const size_t N = (size_t)S.n;
  const int f = W.commit_frame[r];
  if (f < 0) return false;  // nothing committed in this window (step limit reached)
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
    const float Fb = W.fd[(size_t)f * 3 * N + d * N + i];
    const float Ft = W.ft[(size_t)f * 3 * N + d * N + i];
    if (refl) {
      const float Fd = draft_mean_force(W, r, d * N + i, f, Fb);
      const double mut = bob_mean(S.a, S.c1fu, pk[d * N + i], Ft);
      const double mud = bob_mean(S.a, S.c1fu, pk[d * N + i], Fd);
      const double z = ((double)pn - mud) * isg;
      const double dl = S.c1fu * ((double)Fd - (double)Ft) * isg;
      pn = (float)fma(sg, z - coef * dl, mut);
    }
    if (S.obabo) {
      // (OBABO) state of this step (App. E): the midpoint, and the momentum
      // after the first (O) half step drawn from its conditional given
      // pbar_{n-1} = pk, pbar_n = pn and the target force F_n there
      const double Fn = (double)(plain ? Fb : Ft);
      const double pprev = (double)pk[d * N + i];
      const double kick = S.hfu * Fn;
      const double shs = S.sh[sp];
      const double w = ((double)pn - S.a * pprev - (1.0 + S.a) * kick) / shs;
      double eta[3];
      stream_normals3(S.seed, (uint32_t)r, (uint64_t)S.step[r], (uint32_t)(i - S.rep_off[r]), eta,
                      LSD_TAG_OB);
      const double x1 = S.cw * w + S.cs * eta[d];
      S.obabo_p[d * N + i] = (float)(S.ah * (pprev + kick) + shs * x1);
      int dz = 0;
      S.obabo_q[d * N + i] = a_half(xs[d], 0.0f, 0.0, L, &dz);  // the midpoint, wrapped
    }
    const float qn = a_half(xs[d], pn, hm, L, &dimg[d]);
    q[d * N + i] = qn;
    p[d * N + i] = pn;
    if (qc) {
      qc[d] = qn;
      pc[d] = pn;
    }
    img[d * N + i] += dimg[d];
    if (W.ec) {
      // the two last committed errors: frames f-1 and f of this window, or
      // the previous cache and frame f
      if (W.ec_prev) {
        const size_t cp = (size_t)(f - 1) * 3 * N + d * N + i;
        W.ec_prev[d * N + i] = f >= 1 ? W.ft[cp] - W.fd[cp] : W.ec[d * N + i];
      }
      W.ec[d * N + i] = Ft - Fb;
    }
  }
  return true;
}

__global__ __launch_bounds__(256) void k_commit(SysDev S, WinDev W, float* __restrict__ q,
                                                float* __restrict__ p, int* __restrict__ img,
                                                int plain) {
  commit_atom(S, W, q, p, img, plain, blockIdx.x * blockDim.x + threadIdx.x);
}

// Commit of one window fused with the start of the next (graph-replayed
// windows): both are per atom, and the start reads only what the same
// thread has just committed.
__global__ __launch_bounds__(256) void k_commit_start(SysDev S, ListDev Lst, WinDev W, float* q,
                                                      float* p, int* img, int plain) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float qc[3], pc[3];
  const bool done = commit_atom(S, W, q, p, img, plain, i, qc, pc);
  // the next window starts from the values just committed (or, where
  // nothing was committed, from the state as it stands)
  window_start_item(S, Lst, W, q, p, i, done ? qc : nullptr, done ? pc : nullptr);
}

// One small system: the decision, the commit and the next window's start in
// one block, since the commit of every atom waits only for the decision of
// its replica.  The barrier after the decision orders its reads of the
// window's flags before the start rewrites them, and its writes (committed
// frame, reflection, step, list flag) before the commit reads them.
__global__ __launch_bounds__(1024) void k_decide_commit_start(SysDev S, ListDev Lst, WinDev W,
                                                              TileDev Tl, OutDev O, float* q,
                                                              float* p, int* img, int plain) {
  decide_replica(S, W, Tl, O, plain, Lst.rebuild, Lst.always_rebuild, 0);
  __syncthreads();
  const int n = S.n > S.kmax ? S.n : S.kmax;
  for (int base = 0; base < n; base += blockDim.x) {  // uniform trip count
    const int i = base + threadIdx.x;
    float qc[3], pc[3];
    const bool done = commit_atom(S, W, q, p, img, plain, i, qc, pc);
    window_start_item(S, Lst, W, q, p, i, done ? qc : nullptr, done ? pc : nullptr);
  }
}

// (OBABO) start (App. E): frame 0 = the given positions q_0 (wrapped), for
// the lists and the target force at q_0.
__global__ __launch_bounds__(256) void k_obabo_frame0(SysDev S, WinDev W, const float* __restrict__ q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const size_t N = (size_t)S.n;
  W.qmid[i] = make_float4(q[i], q[N + i], q[2 * N + i], pack_img(0, 0, 0));
}

// target forces of frame 0 into f_target (pair potentials and the tether)
__global__ __launch_bounds__(256) void k_frame0_forces(SysDev S, ListDev Lst, WinDev W, PotDev P) {
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int i0 = gt / LSD_LPA, sub = gt % LSD_LPA;
  const bool in = i0 < S.n;
  const int i = in ? i0 : S.n - 1;
  float F[3], e;
  pot_force(P, S, W.qmid, Lst.nbr_t + (size_t)i * Lst.mt, Lst.mt, Lst.cnt_t[i], i,
            S.atom_rep[i], sub, F[0], F[1], F[2], e);
  if (!in || sub != 0) return;
  const size_t N = (size_t)S.n;
  W.ft[i] = F[0];
  W.ft[N + i] = F[1];
  W.ft[2 * N + i] = F[2];
}

// The initial OB half step: pbar_0 = e^{-gamma dt/2} p_0 + Sigma_1/2^{1/2} xi
// + dt/2 F(q_0) (xi from tag 3 at the current step); the staggered state is
// kept as the (ABOBA) state whose next midpoint is q_0 + dt pbar_0 / m.
__global__ __launch_bounds__(256) void k_obabo_begin(SysDev S, WinDev W, float* __restrict__ q,
                                                     float* __restrict__ p, int* __restrict__ img) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int r = S.atom_rep[i];
  const int sp = S.species ? S.species[i] : 0;
  const size_t N = (size_t)S.n;
  const double L = S.box[r];
  double xi[3];
  stream_normals3(S.seed, (uint32_t)r, (uint64_t)S.step[r], (uint32_t)(i - S.rep_off[r]), xi,
                  LSD_TAG_OB);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float q0 = q[d * N + i], p0 = p[d * N + i];
    S.obabo_q[d * N + i] = q0;
    S.obabo_p[d * N + i] = p0;
    const float pb = (float)(S.ah * (double)p0 + S.sh[sp] * xi[d] + S.hfu * (double)W.ft[d * N + i]);
    int dimg = 0;
    q[d * N + i] = a_half(q0, pb, S.hdt_m[sp], L, &dimg);
    p[d * N + i] = pb;
    img[d * N + i] += dimg;
  }
}

hipError_t launch_obabo_begin(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P,
                              bool forces_given, float* q, float* p, int* img, hipStream_t st,
                              int stage) {
  if (stage == 0) {
    hipLaunchKernelGGL(k_obabo_frame0, dim3((S.n + 255) / 256), dim3(256), 0, st, S, W, q);
    return hipGetLastError();
  }
  if (!forces_given) {
    const long long threads = (long long)S.n * LSD_LPA;
    hipLaunchKernelGGL(k_frame0_forces, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st,
                       S, L, W, P);
  }
  hipLaunchKernelGGL(k_obabo_begin, dim3((S.n + 255) / 256), dim3(256), 0, st, S, W, q, p, img);
  return hipGetLastError();
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

__global__ void k_zero_i64(long long* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_zero_i64(long long* p, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i64, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

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

hipError_t launch_build_lists(const SysDev& S, const ListDev& L, const WinDev& W, bool caller_frame0,
                              hipStream_t st) {
  if (S.R == 1 && S.n <= NL_SMALL_MAX) {
    hipLaunchKernelGGL(k_nl_small, dim3((S.n + 3) / 4), dim3(256), 0, st, S, L, W,
                       caller_frame0 ? 1 : 0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_rebuild_bin, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S, L, W,
                     caller_frame0 ? 1 : 0);
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, st, L, S.rep_off, S.R);
  hipLaunchKernelGGL(k_cell_fill, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S.n, S.atom_rep, L);
  hipLaunchKernelGGL(k_cell_sort, dim3(L.n_cells), dim3(64), 0, st, L);
  dim3 grid(L.n_cells, (L.cell_cap + NL_IPB - 1) / NL_IPB);
  hipLaunchKernelGGL(k_nl_build, grid, dim3(NL_NT), 0, st, S, L, W);
  return hipGetLastError();
}

hipError_t launch_draft(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                        const PotDev& P, int k, int use_target_list, hipStream_t st,
                        int forces_given) {
  // one kernel per draft kind (each holds only its own force loop)
  const dim3 tiles(S.n_tiles), block(LSD_VTHREADS);
  if (forces_given) {
    hipLaunchKernelGGL((k_draft<LSD_LPA, 1, LSD_KIND_GIVEN>), tiles, block, 0, st, S, L, W, T, P,
                       k, use_target_list);
  } else if (P.kind == LSD_POT_NET) {
    // the learned draft: a small system's latency-bound loop over more
    // lanes per atom and more compute units
    hipLaunchKernelGGL((k_draft<LSD_NET_LPA, LSD_NET_SUB, LSD_POT_NET>),
                       dim3(S.n_tiles * LSD_NET_SUB), dim3(LSD_TILE / LSD_NET_SUB * LSD_NET_LPA), 0,
                       st, S, L, W, T, P, k, use_target_list);
  } else if (P.kind == LSD_POT_LJ) {
    hipLaunchKernelGGL((k_draft<LSD_LPA, 1, LSD_POT_LJ>), tiles, block, 0, st, S, L, W, T, P, k,
                       use_target_list);
  } else if (P.kind == LSD_POT_PAIR) {
    hipLaunchKernelGGL((k_draft<LSD_LPA, 1, LSD_POT_PAIR>), tiles, block, 0, st, S, L, W, T, P, k,
                       use_target_list);
  } else {
    hipLaunchKernelGGL((k_draft<LSD_LPA, 1, 0>), tiles, block, 0, st, S, L, W, T, P, k,
                       use_target_list);
  }
  return hipGetLastError();
}

// One launch for draft steps k0 .. K-1 (k_draft_tail_net, k_draft_tail_pair)
// on one system: the learned draft with the bfloat16 node pass up to
// LSD_TAIL_MAX_ATOMS atoms, or a pair draft.
bool draft_tail_fits(const SysDev& S, const PotDev& P) {
  if (S.R != 1) return false;
  if (P.kind == LSD_POT_NET) return S.n <= LSD_TAIL_MAX_ATOMS && P.prec == 1;
  return P.kind == LSD_POT_LJ || P.kind == LSD_POT_PAIR;
}

hipError_t launch_draft_tail(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                             const PotDev& P, int k0, int use_target_list, hipStream_t st) {
  if (P.kind == LSD_POT_NET) {
    const int node_blocks = (S.n + NET_IROWS - 1) / NET_IROWS;
    hipLaunchKernelGGL(k_draft_tail_net, dim3(node_blocks), dim3(256), 0, st, S, L, W, T, P, k0);
  } else {
    const dim3 grid(S.n_tiles < LSD_TAIL_PAIR_BLOCKS ? S.n_tiles : LSD_TAIL_PAIR_BLOCKS);
    if (P.kind == LSD_POT_LJ)
      hipLaunchKernelGGL(k_draft_tail_pair<LSD_POT_LJ>, grid, dim3(LSD_VTHREADS), 0, st, S, L, W, T,
                         P, k0, use_target_list);
    else
      hipLaunchKernelGGL(k_draft_tail_pair<LSD_POT_PAIR>, grid, dim3(LSD_VTHREADS), 0, st, S, L, W,
                         T, P, k0, use_target_list);
  }
  return hipGetLastError();
}

hipError_t launch_transport(const SysDev& S, const WinDev& W, const TileDev& T, const double* e_rows,
                            int fbeg, int fend, hipStream_t st) {
  if (fend <= fbeg) return hipSuccess;
  hipLaunchKernelGGL(k_transport, dim3(S.n_tiles, fend - fbeg), dim3(64), 0, st, S, W, T, e_rows,
                     fbeg);
  return hipGetLastError();
}

hipError_t launch_decide_group(const SysDev& S, const WinDev& W, const TileDev& T, int fbeg,
                               int fend, hipStream_t st) {
  const int n = fend - fbeg;
  if (n <= 0) return hipSuccess;
  const int waves = n < 16 ? n : 16;
  hipLaunchKernelGGL(k_decide_group, dim3(S.R), dim3(64 * waves), 0, st, S, W, T, fbeg, fend);
  return hipGetLastError();
}

hipError_t launch_frame_validity(const SysDev& S, const ListDev& L, const WinDev& W,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_frame_validity, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S, L, W);
  return hipGetLastError();
}

// frames per wave: up to LSD_VERIFY_FW_MAX (chosen per window length by the
// caller or the autotuner)
#ifndef LSD_VERIFY_FW_MAX
#define LSD_VERIFY_FW_MAX 8
#endif

// Blocks of the verification grid: every item of a window whose frames are
// all valid, up to about the blocks the GPU holds at once at full occupancy
// (256 CUs x 8 blocks of four waves); beyond that the blocks loop over the
// items.  Items past the window's valid frames launch no block of their own.
#ifndef LSD_VERIFY_MAX_BLOCKS
#define LSD_VERIFY_MAX_BLOCKS 2048
#endif

hipError_t launch_verify(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                         const PotDev& P, int fw, int fbeg, int fend, hipStream_t st) {
  if (fend <= fbeg) return hipSuccess;
  if (fw > LSD_VERIFY_FW_MAX) fw = LSD_VERIFY_FW_MAX;
  fw = fw >= 8 ? 8 : (fw >= 4 ? 4 : (fw == 2 ? 2 : 1));
  const long all_items = (long)S.n_tiles * ((fend - fbeg + fw - 1) / fw);
  const long cap = LSD_VERIFY_MAX_BLOCKS > S.n_tiles ? LSD_VERIFY_MAX_BLOCKS : S.n_tiles;
  const dim3 grid((unsigned)(all_items < cap ? all_items : cap));
  if (fw == 8) {
    hipLaunchKernelGGL(k_verify<8>, grid, dim3(LSD_VTHREADS), 0, st, S, L, W, T, P, fbeg, fend);
  } else if (fw == 4) {
    hipLaunchKernelGGL(k_verify<4>, grid, dim3(LSD_VTHREADS), 0, st, S, L, W, T, P, fbeg, fend);
  } else if (fw == 2) {
    hipLaunchKernelGGL(k_verify<2>, grid, dim3(LSD_VTHREADS), 0, st, S, L, W, T, P, fbeg, fend);
  } else {
    hipLaunchKernelGGL(k_verify<1>, grid, dim3(LSD_VTHREADS), 0, st, S, L, W, T, P, fbeg, fend);
  }
  return hipGetLastError();
}

hipError_t launch_decide(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                         const OutDev& O, int plain, hipStream_t st) {
  // one wave per frame up to 16 waves
  const int waves = plain ? 1 : (W.K < 16 ? W.K : 16);
  hipLaunchKernelGGL(k_decide, dim3(S.R), dim3(64 * waves), 0, st, S, W, T, O, plain, L.rebuild,
                     L.always_rebuild);
  return hipGetLastError();
}

// Decision, commit and the next window's start: one block for one small
// system, else one launch per step.
#ifndef LSD_FUSED_COMMIT_MAX
#define LSD_FUSED_COMMIT_MAX 1024
#endif
hipError_t launch_decide_commit_start(const SysDev& S, const ListDev& L, const WinDev& W,
                                      const TileDev& T, const OutDev& O, float* q, float* p,
                                      int* img, int plain, hipStream_t st) {
  if (S.R == 1 && S.n <= LSD_FUSED_COMMIT_MAX) {
    hipLaunchKernelGGL(k_decide_commit_start, dim3(1), dim3(1024), 0, st, S, L, W, T, O, q, p, img,
                       plain);
    return hipGetLastError();
  }
  hipError_t e = launch_decide(S, L, W, T, O, plain, st);
  if (e != hipSuccess) return e;
  return launch_commit_start(S, L, W, q, p, img, plain, st);
}

hipError_t launch_commit_start(const SysDev& S, const ListDev& L, const WinDev& W, float* q,
                               float* p, int* img, int plain, hipStream_t st) {
  const int n = S.n > S.R * S.kmax ? S.n : S.R * S.kmax;
  hipLaunchKernelGGL(k_commit_start, dim3(blocks_for(n, 256)), dim3(256), 0, st, S, L, W, q, p,
                     img, plain);
  return hipGetLastError();
}

hipError_t launch_commit(const SysDev& S, const WinDev& W, float* q, float* p, int* img,
                         int plain, hipStream_t st) {
  hipLaunchKernelGGL(k_commit, dim3(blocks_for(S.n, 256)), dim3(256), 0, st, S, W, q, p, img,
                     plain);
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
