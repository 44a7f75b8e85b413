// kinetic.hip -- kinetic energy per replica in binary64.
//
// The thermostat observable of Sec. 4.3 (Tab. heating): the kinetic
// temperature T_kin = 2 K / (3 N k_B) of each replica is formed from
// K = sum_i |p_i|^2 / (2 m_i).  The momenta are binary32 (the committed
// state); every square is exact in binary64 and everything after it is
// binary64, summed in a fixed order so that results are reproducible bit for
// bit:
//   pass 1: block (chunk c, replica r) sums the atoms
//           off[r] + c * kChunk + t + 256 m (m = 0, 1, ...) per thread t in
//           order, then a wave butterfly, then its four waves in order, into
//           partial[r][c] (zero for chunks past the replica's end);
//   pass 2: one wave per replica sums partial[r][lane + 64 m] in order, then
//           a butterfly.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "lsd.h"
#include "lsd_device.h"

lsd_status lsd_record_error(lsd_status s, const char* msg);  // lsd_api.hip

// Partial sums of lsd_kinetic_energy_noalloc: a static array, one copy per
// GPU, shared by every call on that GPU (calls that overlap on one GPU race).
// Host code never passes the array's name to a kernel (in host code it is a
// stand-in, not a device address): it uses the address hipGetSymbolAddress
// returns for the current device.
#define LSD_KE_NOALLOC_PARTIALS 65536  // replicas x chunks (512 KiB)
static __device__ __align__(256) double scratch[LSD_KE_NOALLOC_PARTIALS];

namespace {

constexpr int kKeThreads = 256;
constexpr int kChunk = 2048;  // atoms per pass-1 block

struct KeMass {
  double inv2m[LSD_MAX_SPECIES];  // 1 / (2 m) per species
};

__global__ __launch_bounds__(kKeThreads) void k_ke_partial(const float* __restrict__ p, long n,
                                                           const int* __restrict__ species,
                                                           KeMass M, const int* __restrict__ off,
                                                           int chunks, double* __restrict__ part) {
  __shared__ double s_w[kKeThreads / 64];
  const int c = blockIdx.x, r = blockIdx.y, t = threadIdx.x;
  const int lo = off[r], hi = off[r + 1];
  const long a0 = (long)lo + (long)c * kChunk;
  double acc = 0.0;
  for (int m = 0; m < kChunk / kKeThreads; ++m) {
    const long i = a0 + t + (long)m * kKeThreads;
    if (i >= hi) break;
    const double w = M.inv2m[species ? species[i] : 0];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double v = (double)p[d * n + i];
      acc += (v * v) * w;
    }
  }
  acc = wave_sum(acc);
  if ((t & 63) == 0) s_w[t >> 6] = acc;
  __syncthreads();
  if (t == 0) {
    double s = s_w[0];
    for (int q = 1; q < kKeThreads / 64; ++q) s += s_w[q];
    part[(size_t)r * chunks + c] = s;
  }
}

__global__ __launch_bounds__(64) void k_ke_final(const double* __restrict__ part, int chunks,
                                                 const int* __restrict__ off,
                                                 double* __restrict__ ke) {
  const int r = blockIdx.x, lane = threadIdx.x;
  double acc = 0.0;
  for (int c = lane; c < chunks; c += 64) acc += part[(size_t)r * chunks + c];
  acc = wave_sum(acc);
  if (lane == 0) {
    // a replica larger than the chunks cover was only partly summed
    const long size = (long)off[r + 1] - (long)off[r];
    ke[r] = size <= (long)chunks * kChunk ? acc : NAN;
  }
}

int ke_chunks(int max_replica_atoms) {
  return max_replica_atoms <= 0 ? 1 : (max_replica_atoms + kChunk - 1) / kChunk;
}

lsd_status ke_check(const float* p, int n_atoms, const double* species_mass, int n_species,
                    const int* atom_offsets, int n_replicas, int max_replica_atoms, double* ke,
                    KeMass* M) {
  if (!p || !species_mass || !atom_offsets || !ke)
    return lsd_record_error(LSD_ERR_INVALID_ARG, "kinetic energy: null argument");
  if (n_atoms < 0 || n_replicas < 1 || max_replica_atoms < 0 || max_replica_atoms > n_atoms)
    return lsd_record_error(LSD_ERR_INVALID_ARG, "kinetic energy: bad atom or replica count");
  if (n_replicas > 65535)
    return lsd_record_error(LSD_ERR_INVALID_ARG, "kinetic energy: more than 65535 replicas");
  if (n_species < 1 || n_species > LSD_MAX_SPECIES)
    return lsd_record_error(LSD_ERR_INVALID_ARG, "kinetic energy: n_species outside 1..8");
  for (int s = 0; s < LSD_MAX_SPECIES; ++s) {
    const double m = species_mass[s < n_species ? s : 0];
    if (!(m > 0.0) || !std::isfinite(m))
      return lsd_record_error(LSD_ERR_INVALID_ARG, "kinetic energy: masses must be positive");
    M->inv2m[s] = 1.0 / (2.0 * m);
  }
  return LSD_OK;
}

lsd_status ke_launch(const float* p, int n_atoms, const int* species, const KeMass& M,
                     const int* atom_offsets, int n_replicas, int chunks, double* ke,
                     double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_ke_partial, dim3((unsigned)chunks, (unsigned)n_replicas), dim3(kKeThreads),
                     0, st, p, (long)n_atoms, species, M, atom_offsets, chunks, part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_ke_final, dim3((unsigned)n_replicas), dim3(64), 0, st, part, chunks,
                       atom_offsets, ke);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return lsd_record_error(LSD_ERR_HIP, hipGetErrorString(e));
  return LSD_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
lsd_status noalloc_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lsd_record_error(LSD_ERR_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return lsd_record_error(LSD_ERR_UNSUPPORTED, "kinetic energy: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return lsd_record_error(LSD_ERR_HIP, e != hipSuccess ? hipGetErrorString(e)
                                                           : "kinetic energy: null scratch address");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return LSD_OK;
}

}  // namespace

extern "C" {

lsd_status lsd_kinetic_energy_scratch_size(int32_t n_replicas, int32_t max_replica_atoms,
                                           size_t* bytes) {
  if (!bytes || n_replicas < 1 || max_replica_atoms < 0)
    return lsd_record_error(LSD_ERR_INVALID_ARG, "kinetic energy scratch size: bad argument");
  *bytes = (size_t)n_replicas * (size_t)ke_chunks(max_replica_atoms) * sizeof(double);
  return LSD_OK;
}

lsd_status lsd_kinetic_energy(const float* p, int32_t n_atoms, const int32_t* species,
                              const double* species_mass, int32_t n_species,
                              const int32_t* atom_offsets, int32_t n_replicas,
                              int32_t max_replica_atoms, double* ke, void* scratch,
                              size_t scratch_bytes, lsd_stream stream) {
  KeMass M;
  lsd_status s = ke_check(p, n_atoms, species_mass, n_species, atom_offsets, n_replicas,
                          max_replica_atoms, ke, &M);
  if (s != LSD_OK) return s;
  const int chunks = ke_chunks(max_replica_atoms);
  const size_t need = (size_t)n_replicas * (size_t)chunks * sizeof(double);
  if (!scratch || scratch_bytes < need)
    return lsd_record_error(LSD_ERR_CAPACITY, "kinetic energy: scratch smaller than "
                                              "lsd_kinetic_energy_scratch_size");
  return ke_launch(p, n_atoms, species, M, atom_offsets, n_replicas, chunks, ke,
                   static_cast<double*>(scratch), static_cast<hipStream_t>(stream));
}

lsd_status lsd_kinetic_energy_noalloc(const float* p, int32_t n_atoms, const int32_t* species,
                                      const double* species_mass, int32_t n_species,
                                      const int32_t* atom_offsets, int32_t n_replicas,
                                      int32_t max_replica_atoms, double* ke, lsd_stream stream) {
  KeMass M;
  lsd_status s = ke_check(p, n_atoms, species_mass, n_species, atom_offsets, n_replicas,
                          max_replica_atoms, ke, &M);
  if (s != LSD_OK) return s;
  const int chunks = ke_chunks(max_replica_atoms);
  if ((long)n_replicas * (long)chunks > LSD_KE_NOALLOC_PARTIALS)
    return lsd_record_error(LSD_ERR_CAPACITY,
                            "kinetic energy (no allocation): n_replicas x ceil(max_replica_atoms"
                            " / 2048) exceeds 65536");
  double* part = nullptr;
  s = noalloc_scratch(&part);
  if (s != LSD_OK) return s;
  // pass 1 writes every partial it covers (zero past a replica's end), so
  // nothing left by an earlier call is read
  return ke_launch(p, n_atoms, species, M, atom_offsets, n_replicas, chunks, ke, part,
                   static_cast<hipStream_t>(stream));
}

}  // extern "C"
