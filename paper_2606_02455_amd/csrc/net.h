// net.h -- the learned many-body draft: the per-frame node pass that feeds
// drafting (descriptor and dense layers), and force-matching training (loss
// gradient in binary32 with binary64 reductions, Adam).
#pragma once
#include <hip/hip_runtime.h>

#include "lsd_device.h"

#define NET_ROWS 64  // atoms per block of the node and training kernels
// parameter slots of a training partial row (S <= 4 species, so <= 10 pair
// types), then the squared error and the atom-frame count
#define NET_PMAX                                                                 \
  (LSD_NET_HIDDEN * LSD_NET_MAX_DESC + LSD_NET_MAX_SPECIES * LSD_NET_HIDDEN + \
   LSD_NET_MAX_BASIS * LSD_NET_HIDDEN + 10 * LSD_NET_MAX_BASIS)
#define NET_PROW (NET_PMAX + 2)

struct NetTrainDev {
  float* D;         // [K][N][LSD_NET_MAX_DESC] descriptors
  float* z;         // [K][N][LSD_NET_HIDDEN] pre-activations
  float* v;         // [K][N][LSD_NET_MAX_BASIS] edge coefficients
  float* G;         // [K][3][N] dSSE/dF
  float* F;         // [K][3][N] forces (loss of force changes)
  double* partial;  // [K][nblk][NET_PROW]
  int nblk;
};

size_t net_train_bytes(int K, int N);
NetTrainDev net_train_bind(char* base, int K, int N);

// Edge coefficients P.v of frame k of the window (draft list).
hipError_t launch_net_nodes(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P,
                            int k, hipStream_t st);

// grad[0..P) += d/dtheta sum |F - y|^2 over the window's valid frames,
// grad[P] += the squared error, grad[P+1] += atom frames (target list);
// diff: the loss of the changes between consecutive valid frames.
hipError_t launch_net_train(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P,
                            const NetTrainDev& T, int use_target, int diff, double* grad,
                            hipStream_t st);

// amax[0] = max |D|, amax[1] = max |silu(z)| over the window's valid frames.
hipError_t launch_net_amax(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P,
                           const NetTrainDev& T, double* amax, hipStream_t st);

hipError_t launch_net_adam(float* params, double* m, double* v, double* grad, int n_params,
                           double lr, double beta1, double beta2, double eps, long long t,
                           hipStream_t st);
