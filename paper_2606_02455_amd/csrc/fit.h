// fit.h -- force matching of the pair draft (normal equations on the GPU).
#pragma once
#include <hip/hip_runtime.h>

#include "lsd_device.h"

#define FIT_MAX_LP 64  // species x basis columns of one atom's design rows

struct FitDev {
  float rc2, pi_rc;  // fit cutoff squared, pi / cutoff
  int nb, ns;        // basis functions, species
  int LP;            // ns * nb
};

// Entries of one tile's partial normal equations: ns LP^2 + ns LP.
size_t fit_partial_entries(const FitDev& F);

// Adds the normal equations of the window's valid frames (positions q_mid,
// forces f_target if use_target else f_draft) to gram[(P+1)][(P+1)]; with
// diff, of the differences between consecutive valid frames instead.
// partial: n_tiles * fit_partial_entries doubles of scratch.
hipError_t launch_fit(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                      const FitDev& F, int use_target, int diff, double* partial, double* gram,
                      hipStream_t st);
