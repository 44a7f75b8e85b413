// lsd_launch.h -- host-side launchers of the LSD kernels (lsd_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "lsd_device.h"

hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st);
hipError_t launch_zero_i64(long long* p, int n, hipStream_t st);
hipError_t launch_window_start(const SysDev& S, const ListDev& L, const WinDev& W, const float* q,
                               const float* p, hipStream_t st);
// Rebuilds the cell and neighbour lists of the replicas flagged for it, from
// the wrapped first midpoints or (caller_frame0) from the caller's frame 0.
hipError_t launch_build_lists(const SysDev& S, const ListDev& L, const WinDev& W, bool caller_frame0,
                              hipStream_t st);
hipError_t launch_draft(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                        const PotDev& P, int k, int use_target_list, hipStream_t st,
                        int forces_given = 0);
// transport-map sums of frames [fbeg, fend) whose target forces are in the
// window; e_rows: energy per row of those frames, [f - fbeg][N]
hipError_t launch_transport(const SysDev& S, const WinDev& W, const TileDev& T, const double* e_rows,
                            int fbeg, int fend, hipStream_t st);
hipError_t launch_frame_validity(const SysDev& S, const ListDev& L, const WinDev& W,
                                 hipStream_t st);
// verification of frames [fbeg, fend) with fw frames per wave
hipError_t launch_verify(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                         const PotDev& P, int fw, int fbeg, int fend, hipStream_t st);
// decisions of frames [fbeg, fend) of a pipelined window; records the first rejection
hipError_t launch_decide_group(const SysDev& S, const WinDev& W, const TileDev& T, int fbeg,
                               int fend, hipStream_t st);
hipError_t launch_decide(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                         const OutDev& O, int plain, hipStream_t st);
// decision, commit of the window and start of the next one (one launch for a
// single small system, else launch_decide then launch_commit_start)
hipError_t launch_decide_commit_start(const SysDev& S, const ListDev& L, const WinDev& W,
                                      const TileDev& T, const OutDev& O, float* q, float* p,
                                      int* img, int plain, hipStream_t st);
// draft steps k0 .. K-1 in one launch, for the systems draft_tail_fits
// admits (one system: the learned draft with the bfloat16 node pass up to
// LSD_TAIL_MAX_ATOMS atoms, or a pair draft)
#define LSD_TAIL_MAX_ATOMS 2048
bool draft_tail_fits(const SysDev& S, const PotDev& P);
hipError_t launch_draft_tail(const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
                             const PotDev& P, int k0, int use_target_list, hipStream_t st);
// commit of the window and start of the next one in one launch
hipError_t launch_commit_start(const SysDev& S, const ListDev& L, const WinDev& W, float* q,
                               float* p, int* img, int plain, hipStream_t st);
hipError_t launch_commit(const SysDev& S, const WinDev& W, float* q, float* p, int* img,
                         int plain, hipStream_t st);
// (OBABO) start: stage 0 writes the given positions as frame 0; stage 1
// (after the lists are built and, for the network, its forces are in
// f_target) computes the target forces there unless given and applies the
// initial OB half step to (q, p, img).
hipError_t launch_obabo_begin(const SysDev& S, const ListDev& L, const WinDev& W, const PotDev& P,
                              bool forces_given, float* q, float* p, int* img, hipStream_t st,
                              int stage);
hipError_t launch_rng_normals(uint64_t seed, int replica, int64_t step, int n, double* out,
                              hipStream_t st);
hipError_t launch_rng_uniforms(uint64_t seed, int replica, int64_t step0, int count, double* out,
                               hipStream_t st);
