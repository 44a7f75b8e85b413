// mpnn.h -- batched evaluation of the message-passing target on K frames.
//
// Rows are (frame, atom) pairs, row = f_local * N + i; edges are the list
// entries of a row inside the cutoff, compacted row by row in list order
// (capacity: rows x list width).  The dense
// contractions (the per-slot filter MLP 128 -> 128 of every layer, and the
// per-row node MLPs) run as FP32 GEMMs; every gather, activation, reduction
// and the reverse pass to the forces are kernels in mpnn.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include "lsd_device.h"

#define MP_H 128
#define MP_R 16
#define MP_T 3
#define MP_RH 64
#define MP_HT (MP_H * MP_T)  // filter channels of all layers side by side

struct MpnnWeights {
  const float* W_emb;
  const float *A1[MP_T], *a1[MP_T], *A2[MP_T], *a2[MP_T], *B[MP_T], *C1[MP_T], *c1[MP_T];
  const float *C2[MP_T], *c2[MP_T];
  const float *W1, *b1, *w2, *b2;
  long layer_stride;  // floats between consecutive layers' blocks
};

struct MpnnBuffers {
  // per unordered pair (capacity slots / 4 + 1)
  float *S, *DS, *Z, *DZ;  // [pairs][384]
  float* fcd;              // [pairs][2]  f_c, f_c'
  float* uv;               // [pairs][4]  unit vector from the owner row, distance
  float* gr;               // [pairs]     dE/dr summed over both directions and layers
  int *ua, *ub;            // [pairs]     owner row, neighbour row
  // per directed edge (capacity slots = rows x list width)
  int* off;                // [rows+1]    first edge of every (frame, atom) row
  int* erow;               // [slots]     row of an edge's atom
  int* enbr;               // [slots]     row of an edge's neighbour
  int* ecode;              // [slots]     image code of the edge
  int* uid;                // [slots]     pair of the edge: p (owner) or ~p (reverse)
  int* poff;               // [rows+1]    first pair owned by every row
  int* counts;             // [4]         directed edges, pairs, error flag
  float* H;                // [T+1][rows][128]
  float* X;                // [T][rows][128]
  float* U;                // [T][rows][128]
  float *Mm, *Sn;          // [rows][128]
  float *Y, *gY;           // [rows][64]
  float *gH, *gP, *gS, *gM, *gX;  // [rows][128]
};

struct MpnnCtx {
  MpnnWeights w;
  MpnnBuffers b;
  float rc, scale;
  int frames;  // frames per evaluation (buffer capacity)
  rocblas_handle blas = nullptr;
};

// Bytes of the buffers for `frames` frames of N atoms with list width mt.
size_t mpnn_buffer_bytes(int frames, int n, int mt);
// Carves the buffers out of `base` (256-byte aligned) and sets weight views.
void mpnn_bind(MpnnCtx& M, char* base, int frames, int n, int mt, const float* weights,
               int n_model_species);
// Energies (per frame and tile, binary64, into epart[(f0+f) * n_tiles + tile])
// and forces (frame-major [f0+f][3][N] into Fout) of frames f0 .. f0+nf-1.
// Returns false and a message in err on a HIP or rocBLAS failure.
bool mpnn_eval(MpnnCtx& M, const SysDev& S, const ListDev& L, const WinDev& W, const TileDev& T,
               int f0, int nf, float* Fout, double* epart, hipStream_t st, char* err,
               size_t errlen);
