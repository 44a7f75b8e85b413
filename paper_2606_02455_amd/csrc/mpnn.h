// mpnn.h -- batched evaluation of the message-passing target on K frames.
//
// Rows are (frame, atom) pairs, row = f_local * N + i; edges are the list
// entries of a row inside the cutoff, compacted row by row in list order
// (capacity: rows x list width).  The dense contractions (the per-pair filter
// MLP 128 -> 128 of every layer and its r-derivative, and the per-row node
// MLPs) run on the matrix cores as bfloat16 hi/lo splits with binary32
// accumulation; every gather, activation, reduction and the reverse pass to
// the forces are kernels in mpnn.hip.  The counts of edges and pairs stay on
// the device: an evaluation has no host synchronisation and can be captured
// in a graph.
#pragma once
#include <hip/hip_runtime.h>

#include "lsd_device.h"

#define MP_H 128
#define MP_R 16
#define MP_T 3
#define MP_RH 64
#define MP_HT (MP_H * MP_T)  // filter channels of all layers side by side


// bfloat16 hi/lo fragments of a weight matrix, laid out for the operands of
// v_mfma_f32_16x16x32_bf16 (8 values per lane, 16 bytes): element
// [tile][k-step][lane] of hi and of lo
struct MpnnFrag {
  const uint4* hi;
  const uint4* lo;
};

struct MpnnBuffers {
  // per unordered pair (capacity: slots / 4 + 1)
  float *Wf, *Vf;          // [pairs][T][128]  filter W and dW/dr of every layer
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
  int* counts;             // [4]         directed edges, pairs, error flags
  int* tile_sums;          // [tiles][2]  scan of large evaluations: totals per tile of rows
  float* H;                // [T+1][rows][128]
  float* X;                // [T][rows][128]
  float* U;                // [T][rows][128]
  float* Mm;               // [rows][128]  messages of the current layer
  double* Erow;            // [rows]       energy of every row (s_E times its readout)
  float *gH, *gP, *gM, *gX;  // [rows][128]
  // weight fragments (written once by mpnn_prepare)
  uint4* frag;             // all fragment arrays below, contiguous
};

struct MpnnWeights {
  const float* W_emb;
  const float *A1[MP_T], *a1[MP_T], *A2[MP_T], *a2[MP_T], *B[MP_T], *C1[MP_T], *c1[MP_T];
  const float *C2[MP_T], *c2[MP_T];
  const float *W1, *b1, *w2, *b2;
  long layer_stride;  // floats between consecutive layers' blocks
  // A2 of each layer as the first operand of the filter product (channels x
  // inputs); the node matrices as the second operand, forward (W^T) and
  // reverse (W): out[row][n] = sum_k in[row][k] op[k][n]
  MpnnFrag A1f[MP_T];  // A1 [128][16] as the first operand, contraction padded to 32
  MpnnFrag A2f[MP_T];
  MpnnFrag Bf[MP_T], C1f[MP_T], C2f[MP_T];   // forward: B^T, C1^T, C2^T
  MpnnFrag Bb[MP_T], C1b[MP_T], C2b[MP_T];   // reverse: B, C1, C2
  MpnnFrag W1f, W1b;                          // W1^T (128 -> 64), W1 (64 -> 128)
};

// Launch shapes of an evaluation (they change no result: every pair and row
// is computed the same way whichever block takes it)
#define MP_TUNE_CANDIDATES 9  // filter blocks {256, 512, 1024} x chain rows {16, 32, 64}

struct MpnnCtx {
  MpnnWeights w;
  MpnnBuffers b;
  float rc, scale;
  int frames;  // frames per evaluation (buffer capacity)
  long pair_cap;
  unsigned filt_blocks = 512;  // blocks of the filter kernel (two per compute unit)
  int chain_nt = 0;            // row tiles of 16 per chain block; 0: from the row count
};

// Candidate c of the evaluation's launch shapes (0 <= c < MP_TUNE_CANDIDATES).
void mpnn_set_shape(MpnnCtx& M, int c);

// Bytes of the buffers for `frames` frames of N atoms with list width mt.
size_t mpnn_buffer_bytes(int frames, int n, int mt);
// Carves the buffers out of `base` (256-byte aligned) and sets weight views.
void mpnn_bind(MpnnCtx& M, char* base, int frames, int n, int mt, const float* weights,
               int n_model_species);
// Writes the weight fragments (once, after mpnn_bind).
bool mpnn_prepare(MpnnCtx& M, hipStream_t st, char* err, size_t errlen);
// Forces (frame-major [f0+f][3][N] into Fout) of frames f0 .. f0+nf-1, and
// the energy of every row (frame f0+f, atom i) in b.Erow[f N + i] (binary64).
// Asynchronous on `st`, no host synchronisation; a pair count above the
// capacity or inconsistent edge lists are latched in the status word
// (LSD_STATUS_PAIRS, LSD_STATUS_EDGES).  Returns false and a message in err
// on a launch failure.
// Frames past the device bound nvalid (a window's valid frames; nullptr: all
// nf) and frames flagged invalid are not evaluated (no edges; their forces
// and energies are left as they were).
bool mpnn_eval(MpnnCtx& M, const SysDev& S, const ListDev& L, const WinDev& W, int f0, int nf,
               const int* nvalid, float* Fout, hipStream_t st, char* err, size_t errlen);
