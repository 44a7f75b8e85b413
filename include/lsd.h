/*
 * lsd.h -- C ABI of the MI355X (gfx950) batched-verification library for
 * Langevin Speculative Dynamics (LSD).
 *
 * Paper: A. Kosmala, S. Guennemann, M. Gao, B. Wood, "Speculative Sampling
 * For Faster Molecular Dynamics", arXiv 2606.02455.
 *
 * What the library computes (one GPU, R independent replicas batched):
 *   - lsd_draft_steps     : the draft_step procedure of Alg. 2, K times in a
 *                           row: A half step, draft forces, the (BOB)
 *                           Gaussian draw of Eq. bob, A half step (Eq. aboba).
 *   - lsd_verify_window   : verify_step of Alg. 2 for all K drafted frames in
 *                           ONE launch: target forces at every midpoint, the
 *                           target mean of Eq. bob, and the log density ratio
 *                           of Eq. reflectionVerify reduced in binary64.
 *   - lsd_accept_rollback : accept/reject of Eq. reflectionVerify with
 *                           u ~ U(0,1], first rejection of the window (Alg. 1),
 *                           reflection of the rejected momentum, map g of
 *                           Thm. 1, and commit of the kept prefix; everything
 *                           after the first rejection is discarded (rollback).
 *   In LSD_MODE_PLAIN the same kernels run plain target Langevin (ABOBA with
 *   target forces): verify is a no-op and every drafted step is committed.
 *
 * Conventions
 *   - All array arguments are DEVICE pointers unless marked "host".  Device
 *     memory is owned by the caller (e.g. PyTorch tensors); after
 *     lsd_init_system the library allocates no device memory: its scratch
 *     lives in the caller's workspace of lsd_workspace_size() bytes.
 *   - Positions, momenta, forces: binary32, structure-of-arrays [3][N]
 *     (x of all atoms, then y, then z).  Atoms of replica r are the index
 *     range [atom_offsets[r], atom_offsets[r+1]).
 *   - Cubic periodic boxes; positions are kept wrapped in [0, L_r) with
 *     int32 image counters.  Box edges must be binary32-representable and
 *     larger than (target cutoff + skin).
 *   - Units: force_unit converts force*time to momentum and energy to
 *     mass*length^2/time^2 (1.0 in Lennard-Jones reduced units;
 *     9.648533212331e-3 for eV, Angstrom, amu, fs).
 *   - Random numbers: Philox4x32-10 keyed by seed and counter (local atom
 *     index, simulation step n, replica, tag).  Step n (the step being
 *     produced) keys both the noise xi of Eq. aboba and the uniform u of
 *     Eq. reflectionVerify, so a window of any length K commits the same
 *     trajectory.  Tests may replace the stream by replay arrays.
 *   - Every call is asynchronous on the given stream (a hipStream_t; NULL is
 *     the default stream) unless it says it synchronises.
 *   - Errors: every call returns an lsd_status; nothing is thrown across the
 *     ABI.  lsd_last_error() describes the last failure of the calling
 *     thread.  Device-side capacity overflows are latched in a status word
 *     read by lsd_get_status().
 */
#ifndef LSD_H
#define LSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define LSD_API __attribute__((visibility("default")))
#else
#define LSD_API
#endif

typedef struct lsd_system lsd_system; /* opaque, host-side handle */
typedef void *lsd_stream;             /* hipStream_t */

typedef enum {
  LSD_OK = 0,
  LSD_ERR_INVALID_ARG = -1, /* bad size, pointer or parameter */
  LSD_ERR_BAD_STATE = -2,   /* calls out of order (draft -> verify -> accept) */
  LSD_ERR_HIP = -3,         /* a HIP runtime call failed */
  LSD_ERR_CAPACITY = -4,    /* workspace too small / neighbour list overflow */
  LSD_ERR_UNSUPPORTED = -5  /* valid request this build does not implement */
} lsd_status;

typedef enum { LSD_MODE_LSD = 0, LSD_MODE_PLAIN = 1 } lsd_mode;

/* Integrator (Sec. 2.1, App. E).  ABOBA: the committed state is (q, p) of
 * Eq. aboba.  OBABO: LSD runs in the staggered frame of App. E (the ABOBA
 * chain read at its midpoints, which is the staggered (OBABO) chain); on init
 * buf.q/buf.p hold the (OBABO) state y_0, the library applies the initial OB
 * half step (target force at q_0, (O) noise from stream tag 3 at the current
 * step) and keeps its own staggered state in q/p/img from then on; after
 * every window the (OBABO) state of the last committed step is written to
 * buf.obabo_q/obabo_p: its midpoint positions (wrapped) and the momentum
 * recovered by the conditional half step of Eq. obabo_conditional (noise
 * from stream tag 3 at that step). */
typedef enum { LSD_INTEGRATOR_ABOBA = 0, LSD_INTEGRATOR_OBABO = 1 } lsd_integrator;

typedef enum {
  LSD_POT_LJ = 1,       /* truncated, energy-shifted Lennard-Jones */
  LSD_POT_HARMONIC = 2, /* tether U = k/2 |q - anchor|^2 (minimum image) */
  LSD_POT_MPNN = 3,     /* message-passing network (target only), below */
  LSD_POT_PAIR = 4,     /* force-matched pair draft (draft only), below */
  LSD_POT_NET = 5       /* learned many-body draft (draft only), below */
} lsd_pot_kind;

/* Pair-force draft (the fallback of a learned draft: a potential lighter
 * than the target, fitted to its forces; LSD admits any draft, Sec. 3).
 * Central force per unordered species pair t = {s_i, s_j}:
 *   F_i = - sum_(j, image) f_t(r) d / r,  d = q_j + n L - q_i, r = |d| < rc,
 *   f_t(r) = (cos(pi r/rc) + 1)/2 * sum_{b=1..B} w[t][b-1] sin(b pi r/rc) / r,
 * with types ordered (0,0), (0,1), .., (0,S-1), (1,1), .. (S = n_model_species,
 * S(S+1)/2 types).  Weights: device binary32 [S(S+1)/2][B], kept by pointer.
 * Forces only: the draft energy is never needed.  The weights come from
 * force matching: lsd_fit_pair_accumulate / lsd_fit_pair_solve. */
#define LSD_PAIR_MAX_BASIS 32

/* Learned many-body draft (Sec. 3, Sec. 4: the drafts are small learned
 * potentials fitted to the target's forces that predict forces directly; a
 * non-conservative draft is admissible because verification corrects its
 * samples).  A one-layer direct-force network over a species-resolved radial
 * descriptor, H = LSD_NET_HIDDEN hidden units, S species, B radial functions:
 *   e_b(r) = (cos(pi r/rc) + 1)/2 sin(b pi r/rc) / r,  b = 1..B, r < rc
 *   D_i    = sum_(j, image) e(r_ij) placed in the block of species s_j (S B)
 *   h_i    = silu(W1 D_i + b1[s_i]),   v_i = W2 h_i   (B edge coefficients)
 *   f_ij   = sum_b e_b(r_ij) (c[t(s_i, s_j)][b] + v_i[b] + v_j[b])
 *   F_i    = - sum_(j, image) f_ij d / r,  d = q_j + n L - q_i
 * f_ij is symmetric, so the forces obey Newton's third law; with W2 = 0 the
 * draft is the pair draft above with weights c.  Parameters: one flat device
 * binary32 vector kept by pointer (training may update it between windows),
 * matrices [out][in]: W1 [H][S B], b1 [S][H], W2 [B][H], c [S(S+1)/2][B];
 * lsd_net_param_count gives its length.  S = n_model_species (<= 4), B =
 * n_basis (1 .. LSD_NET_MAX_BASIS), S B <= LSD_NET_MAX_DESC.  precision:
 * LSD_PREC_FP32 evaluates the two dense layers in binary32 on the vector
 * ALUs; LSD_PREC_BF16 on the matrix cores with D, h, W1 and W2 rounded to
 * bfloat16 and binary32 accumulation; LSD_PREC_FP8 on the matrix cores in
 * OCP e4m3 with one scale per tensor and binary32 accumulation: W1 and W2
 * are divided by max|W| / 448 (computed from the parameters), D and h by
 * act_amax[0] / 448 and act_amax[1] / 448 (static scales calibrated by
 * lsd_net_activation_amax; larger values saturate at +-448), and the
 * products are scaled back.  Pair terms are binary32 in every mode. */
#define LSD_NET_HIDDEN 32
#define LSD_NET_MAX_BASIS 16
#define LSD_NET_MAX_DESC 64
#define LSD_NET_MAX_SPECIES 4
typedef enum { LSD_PREC_FP32 = 0, LSD_PREC_BF16 = 1, LSD_PREC_FP8 = 2 } lsd_precision;

/* Message-passing potential (a stand-in for the paper's interatomic
 * potentials; architecture fixed here): radial basis
 * e_b(r) = sqrt(2/rc) sin(b pi r/rc)/r (b = 1..16), cutoff
 * f_c(r) = (cos(pi r/rc) + 1)/2, embedding h_i = W_emb[s_i] (128), three
 * layers W_ij = f_c(r) (A2 silu(A1 e(r) + a1) + a2),
 * m_i = sum_j W_ij (.) (B h_j), h_i += C2 silu(C1 m_i + c1) + c2, readout
 * E = s_E sum_i (w2 . silu(W1 h_i + b1) + b2) with W1 64x128, and forces
 * F = -dE/dq.  Weights: one flat binary32 device vector, matrices stored
 * [out][in], in the order W_emb [S][128]; per layer A1 [128][16], a1,
 * A2 [128][128], a2, B [128][128], C1 [128][128], c1, C2 [128][128], c2;
 * then W1 [64][128], b1 [64], w2 [64], b2 [1]. */
#define LSD_MPNN_HIDDEN 128
#define LSD_MPNN_RBF 16
#define LSD_MPNN_LAYERS 3
#define LSD_MPNN_READOUT 64

/* A potential: the target force field of verify_step or the draft force
 * field of draft_step (Alg. 2).  Forces are -dU/dq (Sec. 2.1). */
typedef struct {
  int32_t kind;              /* lsd_pot_kind */
  double cutoff;             /* LJ cutoff r_c (0 for the tether) */
  double epsilon, sigma;     /* LJ parameters */
  double k_spring;           /* tether stiffness */
  const float *anchor;       /* tether anchors, device [3][N] (kept by pointer) */
  const float *force_offset; /* optional constant force field added to the
                                forces, device [3][N] or NULL (test drafts) */
  const float *weights;      /* MPNN / PAIR / NET: flat weights (device, kept by pointer) */
  int32_t n_model_species;   /* MPNN: species rows of W_emb; PAIR, NET: S (>= n_species) */
  double energy_scale;       /* MPNN: s_E */
  int32_t n_basis;           /* PAIR: B, 1 .. LSD_PAIR_MAX_BASIS; NET: B */
  int32_t precision;         /* NET: lsd_precision */
  double act_amax[2];        /* NET, LSD_PREC_FP8: calibrated max |D| and max |h| (> 0) */
} lsd_potential;

typedef struct {
  int32_t n_atoms;             /* N, all replicas */
  int32_t n_replicas;          /* R >= 1 */
  const int32_t *atom_offsets; /* host [R+1], offsets[0] = 0, offsets[R] = N */
  const double *box;           /* host [R] cubic box edges (binary32 values) */
  const int32_t *species;      /* host [N] species index, or NULL for all 0 */
  const double *species_mass;  /* host [n_species] masses, > 0 */
  int32_t n_species;           /* 1 .. 8 */
  double dt, gamma, kT;        /* time step, friction (> 0), k_B T (> 0) */
  double force_unit;           /* see Conventions; > 0 */
  double skin;                 /* Verlet skin added to both cutoffs, > 0 */
  int32_t k_max;               /* largest window, 1 .. 64 */
  int32_t mode;                /* lsd_mode */
  uint64_t seed;               /* Philox key */
  lsd_potential target;        /* verify_step force field */
  lsd_potential draft;         /* draft_step force field (ignored in PLAIN) */
  int32_t max_neighbors_target;/* neighbour-list width; 0 = automatic */
  int32_t max_neighbors_draft; /* 0 = automatic */
  int32_t error_correction;    /* speculative error correction (App. D,
                                  Alg. 3), LSD mode only.  1: every draft of a
                                  window is drawn from the Gaussian of Eq. bob
                                  with F~ + dF, dF = F - F~ (target minus
                                  EC-uncorrected draft force, binary32) of the
                                  last committed step, cached per atom; the
                                  cache starts at 0.  2: as 1, but once two
                                  committed errors dF (step s) and dF' (step
                                  s-1) are held, frame k uses the linear
                                  extrapolation dF + (k+1)(dF - dF').  0: off.
                                  Target forces and the acceptance rule are
                                  unchanged, so the target law is preserved
                                  for any setting. */
  int32_t integrator;          /* lsd_integrator (0 = ABOBA) */
  int32_t no_list_reuse;       /* 0 (default): the neighbour lists of a
                                  replica are kept across windows until one of
                                  its atoms has moved more than skin/4 from
                                  the positions they were built at; != 0:
                                  rebuilt at every window.  Committed results
                                  differ only in summation order. */
} lsd_config;

typedef struct {
  float *q;              /* committed positions [3][N], in/out */
  float *p;              /* committed momenta [3][N], in/out */
  int32_t *img;          /* committed image counters [3][N], in/out */
  int64_t *step;         /* committed step per replica [R], in/out */
  void *workspace;       /* lsd_workspace_size() bytes, 256-byte aligned */
  size_t workspace_bytes;
  double *log_ratio;     /* out [R][k_max]: log N(p~;<p>,S)/N(p~;<p~>,S) */
  double *energy;        /* out [R][k_max]: target potential energy per frame */
  uint8_t *accepted;     /* out [R][k_max]: decision of every verified frame,
                            1 accepted, 0 rejected; 2 not verified (frames
                            from K_eff on, and every frame in PLAIN mode).
                            Only frames 1..n_committed are committed. */
  int32_t *n_committed;  /* out [R]: steps committed by the last window */
  const double *replay_u;  /* optional [R][k_max] uniforms in (0,1] for the
                              frames of the next window; NULL = Philox */
  const double *replay_xi; /* optional [k_max][N][3] normals, frame-major,
                              atom-major within a frame; NULL = Philox */
  float *obabo_q;        /* OBABO integrator: out [3][N] positions of y_n */
  float *obabo_p;        /* OBABO integrator: out [3][N] momenta of y_n */
} lsd_buffers;

/* Workspace bytes needed for cfg (host only; no GPU access). */
LSD_API lsd_status lsd_workspace_size(const lsd_config *cfg, size_t *bytes);

/* Validates cfg, lays out the workspace, uploads the static tables (species,
 * replicas, tiles, cell grids) and returns a handle.  Synchronises `stream`
 * once.  The buffers struct is copied; its pointers must stay valid until
 * lsd_destroy.  Errors: INVALID_ARG (gamma, kT, dt, masses or skin <= 0,
 * k_max outside 1..64, box edge not binary32 or <= cutoff + skin, more than
 * 2^27 atoms), CAPACITY (workspace too small), HIP. */
LSD_API lsd_status lsd_init_system(const lsd_config *cfg, const lsd_buffers *buf,
                           lsd_stream stream, lsd_system **out);

/* draft_step of Alg. 2, K times (1 <= K <= k_max), from the committed
 * state: builds the cell and neighbour lists at the first midpoint, then for
 * each k: draft forces at the midpoint, p~_k = <p~_k> + Sigma^{1/2} xi (Eq.
 * bob, xi keyed by step s + k), position half steps.  Frames whose atoms
 * moved more than skin/2 from the list positions are marked invalid and end
 * the window early (K_eff < K).  Needs state READY or COMMITTED; leaves
 * DRAFTED.  In PLAIN mode the target force field steps the system. */
LSD_API lsd_status lsd_draft_steps(lsd_system *sys, int32_t K, lsd_stream stream);

/* Declares that the caller has written K frames into the window arrays of
 * lsd_window_layout (midpoints, draft momenta 0..K, draft forces) instead of
 * drafting them; builds the neighbour lists at frame 0 and the validity of
 * every frame.  Leaves DRAFTED.  For external drafts and tests. */
LSD_API lsd_status lsd_mark_drafted(lsd_system *sys, int32_t K, lsd_stream stream);

/* verify_step of Alg. 2 for all valid drafted frames of all replicas in one
 * kernel launch: target energy and forces, <p> of Eq. bob, and the binary64
 * sums S1 = delta.z, S2 = delta.delta with z = Sigma^{-1/2}(p~ - <p~>) and
 * delta = Sigma^{-1/2}(<p~> - <p>) (Eq. reflectionVerify).  DRAFTED ->
 * VERIFIED.  No-op in PLAIN mode. */
LSD_API lsd_status lsd_verify_window(lsd_system *sys, lsd_stream stream);

/* Decision and commit: log r_k = -S1 - S2/2, accept frame k iff
 * log u_{s+k} <= log r_k; j = first rejected frame (else K_eff).  Frames
 * 1..j are committed; a rejected frame j takes the reflected momentum
 * <p> + Sigma^{1/2}(I - 2 delta delta^T / delta^T delta) z and map g.  Fills
 * log_ratio, energy, accepted, n_committed and advances step[r] by j.
 * If n_host is not NULL, synchronises and copies n_committed to host [R].
 * VERIFIED (LSD) or DRAFTED (PLAIN) -> COMMITTED. */
LSD_API lsd_status lsd_accept_rollback(lsd_system *sys, int32_t *n_host,
                               lsd_stream stream);

/* Enqueues n_windows x (draft K, verify, accept) without synchronising.
 * By default each window is one launch of a HIP graph (captured once per K
 * on a library stream, replayed on `stream`); with verification timing on,
 * the verification kernel runs between the graph parts that precede and
 * follow it, bracketed by HIP events.  Results are identical either way.
 * In the replayed windows each commit also starts the next window; a call
 * first starts its own first window, so a state the caller writes between
 * calls is taken up (a list rebuild that the previous call's last commit
 * flagged then still happens, which is valid and changes only the order of
 * the list entries). */
LSD_API lsd_status lsd_run_windows(lsd_system *sys, int32_t n_windows, int32_t K,
                           lsd_stream stream);

/* Autotuner of the verification (LSD mode): drafts a window of K frames
 * from the committed state (as lsd_draft_steps; the state is left DRAFTED,
 * so the caller continues with lsd_verify_window), times every candidate on
 * those frames (one untimed and `repeats` timed verifications each, HIP
 * events on `stream`) and keeps the fastest.  Every candidate gives the same
 * results bit for bit.
 *   Pair targets: the verification kernel with 1, 2, 4 and 8 frames per
 *   wave, kept for windows of K frames; chosen = frames per wave, us [4].
 *   Message-passing target: the evaluation's launch shapes, blocks of the
 *   pair-filter kernel {256, 512, 1024} x rows per row-chain block {16, 32,
 *   64} (candidate 3 f + c), kept for every K; chosen = candidate index,
 *   us [9].
 * chosen and us (mean microseconds per verification) are host outputs, each
 * optional.  Captured window graphs are dropped.  Synchronises `stream`. */
LSD_API lsd_status lsd_autotune_verify(lsd_system *sys, int32_t K, int32_t repeats,
                                       int32_t *chosen, double *us, lsd_stream stream);

/* Fixes the verification variant for windows of K frames (1 <= K <=
 * k_max) as lsd_autotune_verify would choose it, without timing (for
 * reproducible profiles): frames_per_wave in {1, 2, 4, 8} for pair targets,
 * the launch-shape candidate 0..8 for the message-passing target (every K).
 * Captured window graphs are dropped.  LSD_ERR_INVALID_ARG for other values. */
LSD_API lsd_status lsd_set_verify_variant(lsd_system *sys, int32_t K, int32_t frames_per_wave);

/* Pipelined windows: the one-GPU form of pipelined LSD (Alg. 2, App. C).
 * With group_frames = G >= 1, lsd_run_windows verifies every group of G
 * drafted frames on a second stream (default priority) as soon as its last
 * frame is drafted, while the draft chain continues on the caller's stream;
 * each group's decisions record the first rejected frame on the device, and
 * the draft and verification launches of later frames of the window then
 * find nothing to do (the flushed drafts of Alg. 2).  The window ends with
 * the decision over every kept frame and the commit, as in a synchronous
 * window: with the step-keyed stream the committed trajectory is the same
 * bit for bit (frames after the first rejection are never kept).  The
 * outputs of frames after the first rejection are reported as not verified
 * (accepted = 2).  Untimed windows run as one two-stream graph; windows
 * whose verification is timed are issued eagerly, each group's verification
 * launch bracketed by events.  0 (the default) restores synchronous windows.
 * LSD mode only (ignored in plain mode); needs graphs on.
 * Errors: INVALID_ARG (G outside 0..64), UNSUPPORTED (graphs off). */
LSD_API lsd_status lsd_set_pipeline(lsd_system *sys, int32_t group_frames);

/* enable != 0 (default): lsd_run_windows replays captured graphs; 0: it
 * issues the kernels of every window one by one. */
LSD_API lsd_status lsd_set_graphs(lsd_system *sys, int32_t enable);

/* Drafting of one system in fewer launches (Alg. 2, the draft chain of a
 * window).  In synchronous windows of a single system with a pair draft
 * (Lennard-Jones or force-matched pairs), or with the learned draft and its
 * bfloat16 node pass up to 2048 atoms, the draft steps first_step .. K-1 run
 * in one launch (the per-step kernels' blocks in turn, a bounded grid
 * barrier after each pass, ending at the first frame past the skin) instead
 * of one or two launches per step; results are bit for bit those of the
 * per-step launches.  Plain stepping with a pair target takes it for a
 * system of one tile (64 atoms), where no grid barrier is needed.
 * first_step = 0 turns it off; the default is 3.  Other systems ignore the
 * setting.  A grid barrier that times out sets bit 5 of the status word.
 * Errors: INVALID_ARG (first_step outside 0..64). */
LSD_API lsd_status lsd_set_draft_tail(lsd_system *sys, int32_t first_step);

/* Byte offsets into the workspace of the window and list arrays (host). */
/* Window frames are continuous with the positions the neighbour lists (and
 * their image codes) were built at: those are the wrapped first midpoints of
 * the window in which the lists were last rebuilt.  Frame 0 is the first
 * midpoint, shifted by whole box edges to lie next to those positions, and
 * frames 1..K-1 follow it without wrapping, so an atom near a face may sit up
 * to skin/2 outside [0, L).  The commit wraps positions and updates the image
 * counters.  lsd_mark_drafted rebuilds the lists from the caller's frame 0,
 * which must be wrapped into [0, L); the caller's later frames must be
 * continuous with it.  A frame in which an atom moved more than skin/2 from
 * the list positions (a wrapped jump included) is not verified. */
typedef struct {
  size_t q_mid;      /* float4 [k_max][N]: x, y, z, packed image deltas of
                        frame 0 relative to the committed counters */
  size_t p_draft;    /* float [k_max+1][3][N]: committed p, then p~_1..p~_K */
  size_t f_draft;    /* float [k_max][3][N]: bare draft forces F~ (the
                        error correction is added where the draft mean is
                        formed, in binary32: F~ + dF) */
  size_t f_target;   /* float [k_max][3][N] */
  size_t frame_invalid; /* int32 [R][k_max] */
  size_t nbr_target; /* uint32 [N][max_neighbors_target]: j << 5 | image code,
                        code = (nx+1) + 3 (ny+1) + 9 (nz+1), n = image */
  size_t cnt_target; /* int32 [N] */
  size_t nbr_draft;  /* uint32 [N][max_neighbors_draft] */
  size_t cnt_draft;  /* int32 [N] */
  size_t error_cache;/* float [3][N] dF of the error correction; 0 (no
                        array) when it is off */
  size_t error_cache_prev; /* float [3][N] dF of the committed step before
                        (linear variant), else 0 */
  int32_t max_neighbors_target, max_neighbors_draft;
  int32_t n_atoms, k_max;
} lsd_window_layout;
LSD_API lsd_status lsd_get_window_layout(const lsd_system *sys, lsd_window_layout *out);

/* Synchronises `stream` and returns the device status word: bit 0 target
 * list overflow, bit 1 draft list overflow, bit 2 cell overflow, bit 3 more
 * in-cutoff pairs of the message-passing target than its buffers hold (a
 * quarter of rows x list width), bit 4 inconsistent pair lists of that
 * target, bit 5 a grid barrier of the one-launch draft chain timed out
 * (lsd_set_draft_tail).  Any set bit means the results since it was set are
 * not valid. */
LSD_API lsd_status lsd_get_status(lsd_system *sys, int32_t *flags, lsd_stream stream);

/* Final step count of the run (Alg. 2 stops when that many steps are
 * verified): frames that would produce a step beyond `limit` are not
 * verified, so every replica stops exactly at step `limit` (a window may then
 * commit 0 steps).  Stopping on a step count rather than after a number of
 * windows keeps the final states target-distributed: window ends follow
 * rejections, so stopping at a window end would select post-rejection
 * states.  Default: no limit.  Takes effect from the next window. */
LSD_API lsd_status lsd_set_step_limit(lsd_system *sys, int64_t limit);

/* Per-replica counters since init or the last reset, copied to host
 * out[R][LSD_NUM_COUNTERS] = {windows, committed steps, rejections (windows
 * ending in a reflected step), frames verified, neighbour-list builds}.  The
 * empirical rejection rate of the paper (Sec. 3.3) is rejections /
 * committed.  Synchronises `stream`. */
#define LSD_NUM_COUNTERS 5
LSD_API lsd_status lsd_get_counters(lsd_system *sys, int64_t *out, lsd_stream stream);
LSD_API lsd_status lsd_reset_counters(lsd_system *sys, lsd_stream stream);

/* Kernel timing of the verification launch with HIP events on `stream`.
 * enable = n > 0 starts recording every n-th verification launch (the n-th,
 * 2n-th, ... after enabling; 1: every one; a sample keeps the graph of the
 * untimed windows whole), 0 stops,
 * n < 0 is LSD_ERR_INVALID_ARG.  lsd_get_verify_timing synchronises and
 * returns the summed milliseconds and the count of timed launches since
 * enabling. */
LSD_API lsd_status lsd_set_verify_timing(lsd_system *sys, int32_t enable);
LSD_API lsd_status lsd_get_verify_timing(lsd_system *sys, double *total_ms,
                                 int64_t *launches);

/* The library's random stream, for parity checks: out[n][3] normals of step
 * `step` (device buffer), and out[count] uniforms of steps step0+1 ..
 * step0+count (device buffer). */
LSD_API lsd_status lsd_rng_normals(uint64_t seed, int32_t replica, int64_t step,
                           int32_t n, double *out, lsd_stream stream);
LSD_API lsd_status lsd_rng_uniforms(uint64_t seed, int32_t replica, int64_t step0,
                            int32_t count, double *out, lsd_stream stream);

/* Force matching of the pair draft (fallback of the learned draft: fitted
 * to forces the target itself produced).  With P = S(S+1)/2 * n_basis
 * weights (S = n_species) in the order of the pair-draft weights, the
 * extended normal equations G = [A | y]^T [A | y] are accumulated, where the
 * rows of A are the pair-draft forces per unit weight of every atom and
 * component of the valid frames (0 .. K_eff-1) of the current window at
 * their midpoints q_mid, and y the forces of those frames: f_target
 * (use_target_forces != 0: LSD mode, a verified window) or f_draft (the
 * stepping forces; in PLAIN mode these are the target's).  differences != 0:
 * the rows are instead the differences between consecutive valid frames
 * (rows of frame k+1 minus rows of frame k, forces likewise), which fits the
 * draft's response to the motion, the part of its error that error
 * correction (App. D) leaves.  Pairs are taken within `cutoff` (<= the
 * target cutoff; the target list is used).
 *   gram: device binary64 [(P+1)][(P+1)] row-major, accumulated (+=) in a
 *         fixed order; zero it before the first call.  Column P = A^T y.
 *   scratch: device memory of lsd_fit_pair_scratch_size bytes.
 * Needs S * n_basis <= 64.  Asynchronous on `stream`.  Errors: INVALID_ARG,
 * BAD_STATE (no drafted window, or no target forces), CAPACITY, HIP. */
LSD_API lsd_status lsd_fit_pair_scratch_size(const lsd_system *sys, int32_t n_basis,
                                             size_t *bytes);
LSD_API lsd_status lsd_fit_pair_accumulate(lsd_system *sys, int32_t n_basis, double cutoff,
                                           int32_t use_target_forces, int32_t differences,
                                           void *scratch, size_t scratch_bytes, double *gram,
                                           lsd_stream stream);
/* Host: weights (host binary64 [P]) minimising |A w - y|^2 + lambda |w|^2
 * from the normal equations `gram` (host copy, layout above), with
 * lambda = ridge * trace(A^T A) / P, by Cholesky factorisation.
 * INVALID_ARG if the system is not positive definite (raise the ridge). */
LSD_API lsd_status lsd_fit_pair_solve(const double *gram, int32_t n_params, double ridge,
                                      double *weights);

/* Training of the learned draft by force matching (host-side count, then
 * device calls).  lsd_net_param_count: length of the parameter vector for S
 * species and B radial functions (0 if out of range).
 *
 * lsd_net_train_accumulate adds, for the valid frames (0 .. K_eff-1) of the
 * current window, the gradient of the summed squared force error
 * sum |F_net(q_mid) - y|^2 (all atoms and components; y = f_target if
 * use_target_forces != 0, else f_draft, the stepping forces, which are the
 * target's in PLAIN mode) in the parameters of `net` (kind LSD_POT_NET, its
 * cutoff <= the target cutoff: the target list is used), evaluated in
 * binary32 (whatever net->precision says) and reduced in binary64 in a fixed
 * order:  grad[0..P) += gradient, grad[P] += the squared error, grad[P+1] +=
 * the number of atom frames.  differences != 0: the loss is instead the
 * squared error of the force changes between consecutive valid frames,
 * sum_k |(F_k+1 - F_k) - (y_k+1 - y_k)|^2, the part of the draft's error
 * that error correction (App. D) leaves, and grad[P+1] counts atom
 * differences.  grad: device binary64 [P+2], zeroed by the
 * caller before the first call.  scratch: device memory of
 * lsd_net_train_scratch_size bytes.  Asynchronous.  Errors: INVALID_ARG,
 * BAD_STATE (no drafted window), CAPACITY, HIP.
 *
 * lsd_net_adam_step: one Adam step (Kingma and Ba, 2015) on the mean
 * squared force component error: g = grad[0..P) / (3 grad[P+1]);
 * m = beta1 m + (1-beta1) g, v = beta2 v + (1-beta2) g^2 (m, v device
 * binary64 [P], zero before step 1), params -= lr m^/(sqrt(v^) + eps) with
 * m^ = m/(1-beta1^t), v^ = v/(1-beta2^t), computed in binary64 and rounded
 * to the binary32 params; then grad[0..P+2) is zeroed.  t >= 1.  Nothing
 * changes if grad[P+1] is 0.  Asynchronous; one work-group. */
LSD_API int32_t lsd_net_param_count(int32_t n_species, int32_t n_basis);
LSD_API lsd_status lsd_net_train_scratch_size(const lsd_system *sys, size_t *bytes);
LSD_API lsd_status lsd_net_train_accumulate(lsd_system *sys, const lsd_potential *net,
                                            int32_t use_target_forces, int32_t differences,
                                            void *scratch,
                                            size_t scratch_bytes, double *grad,
                                            lsd_stream stream);
/* Calibration of the FP8 activation scales: max |D| over the descriptor
 * entries and max |h| over the hidden activations of the learned draft
 * `net` on the valid frames of the current window (binary32 node pass over
 * the target list, as in training; the maximum is order-independent, so
 * the result is exact for those values).  amax: device binary64 [2],
 * overwritten.  scratch as for training.  Asynchronous.  Errors as for
 * lsd_net_train_accumulate. */
LSD_API lsd_status lsd_net_activation_amax(lsd_system *sys, const lsd_potential *net,
                                           void *scratch, size_t scratch_bytes, double *amax,
                                           lsd_stream stream);
LSD_API lsd_status lsd_net_adam_step(float *params, double *m, double *v, double *grad,
                                     int32_t n_params, double lr, double beta1, double beta2,
                                     double eps, int64_t t, lsd_stream stream);

/* Kinetic energy per replica in binary64, the thermostat observable of
 * Sec. 4.3 (Tab. heating; the kinetic temperature of replica r is
 * T_kin = 2 ke[r] / (3 N_r k_B): the paper prints it without the 3 of the
 * three axes):
 *   ke[r] = sum over atoms i of replica r and axes d of p[d][i]^2 / (2 m_i).
 * Stateless; works on any momenta in the library's layout (e.g. the
 * committed state of a system, or frames of a window).
 *   p: device binary32 [3][n_atoms] (SoA); species: device int32 [n_atoms],
 *      or NULL (every atom has species 0); species_mass: host binary64
 *      [n_species], 1 <= n_species <= 8, all > 0 (read during the call);
 *   atom_offsets: device int32 [n_replicas + 1] (replica r = atoms
 *      [atom_offsets[r], atom_offsets[r+1])); max_replica_atoms: host, at
 *      least the largest replica (a replica with more atoms gets NaN);
 *   ke: device binary64 [n_replicas], overwritten.
 * Each square is exact in binary64; the products with 1/(2m) and all sums
 * are binary64 in a fixed order (chunks of 2048 atoms, lane-strided, wave
 * butterfly, chunks in order), so results repeat bit for bit.  All terms
 * are positive, so the relative error against the exact value of the
 * binary32 momenta is at most about (3 N_r + 2) 2^-53.
 *   scratch: device memory of at least lsd_kinetic_energy_scratch_size()
 *      bytes (partial sums; its contents on entry do not matter).
 * Asynchronous on `stream`, no host synchronisation, graph-capturable.
 * Errors: INVALID_ARG (null pointer, bad count or mass), CAPACITY (scratch
 * too small), HIP. */
LSD_API lsd_status lsd_kinetic_energy_scratch_size(int32_t n_replicas,
                                                   int32_t max_replica_atoms, size_t *bytes);
LSD_API lsd_status lsd_kinetic_energy(const float *p, int32_t n_atoms, const int32_t *species,
                                      const double *species_mass, int32_t n_species,
                                      const int32_t *atom_offsets, int32_t n_replicas,
                                      int32_t max_replica_atoms, double *ke, void *scratch,
                                      size_t scratch_bytes, lsd_stream stream);

/* lsd_kinetic_energy without a scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels, summation
 * order and results (bit for bit) as lsd_kinetic_energy; the partial sums go
 * to a static device array of the library instead of caller scratch.
 *   Limit: n_replicas * ceil(max_replica_atoms / 2048) <= 65536 partial sums
 *   (512 KiB, held on every GPU the library runs on until the process
 *   ends); larger requests fail with CAPACITY.
 * The array is shared by every call on a GPU: calls that overlap on one GPU
 * (different streams, or threads) race and must be serialised by the caller.
 * Nothing from an earlier call is read.  Calls no hipMalloc, hipFree or
 * allocating library routine; the first call on a device looks up the
 * array's device address (hipGetSymbolAddress) with that device current.
 * Errors: INVALID_ARG, CAPACITY, UNSUPPORTED (device index above 63), HIP. */
LSD_API lsd_status lsd_kinetic_energy_noalloc(const float *p, int32_t n_atoms,
                                              const int32_t *species,
                                              const double *species_mass, int32_t n_species,
                                              const int32_t *atom_offsets, int32_t n_replicas,
                                              int32_t max_replica_atoms, double *ke,
                                              lsd_stream stream);

/* Verifier state of pipelined LSD (Alg. 2, App. C): host-only bookkeeping
 * for callers that submit every draft step for verification as soon as it
 * is drafted and receive target results in any order (a pool of target
 * workers).  Steps are identified by ids 1, 2, ... in submission order; id
 * 0 is the initial state, verified from the start.  The caller keeps the
 * draft and target states by id.
 *   lsd_pipeline_submit: registers the next draft step as eligible pending
 *     and returns its id.
 *   lsd_pipeline_return: a target result for `id` arrived, accepted != 0
 *     if the coupled target state equals the draft state.  If the step was
 *     flushed by an earlier rejection (or already returned), *ignored = 1
 *     and nothing changes.  Otherwise it becomes conditionally verified; if
 *     rejected, every later step is flushed and *rollback = 1: the caller
 *     continues drafting from this step's target state.  Then every
 *     conditionally verified step that precedes all pending ones is
 *     appended to the verified sequence, in id order.
 *   lsd_pipeline_take_verified: copies up to `cap` ids appended to the
 *     verified sequence since the last call (host array) and their count.
 *   lsd_pipeline_counts: out[3] = {pending, conditionally verified,
 *     verified (including id 0)}.
 * Every verified sequence satisfies the paper's recursive correctness
 * condition: each state is a target sample conditioned on its predecessor.
 * No GPU work; not thread-safe for one handle. */
typedef struct lsd_pipeline lsd_pipeline;
LSD_API lsd_status lsd_pipeline_create(lsd_pipeline **out);
LSD_API lsd_status lsd_pipeline_destroy(lsd_pipeline *pipe);
LSD_API lsd_status lsd_pipeline_submit(lsd_pipeline *pipe, int64_t *id);
LSD_API lsd_status lsd_pipeline_return(lsd_pipeline *pipe, int64_t id, int32_t accepted,
                                       int32_t *ignored, int32_t *rollback);
LSD_API lsd_status lsd_pipeline_take_verified(lsd_pipeline *pipe, int64_t *ids, int32_t cap,
                                              int32_t *n);
LSD_API lsd_status lsd_pipeline_counts(const lsd_pipeline *pipe, int64_t *out);

/* Releases the handle and its HIP events (no device memory is freed). */
LSD_API lsd_status lsd_destroy(lsd_system *sys);

/* Thread-local text of the last error ("" if none). */
LSD_API const char *lsd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LSD_H */
