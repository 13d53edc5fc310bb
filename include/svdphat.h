/*
 * svdphat.h -- C ABI of the MI355X (gfx950) SVD-PHAT sound-source localiser.
 *
 * Method: F. Grondin and J. Glass, "SVD-PHAT: A Fast Sound Source
 * Localization Method" (arXiv 1811.11785).  Section 2 defines SRP-PHAT
 * (far-field delays eq. (2), PHAT cross-spectra eq. (3), steering
 * coefficients eq. (4), powers eq. (5)/(9), argmax eq. (6)); Section 3
 * defines SVD-PHAT (eqs. (7)-(14)) and Algorithm 1 splits it into an offline
 * plan and an online per-frame search.
 *
 * Conventions shared by every call
 *   - Every function returns an int status: SVDPHAT_OK (0) or a negative
 *     SVDPHAT_E_* code.  No C++ exception crosses this boundary.  The
 *     message of the last failure on the calling thread is returned by
 *     svdphat_last_error().  For tests, the environment variable
 *     SVDPHAT_FAULT (comma-separated) forces failures: "alloc" makes every
 *     device allocation of the library fail (SVDPHAT_E_NOMEM), "eig" makes
 *     the plan's eigensolver report no convergence (SVDPHAT_E_NUMERIC).
 *   - "host" pointers are read (or written) before the call returns.
 *     "device" pointers are HIP device memory owned by the caller; the call
 *     enqueues work on the given HIP stream (a hipStream_t passed as void*,
 *     NULL = the null stream) and returns without waiting.  Errors raised by
 *     that work surface at the next call or at svdphat_sync().
 *   - Directions are returned as 0-based indices into the caller's grid.
 *     Directions whose delay rows are identical (within 1e-9 samples in every
 *     pair) have identical rows of W and so identical powers; they form one
 *     class, and the index returned is always the lowest index of the class.
 *   - Inputs: STFT frames X are complex64 (interleaved re, im) laid out
 *     [F][M][N/2+1]: frame-major, then microphone, then bin k = 0 .. N/2
 *     (Section 2, bins k in [0, N/2]).
 */
#ifndef SVDPHAT_H
#define SVDPHAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SVDPHAT_OK              0
#define SVDPHAT_E_INVAL        -1  /* invalid argument (shape, range, NULL) */
#define SVDPHAT_E_NOMEM        -2  /* device or host allocation failed */
#define SVDPHAT_E_DEVICE       -3  /* a HIP / rocBLAS / rocSOLVER call failed */
#define SVDPHAT_E_NUMERIC      -4  /* eigensolver failure or non-finite factors */
#define SVDPHAT_E_NODEV        -5  /* no usable GPU */
#define SVDPHAT_E_UNSUPPORTED  -6  /* request not supported by this plan */
#define SVDPHAT_E_IO           -7  /* a file could not be opened, read or written */

/* ---- plan flags ------------------------------------------------------ */
#define SVDPHAT_KEEP_W    0x1u  /* also store W in FP32 for svdphat_srp_locate */
#define SVDPHAT_NO_DEDUP  0x2u  /* score every direction, not one per class */

/* ---- precision of the two projections in svdphat_locate --------------- */
#define SVDPHAT_FP32  0   /* FP32 operands, FP32 accumulation */
#define SVDPHAT_BF16  1   /* BF16 operands on MFMA, FP32 accumulation */
#define SVDPHAT_FP16  2   /* FP16 operands on MFMA, FP32 accumulation */

/* ---- mode bits of svdphat_locate ------------------------------------- */
#define SVDPHAT_RESCORE  0x1u /* rescore in FP32 every direction whose
                                 low-precision power is within the rounding
                                 bound of the maximum (else only the tiles
                                 holding the maximum are rescored) */
#define SVDPHAT_HILO     0x2u /* recompute Z = S V^H X with a split hi/lo
                                 (compensated) product for frames whose
                                 rescored top-two margin is small */
#define SVDPHAT_HILO_ALL 0x4u /* the hi/lo pass for every frame, whatever
                                 its margin (implies SVDPHAT_HILO; with
                                 FP32 operands there is no hi/lo pass) */
#define SVDPHAT_NORMALIZED 0x8u /* the search of eq. (15) (Section 3):
                                 maximise Re{D^_q Z^} with D^_q = D_q /
                                 ||D_q||, D_q = U_q S, i.e. minimise the
                                 distance ||D^_q - Z^^H||_2 between unit
                                 vectors, instead of Re{D_q Z} of eq. (14);
                                 yhat, margin and y_opt then hold
                                 Re{D_q Z} / ||D_q||, power stays the row
                                 power of the chosen direction */

typedef struct svdphat_plan svdphat_plan;

typedef struct svdphat_info {
    int32_t M;          /* microphones */
    int32_t P;          /* pairs, M(M-1)/2 */
    int32_t B;          /* bins, N/2 + 1 */
    int32_t L;          /* P * B, length of X in eq. (7) */
    int32_t Q;          /* directions */
    int32_t n_classes;  /* rows scored by the reduced search */
    int32_t K;          /* rank used */
    int32_t K_paper;    /* smallest K satisfying eq. (11) */
    int32_t N;          /* frame size */
    int32_t has_w;      /* 1 if the plan keeps W in FP32 */
    double residual;    /* 1 - sum_{k<=K} s_k^2 / ||W||_F^2 */
    double sigma1;      /* largest singular value */
    double sigmaK;      /* K-th singular value */
    double fro2;        /* ||W||_F^2 (= Q * L exactly in exact arithmetic) */
    double u_rownorm_max; /* max_q ||U_q||_2 over the kept rank */
    int64_t device_bytes;
    uint64_t input_hash;  /* svdphat_plan_input_hash of the plan's inputs */
} svdphat_info;

/*
 * svdphat_plan_create -- Algorithm 1, offline steps 1-2 (Section 3).
 *   mic_xyz_m  host, M x 3 doubles, microphone positions in metres.
 *   grid_xyz   host, Q x 3 doubles, candidate directions s_q (any nonzero
 *              length; each row is normalised as in eq. (2)).
 *   fs, c      sample rate (Hz) and speed of sound (m/s), both > 0.
 *   N          STFT frame size, even, >= 2.
 *   delta      tolerated relative reconstruction error of eq. (11), a
 *              small positive value as Section 3 defines it: 0 < delta < 1.
 *              The singular values come from the eigenvalues of the smaller
 *              Gram matrix, which are accurate to about 1e-16 s_1^2 (absolute,
 *              in s^2), so a delta below about 1e-12 can place the cut where
 *              the tail energy is not resolved.
 *   flags      SVDPHAT_KEEP_W | SVDPHAT_NO_DEDUP.
 *   out        receives the new plan (set to NULL on failure).
 * Builds the far-field delays (eq. (2)), W (eqs. (4), (8)) in FP64 on the
 * GPU, its truncated SVD (eq. (10)) through the Hermitian eigen-
 * decomposition of the smaller Gram matrix, chooses K by eq. (11) (extended
 * over a cluster of equal singular values at the cut), and packs the device
 * operands.  Synchronous.  The plan owns all the device memory it creates.
 * Errors: E_INVAL (M < 2 or > 16, Q < 1, N odd or < 2, delta outside (0,1), a zero
 * grid row, non-finite input), E_NODEV, E_NOMEM, E_DEVICE, E_NUMERIC.
 */
int svdphat_plan_create(const double* mic_xyz_m, int32_t M,
                        const double* grid_xyz, int32_t Q,
                        double fs, double c, int32_t N, double delta,
                        uint32_t flags, svdphat_plan** out);

/* svdphat_plan_info -- sizes and factorisation summary of a plan (host). */
int svdphat_plan_info(const svdphat_plan* plan, svdphat_info* out);

/*
 * svdphat_plan_export -- copies the FP64 factors to host memory (a testing
 * aid; any pointer may be NULL to skip it).
 *   sigma      min(Q, L) singular values, descending (eq. (10)).
 *   U          Q x K complex (interleaved), row-major.
 *   V          L x K complex (interleaved), row-major, rows in the order of
 *              eq. (7) (pair-major, bin-minor).
 *   class_rep  Q ints: lowest index of each direction's class.
 */
int svdphat_plan_export(const svdphat_plan* plan, double* sigma, double* U,
                        double* V, int32_t* class_rep);

/*
 * svdphat_plan_save / svdphat_plan_load -- Algorithm 1 computes its offline
 * products once per array and grid (Section 3); these keep them.  save
 * writes the plan's inputs (microphones, grid as given, fs, c, N, delta,
 * flags) and its truncated SVD (sigma, U, V, K, K_paper) to `path` in a
 * versioned little-endian binary with a 64-bit FNV-1a hash of the inputs and
 * a checksum of the file.  load reads such a file and builds a plan on the
 * current HIP device without refactorising W: only the host geometry and
 * the packing of the device operands are repeated, so every result of the
 * loaded plan is identical to the saved one's.  Synchronous.
 *   path  host, NUL-terminated file name.  out: receives the plan (NULL on
 *         failure; the caller destroys it with svdphat_plan_destroy).
 * Errors: E_IO (the file cannot be opened, read or written), E_INVAL (NULL
 * arguments, not a plan file, another version, damaged file: checksum,
 * input hash or sizes), E_NODEV, E_NOMEM, E_DEVICE.
 * svdphat_plan_input_hash -- the hash a saved file records, from the inputs
 * of svdphat_plan_create (host arrays; no device needed), so a caller can
 * match a saved plan to its problem; svdphat_plan_info reports it too.
 */
int svdphat_plan_save(const svdphat_plan* plan, const char* path);
int svdphat_plan_load(const char* path, svdphat_plan** out);
uint64_t svdphat_plan_input_hash(const double* mic_xyz_m, int32_t M,
                                 const double* grid_xyz, int32_t Q, double fs,
                                 double c, int32_t N, double delta,
                                 uint32_t flags);

/*
 * svdphat_locate -- Algorithm 1 online steps 1-4 (Section 3) with the
 * exhaustive search of eq. (14) for F frames.
 *   X          device, complex64 [F][M][N/2+1] STFT frames.
 *   F          number of frames, >= 0 (0 is a no-op).
 *   precision  SVDPHAT_FP32 | SVDPHAT_BF16 | SVDPHAT_FP16.
 *   mode       SVDPHAT_RESCORE | SVDPHAT_HILO | SVDPHAT_HILO_ALL |
 *              SVDPHAT_NORMALIZED.
 *   doa        device, int32 [F]: class-lowest index of argmax_q Y_q.
 *   power      device, f32 [F]: Y at doa from the row of W (step 4, eq. (9)).
 *   yhat       device, f32 [F] or NULL: the reduced power Re{D_q Z} at doa.
 *   margin     device, f32 [F] or NULL: (y1 - y2) / |y1| between the best and
 *              the second-best class of the FP32-rescored reduced powers
 *              (a lower bound where the runner-up was not rescored).
 *   y_opt      device, f32 [F][Q] or NULL: reduced powers of every direction
 *              in the requested precision (debugging; slower).
 *   stream     hipStream_t or NULL.
 * Errors: E_INVAL (NULL plan/X/doa/power with F > 0, bad precision), E_NOMEM
 * (workspace), E_DEVICE.
 */
int svdphat_locate(svdphat_plan* plan, const void* X, int64_t F,
                   int32_t precision, uint32_t mode, int32_t* doa,
                   float* power, float* yhat, float* margin, float* y_opt,
                   void* stream);

/*
 * svdphat_locate_noalloc -- svdphat_locate (same kernels, same results, no
 * y_opt) for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * calls no hipMalloc, hipFree or allocating library routine: its
 * intermediate results live in a fixed device array of
 * svdphat_noalloc_scratch_bytes() bytes (64 MiB) that the library holds on
 * every GPU it runs on until the process ends; the caller still passes X and
 * the outputs.  Every call on a GPU shares that GPU's array (the kernels
 * clear what must start at zero), so calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Errors: as svdphat_locate, and E_INVAL, before anything is enqueued,
 * when F frames need more scratch than the array holds (at the
 * 7-microphone, Q = 10242, K = 48 plan: about 4,800 frames with
 * SVDPHAT_HILO and 16-bit operands, over 30,000 without); split such
 * batches.
 */
int svdphat_locate_noalloc(svdphat_plan* plan, const void* X, int64_t F,
                           int32_t precision, uint32_t mode, int32_t* doa,
                           float* power, float* yhat, float* margin,
                           void* stream);
/* svdphat_noalloc_scratch_bytes -- size of the array above, in bytes. */
int64_t svdphat_noalloc_scratch_bytes(void);

/*
 * svdphat_locate_masked -- svdphat_locate on the cross-spectra of eq. (7)
 * with a binary time-frequency mask applied: the paper names masks (and
 * several sources) as future work in Section 5.  Every pair's x_{p,k} is set
 * to 0 at the bins a frame's mask drops, for the search and for the row
 * power of Algorithm 1 step 4 alike.
 *   mask   device, uint8 [F][N/2+1]: nonzero keeps bin k of frame f, 0 drops
 *          it (a frame with every bin dropped has every power 0 and returns
 *          the lowest index, as a silent frame does).
 *   The other arguments are those of svdphat_locate.  For FP16 and BF16
 *   batches of 6 to 8 microphones, the kernels read the mask with the
 *   frames.  A hi/lo pass still needs a second workspace of the plan and
 *   stream, of F (N/2+1) M 8 bytes, into which its listed frames are copied
 *   masked.  Otherwise (FP32, small batches of 16 frames or fewer, other
 *   plans), every masked frame is written to that workspace first.  The
 *   workspace is grown on demand like the first.  The results are the same
 *   either way: those of svdphat_locate on frames whose dropped bins hold 0.
 * Errors: as svdphat_locate; E_INVAL also for a NULL mask with F > 0.
 */
int svdphat_locate_masked(svdphat_plan* plan, const void* X, int64_t F,
                          const uint8_t* mask, int32_t precision,
                          uint32_t mode, int32_t* doa, float* power,
                          float* yhat, float* margin, float* y_opt,
                          void* stream);

/*
 * svdphat_srp_locate -- plain SRP-PHAT, eqs. (3), (9), (6), in FP32.
 *   X, F, stream as above; doa [F] class-lowest argmax, power [F] its Y,
 *   y_opt [F][Q] or NULL.  Needs a plan created with SVDPHAT_KEEP_W, else
 *   E_UNSUPPORTED.
 */
int svdphat_srp_locate(svdphat_plan* plan, const void* X, int64_t F,
                       int32_t* doa, float* power, float* y_opt, void* stream);

/*
 * Ragged batches: many arrays, each with its own plan (microphones, grid,
 * rank), located in one HIP-graph launch.  The frames of every array are
 * independent (Section 2 omits the frame index without loss of generality),
 * so their searches run side by side; each array follows svdphat_locate
 * with precision SVDPHAT_FP16 and mode SVDPHAT_RESCORE.
 *
 * svdphat_ragged_create
 *   plans       host array of n plans (not owned; they must outlive the batch
 *               and be created without SVDPHAT_NO_DEDUP, on one device).
 *   max_frames  host, n maximum frame counts (>= 1); workspace and work lists
 *               are sized for them.
 *   flags       SVDPHAT_RAGGED_TUNE: time candidate tile settings per array
 *               shape (GEMM1 split, GEMM2 frames per workgroup) and keep the
 *               fastest; otherwise use cached or default settings.
 *   tune_cache  path of a JSON-lines cache of tuned settings keyed by GPU
 *               architecture and shape (read, and appended when tuning), or
 *               NULL.
 *   Synchronous.  Errors: E_INVAL, E_UNSUPPORTED (a plan without classes),
 *   E_NOMEM, E_DEVICE.
 * svdphat_ragged_locate
 *   X, doa, power  host arrays of n device pointers: STFT frames
 *                  complex64 [F_i][M_i][N_i/2+1], int32 [F_i], f32 [F_i].
 *   F              host, n frame counts, 0 <= F_i <= max_frames_i.
 *   precision      SVDPHAT_FP16 (the batch's kernels run FP16 MFMA with FP32
 *                  rescoring); other values give E_UNSUPPORTED.
 *   Copies the per-array descriptors and launches the graph on `stream`;
 *   returns without waiting.
 * svdphat_ragged_info -- how many shapes were tuned now / taken from the cache.
 * svdphat_ragged_destroy -- NULL is a no-op.
 */
#define SVDPHAT_RAGGED_TUNE 0x1u
typedef struct svdphat_ragged svdphat_ragged;
int svdphat_ragged_create(svdphat_plan* const* plans, int32_t n,
                          const int64_t* max_frames, uint32_t flags,
                          const char* tune_cache, svdphat_ragged** out);
int svdphat_ragged_locate(svdphat_ragged* ragged, const void* const* X,
                          const int64_t* F, int32_t* const* doa,
                          float* const* power, int32_t precision,
                          void* stream);
int svdphat_ragged_info(const svdphat_ragged* ragged, int64_t* tuned,
                        int64_t* from_cache);
void svdphat_ragged_destroy(svdphat_ragged* ragged);

/*
 * Learned proposal.  Section 3 replaces the O(Q) scan of eq. (14) by a k-d
 * tree search; here a small network proposes where to look instead: an MLP
 * maps the normalised projection f = [Re Z; Im Z] / ||Z|| (Z of eq. (12))
 * through f -> GELU(W1 f + b1) -> GELU(W2 . + b2) -> W3 . + b3 (GELU with
 * erf to 1.5e-7, `hidden` units) to C coarse cells of the direction grid (the cell of
 * a direction is its nearest coarse direction, ties within 1e-12 to the lowest
 * cell).  The scored directions of the topk most probable cells are rescored
 * exactly in FP32; frames whose top probability is below conf_min take the
 * full search (svdphat_locate, FP16 + rescoring) instead.
 *
 * svdphat_proposal_create  fine: a plan (not owned; must outlive the
 *   proposal; created without SVDPHAT_NO_DEDUP); coarse_xyz: host C x 3
 *   directions; hidden: multiple of 64 in [64, 1024]; seed: weight init.
 * svdphat_proposal_train_step  one Adam step (lr; beta 0.9 / 0.999, eps 1e-8)
 *   on F device frames X [F][M][N/2+1]: labels are the cells of the method's
 *   own argmax (svdphat_locate FP16, rescoring, hi/lo), the loss is the mean
 *   softmax cross-entropy (written to *loss_host).  FP16 operands on MFMA,
 *   FP32 accumulation and master weights.  Synchronous.
 * svdphat_proposal_locate  doa [F] int32, power [F] f32 as svdphat_locate,
 *   fell_back [F] u8 = 1 where the full search was used (top probability
 *   below conf_min, or no scored direction in any of the topk cells): the
 *   search of svdphat_locate with SVDPHAT_FP16 and SVDPHAT_RESCORE, without
 *   the hi/lo pass.  Asynchronous.
 * svdphat_proposal_params  copies the FP32 parameters to (set = 0) or from
 *   (set = 1) a host buffer of svdphat_proposal_nparams() floats laid out
 *   W1 [hidden][2K], b1 [hidden], W2 [hidden][hidden], b2 [hidden],
 *   W3 [C][hidden], b3 [C], row-major.
 * svdphat_proposal_grad  testing aid: mean loss and its gradient (same layout)
 *   for host features [F][2K] and labels [F].
 * svdphat_proposal_cells  host [Q]: cell of every fine direction.
 * svdphat_proposal_save  writes the coarse directions, the FP32 parameters,
 *   the Adam moments and the step count, with the fine plan's input hash,
 *   to `path` (versioned little-endian binary with a checksum).
 * svdphat_proposal_load  reads such a file into a new proposal over `fine`,
 *   which must have the same input hash as the plan the file was saved with
 *   (E_INVAL otherwise); training can continue from the saved state.
 *   Errors of both: E_IO, E_INVAL (as for plans), E_NOMEM, E_DEVICE.
 * svdphat_proposal_features  testing aid: the network input of F device frames
 *   X, written to device f32 [F][2K] (the FP16 values the network reads,
 *   widened); synchronous.  The columns follow the plan's singular vectors,
 *   so they are defined up to a unitary change of basis within each group of
 *   equal singular values (a phase per vector when they are distinct).
 * svdphat_proposal_apply_grad  testing aid: one Adam step (beta 0.9 / 0.999,
 *   eps 1e-8, bias correction at the proposal's next step count) with the
 *   given host mean gradient of svdphat_proposal_nparams() floats in the
 *   layout of svdphat_proposal_params; the same update kernel as the
 *   training step.  Synchronous.
 */
typedef struct svdphat_proposal svdphat_proposal;
int svdphat_proposal_create(svdphat_plan* fine, const double* coarse_xyz,
                            int32_t C, int32_t hidden, uint64_t seed,
                            svdphat_proposal** out);
int svdphat_proposal_train_step(svdphat_proposal* proposal, const void* X,
                                int64_t F, float lr, float* loss_host,
                                void* stream);
int svdphat_proposal_locate(svdphat_proposal* proposal, const void* X,
                            int64_t F, int32_t topk, float conf_min,
                            int32_t* doa, float* power, uint8_t* fell_back,
                            void* stream);
int64_t svdphat_proposal_nparams(const svdphat_proposal* proposal);
int svdphat_proposal_params(svdphat_proposal* proposal, float* host,
                            int64_t n, int32_t set);
int svdphat_proposal_grad(svdphat_proposal* proposal, const float* features,
                          const int32_t* labels, int64_t F, float* grad,
                          float* loss_host);
int svdphat_proposal_cells(const svdphat_proposal* proposal,
                           int32_t* cell_of_direction);
int svdphat_proposal_save(const svdphat_proposal* proposal, const char* path);
int svdphat_proposal_load(svdphat_plan* fine, const char* path,
                          svdphat_proposal** out);
int svdphat_proposal_features(svdphat_proposal* proposal, const void* X,
                              int64_t F, float* feat, void* stream);
int svdphat_proposal_apply_grad(svdphat_proposal* proposal, const float* grad,
                                int64_t n, float lr);
void svdphat_proposal_destroy(svdphat_proposal* proposal);

/* svdphat_plan_destroy -- frees the plan and its device memory; NULL is a no-op. */
void svdphat_plan_destroy(svdphat_plan* plan);

/* svdphat_last_error -- message of the last failure on this thread ("" if none). */
const char* svdphat_last_error(void);

/* svdphat_sync -- waits for the stream and reports any pending device error. */
int svdphat_sync(void* stream);

/* ---- several sources per frame ----------------------------------------- */
/*
 * svdphat_peaks -- the n strongest separated directions of each frame (the
 * paper leaves several sources to future work, Section 5): peak p is the
 * largest y among the directions that are not an earlier peak and whose
 * unit vector has a dot product below cos_sep with every earlier peak's
 * (ties to the lowest index); with no direction left, idx = -1 and
 * val = -inf.  NaN powers never count.  Dot products are rounded product
 * by product, (x x' + y y') + z z', in FP32.
 *   y      device, f32 [F][ldy]: powers of the Q directions of each frame
 *          (e.g. the y_opt output of svdphat_locate, ldy = Q).
 *   dirs   device, f32 [Q][3]: unit vectors of the directions.
 *   n      peaks per frame, 1 <= n <= 16.  cos_sep: cosine of the separation.
 *   idx    device, int32 [F][n];  val  device, f32 [F][n] (written).
 *   stream hipStream_t or NULL; asynchronous.  F = 0 is a no-op.
 * Errors: E_INVAL (F < 0, Q < 1, ldy < Q, n out of range, NULL pointers
 * with F > 0), E_NODEV, E_DEVICE.
 */
int svdphat_peaks(const float* y, int64_t F, int32_t Q, int64_t ldy,
                  const float* dirs, int32_t n, float cos_sep, int32_t* idx,
                  float* val, void* stream);

/* ---- STFT front end ---------------------------------------------------- */
/*
 * svdphat_stft_frames -- number of whole frames in T samples:
 * 1 + (T - N) / hop, or 0 when T < N; -1 for T < 0, N < 1 or hop < 1.
 */
int64_t svdphat_stft_frames(int64_t T, int32_t N, int32_t hop);

/*
 * svdphat_stft -- the short-time Fourier transform that Section 2 applies to
 * each microphone signal before the PHAT (frames of N samples, sine window),
 * on the GPU, writing the STFT frames svdphat_locate reads:
 *   X[f][m][k] = sum_{n<N} w[n] pcm[m][f hop + n] exp(-2 pi i k n / N),
 *   w[n] = sin(pi n / N), k = 0 .. N/2, f < F = svdphat_stft_frames(T, N, hop).
 *   pcm    device, f32: microphone m's T samples at pcm + m * ld.
 *   M      microphones, >= 1.
 *   T      samples per microphone, >= 0;  ld >= T the microphone stride.
 *   N      frame size: a power of two, 16 <= N <= 2048.
 *   hop    samples between frame starts, >= 1.
 *   X      device, complex64 [F][M][N/2+1], written (owned by the caller).
 *   stream hipStream_t or NULL; asynchronous.  The current HIP device runs it.
 * FP32 arithmetic (twiddles and window evaluated in FP64, rounded to FP32).
 * F = 0 is a no-op.  Errors: E_INVAL (M < 1, T < 0, ld < T, hop < 1, NULL
 * pointers with F > 0), E_UNSUPPORTED (N), E_NODEV, E_DEVICE.
 */
int svdphat_stft(const float* pcm, int32_t M, int64_t T, int64_t ld,
                 int32_t N, int32_t hop, void* X, void* stream);

/*
 * Per-kernel timing (instrumentation, not part of the method).
 * svdphat_timing_enable(enable): bit 0 brackets every kernel that the
 * library launches with HIP events on the launch's stream; each call then
 * waits for its own events before returning and adds the elapsed time to a
 * process-wide table keyed by kernel name.  Bit 1 makes the search kernels
 * count events (atomic counters, which slow them; keep it apart from
 * timing).  svdphat_timing_read returns entry `index` (0-based,
 * names in lexicographic order): name (NUL-terminated, truncated to
 * name_len), total milliseconds and launch count; E_INVAL past the last entry.
 * Entries named "count:*" hold event counts in place of milliseconds and
 * the number of frames they were counted over in place of launches
 * ("count:final_tiles_rescored": direction tiles rescored in FP32;
 * "count:frames_hilo": frames recomputed with the hi/lo product).
 * svdphat_timing_reset clears the table.
 */
int svdphat_timing_enable(int enable);
int svdphat_timing_reset(void);
int svdphat_timing_read(int32_t index, char* name, int32_t name_len,
                        double* total_ms, int64_t* launches);

/* svdphat_version -- ABI version (major * 10000 + minor * 100 + patch). */
int svdphat_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SVDPHAT_H */
