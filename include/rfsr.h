/*
 * rfsr.h - C ABI of the MI355X (gfx950) library for recursive frequency
 * selective reconstruction (FSR) of quarter-sampled video with fast motion
 * consistency checks (Grosche, Seiler, Kaup, ICIP 2021).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every image pointer is a DEVICE pointer owned by the caller.  Planes are
 *    row-major H x W with a row stride `pitch` given in ELEMENTS of the
 *    plane's own type (pitch >= W); all planes of one call share `pitch`.
 *  - The library allocates no device memory.  Scratch space is the caller's
 *    `workspace` (device, >= rfsr_workspace_bytes(...) bytes, 256-byte
 *    aligned); its contents on entry are irrelevant and on exit undefined.
 *    (fsr_blocks_noalloc uses a fixed array inside the library instead.)
 *  - All work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *    void*; NULL is the default stream).  The return value reports argument
 *    validation and launch errors synchronously; a device fault of this call
 *    surfaces at the caller's next synchronisation.
 *  - H and W must be positive multiples of 4 (the FSR block size, hence also
 *    of the 2x2 quarter-sampling cell) and at most 16384.
 *  - Masks hold 0 (not measured) or 1 (measured).  Measured-frame values at
 *    unmeasured positions never influence a result (kernels may load them
 *    at in-bounds addresses and discard them), so they may hold anything.
 *  - Motion vectors are (alpha, beta) = (row offset, column offset), int8.
 *  - Calls on different streams do not share state and may run concurrently
 *    as long as their workspaces differ.
 */
#ifndef RFSR_H
#define RFSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RFSR_OK = 0,
    RFSR_EINVAL = -1,        /* null pointer or parameter out of range          */
    RFSR_ESHAPE = -2,        /* H, W or pitch not supported                     */
    RFSR_EWORKSPACE = -3,    /* workspace null, too small or misaligned         */
    RFSR_EDEVICE = -4,       /* HIP runtime error (no device, launch failure)   */
    RFSR_EUNSUPPORTED = -5   /* valid request this library does not implement   */
} rfsr_status;

/* Consistency check applied to the forward motion field.
 *   NONE      every vector accepted.
 *   RME       reverse motion estimation: accept iff the reverse vector at
 *             q = p + v equals -v (Sec. 2.2, the literature check).
 *   RMC       reverse motion check: accept iff the back-pointing candidate
 *             has strictly the lowest normalised cost among the reverse
 *             candidates [-rmc_radius, rmc_radius]^2 placed symmetrically
 *             around it (Sec. 3.1.1, Fig. 2b).
 *   FRMC      the same test with offsets {-7,-3,-1,0,1,3,7}^2 (Sec. 3.1.1,
 *             Fig. 2c), or the set in rfsr_me_params.frmc.
 *   NNC       nearest-neighbour check on the 3x3 median filtered field
 *             (Sec. 3.1.2, Eq. (1), Fig. 2d).
 *   NNC_FRMC  NNC, then FRMC only where NNC accepted (Sec. 3.1.2, Table 3). */
typedef enum {
    RFSR_CHECK_NONE = 0,
    RFSR_CHECK_RME = 1,
    RFSR_CHECK_RMC = 2,
    RFSR_CHECK_FRMC = 3,
    RFSR_CHECK_NNC = 4,
    RFSR_CHECK_NNC_FRMC = 5
} rfsr_check;

/* Final overwrite of the FSR model (Sec. 3.2): D-FSR writes only measured
 * pixels over the model, R-FSR writes measured and projected pixels. */
typedef enum { RFSR_DFSR = 0, RFSR_RFSR = 1 } rfsr_overwrite;

/* Motion estimation by pixel-wise template matching (Sec. 2.2).
 * Cost of vector v at pixel p, template offsets D = {-1,0,1,2}^2:
 *   S(p,v) = sum_{d in D, p+d in frame} b_t(p+d) |f_t(p+d) - Rhat(clamp(p+d+v))|
 * minimised over v in [-search, search]^2 with p+v in the frame, with the
 * total order (S, |v|_1, raster index of v).  Reverse costs (RME, RMC, FRMC)
 * belong to different current-frame pixels and are compared normalised by
 * n, the number of measured template pixels (S_a n_b against S_b n_a).
 *
 * Options beside the paper's setting (defaults reproduce it):
 *   n_frmc, frmc  FRMC's per-axis offset set (Sec. 3.1.1 prints
 *                 {-7,-3,-1,0,1,3,7}; the Fig. 2 caption shows a small range
 *                 {-2,-1,0,1,2}): n_frmc = 0 selects the paper's set, else
 *                 frmc[0..n_frmc-1] (n_frmc <= 15) strictly increasing,
 *                 containing 0, each |d| <= 14.  Used by FRMC and NNC_FRMC.
 *   cost_norm     1: reverse costs compared as S/n (the default reading);
 *                 0: raw S (an ablation of the normalisation).
 *   nnc_center    RFSR_NNC_FILTERED: NNC compares the filtered vector at p
 *                 with the filtered vectors of its four neighbours (the
 *                 reading of Sec. 3.1.2); RFSR_NNC_RAW: the raw vector at p
 *                 with the filtered neighbours. */
typedef enum { RFSR_NNC_FILTERED = 0, RFSR_NNC_RAW = 1 } rfsr_nnc_center;
typedef struct {
    int32_t tmpl;        /* template size; the library supports 4           */
    int32_t search;      /* search radius R, 0..15                            */
    int32_t check;       /* rfsr_check                                        */
    int32_t rmc_radius;  /* RMC radius, 0..15; 0 selects `search`             */
    int32_t n_frmc;      /* 0..15 FRMC offsets in frmc[]; 0: the paper's set  */
    int8_t frmc[16];     /* FRMC per-axis offsets (first n_frmc entries used) */
    int32_t cost_norm;   /* 1: S/n (default); 0: raw S                        */
    int32_t nnc_center;  /* rfsr_nnc_center                                   */
} rfsr_me_params;

/* Block-wise FSR (Sec. 2.1) with concealed weighting 0 (Sec. 4), so blocks
 * are independent.  Each B x B block is modelled on the M x M support
 * centred on it by K greedy iterations over the M x M complex DFT basis:
 * pick the bin with the largest weighted residual energy, add
 * gamma * R_b / W0 to its coefficient, subtract it from the residual.
 * Weights: a * rho^(distance to the support centre), a = 1 measured,
 * proj_weight projected, 0 unknown / outside the frame.  By default the
 * transform, the residual spectrum and its energies are float64 (`precision`
 * below selects the other forms); the list of picks keeps R_b in float32
 * and the output is float32, which bounds the output error near 1e-5 on the
 * 0..255 scale.  In float32 the residual carries rounding of the order of
 * 2^-24 times the block's spectral norm, which turns late near-tie picks the
 * other way in about two blocks per thousand at K = 100. */
typedef struct {
    int32_t block;       /* B; the library supports 4                        */
    int32_t support;     /* M; the library supports 32                       */
    int32_t iters;       /* K, 0..1024                                        */
    int32_t overwrite;   /* rfsr_overwrite                                    */
    double rho;          /* 0 < rho <= 1                                      */
    double gamma;        /* 0 < gamma < 2                                     */
    double proj_weight;  /* >= 0, weight of projected samples                 */
    int32_t precision;   /* rfsr_precision (0 = float64)                      */
    int32_t pairs;       /* 0: complex single bins; 1: conjugate pairs        */
    double concealed_weight; /* delta, 0 <= delta <= 1 (0 = independent blocks) */
    double prior_sigma;  /* frequency-weighting prior, 0 (off) or 0 < sigma <= 1 */
    double stop_ratio;   /* residual-energy early stop, 0 (off) or 0 < ratio < 1 */
    double mixed_bound;  /* RFSR_PREC_MIXED: near-tie bound a > 0 (below)    */
    float* block_margin; /* RFSR_PREC_FP32, nullable: per-block margins (below) */
    unsigned long long* rerun_blocks; /* RFSR_PREC_MIXED, nullable: device
                            counter, ADDED the number of blocks recomputed   */
} rfsr_fsr_params;

/* Basis selection.  pairs = 0 (default): every iteration adds one complex
 * basis function (first maximum in row-major order), the reading used for
 * the paper's FSR.  pairs = 1: real-valued FSR as the FSR literature uses
 * for real images: every iteration adds the conjugate pair
 * dlt phi_b + conj(dlt) phi_-b (one term when b = -b), so the residual stays
 * real and only half of its spectrum is updated (R_k -= dlt W_{k-b} +
 * conj(dlt) W_{k+b}); one pair iteration does the work of about two complex
 * ones.  Not combined with concealed_weight > 0 (RFSR_EUNSUPPORTED).
 *
 * Concealed weighting (the FSR setting Sec. 4 sets to 0): with delta > 0 the
 * blocks are reconstructed in raster order and an unknown pixel of an earlier
 * block enters the supports of later blocks as a sample of weight
 * delta * rho^dist carrying its reconstructed (unclamped) value.  The GPU
 * runs it as a wavefront, one launch per step t = 5 bi + bj (every
 * raster-earlier block within a support has a smaller t; the blocks of one
 * step never share a support), i.e. 5 (H/4 - 1) + W/4 dependent launches per
 * frame.  rfsr_reconstruct_batch runs the steps of all its frames together
 * (one launch per step holding every frame's blocks of that step), so many
 * streams fill the GPU that one frame's wavefront leaves idle.
 *
 * Two options of the FSR literature that the paper's configuration does not
 * use (both 0 = off by default; float64 FFT, complex single bins and
 * independent blocks only, else RFSR_EUNSUPPORTED):
 *   prior_sigma: the pick maximises prior_k |R_k|^2 with prior_k =
 *     sigma^|k|, |k| the Euclidean distance of (min(k1, 32-k1),
 *     min(k2, 32-k2)) from DC, so low frequencies are favoured; the update
 *     is unchanged.
 *   stop_ratio: a block stops before iteration i >= 1 once its pick's
 *     criterion value (prior_b |R_b|^2, or |R_b|^2) falls below stop_ratio
 *     times that of its first iteration.
 * They run in a kernel of their own, so the default loop carries no test
 * for them. */

/* Arithmetic of FSR.  FP64, BF16X3 and FP16X3 select the block DFT that
 * starts FSR (R = DFT(w s), W = DFT(w)) and keep the iterations in float64:
 *   FP64     float64 FFT on the vector ALU (the reference precision).
 *   BF16X3   two 32x32 GEMM stages on the matrix cores (MFMA), operands
 *            split as hi + lo in bfloat16, products hi*hi + hi*lo + lo*hi
 *            accumulated in float32.
 *   FP16X3   the same with float16 operands.
 *   FP32     every step in float32: FFT (w packed at 128 times its scale so
 *            that W and w*s round alike), table, residual and energies (the
 *            plain float32 form).  Complex single bins and independent
 *            blocks only (pairs, concealed_weight > 0 and the literature
 *            options give RFSR_EUNSUPPORTED).
 *   MIXED    FP32 with a near-tie test and float64 for the blocks that fail
 *            it (below); held to the float64 form's tolerance.
 * BF16X3, FP16X3 and FP32 trade accuracy (float32 accumulation, ~2^-16 /
 * ~2^-22 operand splits, float32 rounding of the residual) for throughput;
 * they are not bit-compatible with FP64 and are not held to its 1e-3 output
 * tolerance: they exist to quantify that trade. */
typedef enum {
    RFSR_PREC_FP64 = 0,
    RFSR_PREC_BF16X3 = 1,
    RFSR_PREC_FP16X3 = 2,
    RFSR_PREC_FP32 = 3,
    RFSR_PREC_MIXED = 4
} rfsr_precision;

/* RFSR_PREC_MIXED: the float32 form with a near-tie test, and float64 for
 * the blocks that fail it, so that every block follows the float64 model.
 * The float32 residual differs from the float64 one by rounding of the order
 * of u ||R^0||_2 in every bin (u = 2^-24, R^0 the block's initial weighted
 * residual spectrum; the FFT's rounding dominates and the updates add little),
 * so a float32 pick can differ from the float64 model's only where the pick's
 * energy E_b and the largest other energy E_next (not counting, while the
 * spectrum is still Hermitian, the pick's conjugate partner, which ties
 * exactly and leads to the same real model) are that close.  A block is
 * recomputed by the float64 kernel if at some iteration
 *     E_b - E_next <= 4 a u ||R^0||_2 |R_b|      (a = mixed_bound)
 * i.e. |R_b| - |R_next| below about 2 a u ||R^0||_2; the float32 pass of such
 * a block stops there.  Complex single bins and independent blocks only, as
 * FP32.  RFSR_MIXED_BOUND is the bound the library is measured with: the
 * flips of the plain float32 form were all found at margins far below it.
 *
 * block_margin (RFSR_PREC_FP32 only, a diagnostic that calibrates a): device
 * float per block of the call (flat block index, row-major per frame, frames
 * in call order), receiving the smallest (E_b - E_next) / (4 u ||R^0||_2 |R_b|)
 * over the block's iterations; RFSR_PREC_MIXED with bound a recomputes
 * exactly the blocks whose margin is at most a.  Ignored by other precisions.
 * rerun_blocks (RFSR_PREC_MIXED only): device counter the call adds the
 * number of recomputed blocks to; nullable. */
#define RFSR_MIXED_BOUND 1.0

/* Indices into the optional counters array of rfsr_motion_check. */
enum {
    RFSR_CNT_FORWARD_COSTS = 0,   /* forward template costs evaluated          */
    RFSR_CNT_CHECK_COSTS = 1,     /* reverse template costs evaluated by the
                                     check (RME, RMC, FRMC; RMC stops at the
                                     first losing candidate, FRMC after the
                                     first offset row that holds one)          */
    RFSR_CNT_CHECKED_PIXELS = 2,  /* pixels that entered the RMC/FRMC test     */
    RFSR_CNT_ACCEPTED = 3,        /* accepted pixels                           */
    RFSR_NCOUNTERS = 4
};

/* Bytes of workspace sufficient for any call of this library on an H x W
 * frame with up to `nref` references (0..3) and these parameters.
 * Returns 0 if the arguments are invalid. */
size_t rfsr_workspace_bytes(int32_t H, int32_t W, int32_t nref,
                            const rfsr_me_params* me, const rfsr_fsr_params* fsr);

/* Forward motion estimation of the current frame against one reference
 * reconstruction, followed by the consistency check `me->check`
 * (Sec. 2.2, Sec. 3.1).
 *   cur        uint8 H x W measured frame f_t (used only where cur_mask==1)
 *   cur_mask   uint8 H x W mask b_t
 *   ref_recon  uint8 H x W reconstruction of the past frame
 *   mv         int8 [2][H][W] out: plane 0 alpha (rows), plane 1 beta (cols);
 *              plane 1 starts at mv + H*pitch
 *   accept     uint8 H x W out: 1 accepted, 0 rejected
 *   cost       uint16 H x W out (nullable): S of the chosen vector
 *   counters   uint64 [RFSR_NCOUNTERS] (nullable): ADDED to (caller zeroes)
 * Errors: RFSR_EINVAL (null input/output, bad params), RFSR_ESHAPE,
 * RFSR_EWORKSPACE, RFSR_EUNSUPPORTED (tmpl != 4), RFSR_EDEVICE. */
rfsr_status rfsr_motion_check(const uint8_t* cur, const uint8_t* cur_mask,
                              const uint8_t* ref_recon, int32_t H, int32_t W,
                              int64_t pitch, const rfsr_me_params* me,
                              int8_t* mv, uint8_t* accept, uint16_t* cost,
                              unsigned long long* counters,
                              void* workspace, size_t ws_bytes, void* stream);

/* Block-parallel FSR of one frame (Sec. 2.1; Sec. 3.2 for classes).
 *   values  float32 H x W sample values, used only where cls > 0
 *   cls     uint8 H x W: 0 unknown, 1 measured, 2 projected (others = 0)
 *   out     float32 H x W out: Re of the model, then the overwrite rule;
 *           not clamped
 *   out_u8  uint8 H x W out (nullable): rint(clamp(out, 0, 255)), ties to even
 * Errors: RFSR_EINVAL, RFSR_ESHAPE, RFSR_EWORKSPACE, RFSR_EUNSUPPORTED
 * (block != 4 or support != 32), RFSR_EDEVICE. */
rfsr_status fsr_blocks(const float* values, const uint8_t* cls, int32_t H, int32_t W,
                       int64_t pitch, const rfsr_fsr_params* fsr,
                       float* out, uint8_t* out_u8,
                       void* workspace, size_t ws_bytes, void* stream);

/* fsr_blocks without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  The call allocates nothing; its scratch (the FSR
 * tables, 17 KB, and for RFSR_PREC_MIXED the lists of blocks to recompute,
 * 4 bytes per block + 256) lives in an array inside the library of
 * RFSR_NOALLOC_SCRATCH_BYTES per device (enough for the mixed form up to
 * about a million blocks, i.e. 16 megapixels), which every device that runs
 * the library holds until the process ends.  All calls on one device share that
 * device's array: calls that overlap on one device (different streams or
 * threads) race, and the caller must serialise them.  The array keeps the
 * last call's contents; nothing in it needs to start at zero (each call
 * rewrites what it reads).  Arguments and results as fsr_blocks.
 * Errors: as fsr_blocks; RFSR_EWORKSPACE if the request needs more scratch
 * than the array holds; RFSR_EDEVICE if the array's device address cannot be
 * obtained on the current device. */
#define RFSR_NOALLOC_SCRATCH_BYTES 4194304
rfsr_status fsr_blocks_noalloc(const float* values, const uint8_t* cls, int32_t H, int32_t W,
                               int64_t pitch, const rfsr_fsr_params* fsr,
                               float* out, uint8_t* out_u8, void* stream);

/* One recursive D-FSR / R-FSR frame in the order of Fig. 1: for each of the
 * nref (0..3) references, forward ME against its reconstruction and the
 * consistency check; projection of the measured reference pixels that the
 * accepted vectors point to (averaged over references, Sec. 2.2); FSR with
 * measured and projected samples; overwrite; quantisation.
 *   ref_recon, ref_meas, ref_mask: HOST arrays of nref device pointers,
 *     index k = lag k+1 (uint8 H x W each; ref_meas used only where
 *     ref_mask == 1).  May be NULL when nref == 0 (single-frame FSR).
 *   out     float32 H x W out; out_u8 uint8 H x W out (nullable)
 *   stage_events: NULL, or a HOST array of 4 events (from rfsr_event_create)
 *     recorded on `stream` at: [0] start, [1] after ME and checks,
 *     [2] after projection, [3] after FSR.
 * The frame runs as a batch of one (rfsr_reconstruct_batch below): its job
 * tables are written into a 1 KB slot after the frame's scratch by a kernel,
 * so the call enqueues only kernels and event records, and each stage is one
 * launch over all references.
 * Errors: as rfsr_motion_check and fsr_blocks. */
rfsr_status rfsr_reconstruct_frame(const uint8_t* cur, const uint8_t* cur_mask, int32_t nref,
                                   const uint8_t* const* ref_recon,
                                   const uint8_t* const* ref_meas,
                                   const uint8_t* const* ref_mask,
                                   int32_t H, int32_t W, int64_t pitch,
                                   const rfsr_me_params* me, const rfsr_fsr_params* fsr,
                                   float* out, uint8_t* out_u8, void* const* stage_events,
                                   void* workspace, size_t ws_bytes, void* stream);

/* The same frame in two calls, so that consecutive frames of a recursion can
 * overlap (Fig. 1 order and results unchanged).  Frame t+1's references of
 * lag >= 2 are frames t-1 and t-2, final before frame t is; their motion
 * path can run on a second stream while frame t's FSR runs, and only the
 * lag-1 reference (frame t) waits for frame t.
 *
 * rfsr_frame_motion: the window plane of the current frame and the forward ME
 * and consistency check of references first..nref-1 (lags first+1..nref),
 * into `workspace`.  Arguments as rfsr_reconstruct_frame; 0 <= first <= nref
 * (first == nref: nothing to do).
 *
 * rfsr_frame_finish: the forward ME and check of references 0..first-1, the
 * projection over all nref references, FSR, overwrite and quantisation, i.e.
 * the rest of the frame.  With first < nref it requires a preceding
 * rfsr_frame_motion(..., first, ...) with the same arguments and workspace,
 * ordered before this call by the caller (same stream, or an event); with
 * first == nref it is rfsr_reconstruct_frame.  Its stage events cover its
 * own work ([1]: after the ME and checks of references 0..first-1).  The two
 * calls write their job tables to separate 1 KB slots of the workspace
 * (rfsr_workspace_bytes covers both); the workspace must not be used by
 * another frame until the second call's work has completed.
 * Errors: as rfsr_reconstruct_frame; RFSR_EINVAL for first outside 0..nref. */
rfsr_status rfsr_frame_motion(const uint8_t* cur, const uint8_t* cur_mask, int32_t nref,
                              const uint8_t* const* ref_recon,
                              const uint8_t* const* ref_meas,
                              const uint8_t* const* ref_mask,
                              int32_t H, int32_t W, int64_t pitch,
                              const rfsr_me_params* me, int32_t first,
                              void* workspace, size_t ws_bytes, void* stream);
rfsr_status rfsr_frame_finish(const uint8_t* cur, const uint8_t* cur_mask, int32_t nref,
                              const uint8_t* const* ref_recon,
                              const uint8_t* const* ref_meas,
                              const uint8_t* const* ref_mask,
                              int32_t H, int32_t W, int64_t pitch,
                              const rfsr_me_params* me, const rfsr_fsr_params* fsr,
                              int32_t first, float* out, uint8_t* out_u8,
                              void* const* stage_events,
                              void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- batches ---
 * Many independent streams of recursive reconstruction advance one time step
 * together: every frame of the batch is a separate rfsr_reconstruct_frame
 * problem (its own size, mask, references and outputs; Fig. 1 per stream),
 * but the whole batch runs as ONE launch chain (window planes, forward ME,
 * checks, projection, FSR: each stage one kernel over all frames), so that
 * small and large frames fill the GPU together and the chain can be captured
 * once in a HIP graph and replayed.  Results equal those of
 * rfsr_reconstruct_frame on each frame alone, bit for bit. */
typedef struct {
    const uint8_t* cur;           /* uint8 H x W measured frame (device)        */
    const uint8_t* cur_mask;      /* uint8 H x W mask (device)                  */
    const uint8_t* ref_recon[3];  /* nref reconstructions, index k = lag k+1    */
    const uint8_t* ref_meas[3];   /* their measured frames                      */
    const uint8_t* ref_mask[3];   /* their masks                                */
    float* out;                   /* float32 H x W out                          */
    uint8_t* out_u8;              /* uint8 H x W out (nullable)                 */
    int32_t nref;                 /* 0..3                                       */
    int32_t H, W;                 /* multiples of 4, at most 16384              */
    int32_t reserved;             /* set to 0                                   */
    int64_t pitch;                /* elements, shared by this frame's planes    */
} rfsr_frame_desc;

/* Workspace bytes of rfsr_reconstruct_batch for these frames (1..4096 of
 * them); 0 if the descriptors are invalid. */
size_t rfsr_batch_workspace_bytes(const rfsr_frame_desc* frames, int32_t n,
                                  const rfsr_me_params* me, const rfsr_fsr_params* fsr);

/* Bytes of the batch's job-table image (a multiple of 256); 0 if invalid. */
size_t rfsr_batch_table_bytes(const rfsr_frame_desc* frames, int32_t n);

/* Writes the job-table image of the batch into the HOST buffer `image`
 * (>= rfsr_batch_table_bytes bytes): a header, then the per-frame and
 * per-reference jobs the kernels read (device pointers into the frames and
 * into `workspace`, each job's first workgroup in the merged grids).
 * `workspace` is only used as an address.  The caller copies the image to a
 * device buffer (256-byte aligned) that it passes as `job_tables`; the image
 * stays valid for every later call with the same descriptors, the same
 * me->check and the same workspace (e.g. replays of a captured graph).  The
 * header holds a hash of exactly these; kernels given an image whose hash
 * differs from the call's skip all work (outputs are left unwritten).
 * Errors: RFSR_EINVAL (bad descriptors, image too small), RFSR_EWORKSPACE
 * (null or misaligned workspace), as rfsr_reconstruct_frame otherwise. */
rfsr_status rfsr_batch_write_tables(const rfsr_frame_desc* frames, int32_t n,
                                    const rfsr_me_params* me, const void* workspace,
                                    void* image, size_t image_bytes);

/* One time step of n streams: rfsr_reconstruct_frame on every frame of
 * `frames`, as one chain of kernel launches on `stream`.
 *   job_tables  DEVICE copy of the image rfsr_batch_write_tables wrote for
 *               these descriptors, me->check and workspace (256-byte aligned)
 *   workspace   device, >= rfsr_batch_workspace_bytes, 256-byte aligned
 * The call only enqueues kernels and event records (no copies, no memsets),
 * so it may be captured in a graph.
 * stage_events: NULL or 4 events, as rfsr_reconstruct_frame (for the batch).
 * Errors: as rfsr_reconstruct_frame; RFSR_EINVAL for a null or misaligned
 * job_tables. */
rfsr_status rfsr_reconstruct_batch(const rfsr_frame_desc* frames, int32_t n,
                                   const rfsr_me_params* me, const rfsr_fsr_params* fsr,
                                   const void* job_tables, void* const* stage_events,
                                   void* workspace, size_t ws_bytes, void* stream);

/* A batch split like rfsr_frame_motion / rfsr_frame_finish, for pipelining
 * consecutive time steps of the same streams (results unchanged):
 *   RFSR_PART_MOTION  window planes and motion path of every frame's
 *                     references first..nref-1 (frames with nref <= first:
 *                     nothing); `fsr` may be NULL;
 *   RFSR_PART_FINISH  references 0..first-1, the window planes of frames
 *                     without early references, projections and FSR; the
 *                     MOTION part with the same frames, `first` and workspace
 *                     must be ordered before it by the caller;
 *   RFSR_PART_ALL     whole frames (rfsr_reconstruct_batch; `first` ignored).
 * Each part reads its own job-table image, written by
 * rfsr_batch_write_tables_part with the same part and first (at most
 * rfsr_batch_table_bytes bytes).  0 <= first <= 3.
 * Errors: as rfsr_batch_write_tables / rfsr_reconstruct_batch; RFSR_EINVAL
 * for an unknown part or first outside 0..3. */
typedef enum { RFSR_PART_ALL = 0, RFSR_PART_MOTION = 1, RFSR_PART_FINISH = 2 } rfsr_part;
rfsr_status rfsr_batch_write_tables_part(const rfsr_frame_desc* frames, int32_t n,
                                         const rfsr_me_params* me, int32_t part, int32_t first,
                                         const void* workspace, void* image, size_t image_bytes);
rfsr_status rfsr_reconstruct_batch_part(const rfsr_frame_desc* frames, int32_t n,
                                        const rfsr_me_params* me, const rfsr_fsr_params* fsr,
                                        int32_t part, int32_t first, const void* job_tables,
                                        void* const* stage_events, void* workspace, size_t ws_bytes,
                                        void* stream);

/* ------------------------------------------------------------- quality ---
 * Reconstruction quality as evaluated in Sec. 4: PSNR and mean SSIM of a
 * reconstruction against the ground truth with a border of `border` pixels
 * omitted (the paper omits 40) and the reconstruction clipped to [0, 255]
 * (not rounded).  SSIM as defined by Wang et al. (IEEE TIP 2004, which the
 * paper cites): 11x11 Gaussian window of standard deviation 1.5, unit sum,
 * C1 = (0.01*255)^2, C2 = (0.03*255)^2, averaged over every window position
 * inside the cropped frame.  Accumulation in float64, reduced in a fixed
 * order (the result does not depend on scheduling).
 *   ref     uint8 H x W ground truth (device)
 *   test    float32 H x W reconstruction (device), same pitch
 *   result  DEVICE double[2] out: { PSNR in dB (+inf if identical), mean SSIM }
 * H and W need not be multiples of 4; the cropped frame must be >= 11 x 11.
 * Errors: RFSR_EINVAL (null pointer, border < 0), RFSR_ESHAPE (sizes, pitch,
 * cropped frame < 11 x 11), RFSR_EWORKSPACE, RFSR_EDEVICE. */
size_t rfsr_quality_workspace_bytes(int32_t H, int32_t W, int32_t border);
rfsr_status rfsr_quality(const uint8_t* ref, const float* test, int32_t H, int32_t W,
                         int64_t pitch, int32_t border, double* result,
                         void* workspace, size_t ws_bytes, void* stream);

/* Events for stage_events, benchmarks and ordering between streams (thin
 * wrappers of HIP events).  rfsr_event_elapsed_ms waits for `stop`;
 * rfsr_event_wait makes work enqueued on `stream` after it wait for the
 * event's last record (e.g. a frame's stage event [2], after which only its
 * FSR remains, to start the next frame's early motion path beside that FSR). */
rfsr_status rfsr_event_create(void** event);
rfsr_status rfsr_event_destroy(void* event);
rfsr_status rfsr_event_record(void* event, void* stream);
rfsr_status rfsr_event_elapsed_ms(void* start, void* stop, float* ms);
rfsr_status rfsr_event_wait(void* event, void* stream);

/* Human-readable name of a status code (static storage). */
const char* rfsr_status_string(int32_t status);

/* Library version, major*10000 + minor*100 + patch. */
int32_t rfsr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RFSR_H */
