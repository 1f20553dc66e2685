/* polsar.h -- per-pixel inverse and determinant of 3x3 complex Hermitian
 * positive-definite matrices (PolSAR multilook covariances), and the Wishart
 * log-likelihood with its gradient, on AMD Instinct MI355X (gfx950).
 *
 * Method: Coelho, Cintra, Frery, Dimitrov, "Fast Matrix Inversion and
 * Determinant Computation for Polarimetric Synthetic Aperture Radar":
 * Alg. 2 (adjugate + real-part determinant, Section 3.1) is the method;
 * Alg. 1 (Cholesky, Section 2.2) is built beside it for comparison.
 *
 * DATA LAYOUT.  A batch of n matrices is nine planes of n reals each
 * (structure of arrays).  Plane k starts at base + k*pitch elements:
 *     k = 0:a  1:d  2:f  3:Re b  4:Im b  5:Re c  6:Im c  7:Re e  8:Im e
 * for A = [[a, b, c], [conj(b), d, e], [conj(c), conj(e), f]] (the upper
 * triangle, Section 2.1).  Inverses and gradients use the same packing.
 * Element type is float (POLSAR_F32) or double (POLSAR_F64) for every plane
 * of one call.  pitch >= n.  Pointers must be aligned to the element size;
 * when every plane base is 16-byte aligned (base and pitch*element size
 * multiples of 16, and the status plane 4-byte aligned for F32, 2-byte for
 * F64) the kernels move 64 or 128 bits per access (the launch table's
 * vector_bytes), otherwise one element.
 *
 * MEMORY AND STREAMS.  Unless stated, pointers are DEVICE pointers on the
 * current HIP device; the caller allocates and owns every buffer, the library
 * never frees caller memory.  Every call is asynchronous on `stream` (a
 * hipStream_t; NULL = the default stream); buffers must stay valid until the
 * stream reaches the work.
 *
 * ERRORS.  Calls return POLSAR_OK or a negative polsar_status.  Argument
 * errors are detected before any HIP call.  Per-pixel numerical outcomes are
 * never call errors: they go to the optional status plane (one byte per
 * pixel, POLSAR_PX_*) and to the optional counters (device array of three
 * unsigned 64-bit integers [not_pd, rerouted, nonfinite], ADDED to, so the
 * caller zeroes them).  n == 0 is a no-op returning POLSAR_OK (plane
 * pointers and the workspace may then be NULL; a forward Wishart pass still
 * writes a loss of 0).
 * Reentrant: calls share no mutable state except the launch-configuration
 * table, which is guarded.
 */
#ifndef POLSAR_H
#define POLSAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  POLSAR_OK = 0,
  POLSAR_E_ARG = -1,         /* null/negative/out-of-range argument, pitch < n */
  POLSAR_E_ALIGN = -2,       /* pointer not aligned to its element size */
  POLSAR_E_UNSUPPORTED = -3, /* valid enums, combination not provided */
  POLSAR_E_HIP = -4,         /* a HIP runtime call or launch failed */
  POLSAR_E_WORKSPACE = -5,   /* workspace missing or too small */
  POLSAR_E_ALIAS = -6        /* outputs overlap inputs (other than exact in-place) */
} polsar_status;

typedef enum { POLSAR_F32 = 0, POLSAR_F64 = 1 } polsar_dtype;
typedef enum { POLSAR_ADJUGATE = 0, POLSAR_CHOLESKY = 1 } polsar_method;

/* Arithmetic of one call.
 *   PLAIN        the algorithm in the storage type.
 *   COMPENSATED  ADJUGATE: Dot2-compensated cofactors and determinant (FMA
 *                error-free products and sums); in F32, pixels whose
 *                a-posteriori determinant error bound (a running error
 *                analysis of that evaluation, subnormal results included)
 *                exceeds 1e-6 relative,
 *                or whose det is not positive or not finite, are recomputed
 *                by the compensated F64 path (status POLSAR_PX_REROUTED).
 *                CHOLESKY (F32 only): F32, pixels whose pivots fail
 *                recomputed in F64.
 *   WIDE         F32 storage, F64 arithmetic (F32 only). */
typedef enum { POLSAR_PLAIN = 0, POLSAR_COMPENSATED = 1, POLSAR_WIDE = 2 } polsar_precision;

/* Per-pixel status values.  NOT_PD: the matrix is not positive definite —
 * adjugate forms test the leading principal minors a, a d - |b|^2 and det
 * (Sylvester's criterion; all three are by-products of Alg. 2), Cholesky
 * forms the squared pivots.  NONFINITE: an input or a result is Inf/NaN. */
enum { POLSAR_PX_OK = 0, POLSAR_PX_REROUTED = 1, POLSAR_PX_NOT_PD = 2, POLSAR_PX_NONFINITE = 3 };

/* Inverse and determinant of n packed Hermitian matrices (Alg. 2, Section
 * 3.1: cofactors of Eq. adjoint_elements, determinant of Eq. detr, t = 1/det,
 * inverse = t * adjugate per Eq. inv_adjoint; or Alg. 1 for CHOLESKY).
 *   z       in: 9 planes, pitch z_pitch
 *   inv     out (nullable): 9 planes of the inverse's upper triangle; may be
 *           exactly z with inv_pitch == z_pitch (in place)
 *   det     out (nullable): n determinants
 *   status  out (nullable): n bytes, POLSAR_PX_*
 *   counters in/out (nullable): 3 x uint64 added to
 * Outputs for non-positive-definite or singular pixels are the IEEE results
 * of the formulas (possibly Inf/NaN) with the status set. */
int polsar_inv_det(int dtype, int method, int precision, int64_t n,
                   const void* z, int64_t z_pitch,
                   void* inv, int64_t inv_pitch, void* det,
                   uint8_t* status, unsigned long long* counters, void* stream);

/* Fused multilook front end + inverse and determinant.  From N single-look
 * scattering vectors S(l) = (S_HH, S_HV, S_VV) per pixel (Introduction:
 * reciprocity, the scattering vector, and Eq. ZN read as the outer product)
 * forms Z = (1/N) sum_l S(l) S(l)^H with FP64 accumulation (for F32 looks
 * every product is exact), rounds it to the storage type, optionally stores
 * it, and returns exactly what polsar_inv_det returns for that stored Z.
 *   looks   in: 6*n_looks planes (pitch looks_pitch); plane 6l + 2i + 0/1 is
 *           Re/Im of component i (0 HH, 1 HV, 2 VV) of look l
 *   z       out (nullable): the 9 packed planes of Z (pitch z_pitch)
 *   inv, det, status, counters as for polsar_inv_det.
 * Saves the round trip of Z through memory (36 B/px in FP32 written and read
 * again).  Launch shape: op 2 of polsar_get_launch (unroll must be 1). */
int polsar_multilook_inv_det(int dtype, int method, int precision, int64_t n, int n_looks,
                             const void* looks, int64_t looks_pitch, void* z, int64_t z_pitch,
                             void* inv, int64_t inv_pitch, void* det, uint8_t* status,
                             unsigned long long* counters, void* stream);

/* Spatial (boxcar) multilook fused with the inverse and determinant: Eq. ZN
 * with the looks of pixel (y, x) taken from its (2r+1) x (2r+1)
 * neighbourhood in a single-look image of height x width pixels (row-major),
 * the window clipped at the image border:
 *   Z(y, x) = (1/|W|) sum_{(y', x') in W(y, x)} S(y', x') S(y', x')^H,
 *   W(y, x) = [max(0, y-r), min(H-1, y+r)] x [max(0, x-r), min(W-1, x+r)],
 * summed in FP64 (exact products for F32 input), rounded to the storage type,
 * optionally stored, and inverted exactly as polsar_inv_det inverts that
 * stored Z (same per-pixel function, same bits).
 *   s       in: 6 planes (pitch s_pitch), Re/Im of S_HH, S_HV, S_VV
 *   radius  r, 0..3 (windows 1x1 to 7x7)
 *   z       out (nullable): the 9 packed planes of Z (pitch z_pitch)
 *   inv, det, status, counters as for polsar_inv_det (at least one given).
 * Errors: POLSAR_E_ARG for a bad mode, negative or over-large sizes
 * (height, width <= 2^24, height*width <= 2^32) or radius; the plane checks,
 * alignment and POLSAR_E_ALIAS (any two of s, z, inv, det, status
 * overlapping) as for polsar_multilook_inv_det.  A block stages its tile and
 * halo of S in LDS; the launch shape is fixed. */
int polsar_boxcar_inv_det(int dtype, int method, int precision, int64_t height, int64_t width, int radius,
                          const void* s, int64_t s_pitch, void* z, int64_t z_pitch,
                          void* inv, int64_t inv_pitch, void* det, uint8_t* status,
                          unsigned long long* counters, void* stream);

/* Block-diagonal pixels (closing section: multifrequency data, whose matrix
 * is block diagonal with one Hermitian 3x3 block per band, each block
 * inverted by the proposed method): n_blocks blocks per pixel.
 *   z         in: 9*n_blocks planes; block b is planes 9b..9b+8 (pitch z_pitch)
 *   inv       out (nullable): same layout; may be exactly z (in place)
 *   det       out (nullable): product of the block determinants
 *   block_det out (nullable): n_blocks planes (pitch block_det_pitch)
 *   status    out (nullable): worst block status; counters count pixels.
 * Each block's inverse and determinant are bitwise those of polsar_inv_det. */
int polsar_blockdiag_inv_det(int dtype, int method, int precision, int64_t n, int n_blocks,
                             const void* z, int64_t z_pitch, void* inv, int64_t inv_pitch,
                             void* det, void* block_det, int64_t block_det_pitch,
                             uint8_t* status, unsigned long long* counters, void* stream);

/* Nonlocal-means filtering with stochastic distances between Wishart laws
 * (the use the Introduction gives for fast inverses and determinants: every
 * pixel is compared with each pixel of a (2r+1) x (2r+1) search window).
 *   out_p = sum_q w_pq Z_q / sum_q w_pq,  w_pq = exp(-d(Z_p, Z_q) / h),
 *   KL:            d = N/2 (tr(Z_p^-1 Z_q) + tr(Z_q^-1 Z_p)) - 3N
 *   BHATTACHARYYA: d = N (ln det((Z_p + Z_q)/2) - (ln det Z_p + ln det Z_q)/2)
 * The window is clipped at the image border.  Image: height x width pixels,
 * row-major within each plane.
 *   z     in: 9 planes of Z (pitch z_pitch)
 *   aux   in: KL: the 9 planes of Z^-1; BHATTACHARYYA: the det plane (both as
 *         polsar_inv_det returns them)
 *   out   out: 9 planes of the filtered covariance (pitch out_pitch)
 *   wsum  out (nullable): sum of the weights per pixel
 * radius <= 16, n_looks > 0, h > 0; width <= 2^20, height <= 262140, else
 * POLSAR_E_ARG.  Outputs must not overlap inputs. */
enum { POLSAR_DIST_KL = 0, POLSAR_DIST_BHATTACHARYYA = 1 };
int polsar_nlm_wishart(int dtype, int distance, int64_t height, int64_t width, int radius,
                       double n_looks, double h, const void* z, int64_t z_pitch,
                       const void* aux, int64_t aux_pitch, void* out, int64_t out_pitch,
                       void* wsum, void* stream);

typedef enum { POLSAR_FWD = 1, POLSAR_BWD = 2, POLSAR_FWD_BWD = 3 } polsar_pass;

/* Wishart log-likelihood term, summed over pixels:
 *   L = sum_px N (ln det S + tr(S^-1 Z))
 * (the densities of the Introduction depend on the covariance only through
 * its determinant and inverse; the Sigma-free terms of the complex Wishart
 * density are omitted), with S^-1 and det S from Alg. 2 in the storage type,
 * and its gradient with respect to the packed real parameters of S:
 *   grad = g N (P - P Z P), P = S^-1 recomputed, off-diagonal components
 *   doubled: (M00, M11, M22, 2Re M01, 2Im M01, 2Re M02, 2Im M02, 2Re M12, 2Im M12).
 *   sigma, z   in: 9 planes each (pitches s_pitch, z_pitch)
 *   n_looks    N (> 0)
 *   loss       out (FWD, FWD_BWD): one device double, overwritten with L
 *   ell        out (nullable): n per-pixel terms, storage type
 *   grad_loss  in (BWD, FWD_BWD; nullable = 1.0): device double g
 *   grad       out (BWD, FWD_BWD): 9 planes, pitch g_pitch
 *   workspace  device scratch of at least polsar_wishart_workspace_bytes(n)
 *              bytes (FWD, FWD_BWD), 8-byte aligned; holds per-tile FP64
 *              partial sums, which a second kernel adds in tile order
 *              (deterministic).  Calls that share a workspace must not
 *              overlap in time (one stream, or synchronised streams).
 *   counters   as for polsar_inv_det: [not_pd, low_accuracy, nonfinite] for
 *              S, where low_accuracy counts the positive-definite pixels
 *              whose determinant of S may be off by more than 1e-3 relative
 *              (an a-priori bound of the plain evaluation in the storage
 *              type, gamma_8 sum |x_i| (|c_i| + sum of c_i's product
 *              magnitudes)): their terms and gradient carry errors of that
 *              order or more (ill-conditioned S in FP32).
 * Launch shape: op 1 of polsar_get_launch, op 5 below 2^23 pixels (see
 * polsar_wishart_launch_op); the loss's summation order follows the tiles,
 * so it can differ between the two in the last bits. */
int polsar_wishart_loglik(int dtype, int pass, int64_t n,
                          const void* sigma, int64_t s_pitch,
                          const void* z, int64_t z_pitch, double n_looks,
                          double* loss, void* ell, const double* grad_loss,
                          void* grad, int64_t g_pitch,
                          void* workspace, size_t ws_bytes,
                          unsigned long long* counters, void* stream);
size_t polsar_wishart_workspace_bytes(int dtype, int64_t n);

/* polsar_wishart_loglik without a workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the forward pass keeps its partial sums
 * in a fixed array of this library, 8 MiB on each GPU it runs on,
 * held until the process ends.  Arguments as for polsar_wishart_loglik;
 * same kernels and launch, so the same results bit for bit.  The call
 * allocates nothing (no hipMalloc, no library allocation).  The forward pass
 * takes at most 2^20 tiles of the launch in use: at the default launches
 * FP32 images of up to 2^28 pixels (2^29 where the planes allow vector
 * accesses) and FP64 images of up to 2^27; beyond that POLSAR_E_WORKSPACE,
 * before any HIP call.  Every call on one GPU shares its array: calls that
 * overlap in time on one GPU (other streams, other host threads) race and
 * must not be issued. */
int polsar_wishart_loglik_noalloc(int dtype, int pass, int64_t n,
                                  const void* sigma, int64_t s_pitch,
                                  const void* z, int64_t z_pitch, double n_looks,
                                  double* loss, void* ell, const double* grad_loss,
                                  void* grad, int64_t g_pitch,
                                  unsigned long long* counters, void* stream);

/* Batched launch over many images of uneven sizes: the paper's
 * closing section names, as future work, combining several matrix
 * inversions into a single inversion call; here one call (one graph launch)
 * covers every pixel of every image.  One grid covers the tiles of all
 * images, numbered image after image: one block per tile (the hardware
 * dispatcher balances the blocks over the compute units) or a persistent
 * grid that strides over them; the launch and the per-image loss reduction
 * are captured once in a HIP graph.  Per image, any of: inverse/determinant of Z (ops &
 * POLSAR_OP_INV_DET, Alg. 2 or Alg. 1 as for polsar_inv_det), Wishart
 * forward (loss, ell) and backward (grad) of S against Z (ops &
 * POLSAR_OP_WISHART_FWD / _BWD, as for polsar_wishart_loglik).  Host array
 * `imgs`; the pointers inside are device pointers with the meaning above,
 * `loss` one device double per image.  grad_loss (device double, nullable =
 * 1.0) scales every gradient.  Every image runs in the same grid, so no
 * output of any image (inv, det, status, grad, ell, loss) may overlap an
 * input or another output of any image (POLSAR_E_ALIAS); inputs may be
 * shared between images; in-place is not offered here. */
enum { POLSAR_OP_INV_DET = 1, POLSAR_OP_WISHART_FWD = 2, POLSAR_OP_WISHART_BWD = 4 };
typedef struct {
  int64_t n;
  const void* z;     int64_t z_pitch;
  void* inv;         int64_t inv_pitch;
  void* det;
  uint8_t* status;
  const void* sigma; int64_t s_pitch;
  void* grad;        int64_t g_pitch;
  void* ell;
  double* loss;
  double n_looks;
} polsar_image;
typedef struct polsar_batch polsar_batch;

/* Create: allocates device tables, a workspace and the graph (the only call
 * that allocates).  method: POLSAR_ADJUGATE or POLSAR_CHOLESKY for the inverse;
 * the launch shape is the op-3 entry of the launch table (its grid_per_cu
 * 0: one block per tile; k > 0: a persistent grid of k blocks per compute
 * unit); grid_per_cu > 0 here overrides the entry's.  With counters the grid
 * is persistent, at most 16 blocks per compute unit (one set of atomics per
 * wave).  Returns POLSAR_OK and *out, or an error
 * (no allocation left behind). */
int polsar_batch_create(const polsar_image* imgs, int count, int dtype, int method,
                        int precision, unsigned ops, const double* grad_loss,
                        unsigned long long* counters, int grid_per_cu,
                        polsar_batch** out);
int polsar_batch_run(polsar_batch* b, void* stream);        /* one hipGraphLaunch */
int polsar_batch_run_eager(polsar_batch* b, void* stream);  /* same kernels, no graph */
int64_t polsar_batch_tiles(const polsar_batch* b);
void polsar_batch_destroy(polsar_batch* b);

/* Out-of-core streaming (closing discussion of Section 4: images larger than
 * device memory are streamed through the GPU piece by piece).  A streamer
 * owns two device buffer sets of chunk_pixels pixels and two streams
 * (allocated at creation, freed by destroy).  run() inverts n pixels held in
 * HOST memory (z, inv, det, status are host pointers; pinned memory gives
 * full PCIe speed; counters, if given, is a DEVICE pointer): chunk i is
 * copied in, inverted and copied out on stream i % 2, so transfers of one
 * chunk overlap the other's.  run() returns when all results are in host
 * memory.  Results are bitwise those of polsar_inv_det. */
typedef struct polsar_streamer polsar_streamer;
int polsar_streamer_create(int dtype, int method, int precision, int64_t chunk_pixels,
                           polsar_streamer** out);
int polsar_streamer_run(polsar_streamer* s, int64_t n, const void* z, int64_t z_pitch,
                        void* inv, int64_t inv_pitch, void* det, uint8_t* status,
                        unsigned long long* counters);
void polsar_streamer_destroy(polsar_streamer* s);

/* Launch configuration of the kernels, keyed by op (0 = inv_det,
 * 1 = wishart, 2 = multilook + inv_det, 3 = batch, 4 = the copy probe,
 * 5 = wishart on images of fewer than 2^23 pixels, 6 = inv_det on images of
 * at least 2^25 pixels; ops 2, 3 and 4 take unroll 1, op 4 one tile per
 * block; ops 1, 4 and 5 are keyed with method 0 and
 * precision 0), dtype, method, precision.
 *   block        threads per block: 64, 128 or 256
 *   unroll       vectors per thread per tile: 1, 2 or 4 (the FP32
 *                compensated inverse takes at most 2, sharing one FP64
 *                queue; 1 where that queue would pass 64 KB of LDS)
 *   grid_per_cu  0 = one tile per block; k > 0 = persistent grid of k blocks
 *                per compute unit striding over tiles
 *   nontemporal  1 = streaming (non-temporal) loads and stores
 *   vector_bytes 16 or 8: bytes per lane per plane access on aligned planes
 *   blocks_per_cu 0 = as many resident blocks as registers allow; k > 0 = at
 *                most k blocks resident per compute unit (enforced by padding
 *                the block's LDS).  On MI355X these streaming kernels move
 *                more bytes per second with few waves in flight per CU. */
typedef struct { int block, unroll, grid_per_cu, nontemporal, vector_bytes, blocks_per_cu; } polsar_launch;
int polsar_get_launch(int op, int dtype, int method, int precision, polsar_launch* out);
int polsar_set_launch(int op, int dtype, int method, int precision, const polsar_launch* cfg);
/* The op of the table (1 or 5) whose launch polsar_wishart_loglik uses for
 * n pixels. */
int polsar_wishart_launch_op(int64_t n);
/* The op of the table (0 or 6) whose launch polsar_inv_det (and each chunk of
 * the streamer) uses for n pixels. */
int polsar_inv_det_launch_op(int64_t n);

/* Times each candidate launch configuration of polsar_inv_det on the caller's
 * buffers (same arguments as polsar_inv_det; outputs are overwritten), `reps`
 * timed repetitions each after one warm-up; the six fastest are timed again
 * in three interleaved passes and ranked by their best pass.  Installs the
 * winner in the entry that calls of n pixels use (polsar_inv_det_launch_op)
 * and returns it with that mean time per call in milliseconds.
 * Synchronises `stream`. */
int polsar_autotune_inv_det(int dtype, int method, int precision, int64_t n,
                            const void* z, int64_t z_pitch, void* inv, int64_t inv_pitch,
                            void* det, int reps, polsar_launch* best, float* best_ms,
                            void* stream);

/* Bandwidth probe: copies n_in planes of n elements (pitch src_pitch) to
 * n_out planes (pitch dst_pitch; plane k of dst takes plane k mod n_in, or,
 * with fewer outputs than inputs, the sum of the input planes j with
 * j mod n_out == k, so that every input is read) with
 * the same access pattern as the inverse kernels, for a measured ceiling of
 * each kernel's mix of plane streams: (n_in, n_out) is (9, 10) (inverse),
 * (18, 9) (Wishart forward+backward), (18, 19) (the batch: inverse and
 * Wishart), (24, 10) (four-look multilook), (27, 28) (three-band
 * block-diagonal inverse) or (1, 1) (counter calibration); planes 16-byte
 * aligned.
 * Launch shape: op 4 of polsar_get_launch. */
int polsar_stream_copy(int dtype, int64_t n, const void* src, int64_t src_pitch, int n_in,
                       void* dst, int64_t dst_pitch, int n_out, void* stream);

/* Plane pitch (in elements) recommended for n-element planes of this dtype:
 * n rounded up to 64 KiB, plus 32 KiB, so that consecutive planes start 32 KiB
 * apart modulo 64 KiB instead of at the same offset of every large power of
 * two (on MI355X, power-of-two plane pitches of hundreds of MB cost up to
 * 10% of streaming bandwidth).  Any pitch >= n is accepted by every call. */
int64_t polsar_recommended_pitch(int dtype, int64_t n);

const char* polsar_status_string(int status);
const char* polsar_version(void);
int polsar_device_compute_units(int* cus);

#ifdef __cplusplus
}
#endif
#endif /* POLSAR_H */
