/*
 * sigsep.h -- C ABI of the MI355X (gfx950) signal-separation library.
 *
 * The library implements the per-frame path of Kieffer et al., "Application
 * of signal separation to diffraction image compression and serial
 * crystallography" (2024):
 *
 *   raw Jungfrau words --ss_correct--> corrected intensity v = signal / norm
 *   v --ss_sigma_clip (CSR regroup + iterative clipping)--> 1-D profile
 *   v + profile --ss_compress / ss_peakfind / ss_classify--> kept pixels, peaks
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers marked [dev] are device pointers, [host] host pointers.  The
 *   caller owns every buffer; the library never allocates, frees or keeps a
 *   pointer after the call returns.
 * - Device calls enqueue kernels on `stream` and return at once; they never
 *   synchronise.  Outputs are valid once the stream reaches that point.
 * - Return value: SS_OK (0), or a negative code detected on the host before
 *   anything was enqueued (SS_EINVAL, SS_ESIZE), or SS_EHIP when the HIP
 *   runtime reported a launch error.  ss_strerror() names a code.
 * - Frames are [n_frames][words] float32, row-major (words = n_pix, pixel
 *   index y * width + x) unless a call names a tiled layout (ss_layout):
 *   ss_correct_tiled writes one, ss_sigma_clip reads whatever layout its
 *   CSR indices address, and the ss_classify family reads the layout its
 *   ss_radial names.  Pixel indices in outputs (kept pixels, peaks) are
 *   always y * width + x.
 * - Masks are uint8, nonzero = masked.  A frame value that is not finite
 *   (NaN/Inf, e.g. an invalid gain code) marks that pixel masked in that
 *   frame only.
 * - Statistics are accumulated in float64; frames are float32.
 * - Calls on different streams are independent; calls that share output or
 *   workspace buffers must be ordered by the caller.
 * - ss_sigma_clip / ss_integrate_csr on one or two frames spread their
 *   row-length classes over three side streams that fork from and join back
 *   to `stream` through events (so the call still completes in `stream`
 *   order, and can be captured in a graph).  The side streams and their
 *   events are created once per device, on first use, and kept until the
 *   process ends.  The other piece of library state is the device array that
 *   serves ss_classify_noalloc as workspace (one per GPU).
 */
#ifndef SIGSEP_H
#define SIGSEP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SS_OK 0
#define SS_EINVAL (-1) /* null pointer, bad flag or parameter out of range */
#define SS_ESIZE (-2)  /* size out of range or capacity too small          */
#define SS_EHIP (-3)   /* HIP runtime error at launch                       */

/* Error models of Sec. 2.2 and 2.5. */
#define SS_AZIMUTHAL 0 /* spread of the bin's values (eqs. varA, std2)       */
#define SS_POISSON 1   /* counting statistics (eqs. poisson, varianceP, sem) */
#define SS_HYBRID 2    /* clip with the azimuthal spread, report Poisson     */

/* Pixel splitting of the CSR builder (Sec. 2.2, "Azimuthal averaging"). */
#define SS_SPLIT_NONE 0
#define SS_SPLIT_BBOX 1

/* Radial coordinate code of a pixel (see ss_radial_coords). */
#define SS_RC_FRAC_BITS 20
#define SS_RC_MASKED 0xFFFFFFFFu
#define SS_MAX_BINS 4094
#define SS_MAX_ITER 32
#define SS_MAX_PATCH 15
#define SS_N_CLASSES 8
#define SS_SURROGATE_MAX_CLASS 5 /* the surrogate serves row-length classes 0..5 */

/*
 * Pixel-to-bin matrix in CSR form (rows = radial bins), Sec. 2.2: the
 * regrouping is a sparse matrix times the flattened image.  weight[j] is the
 * per-entry weight omega = c[i, r] * norm_i of eq. omega (the pixel's share
 * of the bin times its normalisation factor).  Row entries have ascending
 * pixel indices.  max_row is the length of the longest row.
 *
 * Optional schedule (from ss_csr_schedule): bin_order lists the bins grouped
 * by row-length class, longest class first, and class_count[c] is the number
 * of bins in class c; the clip then launches one work-group size per class.
 * With bin_order == NULL one work-group size fits the longest row.
 * shape[c] selects the work-group shape the clip uses for class c in
 * batches of more than one frame: 0 (the default) or one of the
 * alternatives 1, 2 (an autotuner's choice); any other value means 0.
 */
typedef struct {
    int32_t n_bins;
    int32_t max_row;
    int64_t n_pix;
    int64_t nnz;
    const int64_t *indptr;    /* [dev] [n_bins + 1]   */
    const int32_t *indices;   /* [dev] [nnz]          */
    const float *weight;      /* [dev] [nnz]          */
    const int32_t *bin_order; /* [dev] [n_bins] or NULL */
    int32_t class_count[SS_N_CLASSES];
    int32_t shape[SS_N_CLASSES];
} ss_csr;

/*
 * Parameters of the path.
 * cutoff    clipping threshold n of eq. clip; <= 0 selects Chauvenet's
 *           value sqrt(2 ln(size / sqrt(2 pi))) per pass (eq. chauvenet)
 * max_iter  maximum number of rejection passes K (Sec. 2.4), 0..SS_MAX_ITER
 * error_model  SS_AZIMUTHAL, SS_POISSON or SS_HYBRID
 * dark_var  sigma_dark^2 of eq. poisson, in signal units squared
 * n_pick    sparsification threshold SNR_pick of Sec. 3
 * noise     noise level added in quadrature to the background std (Sec. 4.1)
 * snr       peak-finder SNR threshold (Sec. 4)
 * patch     odd side P of the peak-finder's square patch, 1..SS_MAX_PATCH
 * min_count minimum number of SNR-passing pixels in the patch
 */
typedef struct {
    float cutoff;
    int32_t max_iter;
    int32_t error_model;
    float dark_var;
    float n_pick;
    float noise;
    float snr;
    int32_t patch;
    int32_t min_count;
} ss_params;

/*
 * 1-D background profile, every array [dev] [n_frames][n_bins].
 * mean = V / Omega (eq. weighted_avg); std = sqrt(VV / OmegaOmega) (eq. std2)
 * or the Poisson std; sem = sqrt(VV) / Omega (eq. sem2) or the Poisson sem;
 * sum_w = Omega (eq. omega); n_members = members of the final set; n_iter =
 * rejection passes that removed something; converged = 1 when a pass removed
 * nothing.  An empty bin has mean = std = sem = 0.
 */
typedef struct {
    double *mean;
    double *std;
    double *sem;
    double *sum_w;
    int32_t *n_members;
    int32_t *n_iter;
    int32_t *converged;
} ss_profile;

/*
 * Frame layout.  Row-major frames (tile_w = tile_h = 0) hold pixel (y, x) at
 * word y * width + x.  A tiled layout cuts the frame into tiles of tile_w x
 * tile_h pixels (powers of two, 4 <= tile_w <= 64, 1 <= tile_h <= 64),
 * tiles row-major, pixels row-major inside a tile: pixel (y, x) sits at word
 *   ((y / tile_h) * tiles_x + x / tile_w) * tile_w * tile_h
 *     + (y % tile_h) * tile_w + x % tile_w,   tiles_x = ceil(width / tile_w),
 * and a frame holds tiles_x * ceil(height / tile_h) * tile_w * tile_h words
 * (ss_layout_words); words of partial tiles past the image edge are NaN.
 * With 8 x 4 tiles (one 128-byte line per tile) the pixels of a thin ring
 * that a line holds are neighbours in two dimensions, not along one image
 * row, so the CSR gathers of the regrouping (Sec. 2.2) touch about half as
 * many lines.  Frames in a tiled layout go with a CSR whose indices are word
 * offsets in it (ss_csr_relayout) and an ss_radial naming the layout.
 */
typedef struct {
    int32_t height;
    int32_t width;
    int32_t tile_w;
    int32_t tile_h;
} ss_layout;

/*
 * Radial position of every pixel for the background lookup of Sec. 3 ("the
 * distance to the centre of every pixel").  Bins are uniform: centre of bin r
 * = centre0 + r * width.  rcoord[i] packs the interval t (bin centre t <=
 * position < centre t+1, t = -1 below the first centre, n_bins - 1 beyond
 * the last) as (t + 1) << SS_RC_FRAC_BITS, plus the position's fraction of
 * that interval in the low SS_RC_FRAC_BITS bits; SS_RC_MASKED marks a
 * statically masked pixel.
 */
typedef struct {
    int32_t n_bins;
    double centre0;
    double width;
    const uint32_t *rcoord; /* [dev] [n_pix] */
    int32_t tile_w;         /* layout of the frames read with it (ss_layout): */
    int32_t tile_h;         /* 0, 0 for row-major frames                     */
} ss_radial;

/* Peak record of Sec. 4: centroid (pixel units, centres at +0.5), sum of
 * background-subtracted intensity and its propagated deviation. */
typedef struct {
    uint32_t index;
    float y;
    float x;
    float intensity;
    float sigma;
} ss_peak;

/* Name of a return code (static string). */
const char *ss_strerror(int code);

/* Library version as major * 10000 + minor * 100 + patch. */
int ss_version(void);

/*
 * ss_build_csr [host] -- the CSR of Sec. 2.2 for a flat detector normal to
 * the beam.  Pixel (y, x) covers [y, y+1) x [x, x+1) in pixel units, the
 * beam centre is (centre_row, centre_col) in the same units, 2theta =
 * atan(pixel_m * r / dist_m) in degrees, and the n_bins bins are uniform on
 * [0, 2theta_max] with 2theta_max the largest pixel-corner angle.
 * split = SS_SPLIT_NONE: a pixel goes whole to the bin of its centre angle.
 * split = SS_SPLIT_BBOX: a pixel spans [min, max] of its corner angles (0 for
 * the pixel holding the beam centre) and c[i, r] = overlap / span; the
 * coefficients of a pixel sum to 1.  Masked pixels (mask [host] [n_pix],
 * may be NULL) get no entries.  weight = c * norm (norm [host] [n_pix], NULL
 * means 1).
 * Call once with indices == NULL to get *nnz and *max_row, then again with
 * indptr [n_bins + 1], indices and weight [capacity >= nnz] to fill them.
 * *tth_max receives 2theta_max in degrees.  Errors: SS_EINVAL, SS_ESIZE.
 */
int ss_build_csr(int32_t height, int32_t width, double pixel_m, double dist_m,
                 double centre_row, double centre_col, int32_t n_bins, int32_t split,
                 const uint8_t *mask, const float *norm,
                 int64_t *indptr, int32_t *indices, float *weight, int64_t capacity,
                 int64_t *nnz, int32_t *max_row, double *tth_max);

/*
 * ss_csr_schedule [host] -- group the bins of a CSR by row length for
 * ss_sigma_clip.  Class c holds the rows of at most ss_class_rows(c) entries
 * not held by a smaller class (the last class: any length); bin_order [host]
 * [n_bins] receives the bins of the longest class first, each class in bin
 * order; class_count [host] [SS_N_CLASSES] the class sizes.
 * Errors: SS_EINVAL, SS_ESIZE.
 */
int ss_csr_schedule(const int64_t *indptr, int32_t n_bins, int32_t *bin_order, int32_t *class_count);

/* Largest row length of class c (0 <= c < SS_N_CLASSES - 1). */
int32_t ss_class_rows(int32_t c);

/*
 * ss_layout_words [host] -- words per frame of a layout (height * width for
 * row-major frames), or a negative code: SS_EINVAL for a null layout,
 * SS_ESIZE for sizes out of range or tiles that are not as ss_layout states.
 */
int64_t ss_layout_words(const ss_layout *layout);

/*
 * ss_csr_relayout [host] -- turn the pixel indices of a CSR from
 * ss_build_csr (layout height x width) into word offsets of the layout and
 * sort every row by offset, moving the weights along (a row's sums are then
 * taken in that order: the same members, rounding of the float64 sums
 * aside).  indptr [host] [n_bins + 1]; indices and weight [host] [nnz],
 * rewritten in place.  Errors: SS_EINVAL (null pointer, an index outside
 * the image, a row that does not ascend in indptr), SS_ESIZE (layout).
 */
int ss_csr_relayout(const ss_layout *layout, int32_t n_bins, const int64_t *indptr, int32_t *indices,
                    float *weight);

/*
 * ss_layout_scatter [host] -- a per-pixel float array (row-major, height x
 * width) rewritten in a layout: dst [host] [ss_layout_words] receives
 * src[y * width + x] at the word of pixel (y, x) and fill elsewhere (for
 * the norm array of ss_sigma_clip on tiled frames).  Errors: SS_EINVAL,
 * SS_ESIZE (layout).
 */
int ss_layout_scatter(const ss_layout *layout, const float *src, float fill, float *dst);

/*
 * ss_radial_coords [host] -- rcoord [host] [n_pix] of the pixel-centre
 * angles for the bins of ss_build_csr (same geometry, n_bins and tth_max);
 * masked pixels (mask may be NULL) get SS_RC_MASKED.  *centre0 and *width
 * receive the first bin centre and the bin width.  Errors: SS_EINVAL,
 * SS_ESIZE (n_bins > SS_MAX_BINS).
 */
int ss_radial_coords(int32_t height, int32_t width, double pixel_m, double dist_m,
                     double centre_row, double centre_col, int32_t n_bins, double tth_max,
                     const uint8_t *mask, uint32_t *rcoord, double *centre0, double *width_out);

/*
 * ss_correct -- Jungfrau pre-processing (Sec. 1.2) and normalisation
 * (eq. norm).  Word bits 15..14 select the gain level (00 -> 0, 01 -> 1,
 * 11 -> 2; 10 is invalid), bits 13..0 are the ADC value; signal = (ADC -
 * pedestal[g]) / gain[g] (float64 arithmetic, rounded to float32, the 32-bit
 * pre-processed frame), then out = signal / norm (float64, rounded to
 * float32).  Invalid words give NaN and are counted.
 *   raw       [dev] uint16 [n_frames][n_pix]
 *   pedestal  [dev] float  [3][n_pix]   (ADU)
 *   gain      [dev] float  [3][n_pix]   (ADU per photon)
 *   norm      [dev] float  [n_pix] or NULL (= 1)
 *   out       [dev] float  [n_frames][n_pix]
 *   n_invalid [dev] int64  [n_frames] or NULL; overwritten
 * Errors: SS_EINVAL (null required pointer), SS_ESIZE (n_pix < 0 or
 * >= 2^31, n_frames < 0), SS_EHIP.
 */
int ss_correct(const uint16_t *raw, int32_t n_frames, int64_t n_pix,
               const float *pedestal, const float *gain, const float *norm,
               float *out, int64_t *n_invalid, hipStream_t stream);

/*
 * ss_correct_indexed -- ss_correct of frames picked from a ring of raw
 * frames by a device-side index (serving support: frames that arrive into a
 * device ring are corrected where they lie, with no copy).  Output frame f
 * is the correction of ring frame frame_index[f]; an index outside
 * [0, ring_frames) gives a frame of invalid words (all NaN, all counted).
 *   ring        [dev] uint16 [ring_frames][n_pix]
 *   frame_index [dev] int64 [n_frames]
 *   other arguments as ss_correct.
 * Errors: those of ss_correct; SS_ESIZE for ring_frames < 0, SS_EINVAL for a
 * null frame_index with n_frames > 0.
 */
int ss_correct_indexed(const uint16_t *ring, int64_t ring_frames, const int64_t *frame_index,
                       int32_t n_frames, int64_t n_pix, const float *pedestal, const float *gain,
                       const float *norm, float *out, int64_t *n_invalid, hipStream_t stream);

/*
 * ss_correct_tiled / ss_correct_indexed_tiled -- ss_correct /
 * ss_correct_indexed writing the corrected frames in a layout: raw words,
 * pedestal, gain and norm stay row-major over layout->height x
 * layout->width pixels; out [dev] float [n_frames][ss_layout_words(layout)],
 * NaN at the words past the image edge.  Errors: those of ss_correct;
 * SS_EINVAL for a null layout, SS_ESIZE for a layout ss_layout_words
 * refuses.
 */
int ss_correct_tiled(const uint16_t *raw, int32_t n_frames, const ss_layout *layout, const float *pedestal,
                     const float *gain, const float *norm, float *out, int64_t *n_invalid, hipStream_t stream);
int ss_correct_indexed_tiled(const uint16_t *ring, int64_t ring_frames, const int64_t *frame_index,
                             int32_t n_frames, const ss_layout *layout, const float *pedestal, const float *gain,
                             const float *norm, float *out, int64_t *n_invalid, hipStream_t stream);

/*
 * ss_integrate_csr -- azimuthal average with uncertainties (Sec. 2.2, eqs. avg
 * to sem2), no clipping: ss_sigma_clip with max_iter forced to 0.
 */
int ss_integrate_csr(const float *frames, const float *norm, const uint8_t *mask,
                     int32_t n_frames, const ss_csr *csr, const ss_params *params,
                     const ss_profile *out, hipStream_t stream);

/* One batch of frames with its own geometry, for ss_sigma_clip_batches. */
typedef struct {
    const float *frames;    /* [dev] [n_frames][csr->n_pix] corrected intensity */
    const float *norm;      /* [dev] [csr->n_pix] or NULL (Poisson / hybrid models) */
    int32_t n_frames;
    const ss_csr *csr;      /* [host] struct of [dev] arrays */
    const ss_profile *out;  /* [host] struct of [dev] [n_frames][csr->n_bins] arrays */
} ss_clip_batch;

/* ss_sigma_clip_batches -- ss_sigma_clip of several batches, each with its
 * own geometry (uneven detectors and bin counts), in one launch per
 * row-length class for all of them: same results as one ss_sigma_clip call
 * per batch.  Every batch needs a scheduled CSR, the azimuthal model and more
 * than one frame for the shared launches (otherwise it is clipped on its own
 * within this call); the work-group shape of each class is taken from
 * batches[0].csr->shape.  Errors: SS_EINVAL, SS_ESIZE, SS_EHIP (checked for
 * every batch before anything is launched). */
int ss_sigma_clip_batches(const ss_clip_batch *batches, int32_t n_batches,
                          const ss_params *params, hipStream_t stream);

/*
 * ss_sigma_clip -- per-bin iterative sigma-clipping (eq. clip, Sec. 2.4).
 * For every frame and bin: members = CSR entries whose pixel is unmasked
 * and finite, value v = frames[f][i], weight omega = csr weight.  Passes
 * k = 0 .. max_iter-1 compute the statistics of the current set and remove
 * members with |v - mean| > n * std (strict; n = cutoff or Chauvenet's value
 * for the current size); the loop stops at the first pass that removes
 * nothing.  The profile holds the statistics of the final set.
 *   frames [dev] float [n_frames][csr->n_pix] (corrected intensities v):
 *          csr->n_pix words per frame, in whatever layout the CSR indices
 *          address (pixel indices, or word offsets after ss_csr_relayout)
 *   norm   [dev] float [csr->n_pix] or NULL, indexed like the frames; used
 *          only by the Poisson and hybrid models, whose pixel variance is
 *          (max(v * norm, 0) + dark_var) / norm^2 in units of v
 *   mask   [dev] uint8 [csr->n_pix] or NULL, indexed like the frames (in
 *          addition to the CSR's own mask)
 *   csr, params, out: [host] structs; their arrays are [dev]
 * Errors: SS_EINVAL, SS_ESIZE (n_bins > SS_MAX_BINS, max_iter out of range),
 * SS_EHIP.
 */
int ss_sigma_clip(const float *frames, const float *norm, const uint8_t *mask,
                  int32_t n_frames, const ss_csr *csr, const ss_params *params,
                  const ss_profile *out, hipStream_t stream);

/*
 * Workspace (device bytes) needed by ss_classify / ss_compress /
 * ss_peakfind for n_frames frames of n_pix pixels and n_bins bins.
 */
size_t ss_classify_workspace(int32_t n_frames, int64_t n_pix, int32_t n_bins);

/*
 * ss_classify -- per-pixel classification against the clipped profile,
 * feeding both applications in one pass over the pixels.
 * Background of pixel i (Sec. 3): mu_i, sigma_i = the profile's mean and std
 * linearly interpolated between the centres of the non-empty bins at the
 * pixel's angle, constant beyond the first and last; sigma_eff =
 * sqrt(sigma_i^2 + noise^2).
 * Sparsification (Sec. 3): keep i when unmasked and v_i - mu_i > n_pick *
 * sigma_eff; kept_index / kept_value receive (i, v_i) in ascending i,
 * [dev] [n_frames][capacity]; n_kept [dev] int64 [n_frames] receives the
 * true count, entries beyond capacity are dropped.
 * Peak finder (Sec. 4): candidate = unmasked and v - mu >= snr * sigma_eff;
 * a peak is a candidate that is the maximum of v over the unmasked pixels
 * of the patch x patch square centred on it (clipped at the border; ties go
 * to the lower index) with at least min_count candidates in the square.
 * Record over the square's candidates j: w_j = v_j - mu_j, intensity =
 * sum w_j, sigma = sqrt(sum sigma_eff_j^2), centroid = sum w_j (y_j + 0.5,
 * x_j + 0.5) / sum w_j.  peaks [dev] [n_frames][peak_capacity] in ascending
 * index; n_peaks [dev] int64 [n_frames] (true count).
 * Either output group may be disabled by passing NULL for all its pointers.
 *   frames [dev] float [n_frames][words], words = ss_layout_words of
 *     (height, width, radial->tile_w, radial->tile_h): height * width for
 *     row-major frames; mask [dev] or NULL
 *   radial, profile, params: [host] structs with [dev] arrays
 *   workspace [dev] >= ss_classify_workspace(...) bytes
 * Errors: SS_EINVAL, SS_ESIZE (workspace too small, capacities < 0,
 * bin count mismatch, height * width >= 2^29), SS_EHIP.
 */
int ss_classify(const float *frames, const uint8_t *mask, int32_t n_frames,
                int32_t height, int32_t width, const ss_radial *radial,
                const ss_profile *profile, const ss_params *params,
                uint32_t *kept_index, float *kept_value, int64_t capacity, int64_t *n_kept,
                ss_peak *peaks, int64_t peak_capacity, int64_t *n_peaks,
                void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * ss_classify_noalloc -- ss_classify for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments and results, without the workspace.  The
 * workspace is a file-scope device array of SS_CLASSIFY_SCRATCH_BYTES bytes
 * inside the library, one per GPU, held from the library's load until the
 * process ends; its device address is looked up once per device on the
 * first call made with that device current.  The call allocates and frees
 * nothing.  Every call on one GPU uses that GPU's array, which keeps the last
 * call's contents (each call writes every byte it reads first, so nothing
 * needs clearing): calls that overlap on one GPU (different streams without
 * ordering, or different host threads) race and give undefined results.
 * Errors: those of ss_classify; SS_ESIZE also when
 * ss_classify_workspace(n_frames, height * width, radial->n_bins) exceeds
 * SS_CLASSIFY_SCRATCH_BYTES (checked before any device call), SS_EHIP when
 * the array's address cannot be obtained.
 */
#define SS_CLASSIFY_SCRATCH_BYTES (64u << 20)
int ss_classify_noalloc(const float *frames, const uint8_t *mask, int32_t n_frames,
                        int32_t height, int32_t width, const ss_radial *radial,
                        const ss_profile *profile, const ss_params *params,
                        uint32_t *kept_index, float *kept_value, int64_t capacity, int64_t *n_kept,
                        ss_peak *peaks, int64_t peak_capacity, int64_t *n_peaks, hipStream_t stream);

/* ss_compress -- the sparsification half of ss_classify (Sec. 3). */
int ss_compress(const float *frames, const uint8_t *mask, int32_t n_frames,
                int32_t height, int32_t width, const ss_radial *radial,
                const ss_profile *profile, const ss_params *params,
                uint32_t *kept_index, float *kept_value, int64_t capacity, int64_t *n_kept,
                void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ss_peakfind -- the peak-finder half of ss_classify (Sec. 4). */
int ss_peakfind(const float *frames, const uint8_t *mask, int32_t n_frames,
                int32_t height, int32_t width, const ss_radial *radial,
                const ss_profile *profile, const ss_params *params,
                ss_peak *peaks, int64_t peak_capacity, int64_t *n_peaks,
                void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Densification (Sec. 3.2) and the peak-count veto (Sec. 4).
 */

/*
 * Noise of a densified background.  The paper regenerates the background
 * "with noise" for analysis programs that measure noise (Sec. 3.2) and fixes
 * no generator; this library's convention: pixel i of absolute frame
 * frame0 + f takes generator block i / 2 of Philox4x32-10 (Salmon et al.,
 * SC 2011) with counter (i / 2, frame0 + f, 0, 0) and key (seed & 0xffffffff,
 * seed >> 32); the even pixel of a block uses words 0, 1, the odd one words
 * 2, 3, as u1 = ((w >> 8) + 1) 2^-24 and u2 = (w >> 8) 2^-24; Box-Muller gives
 * z_a = r cos(2 pi u2), z_b = r sin(2 pi u2), r = sqrt(-2 ln u1); the pixel's
 * draw is the first of z_a, z_b not above trunc, else trunc (pass INFINITY
 * for no bound; n_pick keeps regenerated noise under the sparsification
 * threshold).  Computed in float32; the background in float64.
 */
typedef struct {
    uint64_t seed;
    int64_t frame0;
    float trunc;
} ss_noise;

/* Workspace (device bytes) of ss_densify for n_frames frames and n_bins bins. */
size_t ss_densify_workspace(int32_t n_frames, int32_t n_bins);

/*
 * ss_densify -- dense frames from their sparse representation (Sec. 3.2):
 * the inverse of ss_compress.  Every pixel gets the background mu_i of its
 * frame's profile (interpolated between the centres of the non-empty bins
 * as in ss_classify), plus sigma_i z_i when noise != NULL; masked pixels
 * (mask[i] != 0 or SS_RC_MASKED) get 0; then entries k < min(n_kept[f],
 * capacity) of frame f put kept_value back at kept_index (indices >= n_pix
 * are skipped).
 *   kept_index, kept_value [dev] [n_frames][capacity] (ss_compress layout),
 *     n_kept [dev] int64 [n_frames]; all three may be NULL when capacity = 0
 *   mask [dev] uint8 [n_pix] or NULL; radial, profile: [host] structs with
 *     [dev] arrays (profile mean, std, n_members used)
 *   noise [host] or NULL (noise free)
 *   dense [dev] float [n_frames][n_pix], row-major (the tile fields of
 *     radial are not used), written entirely
 *   workspace [dev] >= ss_densify_workspace(n_frames, radial->n_bins) bytes
 * Errors: SS_EINVAL (null pointers, NaN trunc), SS_ESIZE (sizes,
 * workspace), SS_EHIP.
 */
int ss_densify(const uint32_t *kept_index, const float *kept_value, int64_t capacity,
               const int64_t *n_kept, const uint8_t *mask, int32_t n_frames, int64_t n_pix,
               const ss_radial *radial, const ss_profile *profile, const ss_noise *noise,
               float *dense, void *workspace, size_t workspace_bytes, hipStream_t stream);

#define SS_VETO_BINS 256
#define SS_VETO_COUNTERS (4 + 2 * SS_VETO_BINS)

/*
 * ss_veto -- the peak-count veto of Sec. 4: frame f is a hit when
 * n_peaks[f] >= threshold (the acquisition may discard the others), and the
 * counters from which a live threshold is chosen.  counters [dev] int64
 * [SS_VETO_COUNTERS] are ADDED to (zero them once; they accumulate over
 * calls): [0] hits, [1] non-hits, [2] kept entries of hits, [3] kept entries
 * of non-hits, [4 + p] frames with p peaks, [4 + SS_VETO_BINS + p] their kept
 * entries (p clamped to 0 .. SS_VETO_BINS - 1).  For any threshold
 * T < SS_VETO_BINS, the frames and kept entries a veto at T discards are the
 * sums of the two histograms below T.
 *   n_peaks [dev] int64 [n_frames]; n_kept [dev] int64 [n_frames] or NULL
 *   (counted as 0); hit [dev] uint8 [n_frames] or NULL.
 * Calls that overlap on one counters array add concurrently (atomically).
 * Errors: SS_EINVAL, SS_ESIZE (n_frames < 0), SS_EHIP.
 */
int ss_veto(const int64_t *n_peaks, const int64_t *n_kept, int32_t n_frames, int64_t threshold,
            uint8_t *hit, int64_t *counters, hipStream_t stream);

/*
 * ss_pack_results -- the kept entries and peaks of n_frames frames packed
 * back to back, so that a caller returning results to the host copies one
 * contiguous prefix per kind instead of one piece per frame (serving
 * support; not a step of the paper's method).
 * Frame f contributes its first min(n_kept[f], capacity) entries of
 * kept_index / kept_value (ss_compress layout) and its first
 * min(n_peaks[f], peak_capacity) peaks, in frame order.
 *   offsets [dev] int64 [2 (n_frames + 1)]: written; offsets[f] is frame f's
 *     first packed entry, offsets[n_frames] their total; offsets[n_frames +
 *     1 + f] and offsets[2 n_frames + 1] the same for peaks
 *   packed_index, packed_value [dev] >= n_frames * capacity entries,
 *   packed_peaks [dev] >= n_frames * peak_capacity records
 *   either group (kept: kept_index, kept_value, n_kept, packed_index,
 *   packed_value; peaks: peaks, n_peaks, packed_peaks) may be all NULL; its
 *   offsets are then 0.
 * Errors: SS_EINVAL, SS_ESIZE, SS_EHIP.
 */
int ss_pack_results(const uint32_t *kept_index, const float *kept_value, int64_t capacity,
                    const int64_t *n_kept, const ss_peak *peaks, int64_t peak_capacity,
                    const int64_t *n_peaks, int32_t n_frames, int64_t *offsets, uint32_t *packed_index,
                    float *packed_value, ss_peak *packed_peaks, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned clip surrogate.  Not in the paper: the paper's clip time grows
 * with the number of passes (Sec. 2.4); a small network predicts each bin's
 * converged clipped mean and std from the bin's unclipped statistics and a
 * 16-point sketch of its standardised values, one verification pass checks
 * the prediction, and the plain clip runs wherever the check fails.
 *
 * Features of a bin with n members, unclipped mean m0 and std s0 (azimuthal,
 * eqs. avg, std2): x0 = log(1 + n), x1 = asinh(m0), x2 = asinh(s0),
 * x(3+k) = #{v <= m0 + t_k s0} / n with t_k = -3.75 + 0.5 k, k = 0..15.
 * Targets from a converged clip (mean mc, std sc): y0 = (mc - m0) / s0,
 * y1 = log(sc / s0).  Network 19 -> 64 -> 64 -> 2, GELU (erf) on the hidden
 * layers, float16 parameters, float32 arithmetic.  Parameters are one array
 * of SS_MLP_PARAMS entries: W1 [SS_MLP_K1][64] (rows >= 19 zero), b1 [64],
 * W2 [64][64], b2 [64], W3 [64][SS_MLP_OUT_PAD] (columns >= 2 zero),
 * b3 [SS_MLP_OUT_PAD] (entries >= 2 zero), row-major, at SS_MLP_OFF_*.
 * ---------------------------------------------------------------------- */
#define SS_MLP_IN 19
#define SS_MLP_HID 64
#define SS_MLP_OUT 2
#define SS_MLP_K1 32
#define SS_MLP_OUT_PAD 16
#define SS_MLP_OFF_W1 0
#define SS_MLP_OFF_B1 2048
#define SS_MLP_OFF_W2 2112
#define SS_MLP_OFF_B2 6208
#define SS_MLP_OFF_W3 6272
#define SS_MLP_OFF_B3 7296
#define SS_MLP_PARAMS 7312

/* ss_clip_features -- the surrogate's inputs for every (frame, bin).
 *   frames, norm: as ss_sigma_clip; mask must be NULL (masks are folded into
 *     the CSR) and rows must not exceed ss_class_rows(SS_SURROGATE_MAX_CLASS).
 *   features [dev] float [n_frames][n_bins][SS_MLP_IN] (all 0 for an empty bin)
 *   stats0 [dev] double [n_frames][n_bins][3]: n, m0, s0 (unclipped).
 * Errors: SS_EINVAL (null pointers, a mask, a row too long), SS_ESIZE, SS_EHIP. */
int ss_clip_features(const float *frames, const float *norm, const uint8_t *mask,
                     int32_t n_frames, const ss_csr *csr, float *features, double *stats0,
                     hipStream_t stream);

/* ss_surrogate_targets -- training targets from ss_clip_features' stats0
 * and a converged clip of the same frames (ref, [host] struct of device
 * arrays, count entries each).  target [dev] float [count][2]; use [dev]
 * uint8 [count] = 1 where n0 >= 2, s0 > 0, the clip converged with >= 2
 * members and std > 0 (else the target is 0 and the sample unused). */
int ss_surrogate_targets(const double *stats0, const ss_profile *ref, int64_t count,
                         float *target, uint8_t *use, hipStream_t stream);

/* ss_mlp_forward -- network outputs y [dev] float [n][2] for inputs
 * x [dev] float [n][SS_MLP_IN]; w16 [dev] uint16 [SS_MLP_PARAMS] float16 bits. */
int ss_mlp_forward(const uint16_t *w16, const float *x, int64_t n, float *y, hipStream_t stream);

/* Workspace bytes ss_mlp_grad needs for n samples. */
size_t ss_mlp_grad_workspace(int64_t n);

/* ss_mlp_grad -- loss L = (1/n_used) sum over used samples of
 * sum_o (y_o - target_o)^2 and its gradient with respect to the float16
 * parameters, grad [dev] float [SS_MLP_PARAMS] (0 in the padding), loss
 * [dev] float [1] (may be NULL).  use [dev] uint8 [n] or NULL (all used).
 * Deterministic: fixed reduction order.  Errors: SS_EINVAL, SS_ESIZE
 * (n <= 0, workspace too small), SS_EHIP. */
int ss_mlp_grad(const uint16_t *w16, const float *x, const float *target, const uint8_t *use,
                int64_t n, float *grad, float *loss, void *workspace, size_t workspace_bytes,
                hipStream_t stream);

/* ss_mlp_adam -- one Adam step (Kingma & Ba 2015; step counts from 1) on
 * params / m / v [dev] float [SS_MLP_PARAMS], writing the float16 copy w16. */
int ss_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr,
                float beta1, float beta2, float eps, uint16_t *w16, hipStream_t stream);

/* ss_sigma_clip_surrogate -- the clip of ss_sigma_clip, warm-started by the
 * surrogate.  Per (frame, bin) the network predicts the converged (mean,
 * std); the first clipping pass removes the members outside the intersection
 * of its own bounds (eq. clip on all members) and mean +- cutoff (1 + widen)
 * std; the plain passes follow (params->max_iter in all).  A bin is accepted
 * (state 1) when its clip converged with final bounds inside the predicted
 * ones, so the first pass removed nothing the final bounds keep; a refused
 * bin (state -1) is clipped again from scratch by a second, plain launch on
 * the same stream; a bin without a usable prediction runs the plain clip
 * (state 0): fewer than 64 members, zero spread, or a predicted interval
 * mean - cutoff (1 + widen) std <= 0 (low counts), where the clip can have
 * several fixed points and a warm start could settle on another one.  n_iter counts the passes that
 * removed members, as in ss_sigma_clip.
 * Requires the azimuthal model, cutoff > 0, widen >= 0, mask NULL, rows
 * within ss_class_rows(SS_SURROGATE_MAX_CLASS) and w16 16-byte aligned.
 *   accepted [dev] int32 [n_frames][n_bins], required: the states above.
 * Errors: SS_EINVAL, SS_ESIZE, SS_EHIP. */
int ss_sigma_clip_surrogate(const float *frames, const float *norm, const uint8_t *mask,
                            int32_t n_frames, const ss_csr *csr, const ss_params *params,
                            const uint16_t *w16, float widen, const ss_profile *out,
                            int32_t *accepted, hipStream_t stream);

/* ss_sigma_clip_warm -- the verified warm start of ss_sigma_clip_surrogate
 * with the prediction given instead of computed: pred_mean, pred_std [dev]
 * double [n_frames][n_bins] are each bin's predicted converged mean and std
 * (for instance the previous frame's profile in a stream of similar frames,
 * or any external predictor).  Pass 0 also removes the members outside
 * pred_mean +- cutoff (1 + widen) pred_std; acceptance, refusal (a second,
 * plain launch) and the bins without a warm start (fewer than 64 members,
 * zero spread, a predicted interval reaching zero, or a prediction that is
 * not positive) are exactly those of ss_sigma_clip_surrogate, so every bin
 * ends on the plain clip's fixed point or is clipped plainly.
 * Requirements and errors as ss_sigma_clip_surrogate (pred_mean and
 * pred_std replace w16). */
int ss_sigma_clip_warm(const float *frames, const float *norm, const uint8_t *mask,
                       int32_t n_frames, const ss_csr *csr, const ss_params *params,
                       const double *pred_mean, const double *pred_std, float widen,
                       const ss_profile *out, int32_t *accepted, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SIGSEP_H */
