/*
 * dh.h - C ABI of the MI355X off-axis digital-holography library (libdh.so).
 *
 * The library runs the per-frame pipeline of the digHolo user guide
 * (arXiv 2204.02348, Background, "digHolo processing pipeline"):
 *   1. FFT of the camera-frame window(s) around the beam centre;
 *   2. selection of the off-axis SR* term inside a circular Fourier window
 *      around the reference-tilt position, inverse FFT at the Fourier-window
 *      size (IFFT resolution mode 1), and removal of the reference tilt and
 *      defocus (API section "Alignment");
 *   3. projection of the field on Hermite-Gaussian modes HG(m,n), m+n < G
 *      (API section "Modal basis"), plus a per-frame power normalisation.
 * Every step runs in hand-written gfx950 kernels on the caller's HIP stream.
 *
 * Conventions (all fixed by the plan; see each field):
 *   - frames are row-major [batch][frame_h][frame_w], x fastest;
 *   - two polarisations occupy the left and right halves of the frame width
 *     (pipeline step 1); each has its own FFT window of fft_w x fft_h;
 *   - angles in degrees, lengths in metres, defocus in dioptre ("units");
 *   - complex values are {float re, im} pairs (complex64);
 *   - coefficient layout [batch][pol][mode]: one block of modes per
 *     polarisation (HHH..VVV), as digHoloBasisGetCoefs returns them;
 *   - mode order: group g = m+n ascending, inside a group m descending
 *     (m is the x order, n the y order).
 *
 * Error codes keep the paper's numbering ("Error codes").
 * Thread safety: calls on different handles may run concurrently; a handle
 * is used by one host thread at a time.
 */
#ifndef DH_H
#define DH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DH_SUCCESS 0
#define DH_ERR_ERROR 1
#define DH_ERR_INVALIDHANDLE 2
#define DH_ERR_NULLPOINTER 3
#define DH_ERR_INVALIDDIMENSION 5
#define DH_ERR_INVALIDPOLARISATION 6
#define DH_ERR_INVALIDAXIS 7
#define DH_ERR_INVALIDARGUMENT 8
#define DH_ERR_MEMORYALLOCATION 9

#define DH_INPUT_F32 0  /* frames are float32 */
#define DH_INPUT_U16 1  /* frames are uint16 camera counts */

#define DH_PREC_FP32 0       /* HG overlap on FP32 MFMA */
#define DH_PREC_SPLIT_BF16 1 /* HG overlap as split hi/lo BF16 MFMA, FP32 accumulate */
#define DH_PREC_SPLIT_FP16 2 /* HG overlap as split hi/lo FP16 MFMA, FP32 accumulate */

/* How the coefficients are formed from the masked spectrum (dh_params.path).
 * Both give the same c_mn up to rounding: the inverse DFT of the window, the
 * tilt/defocus removal and the HG quadrature are linear maps, so
 *   c_mn = sum_{u,v} W(u,v) X_m(u) Y_n(v),
 *   X_m(u) = sum_k e^{i phi_x(x'_k)} u_m(x'_k) p'_x e^{2 pi i u x'_k / (Nx p)}
 * (Y alike), with W the masked, normalised window of the cross term.
 *   FIELD:    inverse FFT to the field, tilt/defocus removal, overlap
 *             (the paper's order; needed for dh_get_fields and the split
 *             precision forms).
 *   SPECTRAL: the window contracted with the FP64-built tables X and Y on
 *             FP32 MFMA; no field is formed.
 *   AUTO:     SPECTRAL for the FP32 form with G > 0 and without keep_fields,
 *             else FIELD. */
#define DH_PATH_AUTO 0
#define DH_PATH_FIELD 1
#define DH_PATH_SPECTRAL 2

typedef struct dh_c64 {
  float re, im;
} dh_c64;

typedef int dh_handle;

/* Plan parameters: the paper's statement of the problem. */
typedef struct dh_params {
  int frame_w, frame_h;       /* camera frame, pixels; multiples of 16 ("Frame buffer") */
  int pol_count;              /* 1 or 2 polarisations ("Frame buffer", PolCount) */
  int fft_w, fft_h;           /* FFT window per polarisation, floored to a multiple of 16
                                 ("Window sizes", fftWindowSizeX/Y) */
  double pixel_size;          /* camera pixel pitch, m */
  double wavelength;          /* m */
  double beam_centre[2][2];   /* [pol][x,y], m, from the centre pixel (index half/2) of the
                                 pol's half of the frame ("Alignment", BeamCentre) */
  double window_radius_deg;   /* Fourier window radius w_c, degrees ("Window sizes") */
  double tilt_deg[2][2];      /* [pol][x,y] reference tilt, degrees ("Alignment") */
  double defocus[2];          /* [pol] reference defocus, dioptre ("Alignment") */
  double waist;               /* HG waist (1/e^2 intensity radius), m, shared by both pols */
  int max_mg;                 /* G: modes HG(m,n) with m+n < G; 0 = no decomposition; at most
                                 100 (the paper's largest LG basis, "Basis types"). Above 32 the
                                 spectral path only (FP32, no mode-1 fields, no AutoAlign) */
  int input_dtype;            /* DH_INPUT_F32 or DH_INPUT_U16 */
  int precision;              /* DH_PREC_* */
  int ifft_mode;              /* IFFT resolution mode ("Window sizes", IFFTResolutionMode):
                                 1: the field on the Fourier-window grid (W points, pitch N p / W);
                                 0: the field on the FFT grid (N points, the camera pitch). Mode 0
                                 runs the spectral path (needs FP32): the coefficients take the
                                 overlap over the FFT grid, and fields (keep_fields) are the kept
                                 window zero-padded to the FFT grid and inverse transformed at
                                 full size; with G = 0 only the fields are made */
  int keep_window;            /* nonzero: store each frame's Fourier window (dh_get_window) */
  int keep_fields;            /* nonzero: store each frame's field (dh_get_fields) */
  int path;                   /* DH_PATH_*; SPECTRAL in mode 1 with keep_fields, a split precision
                                 or G = 0 is DH_ERR_INVALIDARGUMENT, as is FIELD in mode 0 */
} dh_params;

/* Geometry derived by the plan (all FP64 on the host). */
typedef struct dh_plan_info {
  int fft_w, fft_h;           /* effective FFT window (after flooring) */
  int ifft_w, ifft_h;         /* Fourier-window grid W: smallest multiple of 16 with prime
                                 factors <= 13 that is >= floor(2 r) + 1 bins (the mode-1 IFFT
                                 size; windows are stored on it in both modes) */
  int box_w, box_h;           /* spectrum bins spanned by the Fourier window (max over pols) */
  int modes;                  /* modes per polarisation, G (G+1) / 2 */
  int x0[2], y0[2];           /* window origins in the frame, pixels */
  double ax[2], ay[2];        /* cross-term position: SR* sits at bins (-ax, -ay) */
  double rx, ry;              /* window radius in bins along x, y */
  double pitch_x, pitch_y;    /* pitch of the W grid, N p / W, m */
  size_t device_bytes;        /* device memory the plan allocates */
  int chunk;                  /* frames per internal launch chunk */
  int path;                   /* DH_PATH_FIELD or DH_PATH_SPECTRAL: the path the plan runs */
  int field_w, field_h;       /* field grid F: W in IFFT mode 1, N in mode 0 */
  double field_pitch_x, field_pitch_y;  /* its pitch N p / F, m (the camera pitch in mode 0) */
  int generic;                /* lengths run by the runtime-length kernels: bit 0 the row
                                 pass (N_x), bit 1 the column pass and mode-0 export (N_y,
                                 or an (N_y, W_y) pair without a compiled column kernel) */
} dh_plan_info;

/*
 * Validate `p` and derive the plan geometry on the host; touches no GPU.
 * Returns DH_SUCCESS and fills *info (if non-NULL), or:
 *   DH_ERR_NULLPOINTER        p is NULL;
 *   DH_ERR_INVALIDDIMENSION   frame or window size not a positive multiple of 16,
 *                             window outside the frame, or an FFT/IFFT length
 *                             the library has no kernel for;
 *   DH_ERR_INVALIDPOLARISATION pol_count not 1 or 2;
 *   DH_ERR_INVALIDARGUMENT    pixel/wavelength/radius/waist not > 0, max_mg outside
 *                             0..100 (or above 32 where the plan would take the field
 *                             path), unknown dtype/precision/ifft_mode/path, a Fourier
 *                             window wider than the spectrum, or DH_PATH_SPECTRAL
 *                             where it does not apply (see DH_PATH_*).
 * max_batch < 1 is taken as 1 (the paper clamps batchCount the same way).
 */
int dh_plan_check(const dh_params* p, int max_batch, dh_plan_info* info);

/*
 * Build a plan: validates like dh_plan_check, then allocates every device
 * table and workspace on the current HIP device and builds the tables
 * (phase tables and masks in FP64 on the host, HG tables by an FP64
 * recurrence on the GPU). The library owns all of it until dh_destroy.
 * hbm_budget: if nonzero and the plan would need more device bytes,
 * DH_ERR_MEMORYALLOCATION is returned before anything is allocated (also on
 * an allocation failure). Writes the new handle to *out.
 */
int dh_plan(const dh_params* p, int max_batch, size_t hbm_budget, dh_handle* out);

/*
 * The largest Fourier window radius (degrees) for the tilts of `p` (the
 * paper's AutoAlignFourierWindowRadius, "as large as possible for the tilt";
 * background section "How do you choose the angle of the Reference Field?"):
 * the window around each pol's cross term stays clear of the autocorrelation
 * terms at the origin (radius twice the window's) and of the conjugate cross
 * term, and, without wrap, inside the resolvable spectrum +-w_max; with wrap
 * the spectrum is periodic (period 2 w_max) and the same gaps hold from every
 * image. The smaller radius of the two pols. Host only: a plan's box is fixed,
 * so a caller plans again with the radius returned. Uses pixel_size,
 * wavelength, pol_count and tilt_deg only. Errors: DH_ERR_NULLPOINTER,
 * DH_ERR_INVALIDPOLARISATION, DH_ERR_INVALIDARGUMENT.
 */
int dh_max_window_radius(const dh_params* p, int wrap, double* radius_deg);

/*
 * Batch processing ("Execute batch processing": digHoloProcessBatch, with the
 * batch count of digHoloConfigSetBatchCount; the pipeline of "digHolo
 * processing pipeline", steps 1-3). Process `batch` frames (device pointer,
 * [batch][frame_h][frame_w] of the plan's input_dtype) asynchronously on
 * `stream` (a hipStream_t; NULL = the default stream). The caller keeps
 * ownership of `frames`; they must stay valid and unchanged until the stream
 * has passed this work. batch < 1 is taken as 1. A batch larger than
 * max_batch is processed in launch chunks like any other; its coefficient
 * outputs (raw, normalised, basis) move to an allocation for `batch` frames,
 * made on the first such call and grown only when a larger batch comes (the
 * call then waits for the device); this is refused with
 * DH_ERR_INVALIDDIMENSION while `stream` is being captured and for plans that
 * keep windows or fields, sweep wavelengths or average (their buffers hold
 * max_batch outputs). With averaging (dh_set_averaging) `batch` counts
 * outputs and batch * count frames are read (DH_ERR_INVALIDDIMENSION above
 * max_batch); with a wavelength sweep (dh_set_wavelengths) batch must be a
 * multiple of the wavelength count (else DH_ERR_INVALIDDIMENSION).
 * Errors: DH_ERR_INVALIDHANDLE, DH_ERR_NULLPOINTER, DH_ERR_INVALIDDIMENSION,
 * DH_ERR_MEMORYALLOCATION (growing the outputs), DH_ERR_ERROR (launch).
 */
int dh_process_batch(dh_handle h, const void* frames, int batch, void* stream);

/* Transfer-matrix metrics ("Transfer matrix analysis parameters"; AutoAlign
 * goal metrics), all in dB. */
#define DH_METRIC_IL 0        /* insertion loss: 10 log10 of the mean squared singular value */
#define DH_METRIC_MDL 1       /* mode dependent loss: 10 log10(min s^2 / max s^2), <= 0 */
#define DH_METRIC_DIAG 2      /* mean power of the diagonal entries */
#define DH_METRIC_SNRAVG 3    /* diagonal power / off-diagonal power */
#define DH_METRIC_DIAGBEST 4  /* largest diagonal power */
#define DH_METRIC_DIAGWORST 5 /* smallest diagonal power */
#define DH_METRIC_SNRBEST 6   /* largest diagonal / off-diagonal power of one row (batch element) */
#define DH_METRIC_SNRWORST 7  /* smallest of the same */
#define DH_METRIC_SNRMG 8     /* as SNRAVG, power between modes of one pol and HG group counted as signal */
#define DH_METRIC_COUNT 9

/*
 * The nine metrics of the last processed batch's transfer matrix A, written
 * to out[DH_METRIC_COUNT] (host memory). A is built from the raw coefficients:
 * pol_independent 0: batch x (pol x mode), row b = frame b; 1: (pol x batch)
 * x (pol x mode), row p*batch + b holds frame b's pol-p coefficients in pol
 * p's columns and zeros in the other pol's (a missing pol gives MDL = -inf).
 * IL and MDL come from the singular values of A (eigenvalues of the smaller
 * Gram matrix, FP64, by the library's eigenvalue kernel; a smaller side
 * above 2048 is refused with DH_ERR_ERROR); the diagonal and SNR metrics from D = A
 * (mul_conj_trans 0) or D = A A^H (1), with entry (i, i) as the diagonal for
 * i < min(rows, cols of D); row i of A stands for the mode of column i, which
 * is what SNRMG compares. Values are +inf / -inf where a ratio's denominator
 * or numerator is zero. Waits for the stream of the last dh_process_batch and
 * runs there; allocates a workspace on first use (kept until dh_destroy).
 * Errors: DH_ERR_INVALIDHANDLE, DH_ERR_NULLPOINTER, DH_ERR_ERROR (no batch
 * processed, G = 0, or the eigen-solver failed), DH_ERR_MEMORYALLOCATION.
 */
int dh_transfer_metrics(dh_handle h, int pol_independent, int mul_conj_trans, double* out);

/*
 * The eigen step of the MDL metric on its own ("Transfer matrix analysis
 * parameters": MDL from the singular values of the transfer matrix, which are
 * the square roots of the eigenvalues of its Gram matrix). a_host: n x n
 * Hermitian matrix in host memory, complex FP64 interleaved (re, im),
 * column-major (only its Hermitian part is meaningful); w_host: n eigenvalues
 * out, ascending. Runs the library's FP64 kernel (Householder reduction to a
 * real tridiagonal matrix, then bisection with Sturm counts; every eigenvalue
 * within a small multiple of n eps |A| of the exact one) on the current device
 * (one workgroup) on `stream` and waits for it; allocates and frees a device
 * copy of the matrix. Errors: DH_ERR_NULLPOINTER, DH_ERR_INVALIDDIMENSION
 * (n < 1 or n > 2048), DH_ERR_MEMORYALLOCATION, DH_ERR_ERROR (entries that are
 * not finite, or a HIP call failed).
 */
int dh_hermitian_eigenvalues(const double* a_host, int n, double* w_host, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the eigen step of
 * dh_hermitian_eigenvalues with no allocation of any kind. a_dev: n x n
 * Hermitian matrix in device memory (layout as above), read only; w_dev: n
 * eigenvalues out in device memory, ascending. The working copy of the matrix
 * lives in a fixed device array of the library (DH_NOALLOC_EIG_MAX_N^2 complex
 * FP64 values, 1 MiB, held on every GPU the library runs on until the process
 * ends). Runs on `stream` on the current device and waits for it. Calls that
 * overlap on one GPU share that array and race: issue them from one thread
 * and stream per GPU. Errors: DH_ERR_NULLPOINTER, DH_ERR_INVALIDDIMENSION
 * (n < 1 or n > DH_NOALLOC_EIG_MAX_N), DH_ERR_ERROR (entries that are not
 * finite, or a HIP call failed).
 */
#define DH_NOALLOC_EIG_MAX_N 256
int dh_hermitian_eigenvalues_noalloc(const double* a_dev, int n, double* w_dev, void* stream);

/*
 * Coefficients of the last processed batch, [batch][pol][mode] complex64.
 * host_out non-NULL: waits for the stream of the last dh_process_batch and
 * copies batch*pols*modes values. dev_out non-NULL: receives the library's
 * device buffer (valid until the next process call or dh_destroy).
 * normalised nonzero: each frame divided by the square root of its total
 * power over both polarisations (computed in FP64); 0: raw coefficients, in
 * field units. batch, modes, pols (each may be NULL) receive the sizes. With
 * max_mg = 0 this succeeds with modes = 0 and *dev_out = NULL.
 */
int dh_mode_coefs(dh_handle h, dh_c64* host_out, const dh_c64** dev_out, int* batch, int* modes,
                  int* pols, int normalised);

/*
 * Fourier windows of the last batch (needs keep_window): [batch][pol][ifft_h][ifft_w]
 * complex64; bin (u, v) of the beam-centred spectrum is stored at
 * (v mod ifft_h, u mod ifft_w) when it lies inside the window, zero elsewhere
 * ("Fourier plane window", digHoloGetFourierPlaneWindow). Sizes as above;
 * DH_ERR_ERROR if the plan does not keep windows.
 */
int dh_get_window(dh_handle h, dh_c64* host_out, const dh_c64** dev_out, int* batch, int* pols,
                  int* width, int* height);

/*
 * Reconstructed fields of the last batch (needs keep_fields):
 * [batch][pol][field_h][field_w] complex64 on the grid x'_k = (k - F/2) p'
 * around the beam centre, F and p' the field grid of the IFFT mode
 * (digHoloGetFields; kept in FP32, dh_get_fields16 gives the int16 form).
 */
int dh_get_fields(dh_handle h, dh_c64* host_out, const dh_c64** dev_out, int* batch, int* pols,
                  int* width, int* height);

/*
 * Axes of the reconstructed field grid (the x and y axis arrays that
 * digHoloGetFields returns with the fields): x[k] = (k - F_x/2) p'_x and
 * y[l] = (l - F_y/2) p'_y in metres from each polarisation's beam centre, F and
 * p' the field grid of the IFFT mode (the same for both polarisations). x, y:
 * host arrays of width / height doubles (each may be NULL); width, height
 * receive the sizes. Host only. Errors: DH_ERR_INVALIDHANDLE.
 */
int dh_get_field_axes(dh_handle h, double* x, double* y, int* width, int* height);

/*
 * Batch summary ("Advanced functions", digHoloBatchGetSummary; "Analysis
 * parameter types"): for every batch element and polarisation, and for the
 * intensity summed over the batch (the last, "+1", entry), the DH_ANALYSIS_*
 * parameters of one plane:
 *   plane 0, the Fourier plane: |FFT|^2 of each polarisation's FFT window on
 *     the real-to-complex half plane, width fft_w/2 + 1 (k_x = 0 .. N_x/2) by
 *     height fft_h (k_y = -N_y/2 .. N_y/2 - 1, ascending); axes in degrees of
 *     paraxial angle (bin k at k lambda/(N p) rad), the units of the tilt.
 *     Computed from `frames` (device pointer, `batch` frames of the plan's
 *     frame size and input type, contiguous) on `stream`.
 *   plane 1, the reconstructed field plane: |E|^2 of the last batch's fields
 *     (needs keep_fields; `frames` and `batch` are ignored), axes as
 *     dh_get_field_axes; runs on the stream of the last dh_process_batch.
 * With I the intensity and dA = |dx dy| the cell of the plane's axes:
 * TOTALPOWER = sum I dA; COMX, COMY = centres of mass on the axes; MAXABS =
 * sqrt(max I); MAXABSIDX = row-major index y W + x of the first maximum,
 * stored as int32 bits in its float slot (as the paper warns); AEFF = (sum I
 * dA)^2 / (sum I^2 dA) (a Gaussian beam I ~ exp(-2 r^2/w^2) gives pi w^2);
 * COMYWRAP = the circular mean of y over the period H dy of the y axis, in
 * the axis' range. Sums in FP64; an all-zero plane gives zeros.
 * Outputs (host memory, each may be NULL): params [DH_ANALYSIS_COUNT][pols]
 * [total_count] float, total_count = batch + 1; x_axis [width], y_axis
 * [height] double; total_intensity [pols][height][width] float, the summed
 * intensity. With params and total_intensity both NULL only the sizes and
 * axes are returned. Allocates and frees device scratch per call and waits
 * for the stream. Errors: DH_ERR_INVALIDHANDLE, DH_ERR_INVALIDARGUMENT (plane),
 * DH_ERR_NULLPOINTER (plane 0 without frames), DH_ERR_ERROR (plane 1 without
 * kept fields or a processed batch), DH_ERR_MEMORYALLOCATION.
 */
#define DH_ANALYSIS_TOTALPOWER 0
#define DH_ANALYSIS_COMX 1
#define DH_ANALYSIS_COMY 2
#define DH_ANALYSIS_MAXABS 3
#define DH_ANALYSIS_MAXABSIDX 4
#define DH_ANALYSIS_AEFF 5
#define DH_ANALYSIS_COMYWRAP 6
#define DH_ANALYSIS_COUNT 7
int dh_batch_summary(dh_handle h, int plane, const void* frames, int batch, void* stream, float* params,
                     double* x_axis, double* y_axis, float* total_intensity, int* total_count, int* pols,
                     int* width, int* height);

/*
 * The fields of the last batch in the paper's 16-bit form (digHoloGetFields16,
 * "Return reconstructed fields"): int16 real and imaginary parts
 * [batch][pol][field_h][field_w] and one float scale per field and pol, the
 * field being (re + i im) / scale. The scale maps the largest real or
 * imaginary magnitude of the field to 32767 (scale 1 for an all-zero field);
 * each part is rounded to the nearest integer, ties to even, in FP32. The
 * device copies live in a buffer the plan makes on the first call and
 * overwrites on each; host pointers, if non-NULL, receive copies. Needs
 * keep_fields (else DH_ERR_ERROR); DH_ERR_MEMORYALLOCATION if the buffer
 * cannot be made. Synchronises the stream of the last dh_process_batch.
 */
int dh_get_fields16(dh_handle h, short* re_host, short* im_host, float* scale_host, const short** re_dev,
                    const short** im_dev, const float** scale_dev, int* batch, int* pols, int* width,
                    int* height);

/*
 * The same conversion for any n_fields complex64 fields of field_len values
 * each, back to back in device memory: re, im (n_fields * field_len each)
 * and scale (n_fields) are device buffers the caller owns. Asynchronous on
 * `stream`. DH_ERR_INVALIDARGUMENT for n_fields < 0 or field_len < 1,
 * DH_ERR_NULLPOINTER for a null buffer (n_fields > 0).
 */
int dh_fields_to_int16(const dh_c64* fields, int n_fields, long long field_len, short* re, short* im,
                       float* scale, void* stream);

/* Copy of the plan's parameters / derived geometry. */
int dh_get_params(dh_handle h, dh_params* out);
int dh_get_plan_info(dh_handle h, dh_plan_info* out);

/*
 * Per-stage timing, the counterpart of the paper's per-stage benchmark rates
 * ("Multi-threading, performance and benchmarking"): while enabled, every
 * dh_process_batch records a HIP event on its stream after each kernel
 * launch. dh_stage_times waits for the last of them and returns, per stage,
 * the summed milliseconds and the number of launches since timing was
 * enabled or last read, then starts a new count. Stages:
 *   0 DH_STAGE_FFT   frame load + FFT along x (row pass)
 *   1 DH_STAGE_CROP  FFT along y + window crop/mask, then the IFFT along y (field
 *                    path) or the contraction with the folded tables (spectral path)
 *   2 DH_STAGE_FIELD IFFT along x + tilt/defocus removal + HG overlap (field path)
 *   3 DH_STAGE_NORM  per-frame FP64 power normalisation
 * ms and launches point to DH_STAGE_COUNT entries each.
 */
#define DH_STAGE_FFT 0
#define DH_STAGE_CROP 1
#define DH_STAGE_FIELD 2
#define DH_STAGE_NORM 3
#define DH_STAGE_COUNT 4
int dh_set_stage_timing(dh_handle h, int enabled);
int dh_stage_times(dh_handle h, double* ms, int* launches);

/*
 * Automatic alignment (the paper's digHoloAutoAlign, "Automatic (AutoAlign)"
 * and "AutoAlign operation modes"): searches the reference tilt and defocus,
 * the beam centre and the HG waist that maximise the goal below, on `batch`
 * frames (device pointer as in dh_process_batch), and leaves the plan at the
 * result.
 *   mode: DH_ALIGN_FULL (snap, then tweak), DH_ALIGN_TWEAK (refine from the
 *         current parameters), DH_ALIGN_ESTIMATE (snap only);
 *   what: bitmask of DH_ALIGN_TILT, DH_ALIGN_DEFOCUS, DH_ALIGN_WAIST,
 *         DH_ALIGN_CENTRE;
 *   tol:  stop when a full sweep over the parameters improves the goal by
 *         less than tol (dB), as the paper's AutoAlignTol.
 * Goal (dh_set_align_goal): by default the captured power,
 * 10 log10(sum |c|^2 / sum |E|^2 p'x p'y) over the batch and both
 * polarisations, computed in FP64 (0 dB: the field is exactly a combination
 * of the basis modes); or one transfer-matrix metric (DH_METRIC_*) of the
 * batch's raw coefficients. With a metric goal every trial evaluates that
 * metric, and each polarisation's tilt, defocus and centre is a coordinate of
 * its own (pol locks: dh_set_pol_lock).
 * Snap: the tilt from scratch, from the whole Fourier plane of the first 32
 * frames: the zero-order region (twice the window radius about the origin)
 * left out, the brightest other bin and its mirror are the cross terms, the
 * one whose tilt is nearer the current tilt is taken (from a zero tilt:
 * positive x, then positive y), at the centroid of its power above the mean
 * (report: plane_tilt_deg); then the tilt at the centroid of the batch power
 * spectrum (above its mean) near that tilt; then, from the fields
 * reconstructed there (G > 0),
 * the beam centre at the centroid of the batch intensity |E|^2 and the waist
 * from its pooled central second moment, w = sqrt(6 (<x^2> + <y^2>) / (2G + 1))
 * (exact when the power is spread evenly over the modes of G groups).
 * Defocus (with DH_ALIGN_DEFOCUS): its magnitude per pol from the window's
 * angular spread beyond the modes' own, 2 (2G + 1) / (3 w^2), over the field's
 * spatial spread (report: snap_defocus); of the start value, +|D| and -|D|
 * each pol keeps the one with its highest captured power (three trials).
 * Tweak: a coordinate search. Tilts stay within 0.6
 * window radii of the snap's (of the start with TWEAK) and beam centres
 * within an eighth of the FFT window of their start; a centre that moves the FFT window out of the frame is a failed
 * trial. Each trial re-runs the window gather, the IFFTs and the overlap from
 * a spectrum kept on the device, computed again only when a centre moves the
 * window by whole pixels.
 * The trials run the field path's overlap, so plans with G > 32 return
 * DH_ERR_INVALIDARGUMENT.
 * The returned value is the goal in dB; -FLT_MAX on failure, with the reason
 * in dh_last_error (DH_ERR_INVALIDHANDLE, NULLPOINTER, INVALIDDIMENSION,
 * INVALIDARGUMENT, MEMORYALLOCATION, ERROR). Synchronises the device.
 */
#define DH_ALIGN_FULL 0
#define DH_ALIGN_TWEAK 1
#define DH_ALIGN_ESTIMATE 2
#define DH_ALIGN_TILT 1u
#define DH_ALIGN_DEFOCUS 2u
#define DH_ALIGN_WAIST 4u
#define DH_ALIGN_CENTRE 8u
float dh_autoalign(dh_handle h, const void* frames, int batch, int mode, unsigned what, float tol, void* stream);

#define DH_GOAL_CAPTURED (-1)
/*
 * Goal of the following dh_autoalign calls on h: DH_GOAL_CAPTURED (default)
 * or a DH_METRIC_* index, with the transfer-matrix options of
 * dh_transfer_metrics (the paper's AutoAlignGoalIdx, AutoAlignPolIndependence,
 * AutoAlignBasisMulConjTrans). Errors: DH_ERR_INVALIDHANDLE,
 * DH_ERR_INVALIDARGUMENT (goal outside -1..DH_METRIC_COUNT-1).
 */
int dh_set_align_goal(dh_handle h, int goal, int pol_independent, int mul_conj_trans);

typedef struct dh_align_report {
  int evaluations;             /* trials of the goal */
  int sweeps;                  /* tweak sweeps over the parameters */
  double start_goal_db;        /* goal after the snap (before the tweak) */
  double goal_db;              /* final goal (dB) */
  double captured;             /* final captured power as a fraction */
  double snap_tilt_deg[2][2];  /* tilt found by the snap ([pol][x,y]) */
  int goal;                    /* the goal optimised: DH_GOAL_CAPTURED or DH_METRIC_* */
  double metrics[DH_METRIC_COUNT];  /* every metric at the final parameters (dh_transfer_metrics) */
  double snap_centre[2][2];    /* beam centre found by the snap ([pol][x,y], metres) */
  double snap_waist;           /* waist found by the snap (metres) */
  double plane_tilt_deg[2][2]; /* the snap's first guess from the whole Fourier plane ([pol][x,y]) */
  double snap_defocus[2];      /* defocus magnitude found by the snap ([pol], dioptre) */
} dh_align_report;

/*
 * Modal basis of the coefficients ("Basis types", digHoloConfigSetBasisType*):
 * fields are always decomposed in HG; another basis is one matrix product of
 * the HG coefficients, c_out = T c_HG, per frame and polarisation, for the raw
 * and the normalised coefficients alike (T applied after the HG power
 * normalisation). After dh_set_basis, dh_mode_coefs returns the basis
 * coefficients (modes = its output count) and dh_transfer_metrics and the
 * metric goals of dh_autoalign take the matrix in that basis.
 *   DH_BASIS_HG      the HG coefficients themselves (default);
 *   DH_BASIS_LG      Laguerre-Gaussian, LG_{p,l} ~ (sqrt2 r/w)^|l| L_p^|l|(2r^2/w^2)
 *                    e^{-r^2/w^2} e^{i l phi}, unit norm, same waist; group
 *                    N = 2p + |l| < G, in group order, l = N, N-2, ..., -N inside
 *                    a group; T[k][j] = <LG_k|HG_j> (unitary, within groups);
 *   DH_BASIS_CUSTOM  the caller's host matrix `transform`, modes_out x modes_in
 *                    row-major complex64; columns past the plan's HG modes are
 *                    not used, missing ones count as zero. The matrix is copied.
 * modes_out, modes_in and transform are read for DH_BASIS_CUSTOM only. A
 * server (dh_serve_create) keeps the basis its plans had when it was made.
 * Errors: DH_ERR_INVALIDHANDLE; DH_ERR_INVALIDARGUMENT (type);
 * DH_ERR_INVALIDDIMENSION (G = 0, or custom sizes < 1 or modes_out > 65536);
 * DH_ERR_NULLPOINTER (custom without a matrix); DH_ERR_MEMORYALLOCATION.
 * Synchronises the device.
 */
#define DH_BASIS_HG 0
#define DH_BASIS_LG 1
#define DH_BASIS_CUSTOM 2
int dh_set_basis(dh_handle h, int type, int modes_out, int modes_in, const dh_c64* transform);

/*
 * Wavelength sweeps ("Wavelength", "Input/output wavelength ordering"): the
 * frames of a batch are taken at `count` wavelengths (m). Each frame is
 * processed at its own wavelength: its tilt angle and defocus are converted
 * with that wavelength, while the window radius in bins, the IFFT size and
 * the field grid stay those of the plan's wavelength (the centre wavelength),
 * so every output has one shape. A batch of N outputs holds I = N / count
 * inputs at every wavelength (N must be a multiple of count); output o holds
 * input i at wavelength w at o = i count + w (out_order DH_WL_FAST) or
 * o = w I + i (DH_WL_SLOW); without averaging, frame j of the batch holds it
 * at j = i count + w (in_order DH_WL_FAST) or w I + i (DH_WL_SLOW). count = 0
 * goes back to every frame at the plan's wavelength.
 * Errors: DH_ERR_INVALIDHANDLE; DH_ERR_INVALIDDIMENSION (count < 0 or > 4096);
 * DH_ERR_NULLPOINTER; DH_ERR_INVALIDARGUMENT (a wavelength not > 0 or not
 * finite, an unknown ordering); DH_ERR_MEMORYALLOCATION. Synchronises the
 * device.
 */
#define DH_WL_FAST 0
#define DH_WL_SLOW 1
int dh_set_wavelengths(dh_handle h, const double* lambdas, int count, int in_order, int out_order);

/*
 * Frame averaging (digHoloSetBatchAvg, "Averaging modes"): each output of
 * dh_process_batch is the average of `count` frames, so a batch of N outputs
 * reads N * count frames (N * count <= max_batch). The repetitions of an
 * output are adjacent (DH_AVG_SEQUENTIAL, AAABBB: frame j count + a), a batch
 * apart (DH_AVG_INTERLACED, ABCABC: frame a N + j), or whole wavelength sweeps
 * apart (DH_AVG_SEQUENTIAL_SWEEP, {A}{A}{B}{B}: frame (i count + a) L + w;
 * the same as sequential for one wavelength), j being the output's frame
 * index without averaging. Their Fourier windows are added in phase: each
 * repetition is turned by exp(-i arg sum W_a conj(W_0)) (over both pols and
 * every window bin; W_0 the first repetition) and the mean is the output's
 * window; its field and coefficients follow (computed per frame and combined
 * the same way, which is equal by linearity), the normalised coefficients
 * from the averaged ones. count = 1 turns averaging off. Sweeps and averaging
 * are not available to dh_autoalign or to servers (DH_ERR_INVALIDARGUMENT).
 * Errors: DH_ERR_INVALIDHANDLE; DH_ERR_INVALIDDIMENSION (count < 1 or > 4096);
 * DH_ERR_INVALIDARGUMENT (mode); DH_ERR_MEMORYALLOCATION.
 */
#define DH_AVG_SEQUENTIAL 0
#define DH_AVG_INTERLACED 1
#define DH_AVG_SEQUENTIAL_SWEEP 2
int dh_set_averaging(dh_handle h, int count, int mode);

/*
 * Polarisation locks of later dh_autoalign calls ("Alignment": PolLockTilt,
 * PolLockDefocus, PolLockBasisWaist): a bitmask of DH_ALIGN_TILT and
 * DH_ALIGN_DEFOCUS; a locked parameter of pol 1 takes pol 0's value after the
 * snap and both move as one coordinate. DH_ALIGN_WAIST is accepted and has no
 * effect: both pols always share one waist here. Errors: DH_ERR_INVALIDHANDLE,
 * DH_ERR_INVALIDARGUMENT (other bits).
 */
int dh_set_pol_lock(dh_handle h, unsigned lock);

/* Report of the last dh_autoalign on h. */
int dh_get_align_report(dh_handle h, dh_align_report* out);

/*
 * Serving form: continuous batching of frames from several cameras, each a
 * resident plan (tables, bases and alignment state stay on the device).
 *
 * dh_serve_create: a server over `ncam` plans (their handles stay owned by the
 * caller and must outlive the server). Every camera gets "lanes" - in-flight
 * batch slots of up to max_batch frames, each with its own HIP stream,
 * workspace, frame-pointer array and pinned result buffer - made round robin
 * over the cameras while their device bytes fit hbm_budget (0: no limit;
 * at least one lane per camera, else DH_ERR_MEMORYALLOCATION; at most four).
 * use_graphs: capture each lane's launch sequence once per batch size as a
 * hipGraph and replay it, for batches of up to 16 requests (larger batches
 * are launched directly). normalised: results are the power-normalised
 * coefficients (else raw). Writes the server handle to *out.
 *
 * Admission: a request waits in its camera's queue until a lane of that
 * camera is free; the lane then takes every waiting request (up to max_batch)
 * as one batch. Batches therefore grow with the load, requests that arrive
 * while others are on the GPU start as soon as a lane frees up, and the lanes
 * of all cameras run concurrently. Each frame's result does not depend on the
 * batch it ran in (no reductions across frames).
 *
 * dh_serve_submit: queue one frame (device pointer, the camera's frame layout
 * and dtype, kept unchanged until its result is done); when it completes its
 * [pol][mode] coefficients are copied to `result` (host, may be NULL).
 * dh_serve_progress: one scheduling round from the calling thread - retire
 * finished batches, start batches on free lanes; *completed = requests done.
 * dh_serve_replay: drive the loop in real time over a trace of n requests:
 * request i arrives t_arrival[i] seconds after the call starts (ascending),
 * for camera[i], frame frames[i], result results[i] (results may be NULL);
 * returns when all are done with t_done[i] = completion time (same clock).
 * dh_serve_info / dh_serve_stats: lanes and bytes per camera; batches and
 * frames processed. dh_serve_destroy: waits for the device, frees the lanes.
 * One host thread drives a server at a time.
 */
typedef int dh_server;
int dh_serve_create(const dh_handle* plans, int ncam, int max_batch, size_t hbm_budget, int use_graphs,
                    int normalised, dh_server* out);
int dh_serve_info(dh_server s, int camera, int* lanes, size_t* lane_bytes, int* per_result);
int dh_serve_submit(dh_server s, int camera, const void* frame, dh_c64* result);
int dh_serve_progress(dh_server s, int* completed);
int dh_serve_replay(dh_server s, int n, const double* t_arrival, const int* camera, const void* const* frames,
                    dh_c64* const* results, double* t_done, double* t_start);
int dh_serve_stats(dh_server s, long long* batches, long long* frames);
int dh_serve_destroy(dh_server s);

/* Error code of the last failing call on h (0 if none), 2 for a bad handle. */
int dh_last_error(dh_handle h);

/* Free every device allocation of h; the handle becomes invalid. */
int dh_destroy(dh_handle h);

#ifdef __cplusplus
}
#endif

#endif /* DH_H */
