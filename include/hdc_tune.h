/*
 * hdc_tune -- parameter choice for the hybrid dealiased convolution: the
 * experience-based autotuner (section 4.2 exhaustive search, section 4.3
 * experience) and the learned predictor (section 4.4; classification over
 * scale-free parameter classes, sections 6.3-6.4).
 *
 * A problem is a 1D convolution of `batch` interleaved copies (section 2.5's
 * C copies) or an N-D convolution (ndim 2 or 3, row-major, last axis
 * contiguous, section 3.6) of equal extents L[a] with output box M[a].
 * Parameters are per axis: the FFT size m, the block counts p and q (0 in
 * requests: derive the ceilings of section 2.5), the residues per pass D, and
 * the column tile (columns per workgroup of the column passes; 0 = the
 * kernels' default).  The tile does not change the result (every column is
 * transformed the same way), only how the work is spread over workgroups.
 *
 * Conventions as in hdc.h (status codes, hdc_last_error).
 */
#ifndef HDC_TUNE_H
#define HDC_TUNE_H

#include <stdint.h>

#include "hdc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t ndim;      /* 1 .. 3                                          */
    int64_t L[3];      /* input extents (equal for f and g)               */
    int64_t M[3];      /* output extents (2 L - 1 for the full convolution) */
    hdc_dtype dtype;   /* HDC_C64 or HDC_C128                             */
    int64_t batch;     /* copies of a 1D problem (1 for N-D)              */
} hdc_problem;

typedef struct {
    int64_t m[3], p[3], q[3], D[3];  /* per axis; p, q = 0: derive            */
    int64_t C[3];                    /* output only: copies of axis a (batch for 1D; for N-D
                                        the product of the inner output extents) */
    int32_t tile[3];                 /* column tile; 0 = default              */
} hdc_params;

/* Plan of `prob` with parameters `prm` (hdc_plan with C = batch for 1D,
 * hdc_plan_nd otherwise, plus the column tiles).  Errors as hdc_plan /
 * hdc_plan_nd; HDC_ERR_UNSUPPORTED for a tile the kernels cannot run
 * (not a power of two, or more than 1024 threads per workgroup). */
hdc_status hdc_plan_params(hdc_plan_t* out, const hdc_problem* prob, const hdc_params* prm);

/* Host-only check of a parameter set (no device is touched): the admissibility
 * rules and kernel limits of hdc_plan / hdc_plan_nd plus the column tiles.  On
 * success, fills `out` (may be NULL) with the derived parameters: p, q, D
 * (clamped), C, and tile[a] = the column tile the plan would use on axis a (0
 * when that axis runs no column pass). */
hdc_status hdc_params_check(const hdc_problem* prob, const hdc_params* prm, hdc_params* out);

/*
 * Autotuner (section 4).  Every candidate is scored by the time of the whole
 * convolution (forward, product and backward fused on the GPU): 2 warm-up
 * runs, then the median of 5 HIP-event-timed runs on inputs allocated and
 * filled by the call (uniform values in [-1, 1]).  Ties within 1 % go to the
 * smaller m, then the smaller D, then the default tile.
 *
 * mode 0 (A0, section 4.2): exhaustive over the candidate grid: power-of-two
 *   m (for 1D problems also m = R 2^k <= 4096 with R odd and 7-smooth, the
 *   mixed-radix fused kernel) with p = ceil(L/m) in {1, 2, 3, 4, 6, 8, 12, 16}
 *   (or q = 1, the explicit case) and q >= p, D in {q, 1, 2, 4, ...} (the
 *   candidates the kernels cannot run are skipped), then the column tile (half and
 *   double the default) of the best.  N-D problems are searched one axis at a
 *   time with the other axes at their defaults (p = 1, D = q): the
 *   separability argument of section 4.2.
 * mode 1 (A1, section 4.3): (1) the best entry of the database for the same
 *   problem, if any, without timing; otherwise (2) the scale-free classes
 *   (p, all residues or one per pass) that won on the two nearest tuned
 *   problems of the same dtype and dimension, (3) two random candidates, and
 *   (4) local refinement (m halved and doubled, D = q) until no new candidate.
 *
 * db: path of an append-only JSON-lines timing database (section 5.1): every
 * timing is appended as it is measured, so an interrupted run resumes; NULL
 * for none.  Rows carry the device name and this library's build id
 * (hdc_build_id); only rows of the current device and build are used.
 * best (required) receives the chosen parameters (p, q and C filled in),
 * best_ms (may be NULL) its time.  Synchronous: allocates its buffers and a
 * stream on the current device and frees them before returning.
 */
hdc_status hdc_tune(const hdc_problem* prob, int mode, const char* db, hdc_params* best, double* best_ms);

/* Cost of one parameter set for hdc_tune_host: milliseconds, or a negative
 * value for a set that cannot run. */
typedef double (*hdc_cost_fn)(const hdc_problem* prob, const hdc_params* prm, void* ctx);

/*
 * The same searches with the time of a candidate given by `cost` instead of a
 * GPU measurement: host only, no device is touched (candidates are checked with
 * hdc_params_check).  `device` and `build` name the cost function in the
 * database rows, in place of the device name and the build id.
 */
hdc_status hdc_tune_host(const hdc_problem* prob, int mode, const char* db, const char* device, const char* build,
                         hdc_cost_fn cost, void* ctx, hdc_params* best, double* best_ms);

/* Identity of this build of the library, as recorded in tuning databases. */
const char* hdc_build_id(void);

/*
 * Uneven batches (hdc_batch_plan) planned from a tuning database: the
 * per-bucket form of the exhaustive search of section 4.2.  The problems of a
 * batch are grouped into buckets by the next power of two of L; a database row
 *     {"key": "{\"bucket\": S, \"dtype\": \"c64\"}", "params": {"m": m}, "ms": t,
 *      "device": ..., "build": ..., "t": ...}
 * records that the problems of bucket S ran in t milliseconds with FFT size m.
 * For each bucket the fastest row of the device and build (equal times: the
 * larger m) gives the m of its problems whose output length is 2L - 1 and that
 * admit it (hdc_derive); other problems, and buckets without a row, take
 * hdc_batch_default_m.  Rows of other
 * kinds in the same file are ignored, and hdc_tune ignores these rows.
 *
 * hdc_batch_db_choose: host only (no device is touched); fills m[i] (n values,
 *   caller-owned) for the n problems of lengths L[i] and output lengths M[i]
 *   (M NULL: 2 L[i] - 1).  db NULL or a missing file: every problem takes the
 *   default.  device / build NULL: the current device's name and hdc_build_id().
 *   HDC_ERR_INVALID_ARG for n < 1, NULL L or m, L[i] < 1 or a non-complex dtype.
 * hdc_batch_db_record: appends one row (bucket a power of two, m >= 1,
 *   ms >= 0; device / build NULL as above).  HDC_ERR_INVALID_ARG for bad
 *   values or a file that cannot be opened for appending.
 * hdc_batch_plan_db: hdc_batch_plan with the m of hdc_batch_db_choose (current
 *   device and build); its errors are those two calls'.
 */
hdc_status hdc_batch_db_choose(int64_t n, const int64_t* L, const int64_t* M, hdc_dtype dtype, const char* db,
                               const char* device, const char* build, int64_t* m);
hdc_status hdc_batch_db_record(const char* db, int64_t bucket, hdc_dtype dtype, int64_t m, double ms,
                               const char* device, const char* build);
hdc_status hdc_batch_plan_db(hdc_batch_t* out, int64_t n, const int64_t* L, const int64_t* M, hdc_dtype dtype,
                             const char* db);

/*
 * Learned predictor (section 4.4; classification, section 6.3).  A checkpoint
 * file holds a multilayer perceptron (ReLU hidden layers, softmax output over
 * scale-free classes (p, D-mode): p in {1, 2, 3, 4, 6, 8, 12, 16}, D-mode 0 = all
 * residues in one pass, 1 = one residue per pass; class index 2 (p index) +
 * D-mode; with 17 outputs, class 16 is explicit padding, q = 1: m the smallest
 * power of two with m >= max(M, 2L - 1), D = 1, section 3.1).  Format (little
 * endian): the 8 bytes "HDCMLP01", int32 format version (1 or 2), int32 layer
 * count n, int32 sizes[n + 1] (sizes[0] = 12 inputs, sizes[n] = 16 or 17
 * classes), then per layer W (out x in, row-major) and b
 * (out), float32; version 2 then holds the minimum and the maximum of every
 * feature over the training rows (12 + 12 float32).
 *
 * hdc_predictor_load reads the file and copies the network to the current
 * device.  hdc_predict evaluates one feature row per axis of `prob` with the
 * HIP kernels of hdc_mlp.h on the current device (synchronously), takes the most
 * probable class per axis (ties: the lowest index) and maps it to parameters:
 * m = the smallest power of two with ceil(L/m) <= p (outer N-D axes at most
 * 2^20; doubled while q < p), D = q or 1 (explicit padding: as above, within the
 * axis limit).  confidence (may be NULL) receives
 * the winning class's probability per axis (prob->ndim values), or 0 for an
 * axis whose features leave the training range (version 2) by more than 1/16
 * (a sixteenth of an octave in the length features): the network abstains
 * there and the caller falls back to hdc_tune.
 * Features per axis (version 1): log2 of this axis's L / 16, log2 of the other
 * two axes' L / 16 (0 if absent, in axis order), one-hot axis (3), one-hot
 * ndim (3), 1 for complex128, log2 batch / 16, log2 of the element count
 * (prod L x batch) / 32.
 */
typedef struct hdc_predictor_s* hdc_predictor_t;
hdc_status hdc_predictor_load(hdc_predictor_t* out, const char* path);
hdc_status hdc_predict(hdc_predictor_t pred, const hdc_problem* prob, hdc_params* out, float* confidence);
hdc_status hdc_predictor_destroy(hdc_predictor_t pred);

#ifdef __cplusplus
}
#endif

#endif /* HDC_TUNE_H */
