/*
 * hdc -- hybrid dealiased convolution for AMD MI355X (gfx950).
 *
 * The operation (section 2.2 eqs. (3)-(4), section 2.3 eq. (5), section 3.3):
 *   given f, g of length L, compute the linear convolution
 *       h_k = sum_j f_j g_{k-j},  k = 0 .. M-1,
 *   (all 2L-1 terms and zeros beyond when M >= 2L-1; the first M terms when
 *   M < 2L-1, e.g. M = L, the backward range t < p of section 2.2),
 *   by hybrid dealiasing: choose an FFT size m, explicitly extend the inputs
 *   to p*m >= L (p = ceil(L/m), zeros never stored), implicitly pad to
 *   N = q*m >= max(M, 2L-1) (q = ceil(max(M, 2L-1)/m)), and compute the length-N transform as q
 *   "residues" r = 0..q-1, each an m-point DFT of the block sum
 *       w^(r)_s = zeta_N^{r s} sum_{t<p} zeta_q^{r t} f_{t m + s}
 *   (forward, eq. (3), zeta_n = exp(+2 pi i / n), unscaled).  The product
 *   H = F.G is taken residue by residue and the backward, eq. (4),
 *       h_{t m + s} = (1/N) sum_r zeta_q^{-t r} zeta_N^{-s r} sum_l zeta_m^{-s l} H_{q l + r}
 *   is accumulated over output blocks t < ceil(M/m).  Residues are taken D
 *   at a time (section 2.5); C copies are transformed together.
 *
 * Conventions for every entry point:
 *   - all sizes are int64_t; complex data are interleaved (re, im) pairs of
 *     float (HDC_C64) or double (HDC_C128), i.e. torch.complex64/complex128;
 *   - data pointers (f, g, h, residue buffers, workspaces) are DEVICE
 *     pointers owned by the caller; the plan owns only its twiddle tables;
 *   - a 1D problem with C copies stores element j of copy c at j*C + c;
 *     N-D arrays are row-major with the last axis contiguous;
 *   - h must not alias f or g; f == g (autoconvolution) is allowed;
 *   - calls enqueue work on `stream` and never synchronise; errors in
 *     arguments are reported before any launch, asynchronous device faults
 *     surface at the caller's next synchronisation;
 *   - on failure a status other than HDC_OK is returned and
 *     hdc_last_error() describes it (thread-local string).
 *   - a plan is immutable after creation and may be used concurrently on
 *     different streams with different workspaces.
 */
#ifndef HDC_H
#define HDC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Data types: complex64 / complex128 (interleaved re, im), and real float32 /
 * float64 (the real case of section 7: 1D plans, see hdc_plan, and N-D plans,
 * see hdc_plan_nd). */
typedef enum { HDC_C64 = 0, HDC_C128 = 1, HDC_R32 = 2, HDC_R64 = 3 } hdc_dtype;

typedef enum {
    HDC_OK = 0,
    HDC_ERR_INVALID_ARG = 1, /* inadmissible parameters or null pointers */
    HDC_ERR_UNSUPPORTED = 2, /* admissible but outside what the kernels implement */
    HDC_ERR_WORKSPACE = 3,   /* workspace missing or too small */
    HDC_ERR_HIP = 4          /* a HIP runtime call failed */
} hdc_status;

typedef struct hdc_plan_s* hdc_plan_t;
typedef struct hdc_batch_s* hdc_batch_t;

/* Derived description of one axis of a plan (filled by hdc_derive / hdc_plan_axis). */
typedef struct {
    int64_t L, M;     /* input length, output length                         */
    int64_t m, p, q;  /* FFT size, explicit blocks ceil(L/m), residues ceil(M/m) */
    int64_t N;        /* transform length q*m                                 */
    int64_t D;        /* residues per pass (clamped to 1..q)                  */
    int64_t C;        /* copies                                               */
    int64_t q_out;    /* output blocks ceil(M/m)                              */
    int64_t m1, m2;   /* m = m1*m2: column-stage and row-stage FFT lengths    */
    int32_t variant;  /* 0 = fused single kernel, 1 = column/row/column passes,
                         2 = raw residue rows + output sums (one-row residues),
                         3 = whole-row convolution (innermost N-D axis)       */
    int32_t reserved;
} hdc_axis_desc;

/*
 * Admissibility and derivation, host only (no device is touched).
 * Section 2.5 defines p = ceil(L/m), q = ceil(M/m) as the smallest values with
 * p m >= L and q m >= M; section 2.2 requires q >= p.  Admissible means
 * m >= 1, L >= 1, M >= 1, p m >= L, q m >= max(M, 2L-1) (else the outputs
 * alias), q >= p, C >= 1, 1 <= D.  p or q = 0 derives the ceiling (q from
 * max(M, 2L-1)); M below 2L-1 writes the first M outputs only; D = 0
 * means D = q; D > q is clamped to q.  Returns HDC_ERR_INVALID_ARG for
 * inadmissible input and HDC_ERR_UNSUPPORTED when m > 2^22, when the
 * transform does not fit the kernels' index range, or when m is not a power of
 * two and either its odd factor R (m = R 2^k) has a prime factor above 7 or
 * exceeds 63, or the residues do not fit the fused kernel (m <= 4096 and
 * q m b 9/8 <= 80 KiB): such m (section 3.1's FFT-friendly sizes) run on the
 * mixed-radix fused kernel only, in 1D complex plans and batches.
 */
hdc_status hdc_derive(int64_t L, int64_t M, int64_t m, int64_t p, int64_t q, int64_t C, int64_t D,
                      hdc_dtype dtype, hdc_axis_desc* out);

/* 1D plan (eqs. (3)-(4)).  Allocates the device twiddle tables on the current device
 * (the only allocation a plan makes).  Errors as hdc_derive, plus HDC_ERR_HIP.
 *
 * Real data (dtype HDC_R32 or HDC_R64; the real case that section 7 names as
 * future work): f, g and h are real arrays of float or double, L x C and M x C
 * values with element j of copy c at j*C + c, and the plan computes in
 * complex64 / complex128.  The two inputs are transformed together as
 * z = f + i g (one forward transform instead of two): with k = q l + r,
 *     F_k = (Z_k + conj Z_{N-k}) / 2,  G_k = (Z_k - conj Z_{N-k}) / (2i),
 * and N - k lies in residue q - r.  The product H is Hermitian, so only the
 * residues r <= q/2 are multiplied and inverted, D of them per pass (D is
 * clamped to q/2 + 1), and h is the real part of their sum weighted 2 (1 for
 * r = 0 and r = q/2).  Such a plan supports hdc_convolve, hdc_time_convolve
 * and hdc_convolve_profiled; the residue-level calls (hdc_forward,
 * hdc_multiply, hdc_backward, hdc_residues_natural, hdc_residue_buffer_size)
 * return HDC_ERR_UNSUPPORTED for it, as do hdc_plan_uneq* and hdc_batch_plan
 * given a real dtype.  Pointers need 4-byte (HDC_R32) or 8-byte (HDC_R64)
 * alignment. */
hdc_status hdc_plan(hdc_plan_t* out, int64_t L, int64_t M, int64_t m, int64_t p, int64_t q, int64_t C,
                    int64_t D, hdc_dtype dtype);

/* N-D plan, ndim = 1..3 (section 3.6): per-axis L, M, m, p, q, D (p, q, D may
 * be 0 to derive).  The outer axes are transformed as strided column passes
 * whose copies are the inner extents (section 2.5's C copies; outer m up to
 * 2^20, split into two column stages when above 1024); the innermost axis is a
 * 1D hybrid convolution per outer-residue row.
 *
 * Real data (HDC_R32 / HDC_R64, ndim 2 or 3; the real case of section 7): f, g
 * and h are real boxes.  Because the convolution is bilinear,
 *     z * z = f * f - s^2 g * g + 2 i s f * g   for z = f + i s g,
 * so h = Im(z * z) / (2 s): one complex autoconvolution (one forward transform
 * per axis instead of two) of z.  s = max|f| / max|g| (1 if
 * either is 0) keeps the two terms at one scale, so the rounding error relative
 * to |f| |g| stays that of a complex plan (with g = 0, h is rounding noise at
 * the scale of f * f rather than exact zeros).  z is never stored: the outer
 * axis's forward column pass reads f and s g as z, and its backward pass
 * writes h; the workspace is the complex plan's plus 256 bytes.  ndim = 1 returns
 * HDC_ERR_UNSUPPORTED (hdc_plan's Hermitian pairing serves 1D real data). */
hdc_status hdc_plan_nd(hdc_plan_t* out, int ndim, const int64_t* L, const int64_t* M, const int64_t* m,
                       const int64_t* p, const int64_t* q, const int64_t* D, hdc_dtype dtype);

/* Host-only check of an N-D plan (no device memory is touched): the
 * admissibility of every axis and the kernel geometry (LDS needs against the
 * device's, or gfx950's 160 KiB when no device is visible).  Fills
 * out[0 .. ndim-1] when out is non-NULL. */
hdc_status hdc_plan_nd_check(int ndim, const int64_t* L, const int64_t* M, const int64_t* m, const int64_t* p,
                             const int64_t* q, const int64_t* D, hdc_dtype dtype, hdc_axis_desc* out);

/*
 * Unequal operand lengths (section 3.5): h = f * g for f of length Lf and g of
 * length Lg, k = 0 .. M-1 (M >= 1; the transforms cover max(M, Lf + Lg - 1)
 * points, so M < Lf + Lg - 1 writes the first M outputs), C copies.  Roles follow the
 * lengths: the shorter operand is cut into m-point residues and the longer
 * into Lambda m-point residues,
 *     p_f = ceil(Ls/m), p_g = ceil(Ll/(Lambda m)), q_g = ceil(M/(Lambda m)), q_f = Lambda q_g,
 * both of transform length N = q_g Lambda m.  Residue r_g of the longer operand
 * meets, at its point l_g, point floor(l_g/Lambda) of the shorter operand's
 * residue r_f = q_g (l_g mod Lambda) + r_g; the product and the backward run in
 * the longer operand's geometry, D residues of it per pass.
 * m = 0 derives m (and Lambda if 0) so that both operands fit one block
 * (p_f = p_g = 1) within the limits below; Lambda = 0 with m > 0 derives Lambda
 * the same way.  Admissible: Lf, Lg, C, M >= 1, D >= 0.
 * HDC_ERR_UNSUPPORTED unless m and Lambda are powers of two with
 * Lambda <= 1024 and Lambda m <= 2^22.
 *
 * hdc_uneq_derive is host-only: it fills the shorter operand's description
 * (m, p_f, q_f, its four-step split) and the longer one's (Lambda m, p_g, q_g,
 * D, q_out), and *swapped = 1 when Lf > Lg (then g plays the shorter role).
 * Any output pointer may be NULL.
 */
hdc_status hdc_uneq_derive(int64_t Lf, int64_t Lg, int64_t M, int64_t m, int64_t Lambda, int64_t C, int64_t D,
                           hdc_dtype dtype, hdc_axis_desc* short_out, hdc_axis_desc* long_out, int* swapped);

/* Plan of the unequal-length convolution above (allocates its twiddle tables).
 * hdc_convolve(plan, f, g, h, ws, s) then reads Lf x C values of f and
 * Lg x C of g.  hdc_plan_axis reports ndim = 1, axis 0 the longer operand's
 * description and axis 1 the shorter one's.  hdc_forward is rejected for such
 * a plan (use hdc_forward_operand); hdc_multiply, hdc_backward,
 * hdc_residues_natural and hdc_residue_buffer_size use the longer operand's
 * geometry. */
hdc_status hdc_plan_uneq(hdc_plan_t* out, int64_t Lf, int64_t Lg, int64_t M, int64_t m, int64_t Lambda, int64_t C,
                         int64_t D, hdc_dtype dtype);

/*
 * Unequal extents in 2D/3D (section 3.6 with section 3.5's lengths): f of
 * extents Lf[0..ndim), g of extents Lg[0..ndim), both row-major with the last
 * axis contiguous, output box M[a] >= 1 (the first M[a] of the Lf[a] + Lg[a] - 1
 * terms, zeros beyond).  Every axis follows
 * the 1D rules above on its own, the roles too (f may be the shorter operand
 * on one axis and the longer on another); m, Lambda and D may be NULL or hold
 * 0 to derive.  Outer axes are column passes over the inner extents: there
 * Lambda m <= 2^20, split into a first column stage of min(Lambda m, 1024)
 * points and a second strided one.  The innermost axis is a batched 1D
 * unequal convolution per row pair (the fused kernel when Lambda = 1 and it
 * fits a workgroup's LDS).
 *
 * hdc_uneq_nd_check is host-only and fills, per axis, the shorter operand's
 * description, the longer one's and whether f is the longer one (any output
 * array may be NULL).  hdc_plan_axis on such a plan: axis a < ndim gives the
 * longer operand's description, axis ndim + a the shorter one's.
 * hdc_convolve(plan, f, g, h, ws, s) reads prod(Lf) and prod(Lg) values.
 */
hdc_status hdc_uneq_nd_check(int ndim, const int64_t* Lf, const int64_t* Lg, const int64_t* M, const int64_t* m,
                             const int64_t* Lambda, const int64_t* D, hdc_dtype dtype, hdc_axis_desc* short_out,
                             hdc_axis_desc* long_out, int* swapped);
hdc_status hdc_plan_uneq_nd(hdc_plan_t* out, int ndim, const int64_t* Lf, const int64_t* Lg, const int64_t* M,
                            const int64_t* m, const int64_t* Lambda, const int64_t* D, hdc_dtype dtype);

/*
 * Multi-convolution (section 6.1, the convolution applied to N arrays rather
 * than two): h = x_0 * x_1 * ... * x_{A-1} for A = 2 .. 8 sequences of length L,
 *     h_k = sum over j_0 + ... + j_{A-1} = k of prod_a x_a[j_a],  k = 0 .. M-1,
 * C copies (element j of copy c at j*C + c).  The linear result has A(L-1)+1
 * terms, so the transform length N = q m must reach max(M, A(L-1)+1) (q = 0
 * derives it; M below A(L-1)+1 writes the first M terms).  Every residue of
 * every operand is formed as in eq. (3), the A residues multiply pointwise and
 * one backward, eq. (4), accumulates h.  Other arguments and errors as
 * hdc_plan; complex types only (HDC_ERR_UNSUPPORTED for real ones).
 * hdc_convolve_multi(plan, x, h, ws, stream): x is a HOST array of plan's A
 * DEVICE pointers (A = 2 for a plan of hdc_plan or hdc_plan_nd), each of L x C
 * values (the operand box for N-D plans); h must
 * not alias any operand; ws as hdc_workspace_size.  hdc_convolve refuses a
 * plan of more than two operands.  The residue-level calls work on such a plan
 * operand by operand: hdc_forward of each, hdc_multiply of the first buffer by
 * every other, hdc_backward of the product.
 */
hdc_status hdc_plan_multi(hdc_plan_t* out, int A, int64_t L, int64_t M, int64_t m, int64_t p, int64_t q, int64_t C,
                          int64_t D, hdc_dtype dtype);
hdc_status hdc_convolve_multi(hdc_plan_t plan, const void* const* x, void* h, void* ws, hipStream_t stream);

/*
 * Multi-convolution of A = 2 .. 8 arrays in 2 or 3 dimensions (section 6.1's
 * 1D/2D multi-convolution, applied axis by axis as section 3.6 does for two
 * operands): every operand an L[0] x .. x L[ndim-1] row-major box, h the
 * M[0] x .. box of the first M[a] terms per axis of the A-fold linear result
 * (M == NULL: all A(L[a]-1)+1 terms).  Per axis m[a] (a power of two, at
 * most 2^20 on outer axes, 2^22 on the innermost) and D[a] (NULL or 0: all
 * residues per pass) as hdc_plan_nd; q[a] is derived from max(M[a],
 * A(L[a]-1)+1).  Outer axes run the column passes on each operand; the
 * innermost axis the multi-operand rows.  Convolve with hdc_convolve_multi;
 * the residue-level calls are 1D only.  Errors as hdc_plan_nd and
 * hdc_plan_multi.
 */
hdc_status hdc_plan_multi_nd(hdc_plan_t* out, int A, int ndim, const int64_t* L, const int64_t* M, const int64_t* m,
                             const int64_t* D, hdc_dtype dtype);

/* Frees the plan and its device twiddle tables (hipFree: synchronises with the
 * device).  No call that uses the plan may still be in flight.  NULL is a no-op. */
hdc_status hdc_plan_destroy(hdc_plan_t plan);

/* Number of axes and the description of axis `axis`. */
hdc_status hdc_plan_axis(hdc_plan_t plan, int axis, int* ndim, hdc_axis_desc* out);

/* Bytes of device workspace that hdc_convolve (and hdc_forward/backward) need;
 * the caller allocates it (256-byte alignment).  May be 0. */
hdc_status hdc_workspace_size(hdc_plan_t plan, size_t* bytes);

/* Bytes of one residue buffer (D residues x m x C complex values), 1D plans. */
hdc_status hdc_residue_buffer_size(hdc_plan_t plan, size_t* bytes);

/*
 * Full convolution: h[0 .. M) (x C copies, or the N-D output box) from f, g
 * (L values each).  All residue groups, the products and the backward
 * accumulation run on `stream`.  f == g allowed; h must not alias f or g.
 */
hdc_status hdc_convolve(hdc_plan_t plan, const void* f, const void* g, void* h, void* ws, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * work as hdc_convolve(plan, f, g, h, ws, stream), with the workspace taken
 * from a library-owned device array of HDC_SCRATCH_BYTES bytes per GPU instead
 * of a caller buffer.  The array is set up on a device by the first call made
 * with that device current (one symbol-address lookup, no allocation) and
 * stays until the process ends.  The call itself allocates nothing: no
 * hipMalloc, hipFree or allocating library routine.  Every call on a GPU
 * shares that GPU's array, which keeps the last call's contents; calls that
 * overlap on one GPU (different streams, threads, or a captured graph replayed
 * while another call runs) race on it and must be serialised by the caller.
 * HDC_ERR_WORKSPACE when hdc_workspace_size(plan) exceeds HDC_SCRATCH_BYTES;
 * other errors as hdc_convolve.  Multi-operand plans take hdc_convolve_multi.
 */
#define HDC_SCRATCH_BYTES ((size_t)64 << 20)
hdc_status hdc_convolve_noalloc(hdc_plan_t plan, const void* f, const void* g, void* h, hipStream_t stream);

/*
 * Forward residues [r0, r0 + D') of a 1D plan, D' = min(D, q - r0): the m-point
 * DFTs of eq. (3).  F holds D' x m x C values; within a residue the order is
 * implementation-defined (hdc_residues_natural gives the natural order).
 * r0 must be a multiple of D.  ws: hdc_workspace_size bytes.  The separate
 * stages (hdc_forward, hdc_forward_operand, hdc_multiply, hdc_backward,
 * hdc_residues_natural) take power-of-two m: HDC_ERR_UNSUPPORTED otherwise
 * (a plan with m = R 2^k, R > 1, convolves with hdc_convolve only).
 */
hdc_status hdc_forward(hdc_plan_t plan, const void* f, void* F, int64_t r0, void* ws, hipStream_t stream);

/*
 * hdc_forward for one operand: operand 0 is f, 1 is g.  For an equal-length
 * plan it is hdc_forward.  For an unequal-length plan it fills the residue
 * buffer of group [r0, r0 + D') of the longer operand's geometry (D' x Lambda m
 * x C values): for the longer operand its Lambda m-point residues; for the
 * shorter one the matching values of its m-point residues (section 3.5),
 * which sit at the same indices k = q_g l_g + r of the length-N transform, so
 * hdc_multiply pairs them point by point.
 */
hdc_status hdc_forward_operand(hdc_plan_t plan, int operand, const void* x, void* F, int64_t r0, void* ws,
                               hipStream_t stream);

/* Pointwise product of two residue buffers of the same group: F <- F . G. */
hdc_status hdc_multiply(hdc_plan_t plan, void* F, const void* G, int64_t r0, hipStream_t stream);

/*
 * Backward, eq. (4), for residues [r0, r0 + D'): inverse m-point DFTs,
 * twiddle, and accumulation into the output blocks t < ceil(M/m) of h.
 * r0 == 0 overwrites h; r0 > 0 adds to it, so calling r0 = 0, D, 2D, ... in
 * order on one stream yields the convolution.  F is overwritten.
 */
hdc_status hdc_backward(hdc_plan_t plan, void* F, void* h, int64_t r0, void* ws, hipStream_t stream);

/* Debug view: copy residues [r0, r0 + D') of F into `out` in the natural order,
 * out[(d*m + l)*C + c] = F_{q l + r0 + d} of copy c (= the length-N zero-extended
 * DFT of f at index k = q l + r).  `out` (D' m C values) must not alias F;
 * HDC_ERR_INVALID_ARG for r0 outside the plan's groups or misaligned pointers. */
hdc_status hdc_residues_natural(hdc_plan_t plan, const void* F, int64_t r0, void* out, hipStream_t stream);

/*
 * Batched uneven 1D convolutions (n independent problems of lengths L[i], output
 * lengths M[i], M == NULL means 2 L[i] - 1).  Operands are packed back to back:
 * f and g at offsets sum_{j<i} L[j], h at sum_{j<i} M[j].  Problems are grouped
 * into buckets that share (m, p, q, D); `bucket_m` (length n, may be NULL) gives
 * the FFT size chosen for each problem, 0 meaning the built-in default
 * (hdc_batch_default_m).  The buckets that fit the fused kernel (m <= 4096
 * for HDC_C64, m <= 512 for HDC_C128) are served by one persistent launch
 * whose workgroups take (bucket, block of problems) items from a queue with
 * an integer atomic counter.  Buckets whose residue transform is a single row
 * (m <= 4096) and does not fit the fused kernel, with p <= 4 and q <= 32, are
 * served together, per m, by one launch of residue rows formed from the raw
 * inputs and one launch of the output sums.  Other buckets run their own
 * launches.
 * The first hdc_batch_convolve captures the launches in a HIP graph on a private
 * stream of the batch; later calls with the same buffers replay it.  Every
 * call is ordered after the work already on `stream`, and work enqueued on
 * `stream` afterwards runs after it.  Inside the graph the buckets run on up to
 * four concurrent lanes (dealt longest first onto the least-loaded lane; the
 * buckets of one lane run in turn), each lane with its own region of `ws`, so
 * the workspace is the sum over lanes of the largest bucket need of each.
 * Results do not depend on the lanes: every problem is computed by the same
 * launches as in hdc_batch_convolve_eager, which runs the buckets in turn on
 * `stream`.  Calls on one batch must not overlap (they share its graph).
 */
hdc_status hdc_batch_plan(hdc_batch_t* out, int64_t n, const int64_t* L, const int64_t* M, const int64_t* bucket_m,
                          hdc_dtype dtype);
/* The FFT size hdc_batch_plan gives a problem of length L by default (host
 * only): the smallest power of two >= L, except 4096 (p = 2) for lengths in
 * (4096, 8192]. */
hdc_status hdc_batch_default_m(int64_t L, int64_t* m);
hdc_status hdc_batch_workspace_size(hdc_batch_t batch, size_t* bytes);
hdc_status hdc_batch_convolve(hdc_batch_t batch, const void* f, const void* g, void* h, void* ws,
                              hipStream_t stream);
/* Same work as hdc_batch_convolve, launched directly without a graph: the call to
 * use inside a caller's stream capture (hdc_batch_convolve returns
 * HDC_ERR_INVALID_ARG on a capturing stream, since it captures a graph of its own). */
hdc_status hdc_batch_convolve_eager(hdc_batch_t batch, const void* f, const void* g, void* h, void* ws,
                                   hipStream_t stream);
hdc_status hdc_batch_info(hdc_batch_t batch, int64_t* n_buckets, int64_t* total_L, int64_t* total_M);
hdc_status hdc_batch_destroy(hdc_batch_t batch);

/*
 * Timing core for the autotuner (sections 4.2-4.3): runs hdc_convolve
 * `warmup` times, then `reps` times each bracketed by HIP events on `stream`,
 * and writes the per-repetition milliseconds to ms_out[reps].  Synchronises
 * the stream.
 */
hdc_status hdc_time_convolve(hdc_plan_t plan, const void* f, const void* g, void* h, void* ws, hipStream_t stream,
                             int warmup, int reps, float* ms_out);

/*
 * Instrumented hdc_convolve: the same launches, each bracketed by HIP events on
 * `stream`; synchronises the stream.  For launch i < min(*n_launches,
 * max_launches): kinds[i] (0 fused, 1 forward column, 2 row, 3 backward
 * column, 4 raw residue rows, 5 output sums, 6 whole-row convolution, 7 the
 * maxima of real N-D inputs), ms[i] (event-measured duration) and bytes[i] (the launch's
 * algorithmic HBM bytes: compulsory reads plus writes).  Any output array may
 * be NULL.  *n_launches receives the total number of launches.
 */
hdc_status hdc_convolve_profiled(hdc_plan_t plan, const void* f, const void* g, void* h, void* ws, hipStream_t stream,
                                 int max_launches, int* n_launches, int32_t* kinds, float* ms, double* bytes);

/*
 * Per-launch timing over a region of the caller's choosing: after
 * hdc_profile_begin(filter), every kernel launched on this thread by
 * hdc_convolve of plan `filter` (of any plan if filter is NULL) is bracketed
 * by HIP events on its stream.  hdc_profile_end synchronises the device and
 * reports the launches as hdc_convolve_profiled does.
 */
hdc_status hdc_profile_begin(hdc_plan_t filter);
hdc_status hdc_profile_end(int max_launches, int* n_launches, int32_t* kinds, float* ms, double* bytes);

/* Thread-local description of the last error (never NULL). */
const char* hdc_last_error(void);

/* Library version string. */
const char* hdc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HDC_H */
