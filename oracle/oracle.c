/*
 * CPU FP64 oracle for the linear convolution computed by hybrid dealiasing.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the GPU library.
 *
 * What it computes (the method reaches this result exactly, up to rounding):
 *   the linear convolution of two length-L sequences, eq. (5) of section 2.3,
 *       h_k = sum_{j} f_j g_{k-j},   0 <= j < L, 0 <= k-j < L,
 *   reported over the output length M (M >= 2L-1); entries k >= 2L-1 are 0.
 *   Unequal lengths (section 3.5): f of length Lf, g of length Lg, the same sum
 *   with 0 <= j < Lf, 0 <= k-j < Lg, over M >= Lf + Lg - 1.
 *   N-D: the same sum per axis over the box [0, M_1) x ... x [0, M_d).
 *
 * Two independent routes, deliberately plain:
 *   1. direct summation of eq. (5)                           (O(L^2));
 *   2. explicit dealiasing (section 3.1): zero-pad both operands to the
 *      smallest size 2^a 3^b 5^c 7^d >= 2L-1, forward DFT (zeta = e^{+2 pi i/n}),
 *      pointwise product, backward DFT with 1/n, crop.
 * The DFT is a recursive decimation-in-time transform that splits off the
 * smallest prime factor and recombines the sub-transforms by direct sums
 * (section 2.2 generalised from radix 2 to any prime); every twiddle is
 * cos/sin of 2*pi*e/n with the exponent e reduced mod n in integer arithmetic.
 *
 * Complex arrays are interleaved (re, im) doubles.  1D arrays with C copies
 * place element j of copy c at j*C + c.  N-D arrays are row-major with the
 * last axis contiguous.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cd;

static inline cd cmul(cd a, cd b) { cd r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cd cadd(cd a, cd b) { cd r = {a.re + b.re, a.im + b.im}; return r; }

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- direct -- */

/* eq. (5) for operands of lengths Lf and Lg (f_j = 0 for j >= Lf, g_j = 0 for
 * j >= Lg, the unequal case of section 3.5), all copies, all k < M. */
int oracle_direct_1d_uneq(int64_t Lf, int64_t Lg, int64_t M, int64_t C, const double* f_, const double* g_,
                          double* h_) {
    if (Lf < 0 || Lg < 0 || M < 0 || C < 1) return 1;
    const cd* f = (const cd*)f_;
    const cd* g = (const cd*)g_;
    cd* h = (cd*)h_;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < M; ++k) {
        for (int64_t c = 0; c < C; ++c) {
            cd acc = {0.0, 0.0};
            int64_t jlo = k - (Lg - 1) > 0 ? k - (Lg - 1) : 0;
            int64_t jhi = k < Lf - 1 ? k : Lf - 1;
            for (int64_t j = jlo; j <= jhi; ++j) acc = cadd(acc, cmul(f[j * C + c], g[(k - j) * C + c]));
            h[k * C + c] = acc;
        }
    }
    return 0;
}

/* eq. (5) for real sequences (the real case the paper leaves to future work,
 * section 7): real arithmetic throughout, all copies, all k < M. */
int oracle_direct_1d_real(int64_t L, int64_t M, int64_t C, const double* f, const double* g, double* h) {
    if (L < 0 || M < 0 || C < 1) return 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < M; ++k) {
        for (int64_t c = 0; c < C; ++c) {
            double acc = 0.0;
            int64_t jlo = k - (L - 1) > 0 ? k - (L - 1) : 0;
            int64_t jhi = k < L - 1 ? k : L - 1;
            for (int64_t j = jlo; j <= jhi; ++j) acc += f[j * C + c] * g[(k - j) * C + c];
            h[k * C + c] = acc;
        }
    }
    return 0;
}

/* eq. (5), all copies, all k < M. */
int oracle_direct_1d(int64_t L, int64_t M, int64_t C, const double* f_, const double* g_, double* h_) {
    return oracle_direct_1d_uneq(L, L, M, C, f_, g_, h_);
}

/* eq. (5) for the listed output indices only (copy 0 .. C-1 of each), operands
 * of lengths Lf and Lg (section 3.5; Lf = Lg is the equal case). */
int oracle_direct_1d_uneq_sampled(int64_t Lf, int64_t Lg, int64_t C, const double* f_, const double* g_,
                                  const int64_t* ks, int64_t nk, double* out_) {
    if (Lf < 0 || Lg < 0 || C < 1 || nk < 0) return 1;
    const cd* f = (const cd*)f_;
    const cd* g = (const cd*)g_;
    cd* out = (cd*)out_;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nk; ++i) {
        int64_t k = ks[i];
        for (int64_t c = 0; c < C; ++c) {
            cd acc = {0.0, 0.0};
            int64_t jlo = k - (Lg - 1) > 0 ? k - (Lg - 1) : 0;
            int64_t jhi = k < Lf - 1 ? k : Lf - 1;
            for (int64_t j = jlo; j <= jhi; ++j) acc = cadd(acc, cmul(f[j * C + c], g[(k - j) * C + c]));
            out[i * C + c] = acc;
        }
    }
    return 0;
}

/* eq. (5) for the listed output indices only (copy 0 .. C-1 of each). */
int oracle_direct_1d_sampled(int64_t L, int64_t C, const double* f_, const double* g_,
                             const int64_t* ks, int64_t nk, double* out_) {
    return oracle_direct_1d_uneq_sampled(L, L, C, f_, g_, ks, nk, out_);
}

static void unravel(int ndim, const int64_t* ext, int64_t lin, int64_t* idx) {
    for (int a = ndim - 1; a >= 0; --a) { idx[a] = lin % ext[a]; lin /= ext[a]; }
}

/* N-D eq. (5) for the listed output multi-indices (given as row-major linear
 * indices into the M box), f of extents Lf and g of extents Lg (equal or not,
 * section 3.6 with the lengths of section 3.5). ndim <= 3. */
int oracle_direct_nd_uneq_sampled(int ndim, const int64_t* Lf, const int64_t* Lg, const int64_t* M, const double* f_,
                                  const double* g_, const int64_t* ks, int64_t nk, double* out_) {
    if (ndim < 1 || ndim > 3) return 1;
    const cd* f = (const cd*)f_;
    const cd* g = (const cd*)g_;
    cd* out = (cd*)out_;
    int64_t F3[3] = {1, 1, 1}, G3[3] = {1, 1, 1};
    for (int a = 0; a < ndim; ++a) {
        F3[3 - ndim + a] = Lf[a];
        G3[3 - ndim + a] = Lg[a];
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nk; ++i) {
        int64_t k[3] = {0, 0, 0}, kk[3];
        unravel(ndim, M, ks[i], kk);
        for (int a = 0; a < ndim; ++a) k[3 - ndim + a] = kk[a];
        cd acc = {0.0, 0.0};
        for (int64_t j0 = 0; j0 < F3[0]; ++j0) {
            int64_t d0 = k[0] - j0;
            if (d0 < 0 || d0 >= G3[0]) continue;
            for (int64_t j1 = 0; j1 < F3[1]; ++j1) {
                int64_t d1 = k[1] - j1;
                if (d1 < 0 || d1 >= G3[1]) continue;
                for (int64_t j2 = 0; j2 < F3[2]; ++j2) {
                    int64_t d2 = k[2] - j2;
                    if (d2 < 0 || d2 >= G3[2]) continue;
                    int64_t a = (j0 * F3[1] + j1) * F3[2] + j2;
                    int64_t b = (d0 * G3[1] + d1) * G3[2] + d2;
                    acc = cadd(acc, cmul(f[a], g[b]));
                }
            }
        }
        out[i] = acc;
    }
    return 0;
}

/* N-D eq. (5) for the listed output multi-indices, equal extents L. */
int oracle_direct_nd_sampled(int ndim, const int64_t* L, const int64_t* M, const double* f_, const double* g_,
                             const int64_t* ks, int64_t nk, double* out_) {
    return oracle_direct_nd_uneq_sampled(ndim, L, L, M, f_, g_, ks, nk, out_);
}

/* ------------------------------------------------------------------- DFT -- */

/* Smallest n' >= n of the form 2^a 3^b 5^c 7^d (section 3.1's FFT-friendly sizes,
 * without the factor 11). */
int64_t oracle_friendly_size(int64_t n) {
    if (n <= 1) return 1;
    for (int64_t c = n;; ++c) {
        int64_t r = c;
        const int64_t pr[4] = {2, 3, 5, 7};
        for (int i = 0; i < 4; ++i) while (r % pr[i] == 0) r /= pr[i];
        if (r == 1) return c;
    }
}

static int64_t smallest_prime_factor(int64_t n) {
    if (n % 2 == 0) return 2;
    for (int64_t d = 3; d * d <= n; d += 2) if (n % d == 0) return d;
    return n;
}

/* table[e] = zeta_n^{e} = exp(sign * 2 pi i e / n), e < n. */
static cd* root_table(int64_t n, int sign) {
    cd* t = (cd*)malloc(sizeof(cd) * (size_t)(n > 0 ? n : 1));
    for (int64_t e = 0; e < n; ++e) {
        double a = 2.0 * M_PI * (double)e / (double)n;
        t[e].re = cos(a);
        t[e].im = (double)sign * sin(a);
    }
    return t;
}

/* out[k] = sum_j zeta_n^{k j} in[j*stride], recursive DIT.  `root` is the
 * table of zeta_ntop^e for the top-level size ntop; zeta_n = zeta_ntop^{ntop/n}. */
static void dft_rec(const cd* in, int64_t stride, int64_t n, cd* out, const cd* root, int64_t ntop, cd* scratch) {
    if (n == 1) { out[0] = in[0]; return; }
    int64_t R = smallest_prime_factor(n);
    int64_t s = n / R;
    /* sub-transform i: the samples j = i + R*u, u < s */
    for (int64_t i = 0; i < R; ++i) dft_rec(in + i * stride, stride * R, s, scratch + i * s, root, ntop, out);
    int64_t scale = ntop / n;
    for (int64_t a = 0; a < R; ++a) {
        for (int64_t k = 0; k < s; ++k) {
            int64_t kk = k + a * s; /* output index */
            cd acc = {0.0, 0.0};
            for (int64_t i = 0; i < R; ++i) {
                int64_t e = (i * kk) % n; /* zeta_n^{i kk} */
                acc = cadd(acc, cmul(root[e * scale], scratch[i * s + k]));
            }
            out[kk] = acc;
        }
    }
}

/* In-place DFT of x (n complex values): X_k = sum_j exp(sign 2 pi i k j / n) x_j, unscaled. */
int oracle_dft(int64_t n, double* x_, int sign) {
    if (n < 1 || (sign != 1 && sign != -1)) return 1;
    cd* x = (cd*)x_;
    cd* root = root_table(n, sign);
    cd* out = (cd*)malloc(sizeof(cd) * (size_t)n);
    cd* scr = (cd*)malloc(sizeof(cd) * (size_t)n);
    /* dft_rec alternates `out` and `scratch` roles level by level; give it two
     * buffers of size n each: the recursion writes level results into the
     * buffer it is handed and uses the other one for its children. */
    dft_rec(x, 1, n, out, root, n, scr);
    memcpy(x, out, sizeof(cd) * (size_t)n);
    free(root); free(out); free(scr);
    return 0;
}

/* -------------------------------------------------------- explicit padding -- */

/* Explicitly zero-padded FFT convolution of lengths Lf and Lg, 1D with C copies
 * (section 3.1; padding to the smallest friendly size >= Lf + Lg - 1). */
int oracle_padded_1d_uneq(int64_t Lf, int64_t Lg, int64_t M, int64_t C, const double* f_, const double* g_,
                          double* h_) {
    if (Lf < 1 || Lg < 1 || M < 1 || C < 1) return 1;
    const cd* f = (const cd*)f_;
    const cd* g = (const cd*)g_;
    cd* h = (cd*)h_;
    int64_t Ne = oracle_friendly_size(Lf + Lg - 1);
    int64_t Kmax = Lf + Lg - 1 < M ? Lf + Lg - 1 : M;
    cd* rp = root_table(Ne, +1);
    cd* rm = root_table(Ne, -1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        cd* a = (cd*)calloc((size_t)Ne, sizeof(cd));
        cd* b = (cd*)calloc((size_t)Ne, sizeof(cd));
        cd* o = (cd*)malloc(sizeof(cd) * (size_t)Ne);
        cd* s = (cd*)malloc(sizeof(cd) * (size_t)Ne);
        for (int64_t j = 0; j < Lf; ++j) a[j] = f[j * C + c];
        for (int64_t j = 0; j < Lg; ++j) b[j] = g[j * C + c];
        dft_rec(a, 1, Ne, o, rp, Ne, s); memcpy(a, o, sizeof(cd) * (size_t)Ne);
        dft_rec(b, 1, Ne, o, rp, Ne, s); memcpy(b, o, sizeof(cd) * (size_t)Ne);
        for (int64_t k = 0; k < Ne; ++k) a[k] = cmul(a[k], b[k]);
        dft_rec(a, 1, Ne, o, rm, Ne, s);
        for (int64_t k = 0; k < M; ++k) {
            cd v = {0.0, 0.0};
            if (k < Kmax) { v.re = o[k].re / (double)Ne; v.im = o[k].im / (double)Ne; }
            h[k * C + c] = v;
        }
        free(a); free(b); free(o); free(s);
    }
    free(rp); free(rm);
    return 0;
}

/* Explicitly zero-padded FFT convolution, 1D with C copies (section 3.1). */
int oracle_padded_1d(int64_t L, int64_t M, int64_t C, const double* f_, const double* g_, double* h_) {
    return oracle_padded_1d_uneq(L, L, M, C, f_, g_, h_);
}

/* DFT along one axis of a row-major array with extents ext[0..nd-1]. */
static void dft_axis(cd* x, int nd, const int64_t* ext, int axis, int sign) {
    int64_t n = ext[axis];
    int64_t inner = 1, outer = 1;
    for (int a = axis + 1; a < nd; ++a) inner *= ext[a];
    for (int a = 0; a < axis; ++a) outer *= ext[a];
    cd* root = root_table(n, sign);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t o = 0; o < outer; ++o) {
        for (int64_t i = 0; i < inner; ++i) {
            cd* line = (cd*)malloc(sizeof(cd) * (size_t)n);
            cd* res = (cd*)malloc(sizeof(cd) * (size_t)n);
            cd* scr = (cd*)malloc(sizeof(cd) * (size_t)n);
            cd* base = x + o * n * inner + i;
            for (int64_t j = 0; j < n; ++j) line[j] = base[j * inner];
            dft_rec(line, 1, n, res, root, n, scr);
            for (int64_t j = 0; j < n; ++j) base[j * inner] = res[j];
            free(line); free(res); free(scr);
        }
    }
    free(root);
}

/* Explicitly zero-padded FFT convolution in 1..3 dimensions (per-axis padding
 * to the smallest friendly size >= 2 L_a - 1). */
int oracle_padded_nd_uneq(int ndim, const int64_t* Lf, const int64_t* Lg, const int64_t* M, const double* f_,
                          const double* g_, double* h_) {
    if (ndim < 1 || ndim > 3) return 1;
    const cd* f = (const cd*)f_;
    const cd* g = (const cd*)g_;
    cd* h = (cd*)h_;
    int64_t Ne[3], K[3], tot = 1, totF = 1, totG = 1, totM = 1;
    for (int a = 0; a < ndim; ++a) {
        if (Lf[a] < 1 || Lg[a] < 1 || M[a] < 1) return 1;
        K[a] = Lf[a] + Lg[a] - 1;
        Ne[a] = oracle_friendly_size(K[a]);
        tot *= Ne[a]; totF *= Lf[a]; totG *= Lg[a]; totM *= M[a];
    }
    cd* A = (cd*)calloc((size_t)tot, sizeof(cd));
    cd* B = (cd*)calloc((size_t)tot, sizeof(cd));
    int64_t idx[3];
    for (int64_t lin = 0; lin < totF; ++lin) {
        unravel(ndim, Lf, lin, idx);
        int64_t p = 0;
        for (int a = 0; a < ndim; ++a) p = p * Ne[a] + idx[a];
        A[p] = f[lin];
    }
    for (int64_t lin = 0; lin < totG; ++lin) {
        unravel(ndim, Lg, lin, idx);
        int64_t p = 0;
        for (int a = 0; a < ndim; ++a) p = p * Ne[a] + idx[a];
        B[p] = g[lin];
    }
    for (int a = 0; a < ndim; ++a) { dft_axis(A, ndim, Ne, a, +1); dft_axis(B, ndim, Ne, a, +1); }
    for (int64_t i = 0; i < tot; ++i) A[i] = cmul(A[i], B[i]);
    for (int a = 0; a < ndim; ++a) dft_axis(A, ndim, Ne, a, -1);
    for (int64_t lin = 0; lin < totM; ++lin) {
        unravel(ndim, M, lin, idx);
        int inside = 1;
        int64_t p = 0;
        for (int a = 0; a < ndim; ++a) {
            if (idx[a] >= K[a]) inside = 0;
            p = p * Ne[a] + (inside ? idx[a] : 0);
        }
        cd v = {0.0, 0.0};
        if (inside) { v.re = A[p].re / (double)tot; v.im = A[p].im / (double)tot; }
        h[lin] = v;
    }
    free(A); free(B);
    return 0;
}

/* Explicitly zero-padded FFT convolution in 1..3 dimensions, equal extents L. */
int oracle_padded_nd(int ndim, const int64_t* L, const int64_t* M, const double* f_, const double* g_, double* h_) {
    return oracle_padded_nd_uneq(ndim, L, L, M, f_, g_, h_);
}

/* Zero-extended forward DFT (the transform that the residues of section 2.2,
 * eq. (3), enumerate): X_k = sum_{j<L} zeta_N^{+kj} x_j for k < N. */
int oracle_padded_dft(int64_t L, int64_t N, const double* x_, double* X_) {
    if (L < 0 || N < 1 || L > N) return 1;
    cd* buf = (cd*)calloc((size_t)N, sizeof(cd));
    memcpy(buf, x_, sizeof(cd) * (size_t)L);
    oracle_dft(N, (double*)buf, +1);
    memcpy(X_, buf, sizeof(cd) * (size_t)N);
    free(buf);
    return 0;
}
