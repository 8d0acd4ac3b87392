// Internal interface between the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hdc.h"

// Records the thread-local message returned by hdc_last_error(); returns st.
hdc_status set_error(hdc_status st, const char* msg);

namespace hdc {

// zeta_N^e = lo[e & mask] * hi[e >> lgB]  (two-level table of exp(+2 pi i e / N), FP64).
struct TwN {
    const double2* lo;
    const double2* hi;
    int32_t lgB;
    int32_t mask;
};

// Addressing of independent rows: base(row) = (row / inner_cnt) * outer_stride
// + (row % inner_cnt) * inner_stride, element j of the row at base + j * es.
struct RowAddr {
    int64_t inner_cnt;
    int64_t outer_stride;
    int64_t inner_stride;
    int64_t es;
};

// Fused small-transform convolution: every residue of one row in one workgroup.
struct FusedArgs {
    const void* f;
    const void* g;
    void* h;
    int64_t nrows;
    RowAddr in;   // f and g (f only when Lg > 0)
    RowAddr ing;  // g when Lg > 0
    RowAddr out;  // h
    const int64_t* desc;  // optional per-row {f_off, h_off, L, M}; in/out then give es only
    int32_t L, M;         // uniform lengths when desc == nullptr
    int32_t Lg;           // g's length when it differs from f's (section 3.5 with Lambda = 1), else 0
    int32_t p, q, qout;   // qout = max output blocks ceil(M/m)
    int32_t N;            // q * m
    int32_t Dc;           // residues processed concurrently
    int32_t rpw;          // rows per workgroup
    int32_t same;         // f == g
    int32_t hiprec;       // FP64 twiddle products for complex64
    TwN tw;
    const void* twm;      // zeta_m^e, e < m, in the data type
    double invN;
    // multi-convolution (section 6.1): nops > 2 operands, f and g the first two,
    // xm[o - 2] the others (same lengths and layout as f)
    int32_t nops;
    const void* xm[6];
    // m = R msz with R odd (R = 1: m a power of two): the mixed-radix fused kernel
    int32_t R;
};

// Persistent fused kernel of a batch: items[3 i .. 3 i + 2] = {bucket, FFT size m,
// block of rows} read in queue order through the atomic counter; args[bucket]
// holds the bucket's fused arguments (their f, g, h unused: these are f, g, h).
struct FusedQueueArgs {
    const void* f;
    const void* g;
    void* h;
    int32_t same, nitems;
    const FusedArgs* args;
    const int32_t* items;
    int* counter;
};

struct ColFwdArgs {
    const void* x;
    const void* x2;            // real case: g (x is f), both real
    void* X;
    int64_t B, in_bs, out_bs;  // batch count and strides (elements)
    int32_t L, Ccols, C1, m2, m, q, p, N;
    int32_t r0, Dg;            // Dg residue slots; slot d lam + li is residue r0 + d + li rstride
    int32_t lam, rstride;      // lam = 1 (rstride unused): residues [r0, r0 + Dg)
    int32_t nsec, r2;          // the last nsec slots hold residues r2, r2 - 1, ... (real case)
    int32_t tile, ntiles;
    int32_t hiprec;
    TwN tw;
    const void* tw1;           // per-pass twiddle table of the m1-point transform, data type
    const int64_t* desc;       // optional per-batch {input offset, L}; replaces b*in_bs and L
    const void* gs;            // real N-D: scale words (z = f + i s g); nullptr: s = 1
};

struct ColBwdArgs {
    const void* Y;
    void* h;
    int64_t B, in_bs, out_bs;
    int32_t M, Ccols, C1, m2, m, q, N, qout;
    int32_t r0, Dg, accumulate;
    int32_t tile, ntiles;
    int32_t hiprec;
    TwN tw;
    const void* tw1;
    double invN;
    const int64_t* desc;  // optional per-batch {output offset, M}; replaces b*out_bs and M
    const void* gs;       // real N-D (REAL): scale words, h = Im(...) / (2 s); nullptr: Hermitian weights
};

struct RowArgs {
    const void* a;
    const void* b;
    void* out;
    int64_t nrows;
    RowAddr addr;
    int32_t mode;  // 0 forward DFT, 1 inverse DFT, 2 forward a and b, product, inverse
    int32_t same;
    int32_t rpw;
    const void* tw;   // zeta_{m2}^e, e < m2
    const void* twp;  // per-pass twiddle table of the m2-point transform
    // MODE_CONV with fraw != nullptr (section 3.5, shorter operand with a
    // trivial column stage): operand a is formed from the raw input fraw
    // (batches fbs apart, Lf x C1 values each, pf blocks of m2) instead of being
    // read; row ((b Dg + d) m1g + l1g) C1 + c1 then holds residue
    // r0 + d + l1g qg of length qf m2 = N of batch b
    const void* fraw;
    TwN twN;
    int64_t fbs;
    int32_t Lf, pf, qf, N, r0, qg, m1g, Dg, hiprec;
    // real case (k_row_real): product rows of residues r0 + d (d < Dg, each
    // q = qg), Z with S slots per batch, partner slots from residue pfirst on
    int32_t S, pfirst;
    // multi-convolution (k_row_multi): nops operands' rows at a + o * ostride
    int32_t nops;
    int64_t ostride;
};

// One problem of the raw-residue-row path (m1 = 1: a residue transform is one
// row of m <= 4096 points): its inputs' and output's element offsets, lengths,
// blocks p and residues q (N = q m), and its zeta_N table.
struct RawProb {
    int64_t f_off, h_off;
    int32_t L, M, p, q;
    int32_t qout, hiprec;
    TwN tw;
    double invN;
};

// Raw residue rows (k_row_rr) and the q-point output sums (k_qsum).
// Plain mode (rowmap == nullptr): one problem p0 over B batches (strides fbs,
// ybs, hbs in elements) of C1 interleaved copies, residues [r0, r0 + Dg); row
// (b Dg + d) C1 + c1 of Y holds residue r0 + d of copy c1 at
// Y[b ybs + d m C1 + s C1 + c1].  Batch mode: problems probs[], row k of Y
// (m values) holds residue rowmap[2k + 1] of problem rowmap[2k], the rows of
// problem i starting at ybase[i]; k_qsum workgroup w covers columns
// [tilemap[2w + 1], + blockDim) of problem tilemap[2w].
struct RawArgs {
    const void* f;
    const void* g;
    void* Y;
    void* h;
    int64_t nrows;
    int32_t m, rpw, C1, Dg, r0, same, accumulate, ntiles;
    int64_t fbs, ybs, hbs;
    RawProb p0;
    const RawProb* probs;
    const int32_t* rowmap;
    const int64_t* ybase;
    const int32_t* tilemap;
    const void* twp;  // per-pass table of the m-point transform, data type
};

// Largest FFT size the persistent fused batch kernel serves, per type.
constexpr int kQueueMaxM64 = 4096;   // complex64
constexpr int kQueueMaxM128 = 512;   // complex128

// Largest residue group the q-point output sums keep in registers, and the
// most blocks the raw-row path re-reads per residue.
constexpr int kMaxQsum = 32;
constexpr int kMaxRawP = 4;

// Whole-row convolution of an innermost N-D axis (k_rowconv, complex64): FFT
// sizes, the output blocks its registers hold, the most input blocks each
// residue re-reads.
constexpr int kRowconvMinM = 1024;
constexpr int kRowconvMaxM = 4096;
constexpr int kRowconvQO = 4;
constexpr int kRowconvMaxP = 4;

enum { MODE_FWD = 0, MODE_INV = 1, MODE_CONV = 2 };

// Compute units of the current device (cached).
int cu_count();

// Launchers (return hipSuccess or the launch error).  `dbl` selects complex128.
hipError_t launch_fused(bool dbl, int m, const FusedArgs& a, int threads, int64_t blocks, size_t lds,
                        hipStream_t s);
hipError_t launch_col_fwd(bool dbl, int m1, const ColFwdArgs& a, int threads, int64_t gx, int64_t gy,
                          size_t lds, hipStream_t s, bool real = false);
hipError_t launch_col_bwd(bool dbl, int m1, const ColBwdArgs& a, int threads, int64_t gx, int64_t gy,
                          size_t lds, hipStream_t s, bool real = false);
hipError_t launch_row_real(bool dbl, int m2, const RowArgs& a, int threads, int64_t blocks, size_t lds,
                           hipStream_t s);
hipError_t launch_fused_real(bool dbl, int m, const FusedArgs& a, int threads, int64_t blocks, size_t lds,
                             hipStream_t s);
hipError_t launch_row(bool dbl, int m2, const RowArgs& a, int threads, int64_t blocks, size_t lds,
                      hipStream_t s);
hipError_t launch_row_multi(bool dbl, int m2, const RowArgs& a, int threads, int64_t blocks, size_t lds,
                            hipStream_t s);
hipError_t launch_row_rr(bool dbl, int m, const RawArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s);
hipError_t launch_qsum(bool dbl, const RawArgs& a, int64_t gx, int64_t gy, hipStream_t s);
hipError_t launch_rowconv(bool dbl, int m, const FusedArgs& a, int threads, int64_t blocks, size_t lds,
                          hipStream_t s);
hipError_t launch_fused_queue(bool dbl, const FusedQueueArgs& a, int64_t nitems, size_t lds, hipStream_t s);
hipError_t launch_mul(bool dbl, void* F, const void* G, int64_t n, hipStream_t s);
// Real N-D data: the scale words max|f|, max|g| (cleared and filled) that the
// column passes turn into s = max|f| / max|g| for z = f + i s g, h = Im(z * z) / (2 s).
hipError_t launch_real_scale(bool dbl, const void* f, const void* g, int64_t n, void* mx, hipStream_t s);
hipError_t launch_natural(bool dbl, const void* F, void* out, int64_t Dg, int64_t m1, int64_t m2, int64_t C,
                          hipStream_t s);

// Slots of a contiguous n-point LDS buffer (one pad slot per 8 values).
inline int64_t padded_len(int64_t n) { return n + (n >> 3); }

// Entries of the per-pass twiddle table of an n-point row transform (radix R0
// first, then radix 8 at Ns = R0, 8 R0, ...: three arrays of Ns values each).
inline int64_t pass_tab_len(int64_t n) {
    int lg = 0;
    while ((int64_t(1) << lg) < n) ++lg;
    if (n < 8) return 0;
    const int r0 = lg % 3 == 0 ? 8 : (1 << (lg % 3));
    const int np = lg % 3 == 0 ? lg / 3 : lg / 3 + 1;
    return np > 1 ? 3 * (int64_t)r0 * ((int64_t(1) << (3 * (np - 1))) - 1) / 7 : 0;
}

// Points per thread of the Stockham transforms for size n.
inline int ppt_for(int n) { return n >= 8 ? 8 : n; }

// m = R 2^k: the odd factor R, and the threads of one m-point residue transform
// (R sub-transforms of 2^k points side by side).
inline int64_t odd_part(int64_t m) {
    while (m > 0 && (m & 1) == 0) m >>= 1;
    return m;
}
inline int res_threads(int64_t m) {
    const int64_t R = odd_part(m), p2 = m / R;
    return (int)(R * (p2 / ppt_for((int)p2)));
}

// Largest odd factor of m the mixed-radix fused kernel takes (its direct
// R-point stage costs R products per point).
constexpr int kMaxOddR = 63;

// Largest column-stage transform and row-stage transform the kernels implement.
constexpr int kMaxM1 = 1024;
constexpr int kMaxRow = 4096;
constexpr int kMaxFused = 4096;
// Largest number of operands of a multi-convolution.
constexpr int kMaxOps = 8;

}  // namespace hdc
