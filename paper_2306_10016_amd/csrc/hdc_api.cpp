// Host side of the hdc library: parameter derivation (section 2.5), FP64
// twiddle tables, kernel-variant choice, the N-D recursion over axes
// (section 3.6) and the C-ABI entry points declared in include/hdc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hdc.h"
#include "../../include/hdc_tune.h"
#include "hdc_internal.h"

using namespace hdc;

namespace {

thread_local std::string g_err = "no error";

hdc_status fail(hdc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

hdc_status hip_fail(hipError_t e, const char* what) {
    return fail(HDC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return hip_fail(_e, #expr); \
    } while (0)

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
// no prime factor above 7
bool smooth7(int64_t x) {
    if (x < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (x % p == 0) x /= p;
    return x == 1;
}
int ilog2i(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

size_t elem_bytes(hdc_dtype t) { return (t == HDC_C128 || t == HDC_R64) ? 16 : 8; }
bool is_real(hdc_dtype t) { return t == HDC_R32 || t == HDC_R64; }
// the complex type a real plan computes in (z = f + i g)
hdc_dtype complex_of(hdc_dtype t) { return t == HDC_R64 ? HDC_C128 : (t == HDC_R32 ? HDC_C64 : t); }

// exp(+2 pi i e / n) from an exactly reduced exponent, evaluated in long double.
void root(int64_t e, int64_t n, double* re, double* im) {
    e %= n;
    if (e < 0) e += n;
    const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)e / (long double)n;
    *re = (double)cosl(a);
    *im = (double)sinl(a);
}

size_t device_lds_max() {
    static size_t cached = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, v = 0;
        cached = 163840;  // gfx950: 160 KiB of LDS per workgroup
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            cached = (size_t)v;
    });
    return cached;
}

// LDS budget the fused kernel may use for one row (q padded residues + q twiddles):
// two such workgroups fit the 160 KiB of a gfx950 CU.
constexpr size_t kFusedRowLds = 81920;

int64_t round8(int64_t x) { return (x + 7) / 8 * 8; }

// Largest y extent of a launch grid; column launches over more batches are split.
constexpr int64_t kMaxGridY = 65535;

// Optional per-launch timing: when a recorder is installed on this thread,
// every kernel launch is bracketed by HIP events on its stream and its
// algorithmic bytes (compulsory reads + writes of that launch) are noted.
struct Recorder {
    const void* filter = nullptr;  // record only launches of this plan (NULL: all)
    std::vector<hipEvent_t> ev;
    std::vector<int32_t> kind;
    std::vector<double> bytes;
};
thread_local Recorder* g_rec = nullptr;
thread_local const void* g_cur_plan = nullptr;  // plan whose launches are being issued

struct LaunchScope {
    bool on = false;
    LaunchScope(hipStream_t s, int kind, double bytes) {
        if (!g_rec) return;
        if (g_rec->filter && g_rec->filter != g_cur_plan) return;
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
        g_rec->ev.push_back(a);
        g_rec->ev.push_back(b);
        g_rec->kind.push_back(kind);
        g_rec->bytes.push_back(bytes);
        (void)hipEventRecord(a, s);
        on = true;
        end = b;
        st = s;
    }
    ~LaunchScope() {
        if (on) (void)hipEventRecord(end, st);
    }
    hipEvent_t end = nullptr;
    hipStream_t st = nullptr;
};

}  // namespace

hdc_status set_error(hdc_status st, const char* msg) { return fail(st, "%s", msg); }

// ------------------------------------------------------------------ plans --

struct AxisPlan {
    hdc_axis_desc d{};
    bool dbl = false;
    bool hiprec = false;
    // fused geometry
    int Dc = 1, f_rpw = 1, f_threads = 1;
    size_t f_lds = 0;
    // whole-row convolution (variant 3)
    int rc_rpw = 1, rc_threads = 1;
    size_t rc_lds = 0;
    // column/row geometry
    int cf_tile = 1, cf_threads = 1, cb_tile = 1, cb_threads = 1, r_rpw = 1, r_threads = 1;
    size_t cf_lds = 0, cb_lds = 0, r_lds = 0;
    // requested columns per workgroup of the column passes (0: the default below)
    int tile_req = 0;
    // outer N-D axes with m2 > 1: plain strided m2-point DFT passes (column kernels)
    int mf_tile = 1, mf_threads = 1, mb_tile = 1, mb_threads = 1;
    size_t mf_lds = 0, mb_lds = 0;
    // device tables
    TwN tw{};
    const void* tw_m = nullptr;
    const void* tw_m1 = nullptr;
    const void* tw_m2 = nullptr;
    // per-pass twiddle tables of the m1- and m2-point transforms (the layout the
    // kernels keep in LDS: for each radix-8 pass of length Ns, three arrays of
    // Ns values zeta_{8 Ns}^{i k}, i = 1, 2, 4)
    const void* tw_p1 = nullptr;
    const void* tw_p2 = nullptr;
    // table layout offsets (bytes) inside the plan's table block
    size_t off_lo = 0, off_hi = 0, off_m = 0, off_m1 = 0, off_m2 = 0, off_p1 = 0, off_p2 = 0;
    int64_t nlo = 0, nhi = 0;
};

struct hdc_plan_s {
    int ndim = 1;
    hdc_dtype dtype = HDC_C128;
    AxisPlan ax[3];
    // unequal lengths (sections 3.5-3.6): per axis, ax[a] is the longer
    // operand's geometry (Lambda m-point residues) and fx[a] the shorter one's
    // (m-point residues); swap[a]: the caller's f is the longer one on axis a
    bool uneq = false;
    // real f, g and h (HDC_R32 / HDC_R64, 1D); dtype is then the complex type computed in
    bool real = false;
    // real f, g and h of an N-D plan: one complex autoconvolution of z = f + i s g
    bool real_nd = false;
    // operands of a multi-convolution (section 6.1), 2 for every other plan
    int nops = 2;
    bool swap[3] = {false, false, false};
    int64_t lam[3] = {1, 1, 1};
    int64_t Lf[3] = {1, 1, 1}, Lg[3] = {1, 1, 1};
    AxisPlan fx[3];
    void* tables = nullptr;
    size_t ws_bytes = 0;
};

namespace {

// Derivation and admissibility (section 2.5, section 2.2's q >= p).  K is the
// length of the linear convolution (2L-1 for equal lengths): the transform
// length N = q m must reach max(M, K) or the outputs alias; M is the number of
// outputs written, so M < K gives the first M outputs only (the backward range
// t < p of section 2.2 gives the first L).
hdc_status derive_axis(int64_t L, int64_t M, int64_t m, int64_t p, int64_t q, int64_t C, int64_t D, hdc_dtype dtype,
                       hdc_axis_desc* o, int64_t K = -1) {
    if (is_real(dtype))
        return fail(HDC_ERR_UNSUPPORTED, "real data (HDC_R32 / HDC_R64) are implemented for 1D plans (hdc_plan) only");
    if (dtype != HDC_C64 && dtype != HDC_C128) return fail(HDC_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (L < 1) return fail(HDC_ERR_INVALID_ARG, "L = %lld must be >= 1", (long long)L);
    // no admissible size comes near 2^40; bounding every argument first keeps
    // the products below (2L, p m, q m) inside 64 bits
    constexpr int64_t kHuge = int64_t(1) << 40;
    if (L >= kHuge || M >= kHuge || m >= kHuge || p >= kHuge || q >= kHuge || C >= kHuge || D >= kHuge ||
        K >= kHuge)
        return fail(HDC_ERR_UNSUPPORTED, "sizes of 2^40 and beyond are not supported");
    if (K < 0) K = 2 * L - 1;
    if (M < 1) return fail(HDC_ERR_INVALID_ARG, "M = %lld must be >= 1", (long long)M);
    const int64_t Mt = std::max(M, K);
    if (m < 1) return fail(HDC_ERR_INVALID_ARG, "m = %lld must be >= 1", (long long)m);
    if (C < 1) return fail(HDC_ERR_INVALID_ARG, "C = %lld must be >= 1", (long long)C);
    if (p < 0 || q < 0 || D < 0) return fail(HDC_ERR_INVALID_ARG, "p, q, D must be >= 0 (0 derives)");
    if (p == 0) p = ceil_div(L, m);
    if (q == 0) q = ceil_div(Mt, m);
    if (p * m < L) return fail(HDC_ERR_INVALID_ARG, "p m = %lld < L = %lld", (long long)(p * m), (long long)L);
    if (q * m < M) return fail(HDC_ERR_INVALID_ARG, "q m = %lld < M = %lld", (long long)(q * m), (long long)M);
    if (q * m < K)
        return fail(HDC_ERR_INVALID_ARG, "q m = %lld < %lld: the transform would alias the linear convolution",
                    (long long)(q * m), (long long)K);
    if (q < p) return fail(HDC_ERR_INVALID_ARG, "q = %lld < p = %lld", (long long)q, (long long)p);
    if (D == 0 || D > q) D = q;
    // m = R 2^k with R odd and 7-smooth (section 3.1's FFT-friendly sizes);
    // R > 1 runs on the mixed-radix fused kernel only
    const int64_t Rodd = odd_part(m);
    if (!is_pow2(m) && !(Rodd <= kMaxOddR && smooth7(Rodd)))
        return fail(HDC_ERR_UNSUPPORTED, "m = %lld: the kernels take m = R 2^k with R odd, 7-smooth and at most %d",
                    (long long)m, kMaxOddR);
    const int64_t N = q * m;
    if (N >= (int64_t(1) << 31))
        return fail(HDC_ERR_UNSUPPORTED, "N = %lld exceeds the 32-bit twiddle index range", (long long)N);
    if (C > (int64_t(1) << 40) / M)
        return fail(HDC_ERR_UNSUPPORTED, "M C = %lld x %lld outputs exceed 2^40", (long long)M, (long long)C);
    o->L = L;
    o->M = M;
    o->m = m;
    o->p = p;
    o->q = q;
    o->N = N;
    o->D = D;
    o->C = C;
    o->q_out = ceil_div(M, m);
    // four-step split of the m-point DFT for the column/row passes
    const int64_t rowmax = kMaxRow;
    int64_t m2 = std::min<int64_t>(m, rowmax);
    int64_t m1 = m / m2;
    if (m1 > kMaxM1)
        return fail(HDC_ERR_UNSUPPORTED, "m = %lld exceeds %lld (column stage %d x row stage %d)", (long long)m,
                    (long long)(kMaxM1 * rowmax), kMaxM1, (int)rowmax);
    o->m1 = m1;
    o->m2 = m2;
    const size_t b = elem_bytes(dtype);
    const size_t fused_lds = (size_t)(q * padded_len(m)) * b + (size_t)q * 16 + 16;
    o->variant = (m <= kMaxFused && fused_lds <= kFusedRowLds) ? 0 : 1;
    o->reserved = 0;
    if (!is_pow2(m) && (o->variant != 0 || res_threads(m) > 512))
        return fail(HDC_ERR_UNSUPPORTED,
                    "m = %lld is not a power of two: it needs the fused kernel (q m b 9/8 = %zu bytes of LDS within "
                    "%zu, m <= %d)", (long long)m, fused_lds, kFusedRowLds, kMaxFused);
    return HDC_OK;
}

int tile_for(int tpf, int tmin, int maxthreads) {
    int t = std::max(tmin, 256 / std::max(tpf, 1));
    while (t > 1 && t * tpf > maxthreads) t /= 2;
    return std::max(t, 1);
}

// Geometry of every kernel for one axis; `outer` = transformed as a column
// stage of an N-D problem (m1 = m, m2 = 1).
hdc_status geometry(AxisPlan& A, bool outer, bool many_rows = false, bool keep_split = false) {
    hdc_axis_desc& d = A.d;
    const size_t b = A.dbl ? 16 : 8;
    if (!is_pow2(d.m) && (outer || many_rows))
        return fail(HDC_ERR_UNSUPPORTED, "m = %lld: N-D axes take powers of two", (long long)d.m);
    if (outer) {
        // an outer axis is transformed down strided columns: m = m1 * m2 with both
        // factors column passes (the second one a plain strided m2-point DFT)
        if (d.m > (int64_t)kMaxM1 * kMaxM1)
            return fail(HDC_ERR_UNSUPPORTED, "outer-axis m = %lld exceeds %d", (long long)d.m, kMaxM1 * kMaxM1);
        if (!keep_split) {
            d.m1 = std::min<int64_t>(d.m, kMaxM1);
            d.m2 = d.m / d.m1;
        }
        d.variant = 1;
        const int ppt = ppt_for((int)d.m2);
        const int tpf = (int)d.m2 / ppt;
        const int tmin0 = A.dbl ? 8 : 16;
        A.mf_tile = tile_for(tpf, tmin0, 1024);
        A.mf_threads = A.mf_tile * tpf;
        A.mf_lds = (size_t)d.m2 * A.mf_tile * b;
        A.mb_tile = tile_for(tpf, tmin0, 512);
        while (A.mb_tile > 1 && (size_t)d.m2 * A.mb_tile * b > 65536) A.mb_tile /= 2;
        A.mb_threads = A.mb_tile * tpf;
        A.mb_lds = (size_t)d.m2 * A.mb_tile * b;
    }
    const int tmin = A.dbl ? 8 : 16;
    // fused (m = R 2^k: R sub-transforms side by side)
    {
        const int tpf = res_threads(d.m);
        // every residue of a row stays in LDS whatever D is (D bounds the
        // workspace of the multi-pass variant), so D does not limit concurrency
        int Dc = (int)d.q;
        Dc = std::max(1, std::min(Dc, 512 / tpf));
        const int rowthreads = tpf * Dc;
        const size_t rowlds = (size_t)(d.q * padded_len(d.m)) * b;
        int rpw = std::max(1, 256 / rowthreads);
        while (rpw > 1 && (size_t)rpw * rowlds > kFusedRowLds) rpw /= 2;
        A.Dc = Dc;
        A.f_rpw = rpw;
        A.f_threads = rowthreads * rpw;
        A.f_lds = ((size_t)rpw * rowlds + 15) / 16 * 16 + (size_t)d.q * 16;
    }
    // columns
    {
        const int ppt = ppt_for((int)d.m1);
        const int tpf = (int)d.m1 / ppt;
        // the backward kernel keeps at most 64 KiB of LDS per workgroup; narrower
        // tiles still fetch whole cache lines once, because the XCD map runs
        // neighbouring tiles on the same L2
        A.cf_tile = tile_for(tpf, tmin, 1024);
        A.cf_threads = A.cf_tile * tpf;
        A.cf_lds = (size_t)d.m1 * A.cf_tile * b;
        A.cb_tile = tile_for(tpf, tmin, 512);
        while (A.cb_tile > 1 && (size_t)d.m1 * A.cb_tile * b > 65536) A.cb_tile /= 2;
        if (A.tile_req > 0) {
            // a tuner's choice: the forward tile as requested, the backward one the
            // same within its 512 threads and 64 KiB of LDS
            if (!is_pow2(A.tile_req) || A.tile_req * tpf > 1024)
                return fail(HDC_ERR_UNSUPPORTED, "column tile %d: a power of two with %d threads per column and "
                            "at most 1024 threads", A.tile_req, tpf);
            A.cf_tile = A.tile_req;
            A.cf_threads = A.cf_tile * tpf;
            A.cf_lds = (size_t)d.m1 * A.cf_tile * b;
            A.cb_tile = A.tile_req;
            while (A.cb_tile > 1 && (A.cb_tile * tpf > 512 || (size_t)d.m1 * A.cb_tile * b > 65536)) A.cb_tile /= 2;
        }
        A.cb_threads = A.cb_tile * tpf;
        A.cb_lds = (size_t)d.m1 * A.cb_tile * b;
        const size_t tab = (size_t)pass_tab_len(d.m1) * b;
        if (A.cf_lds + tab > device_lds_max() || A.cb_lds + tab > device_lds_max())
            return fail(HDC_ERR_UNSUPPORTED, "column stage m1 = %lld needs %zu bytes of LDS", (long long)d.m1,
                        A.cf_lds);
    }
    // rows
    {
        const int ppt = ppt_for((int)d.m2);
        const int tpf = (int)d.m2 / ppt;
        int rpw = std::max(1, 256 / tpf);
        A.r_rpw = rpw;
        A.r_threads = rpw * tpf;
        A.r_lds = (size_t)rpw * 2 * d.m2 * b;  // two exchange buffers per row
        // plus the pass table and (real-data rows) the two-level zeta_m2 table
        if (A.r_lds + (size_t)(pass_tab_len(d.m2) + 128) * b > device_lds_max())
            return fail(HDC_ERR_UNSUPPORTED, "row stage m2 = %lld needs %zu bytes of LDS", (long long)d.m2, A.r_lds);
    }
    // with many independent rows (the innermost axis of an N-D problem) one
    // workgroup per row keeps the machine busy, and the fused kernel may use all
    // the LDS a workgroup can have instead of the 80 KiB that leaves room for two
    if (many_rows && !outer && d.m <= kMaxFused && A.f_lds + 4096 <= device_lds_max()) d.variant = 0;
    if (d.variant == 0 && A.f_lds > device_lds_max()) d.variant = 1;
    // long one-row residues of an innermost N-D axis: a workgroup per (row,
    // residue) on the raw-row path rather than every residue of a row in turn
    // in one fused workgroup
    if (many_rows && !outer && d.m >= 2048 && d.m <= kMaxRow && d.q <= kMaxQsum && d.p <= kMaxRawP &&
        d.C * d.m <= (int64_t(1) << 30))
        d.variant = 2;
    // ... and when the output blocks fit the registers, the whole row in one
    // workgroup: residues in turn, output sums accumulated in registers
    if (many_rows && !outer && !A.dbl && is_pow2(d.m) && d.m >= kRowconvMinM && d.m <= kRowconvMaxM &&
        d.q_out <= kRowconvQO && d.p <= kRowconvMaxP) {
        // two exchange buffers per row, the m-point pass table, q twiddles
        const int tpf = (int)d.m / 8;
        A.rc_rpw = std::max(1, 256 / tpf);
        A.rc_threads = A.rc_rpw * tpf;
        A.rc_lds = (((size_t)A.rc_rpw * 2 * d.m + (size_t)pass_tab_len(d.m)) * b + 15) / 16 * 16 + (size_t)d.q * 16;
        if (A.rc_lds <= device_lds_max()) d.variant = 3;
    }
    A.hiprec = !A.dbl && d.N > (int64_t(1) << 20);
    return HDC_OK;
}

// Plain complex 1D plans whose residue transform is one row (m1 = 1) and does
// not fit the fused kernel take the raw-row path (variant 2) when every residue
// group fits the output sums' registers (q <= 32) and the inputs are re-read
// little (every residue reads all p blocks: p <= 4).
void enable_raw_rows(AxisPlan& A) {
    if (A.d.variant == 1 && A.d.m1 == 1 && A.d.q <= kMaxQsum && A.d.p <= kMaxRawP &&
        A.d.C * A.d.m <= (int64_t(1) << 30))
        A.d.variant = 2;
}

int64_t pow2_ceil(int64_t x) {
    int64_t v = 1;
    while (v < x) v <<= 1;
    return v;
}

// Section 3.5: the shorter operand (length Ls) is cut into m-point residues,
// the longer one (length Ll) into Lambda m-point residues, with
//   p_f = ceil(Ls/m), p_g = ceil(Ll/(Lambda m)), q_g = ceil(M/(Lambda m)),
//   q_f = Lambda q_g,
// so both transforms have length N = q_g Lambda m = q_f m.  The longer
// operand's four-step split m1g x m2g takes m1g a multiple of Lambda; the
// shorter one's is (m1g/Lambda) x m2g, so its row l1f of residue r_f is the
// longer operand's row Lambda l1f + lambda of residue r_f - q_g lambda.
// `outer`: an outer axis of an N-D problem; `inner_nd`: the innermost axis of one.
hdc_status derive_uneq(int64_t Lf, int64_t Lg, int64_t M, int64_t m, int64_t lam, int64_t C, int64_t D,
                       hdc_dtype dtype, hdc_axis_desc* fo, hdc_axis_desc* go, bool* swapped, bool outer = false,
                       bool inner_nd = false) {
    if (Lf < 1 || Lg < 1) return fail(HDC_ERR_INVALID_ARG, "Lf = %lld and Lg = %lld must be >= 1", (long long)Lf,
                                      (long long)Lg);
    constexpr int64_t kHuge = int64_t(1) << 40;  // as in derive_axis: keeps Lf + Lg and Lambda m in range
    if (Lf >= kHuge || Lg >= kHuge || M >= kHuge || m >= kHuge || lam >= kHuge)
        return fail(HDC_ERR_UNSUPPORTED, "sizes of 2^40 and beyond are not supported");
    const bool sw = Lf > Lg;
    const int64_t Ls = sw ? Lg : Lf, Ll = sw ? Lf : Lg;
    if (M < 1) return fail(HDC_ERR_INVALID_ARG, "M = %lld must be >= 1", (long long)M);
    // the transform must reach the linear convolution's Lf + Lg - 1 terms
    const int64_t Mo = M;
    M = std::max(M, Ls + Ll - 1);
    if (m < 0 || lam < 0) return fail(HDC_ERR_INVALID_ARG, "m and Lambda must be >= 0 (0 derives)");
    // an outer N-D axis is two column stages of at most kMaxM1 each
    const int64_t mg_max = int64_t(kMaxM1) * (outer ? kMaxM1 : kMaxRow);
    if (m == 0 && lam == 0 && outer) {
        // outer axes (measured): the smallest Lambda m with at most four blocks of
        // the longer operand, and m the smallest power of two holding the shorter
        // operand in one block
        int64_t mg = 1;
        while (mg * 4 < Ll && mg < mg_max) mg <<= 1;
        lam = std::max<int64_t>(1, std::min<int64_t>({mg / pow2_ceil(Ls), kMaxM1, mg}));
        m = mg / lam;
    } else if (m == 0 && lam == 0 && inner_nd) {
        // the innermost axis of an N-D problem (measured): Lambda = 1, so that its
        // many rows run in the fused kernel when the transform fits, in as few
        // blocks and residues as it allows (one residue, else one block)
        int64_t best = pow2_ceil(M);
        if (best > kMaxFused) best = pow2_ceil(Ll);
        const size_t lds = (size_t)(ceil_div(M, best) * padded_len(best)) * elem_bytes(dtype) + 4096;
        if (lds <= device_lds_max()) {
            lam = 1;
            m = best;
        }
    }
    if (m == 0 || lam == 0) {
        // Lambda m: up to 2^17 output points a single block (q_g = 1: one
        // residue, the fewest launches); beyond, the power of two with at most
        // four blocks of the longer operand and the shortest transform
        // N = ceil(M/(Lambda m)) Lambda m (ties: the larger)
        int64_t best = 0, bestN = 0;
        for (int64_t mg = 1; mg <= mg_max; mg <<= 1) {
            if (m > 0 && (mg < m || mg / m > kMaxM1)) continue;
            if (lam > 0 && mg < lam) continue;
            if (mg * 4 < Ll && mg < mg_max) continue;
            if (M <= 131072 && mg < M && mg < mg_max) continue;
            const int64_t N = ceil_div(M, mg) * mg;
            if (best == 0 || N <= bestN) {
                if (best != 0 && M <= 131072 && N == bestN) continue;
                best = mg, bestN = N;
            }
        }
        if (best == 0) return fail(HDC_ERR_UNSUPPORTED, "no admissible Lambda m for m = %lld", (long long)m);
        if (m > 0) lam = best / m;
        else if (lam > 0) m = best / lam;
        else {
            // a balanced four-step split m1g x m2g, m2g = 2^ceil(lg(Lambda m)/2),
            // with the shorter operand's column stage trivial: m = m2g, Lambda = m1g
            int64_t m2 = 1;
            while (m2 * m2 < best) m2 <<= 1;
            m2 = std::min<int64_t>(m2, kMaxRow);
            lam = std::min<int64_t>(kMaxM1, best / m2);
            m = best / lam;
        }
    }
    if (!is_pow2(m) || !is_pow2(lam))
        return fail(HDC_ERR_UNSUPPORTED, "m = %lld and Lambda = %lld: only powers of two are implemented",
                    (long long)m, (long long)lam);
    if (lam > kMaxM1)
        return fail(HDC_ERR_UNSUPPORTED, "Lambda = %lld exceeds the column stage's %d", (long long)lam, kMaxM1);
    hdc_axis_desc g{};
    hdc_status st = derive_axis(Ll, Mo, lam * m, 0, 0, C, D, dtype, &g, Ls + Ll - 1);
    if (st != HDC_OK) return st;
    if (g.m > mg_max)
        return fail(HDC_ERR_UNSUPPORTED, "Lambda m = %lld exceeds %lld", (long long)g.m, (long long)mg_max);
    // split with Lambda | m1g: a 1D axis (and the innermost N-D axis) puts at
    // most kMaxRow points in the row stage; an outer axis puts up to kMaxM1 in
    // its first column stage (Lambda <= kMaxM1 divides it)
    if (outer) {
        g.m1 = std::min<int64_t>(g.m, kMaxM1);
        if (g.m1 < lam) g.m1 = lam;
    } else {
        g.m1 = std::max<int64_t>(lam, g.m / kMaxRow);
    }
    g.m2 = g.m / g.m1;
    if (g.m1 > kMaxM1 || (outer && g.m2 > kMaxM1))
        return fail(HDC_ERR_UNSUPPORTED, "Lambda m = %lld does not split for Lambda = %lld", (long long)g.m,
                    (long long)lam);
    // Lambda = 1 keeps the single-kernel variant when it fits (both operands
    // then share m and differ only in their lengths)
    if (lam > 1 || outer) g.variant = 1;
    hdc_axis_desc f = g;
    f.L = Ls;
    f.m = m;
    f.p = ceil_div(Ls, m);
    f.q = lam * g.q;
    f.D = lam * g.D;
    f.q_out = ceil_div(Mo, m);
    f.m1 = g.m1 / lam;
    f.m2 = g.m2;
    if (fo) *fo = f;
    if (go) *go = g;
    if (swapped) *swapped = sw;
    return HDC_OK;
}

// Append tables for one axis to the host staging blob.
void stage_tables(AxisPlan& A, std::vector<unsigned char>& blob) {
    auto align = [&](size_t a) {
        while (blob.size() % a) blob.push_back(0);
    };
    const int64_t N = A.d.N;
    const int lgN = ilog2i(N);
    const int lgB = (lgN + 1) / 2;
    const int64_t B = int64_t(1) << lgB;
    A.nlo = B;
    A.nhi = ceil_div(N, B);
    align(256);
    A.off_lo = blob.size();
    for (int64_t e = 0; e < B; ++e) {
        double v[2];
        root(e, N, &v[0], &v[1]);
        blob.insert(blob.end(), (unsigned char*)v, (unsigned char*)v + 16);
    }
    A.off_hi = blob.size();
    for (int64_t e = 0; e < A.nhi; ++e) {
        double v[2];
        root(e * B, N, &v[0], &v[1]);
        blob.insert(blob.end(), (unsigned char*)v, (unsigned char*)v + 16);
    }
    auto small_table = [&](int64_t n) {
        align(256);
        size_t off = blob.size();
        for (int64_t e = 0; e < n; ++e) {
            double re, im;
            root(e, n, &re, &im);
            if (A.dbl) {
                double v[2] = {re, im};
                blob.insert(blob.end(), (unsigned char*)v, (unsigned char*)v + 16);
            } else {
                float v[2] = {(float)re, (float)im};
                blob.insert(blob.end(), (unsigned char*)v, (unsigned char*)v + 8);
            }
        }
        return off;
    };
    // the radix-8 passes after the first (radix R0 at Ns = 1): Ns = R0, 8 R0, ...
    auto pass_table = [&](int64_t n) {
        align(256);
        size_t off = blob.size();
        if (n < 8) return off;
        const int lg = ilog2i(n);
        const int64_t r0 = lg % 3 == 0 ? 8 : (int64_t(1) << (lg % 3));
        const int np = lg % 3 == 0 ? lg / 3 : lg / 3 + 1;
        int64_t Ns = r0;
        for (int ps = 1; ps < np; ++ps, Ns *= 8) {
            for (int i = 0; i < 3; ++i) {
                for (int64_t k = 0; k < Ns; ++k) {
                    double re, im;
                    root((k << i) * (n / (8 * Ns)), n, &re, &im);
                    if (A.dbl) {
                        double v[2] = {re, im};
                        blob.insert(blob.end(), (unsigned char*)v, (unsigned char*)v + 16);
                    } else {
                        float v[2] = {(float)re, (float)im};
                        blob.insert(blob.end(), (unsigned char*)v, (unsigned char*)v + 8);
                    }
                }
            }
        }
        return off;
    };
    A.off_m = small_table(A.d.m <= kMaxFused ? A.d.m : 1);
    A.off_m1 = small_table(A.d.m1);
    A.off_m2 = small_table(A.d.m2);
    A.off_p1 = pass_table(A.d.m1);
    A.off_p2 = pass_table(A.d.m2);
    A.tw.lgB = lgB;
    A.tw.mask = (int32_t)(B - 1);
}

void bind_tables(AxisPlan& A, unsigned char* base) {
    A.tw.lo = reinterpret_cast<const double2*>(base + A.off_lo);
    A.tw.hi = reinterpret_cast<const double2*>(base + A.off_hi);
    A.tw_m = base + A.off_m;
    A.tw_m1 = base + A.off_m1;
    A.tw_m2 = base + A.off_m2;
    A.tw_p1 = base + A.off_p1;
    A.tw_p2 = base + A.off_p2;
}

// ---------------------------------------------------------------- launches --

// Whole-row convolutions (variant 3) of nrows rows addressed by in / out.
hdc_status run_rowconv(const AxisPlan& A, const void* f, const void* g, void* h, int64_t nrows, RowAddr in,
                       RowAddr out, hipStream_t s) {
    if (nrows <= 0) return HDC_OK;
    FusedArgs a{};
    a.f = f;
    a.g = g;
    a.h = h;
    a.nrows = nrows;
    a.in = in;
    a.out = out;
    a.L = (int32_t)A.d.L;
    a.M = (int32_t)A.d.M;
    a.p = (int32_t)A.d.p;
    a.q = (int32_t)A.d.q;
    a.qout = (int32_t)A.d.q_out;
    a.N = (int32_t)A.d.N;
    a.rpw = A.rc_rpw;
    a.same = f == g ? 1 : 0;
    a.hiprec = A.hiprec ? 1 : 0;
    a.tw = A.tw;
    a.twm = A.tw_p2;  // the pass table of the m-point transform (m2 = m)
    a.invN = 1.0 / (double)A.d.N;
    a.R = 1;
    const int64_t blocks = ceil_div(nrows, A.rc_rpw);
    if (blocks > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "too many rows");
    const double eb = A.dbl ? 16.0 : 8.0;
    LaunchScope ls(s, 6, eb * (double)nrows * ((a.same ? 1.0 : 2.0) * (double)A.d.L + (double)A.d.M));
    hipError_t e = launch_rowconv(A.dbl, (int)A.d.m, a, A.rc_threads, blocks, A.rc_lds, s);
    if (e != hipSuccess) return hip_fail(e, "row convolution launch");
    return HDC_OK;
}

// Lf >= 0: f has length Lf and g the axis length, g's rows addressed by ing
// (section 3.5 with Lambda = 1).
hdc_status run_fused(const AxisPlan& A, const void* f, const void* g, void* h, int64_t nrows, RowAddr in, RowAddr out,
                     const int64_t* desc, hipStream_t s, int64_t Lf = -1, RowAddr ing = RowAddr{},
                     const void* const* xs = nullptr, int nops = 2) {
    if (nrows <= 0) return HDC_OK;
    FusedArgs a{};
    a.f = f;
    a.g = g;
    a.h = h;
    a.nrows = nrows;
    a.in = in;
    a.out = out;
    a.desc = desc;
    a.L = (int32_t)A.d.L;
    a.M = (int32_t)A.d.M;
    a.p = (int32_t)A.d.p;
    a.q = (int32_t)A.d.q;
    a.qout = (int32_t)A.d.q_out;
    a.N = (int32_t)A.d.N;
    a.Dc = A.Dc;
    a.rpw = A.f_rpw;
    a.same = (f == g && Lf < 0) ? 1 : 0;
    if (Lf >= 0) {
        a.L = (int32_t)Lf;
        a.Lg = (int32_t)A.d.L;
        a.ing = ing;
    }
    a.hiprec = A.hiprec ? 1 : 0;
    a.tw = A.tw;
    a.twm = A.tw_m;
    a.invN = 1.0 / (double)A.d.N;
    a.nops = nops;
    for (int o = 2; o < nops; ++o) a.xm[o - 2] = xs[o];
    a.R = (int32_t)odd_part(A.d.m);
    const int64_t blocks = ceil_div(nrows, A.f_rpw);
    if (blocks > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "too many rows");
    const double eb = A.dbl ? 16.0 : 8.0;
    const double lin = Lf >= 0 ? (double)(Lf + A.d.L)
                               : (a.same ? (double)(nops - 1) : (double)nops) * (double)A.d.L;
    LaunchScope ls(s, 0, eb * (double)nrows * (lin + (double)A.d.M));
    hipError_t e = launch_fused(A.dbl, (int)A.d.m, a, A.f_threads, blocks, A.f_lds, s);
    if (e != hipSuccess) return hip_fail(e, "fused convolution launch");
    return HDC_OK;
}

// Forward column stage of residues r0 + d (d < Dg).  With lam > 1 (section 3.5)
// every d also yields residues r0 + d + li rstride, li < lam, interleaved so
// that slot (d, l1, li) lands on row (d m1 + l1) lam + li.
hdc_status run_col_fwd(const AxisPlan& A, const void* x, void* X, int64_t B, int64_t in_bs, int64_t out_bs,
                       int64_t C1, int64_t r0, int64_t Dg, hipStream_t s, const int64_t* desc = nullptr,
                       int64_t lam = 1, int64_t rstride = 0, const void* x2 = nullptr, int64_t nsec = 0,
                       int64_t r2 = 0, const void* gs = nullptr) {
    ColFwdArgs a{};
    a.desc = desc;
    a.gs = gs;
    a.x = x;
    a.x2 = x2;
    a.nsec = (int32_t)nsec;
    a.r2 = (int32_t)r2;
    a.X = X;
    a.B = B;
    a.in_bs = in_bs;
    a.out_bs = out_bs;
    a.L = (int32_t)A.d.L;
    a.Ccols = (int32_t)(A.d.m2 * C1);
    a.C1 = (int32_t)C1;
    a.m2 = (int32_t)A.d.m2;
    a.m = (int32_t)A.d.m;
    a.q = (int32_t)A.d.q;
    a.p = (int32_t)A.d.p;
    a.N = (int32_t)A.d.N;
    a.r0 = (int32_t)r0;
    a.Dg = (int32_t)(Dg * lam);
    a.lam = (int32_t)lam;
    a.rstride = (int32_t)rstride;
    const bool real = x2 != nullptr;
    // the real-input kernel gives each thread 16 points (m1 >= 16) and runs at
    // most 512 threads: at most 8 columns per tile for m1 = 1024
    const int64_t tpf = real && A.d.m1 >= 16 ? A.d.m1 / 16 : A.d.m1 / ppt_for((int)A.d.m1);
    int rtile = A.cf_tile;
    while (real && rtile > 1 && rtile * tpf > 512) rtile /= 2;
    a.tile = rtile;
    a.ntiles = (int32_t)ceil_div(a.Ccols, a.tile);
    a.hiprec = A.hiprec ? 1 : 0;
    a.tw = A.tw;
    a.tw1 = A.tw_p1;
    const int64_t gx = round8((int64_t)a.ntiles * a.Dg);
    if (gx > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "column grid too large");
    const double eb = A.dbl ? 16.0 : 8.0;  // real: two inputs of L reals = L complex values
    const size_t esz = (A.dbl ? 16 : 8) / (real ? 2 : 1);
    LaunchScope ls(s, 1, eb * (double)B * (double)C1 * ((double)A.d.L + (double)(a.Dg * A.d.m)));
    for (int64_t b0 = 0; b0 < B; b0 += kMaxGridY) {  // the grid's y extent is limited
        ColFwdArgs c = a;
        c.B = std::min<int64_t>(kMaxGridY, B - b0);
        if (desc) c.desc = desc + 2 * b0;
        else c.x = (const char*)x + (size_t)(b0 * in_bs) * esz;
        if (real) c.x2 = (const char*)x2 + (size_t)(b0 * in_bs) * esz;
        c.X = (char*)X + (size_t)(b0 * out_bs) * (A.dbl ? 16 : 8);
        hipError_t e = launch_col_fwd(A.dbl, (int)A.d.m1, c, (int)(a.tile * tpf), gx, c.B,
                                      A.cf_lds / A.cf_tile * a.tile, s, real);
        if (e != hipSuccess) return hip_fail(e, "column forward launch");
    }
    return HDC_OK;
}

hdc_status run_col_bwd(const AxisPlan& A, const void* Y, void* h, int64_t B, int64_t in_bs, int64_t out_bs,
                       int64_t C1, int64_t r0, int64_t Dg, bool accumulate, hipStream_t s,
                       const int64_t* desc = nullptr, bool real = false, const void* gs = nullptr) {
    ColBwdArgs a{};
    a.desc = desc;
    a.gs = gs;
    a.Y = Y;
    a.h = h;
    a.B = B;
    a.in_bs = in_bs;
    a.out_bs = out_bs;
    a.M = (int32_t)A.d.M;
    a.Ccols = (int32_t)(A.d.m2 * C1);
    a.C1 = (int32_t)C1;
    a.m2 = (int32_t)A.d.m2;
    a.m = (int32_t)A.d.m;
    a.q = (int32_t)A.d.q;
    a.N = (int32_t)A.d.N;
    a.qout = (int32_t)A.d.q_out;
    a.r0 = (int32_t)r0;
    a.Dg = (int32_t)Dg;
    a.accumulate = accumulate ? 1 : 0;
    a.tile = A.cb_tile;
    a.ntiles = (int32_t)ceil_div(a.Ccols, A.cb_tile);
    a.hiprec = A.hiprec ? 1 : 0;
    a.tw = A.tw;
    a.tw1 = A.tw_p1;
    a.invN = 1.0 / (double)A.d.N;
    const double eb = A.dbl ? 16.0 : 8.0;
    const size_t esz = A.dbl ? 16 : 8;
    const size_t hsz = real ? esz / 2 : esz;  // real output: M reals per copy
    LaunchScope ls(s, 3, eb * (double)B * (double)C1 *
                             ((double)(Dg * A.d.m) + (accumulate ? 2.0 : 1.0) * (double)A.d.M * (real ? 0.5 : 1.0)));
    for (int64_t b0 = 0; b0 < B; b0 += kMaxGridY) {  // the grid's y extent is limited
        ColBwdArgs c = a;
        c.B = std::min<int64_t>(kMaxGridY, B - b0);
        c.Y = (const char*)Y + (size_t)(b0 * in_bs) * esz;
        if (desc) c.desc = desc + 2 * b0;
        else c.h = (char*)h + (size_t)(b0 * out_bs) * hsz;
        hipError_t e =
            launch_col_bwd(A.dbl, (int)A.d.m1, c, A.cb_threads, round8(a.ntiles), c.B, A.cb_lds, s, real);
        if (e != hipSuccess) return hip_fail(e, "column backward launch");
    }
    return HDC_OK;
}

// Plain strided m2-point DFTs of an outer axis split four-step: B slabs of
// [m2][cols], in place; sign +1 uses the forward column kernel with one
// residue and no twiddles, sign -1 the backward one with no 1/N scaling.
hdc_status run_col_plain(const AxisPlan& A, void* x, int64_t B, int64_t cols, int sign, hipStream_t s) {
    const int m2 = (int)A.d.m2;
    const int64_t bs = (int64_t)m2 * cols;
    if (B > kMaxGridY) {  // the grid's y extent is limited
        const size_t esz = A.dbl ? 16 : 8;
        for (int64_t b0 = 0; b0 < B; b0 += kMaxGridY) {
            hdc_status st = run_col_plain(A, (char*)x + (size_t)(b0 * bs) * esz, std::min<int64_t>(kMaxGridY, B - b0),
                                          cols, sign, s);
            if (st != HDC_OK) return st;
        }
        return HDC_OK;
    }
    const double eb = A.dbl ? 16.0 : 8.0;
    if (sign > 0) {
        ColFwdArgs a{};
        a.x = x;
        a.X = x;
        a.B = B;
        a.in_bs = bs;
        a.out_bs = bs;
        a.L = m2;
        a.Ccols = (int32_t)cols;
        a.C1 = (int32_t)cols;
        a.m2 = 1;
        a.m = m2;
        a.q = 1;
        a.p = 1;
        a.N = m2;
        a.r0 = 0;
        a.Dg = 1;
        a.lam = 1;
        a.rstride = 0;
        a.tile = A.mf_tile;
        a.ntiles = (int32_t)ceil_div(cols, A.mf_tile);
        a.hiprec = 0;
        a.tw = A.tw;
        a.tw1 = A.tw_p2;
        LaunchScope ls(s, 1, eb * 2.0 * (double)B * (double)bs);
        hipError_t e = launch_col_fwd(A.dbl, m2, a, A.mf_threads, round8(a.ntiles), B, A.mf_lds, s);
        if (e != hipSuccess) return hip_fail(e, "strided DFT launch");
        return HDC_OK;
    }
    ColBwdArgs a{};
    a.Y = x;
    a.h = x;
    a.B = B;
    a.in_bs = bs;
    a.out_bs = bs;
    a.M = m2;
    a.Ccols = (int32_t)cols;
    a.C1 = (int32_t)cols;
    a.m2 = 1;
    a.m = m2;
    a.q = 1;
    a.N = m2;
    a.qout = 1;
    a.r0 = 0;
    a.Dg = 1;
    a.accumulate = 0;
    a.tile = A.mb_tile;
    a.ntiles = (int32_t)ceil_div(cols, A.mb_tile);
    a.hiprec = 0;
    a.tw = A.tw;
    a.tw1 = A.tw_p2;
    a.invN = 1.0;
    LaunchScope ls(s, 3, eb * 2.0 * (double)B * (double)bs);
    hipError_t e = launch_col_bwd(A.dbl, m2, a, A.mb_threads, round8(a.ntiles), B, A.mb_lds, s);
    if (e != hipSuccess) return hip_fail(e, "strided inverse DFT launch");
    return HDC_OK;
}

// Rows of the residue buffer [B][Dg][m1][m2*C1]: row = ((b Dg + d) m1 + l1) C1 + c1.
hdc_status run_rows(const AxisPlan& A, const void* a_, const void* b_, void* out, int64_t nrows, int64_t C1, int mode,
                    hipStream_t s) {
    if (nrows <= 0) return HDC_OK;
    RowArgs a{};
    a.a = a_;
    a.b = b_;
    a.out = out;
    a.nrows = nrows;
    a.addr.inner_cnt = C1;
    a.addr.outer_stride = A.d.m2 * C1;
    a.addr.inner_stride = 1;
    a.addr.es = C1;
    a.mode = mode;
    a.same = (a_ == b_) ? 1 : 0;
    a.rpw = A.r_rpw;
    a.tw = A.tw_m2;
    a.twp = A.tw_p2;
    const int64_t blocks = ceil_div(nrows, A.r_rpw);
    if (blocks > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "too many rows");
    const double eb = A.dbl ? 16.0 : 8.0;
    const double nio = mode == MODE_CONV ? (a.same ? 2.0 : 3.0) : 2.0;
    LaunchScope ls(s, 2, eb * nio * (double)nrows * (double)A.d.m2);
    hipError_t e = launch_row(A.dbl, (int)A.d.m2, a, A.r_threads, blocks, A.r_lds, s);
    if (e != hipSuccess) return hip_fail(e, "row launch");
    return HDC_OK;
}

// Row pass of section 3.5 whose first operand is formed from the raw shorter
// operand xs (plan F, column stage trivial) for the group at r0; the second is
// the longer operand's column-stage output Xg (plan G); the product's inverse
// rows go to out.
hdc_status run_rows_raw(const AxisPlan& G, const AxisPlan& F, const void* xs, const void* Xg, void* out, int64_t nrows,
                        int64_t C1, int64_t r0, int64_t Dg, int64_t xs_bs, hipStream_t s) {
    if (nrows <= 0) return HDC_OK;
    RowArgs a{};
    a.a = nullptr;
    a.b = Xg;
    a.out = out;
    a.nrows = nrows;
    a.addr.inner_cnt = C1;
    a.addr.outer_stride = G.d.m2 * C1;
    a.addr.inner_stride = 1;
    a.addr.es = C1;
    a.mode = MODE_CONV;
    a.same = 0;
    a.rpw = G.r_rpw;
    a.tw = G.tw_m2;
    a.twp = G.tw_p2;
    a.fraw = xs;
    a.twN = F.tw;
    a.Lf = (int32_t)F.d.L;
    a.pf = (int32_t)F.d.p;
    a.qf = (int32_t)F.d.q;
    a.N = (int32_t)F.d.N;
    a.r0 = (int32_t)r0;
    a.qg = (int32_t)G.d.q;
    a.m1g = (int32_t)G.d.m1;
    a.Dg = (int32_t)Dg;
    a.fbs = xs_bs;
    a.hiprec = F.hiprec ? 1 : 0;
    const int64_t blocks = ceil_div(nrows, G.r_rpw);
    if (nrows > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "too many rows");
    const double eb = G.dbl ? 16.0 : 8.0;
    const double batches = (double)nrows / (double)(Dg * G.d.m1 * C1);
    LaunchScope ls(s, 2, eb * (2.0 * (double)nrows * (double)G.d.m2 + batches * (double)(F.d.L * C1)));
    hipError_t e = launch_row(G.dbl, (int)G.d.m2, a, G.r_threads, blocks, G.r_lds, s);
    if (e != hipSuccess) return hip_fail(e, "row launch");
    return HDC_OK;
}

size_t elem(const hdc_plan_s* P) { return elem_bytes(P->dtype); }

// Workspace (elements) of a 1D convolution of B rows x C1 copies on axis A.
int64_t ws1d(const AxisPlan& A, int64_t B, int64_t C1) {
    if (A.d.variant == 0 || A.d.variant == 3) return 0;
    const int64_t Dg = std::min(A.d.D, A.d.q);
    if (A.d.variant == 2) return B * Dg * A.d.m * C1;  // the product rows only
    return 2 * B * Dg * A.d.m * C1;
}

// The problem record of the raw-row path for axis A (plain mode).
RawProb raw_prob(const AxisPlan& A) {
    RawProb p{};
    p.L = (int32_t)A.d.L;
    p.M = (int32_t)A.d.M;
    p.p = (int32_t)A.d.p;
    p.q = (int32_t)A.d.q;
    p.qout = (int32_t)A.d.q_out;
    p.hiprec = A.hiprec ? 1 : 0;
    p.tw = A.tw;
    p.invN = 1.0 / (double)A.d.N;
    return p;
}

// Raw residue rows of group [r0, r0 + Dg) for B batches of C1 copies into Y,
// then the output sums into h (added to h for r0 > 0).
hdc_status run_raw_group(const AxisPlan& A, const void* xf, const void* xg, void* Y, void* out, int64_t B,
                         int64_t in_bs, int64_t out_bs, int64_t C1, int64_t r0, int64_t Dg, hipStream_t s) {
    RawArgs a{};
    a.f = xf;
    a.g = xg;
    a.Y = Y;
    a.h = out;
    a.m = (int32_t)A.d.m;
    a.rpw = A.r_rpw;
    a.C1 = (int32_t)C1;
    a.Dg = (int32_t)Dg;
    a.r0 = (int32_t)r0;
    a.same = xf == xg ? 1 : 0;
    a.accumulate = r0 > 0 ? 1 : 0;
    a.fbs = in_bs;
    a.ybs = Dg * A.d.m * C1;
    a.hbs = out_bs;
    a.p0 = raw_prob(A);
    a.twp = A.tw_p2;
    a.nrows = B * Dg * C1;
    const double eb = A.dbl ? 16.0 : 8.0;
    {
        const int64_t blocks = ceil_div(a.nrows, A.r_rpw);
        if (a.nrows > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "too many rows");
        // compulsory: the inputs once, the product rows written
        LaunchScope ls(s, 4, eb * (double)B * (double)C1 * ((a.same ? 1.0 : 2.0) * (double)A.d.L + (double)(Dg * A.d.m)));
        hipError_t e = launch_row_rr(A.dbl, (int)A.d.m, a, A.r_threads, blocks, A.r_lds, s);
        if (e != hipSuccess) return hip_fail(e, "raw row launch");
    }
    const int64_t gx = ceil_div(A.d.m * C1, 256);
    if (B > kMaxGridY) return fail(HDC_ERR_UNSUPPORTED, "too many batches for the output sums");
    LaunchScope ls(s, 5, eb * (double)B * (double)C1 * ((double)(Dg * A.d.m) + (r0 > 0 ? 2.0 : 1.0) * (double)A.d.M));
    hipError_t e = launch_qsum(A.dbl, a, gx, B, s);
    if (e != hipSuccess) return hip_fail(e, "output sum launch");
    return HDC_OK;
}

// 1D convolution along axis A: B batches (strides in_bs / out_bs) of C1 interleaved copies.
hdc_status conv1d(const AxisPlan& A, const void* xf, const void* xg, void* out, int64_t B, int64_t in_bs, int64_t out_bs,
                  int64_t C1, char* ws, size_t eb, hipStream_t s) {
    if (A.d.variant == 0 || A.d.variant == 3) {
        RowAddr in{C1, in_bs, 1, C1};
        RowAddr ou{C1, out_bs, 1, C1};
        if (A.d.variant == 3) return run_rowconv(A, xf, xg, out, B * C1, in, ou, s);
        return run_fused(A, xf, xg, out, B * C1, in, ou, nullptr, s);
    }
    const bool same = xf == xg;
    const int64_t D = std::min(A.d.D, A.d.q);
    if (A.d.variant == 2) {
        for (int64_t r0 = 0; r0 < A.d.q; r0 += D) {
            hdc_status st = run_raw_group(A, xf, xg, ws, out, B, in_bs, out_bs, C1, r0, std::min(D, A.d.q - r0), s);
            if (st != HDC_OK) return st;
        }
        return HDC_OK;
    }
    char* Xf = ws;
    char* Xg = same ? ws : ws + (size_t)(B * D * A.d.m * C1) * eb;
    for (int64_t r0 = 0; r0 < A.d.q; r0 += D) {
        const int64_t Dg = std::min(D, A.d.q - r0);
        const int64_t xbs = Dg * A.d.m * C1;
        hdc_status st = run_col_fwd(A, xf, Xf, B, in_bs, xbs, C1, r0, Dg, s);
        if (st != HDC_OK) return st;
        if (!same) {
            st = run_col_fwd(A, xg, Xg, B, in_bs, xbs, C1, r0, Dg, s);
            if (st != HDC_OK) return st;
        }
        st = run_rows(A, Xf, Xg, Xf, B * Dg * A.d.m1 * C1, C1, MODE_CONV, s);
        if (st != HDC_OK) return st;
        st = run_col_bwd(A, Xf, out, B, xbs, out_bs, C1, r0, Dg, r0 > 0, s);
        if (st != HDC_OK) return st;
    }
    return HDC_OK;
}

// ---------------------------------------------------------------- real data --
//
// Real f and g (the real case section 7 leaves to future work): the complex
// sequence z = f + i g is transformed once.  Because f and g are real,
// F_k = (Z_k + conj Z_{N-k}) / 2 and G_k = (Z_k - conj Z_{N-k}) / (2i), and with
// k = q l + r the index N - k lies in residue q - r (residue 0 for r = 0).  The
// product H is Hermitian, so only residues r <= q/2 are formed and inverted; the
// backward sums them with weight 2 (1 for r = 0 and r = q/2) and keeps the real
// part.  A pass over the group [r0, r0 + Dg) of those residues transforms Z for
// the group and for the partners q - r it needs.

struct RealGroup {
    int64_t Dg, pfirst, npart;  // residues r0 .. r0+Dg-1; partners q - pfirst, q - pfirst - 1, ...
};

RealGroup real_group(const hdc_axis_desc& d, int64_t r0) {
    const int64_t qh = d.q / 2 + 1;
    const int64_t D = std::min(d.D, qh);
    RealGroup g{};
    g.Dg = std::min(D, qh - r0);
    g.pfirst = std::max<int64_t>(r0, 1);
    const int64_t plast = std::min(r0 + g.Dg - 1, (d.q - 1) / 2);
    g.npart = std::max<int64_t>(0, plast - g.pfirst + 1);
    return g;
}

// Workspace (complex elements) of the column/row/column real convolution:
// Z (Dg + npart slots) and the product rows (Dg slots) of the largest group.
int64_t ws_real(const AxisPlan& A, int64_t B, int64_t C1) {
    if (A.d.variant == 0) return 0;
    const int64_t qh = A.d.q / 2 + 1;
    const int64_t D = std::min(A.d.D, qh);
    int64_t slots = 0;
    for (int64_t r0 = 0; r0 < qh; r0 += D) {
        const RealGroup g = real_group(A.d, r0);
        slots = std::max(slots, 2 * g.Dg + g.npart);
    }
    return B * slots * A.d.m * C1;
}

hdc_status run_fused_real(const AxisPlan& A, const void* f, const void* g, void* h, int64_t nrows, RowAddr in,
                          RowAddr out, hipStream_t s) {
    if (nrows <= 0) return HDC_OK;
    FusedArgs a{};
    a.f = f;
    a.g = g;
    a.h = h;
    a.nrows = nrows;
    a.in = in;
    a.out = out;
    a.L = (int32_t)A.d.L;
    a.M = (int32_t)A.d.M;
    a.p = (int32_t)A.d.p;
    a.q = (int32_t)A.d.q;
    a.qout = (int32_t)A.d.q_out;
    a.N = (int32_t)A.d.N;
    a.Dc = A.Dc;
    a.rpw = A.f_rpw;
    a.hiprec = A.hiprec ? 1 : 0;
    a.tw = A.tw;
    a.twm = A.tw_m;
    a.invN = 1.0 / (double)A.d.N;
    const int64_t blocks = ceil_div(nrows, A.f_rpw);
    if (blocks > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "too many rows");
    const double rb = A.dbl ? 8.0 : 4.0;  // bytes per real value
    LaunchScope ls(s, 0, rb * (double)nrows * (2.0 * (double)A.d.L + (double)A.d.M));
    hipError_t e = launch_fused_real(A.dbl, (int)A.d.m, a, A.f_threads, blocks, A.f_lds, s);
    if (e != hipSuccess) return hip_fail(e, "fused real convolution launch");
    return HDC_OK;
}

// Product rows of the group at r0: Z has S = Dg + npart slots per batch, the
// output Dg slots; row ((b Dg + d) m1 + l1) C1 + c1.  The residues 0 and q/2
// pair rows of their own (one work item gives rows l1 and its mirror), so the
// launch covers m1/2 + 1 (residue 0) and m1/2 (q/2) items for them, m1 for the
// others (one item each when m1 = 1).
hdc_status run_rows_real(const AxisPlan& A, const void* Z, void* O, int64_t B, int64_t C1, int64_t r0,
                         const RealGroup& g, hipStream_t s) {
    const int64_t m1 = A.d.m1, q = A.d.q;
    const int64_t n0 = m1 == 1 ? 1 : m1 / 2 + 1, nh = m1 == 1 ? 1 : m1 / 2;
    const bool has0 = r0 == 0;
    const bool hash = q % 2 == 0 && r0 + g.Dg - 1 == q / 2 && q / 2 != 0;
    const int64_t W = g.Dg * m1 - (has0 ? m1 - n0 : 0) - (hash ? m1 - nh : 0);
    const int64_t nrows = B * W * C1;
    if (nrows <= 0) return HDC_OK;
    RowArgs a{};
    a.a = Z;
    a.out = O;
    a.nrows = nrows;
    a.addr.inner_cnt = C1;
    a.addr.outer_stride = A.d.m2 * C1;
    a.addr.inner_stride = 1;
    a.addr.es = C1;
    a.mode = MODE_CONV;
    a.rpw = A.r_rpw;
    a.tw = A.tw_m2;
    a.twp = A.tw_p2;
    a.r0 = (int32_t)r0;
    a.qg = (int32_t)A.d.q;
    a.m1g = (int32_t)A.d.m1;
    a.Dg = (int32_t)g.Dg;
    a.S = (int32_t)(g.Dg + g.npart);
    a.pfirst = (int32_t)g.pfirst;
    const int64_t blocks = ceil_div(nrows, A.r_rpw);
    if (blocks > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "too many rows");
    // algorithmic bytes: a self-paired residue reads and writes each of its m1
    // rows once, any other reads its rows and its partner's and writes its own
    const double eb = A.dbl ? 16.0 : 8.0;
    const int64_t nself = (has0 ? 1 : 0) + (hash ? 1 : 0);
    const double rows_rw = (double)(2 * nself + 3 * (g.Dg - nself)) * (double)(m1 * C1 * B);
    LaunchScope ls(s, 2, eb * rows_rw * (double)A.d.m2);
    hipError_t e = launch_row_real(A.dbl, (int)A.d.m2, a, A.r_threads, blocks, A.r_lds, s);
    if (e != hipSuccess) return hip_fail(e, "real row launch");
    return HDC_OK;
}

// Real 1D convolution along axis A: B batches (strides in_bs / out_bs, in real
// elements) of C1 interleaved copies.
hdc_status conv1d_real(const AxisPlan& A, const void* xf, const void* xg, void* out, int64_t B, int64_t in_bs,
                       int64_t out_bs, int64_t C1, char* ws, size_t eb, hipStream_t s) {
    if (A.d.variant == 0) {
        RowAddr in{C1, in_bs, 1, C1};
        RowAddr ou{C1, out_bs, 1, C1};
        return run_fused_real(A, xf, xg, out, B * C1, in, ou, s);
    }
    const int64_t qh = A.d.q / 2 + 1;
    const int64_t D = std::min(A.d.D, qh);
    for (int64_t r0 = 0; r0 < qh; r0 += D) {
        const RealGroup g = real_group(A.d, r0);
        const int64_t S = g.Dg + g.npart;
        char* Z = ws;
        char* O = ws + (size_t)(B * S * A.d.m * C1) * eb;
        hdc_status st = run_col_fwd(A, xf, Z, B, in_bs, S * A.d.m * C1, C1, r0, S, s, nullptr, 1, 0, xg, g.npart,
                                    A.d.q - g.pfirst);
        if (st != HDC_OK) return st;
        st = run_rows_real(A, Z, O, B, C1, r0, g, s);
        if (st != HDC_OK) return st;
        st = run_col_bwd(A, O, out, B, g.Dg * A.d.m * C1, out_bs, C1, r0, g.Dg, r0 > 0, s, nullptr, true);
        if (st != HDC_OK) return st;
    }
    return HDC_OK;
}

// ------------------------------------------------------- multi-convolution --
//
// The convolution of A >= 2 sequences (section 6.1): every residue of every
// operand is formed as in eq. (3), the A residues multiply pointwise, and one
// backward, eq. (4), gives h.  The transform must cover the A(L - 1) + 1 terms.

// Rows of the A residue buffers of a group: operand o's at X + o ostride; the
// product overwrites operand 0's.
hdc_status run_rows_multi(const AxisPlan& A, void* X, int64_t ostride, int64_t nrows, int64_t C1, int nops,
                          hipStream_t s) {
    if (nrows <= 0) return HDC_OK;
    RowArgs a{};
    a.a = X;
    a.out = X;
    a.nrows = nrows;
    a.addr.inner_cnt = C1;
    a.addr.outer_stride = A.d.m2 * C1;
    a.addr.inner_stride = 1;
    a.addr.es = C1;
    a.mode = MODE_CONV;
    a.rpw = A.r_rpw;
    a.tw = A.tw_m2;
    a.twp = A.tw_p2;
    a.nops = nops;
    a.ostride = ostride;
    const int64_t blocks = ceil_div(nrows, A.r_rpw);
    if (blocks > 0x7fffffff) return fail(HDC_ERR_UNSUPPORTED, "too many rows");
    const double eb = A.dbl ? 16.0 : 8.0;
    LaunchScope ls(s, 2, eb * (double)(nops + 1) * (double)nrows * (double)A.d.m2);
    hipError_t e = launch_row_multi(A.dbl, (int)A.d.m2, a, A.r_threads, blocks, A.r_lds, s);
    if (e != hipSuccess) return hip_fail(e, "multi row launch");
    return HDC_OK;
}

int64_t ws_multi(const AxisPlan& A, int nops, int64_t B, int64_t C1) {
    if (A.d.variant == 0) return 0;
    return (int64_t)nops * B * std::min(A.d.D, A.d.q) * A.d.m * C1;
}

hdc_status conv1d_multi(const AxisPlan& A, const void* const* xs, int nops, void* out, int64_t B, int64_t in_bs,
                        int64_t out_bs, int64_t C1, char* ws, size_t eb, hipStream_t s) {
    if (A.d.variant == 0) {
        RowAddr in{C1, in_bs, 1, C1};
        RowAddr ou{C1, out_bs, 1, C1};
        return run_fused(A, xs[0], xs[1], out, B * C1, in, ou, nullptr, s, -1, RowAddr{}, xs, nops);
    }
    const int64_t D = std::min(A.d.D, A.d.q);
    const int64_t ostride = B * D * A.d.m * C1;
    for (int64_t r0 = 0; r0 < A.d.q; r0 += D) {
        const int64_t Dg = std::min(D, A.d.q - r0);
        const int64_t xbs = Dg * A.d.m * C1;
        for (int o = 0; o < nops; ++o) {
            hdc_status st = run_col_fwd(A, xs[o], ws + (size_t)(o * ostride) * eb, B, in_bs, xbs, C1, r0, Dg, s);
            if (st != HDC_OK) return st;
        }
        hdc_status st = run_rows_multi(A, ws, ostride, B * Dg * A.d.m1 * C1, C1, nops, s);
        if (st != HDC_OK) return st;
        st = run_col_bwd(A, ws, out, B, xbs, out_bs, C1, r0, Dg, r0 > 0, s);
        if (st != HDC_OK) return st;
    }
    return HDC_OK;
}

int64_t prod_L(const hdc_plan_s* P, int from) {
    int64_t v = 1;
    for (int a = from; a < P->ndim; ++a) v *= P->ax[a].d.L;
    return v;
}
int64_t prod_M(const hdc_plan_s* P, int from) {
    int64_t v = 1;
    for (int a = from; a < P->ndim; ++a) v *= P->ax[a].d.M;
    return v;
}

// Workspace (elements) of the N-D recursion from `level` with B batches.
int64_t wsnd(const hdc_plan_s* P, int level, int64_t B) {
    const AxisPlan& A = P->ax[level];
    if (level == P->ndim - 1) return ws1d(A, B, 1);
    const int64_t Dg = std::min(A.d.D, A.d.q);
    const int64_t inner_in = prod_L(P, level + 1), inner_out = prod_M(P, level + 1);
    const int64_t nb = B * Dg * A.d.m;
    return 2 * nb * inner_in + nb * inner_out + wsnd(P, level + 1, nb);
}

// Section 3.6: forward along the outer axis for a residue group, recurse on the
// inner (N-1)-D problem for every residue row, backward along the outer axis.
hdc_status convnd(const hdc_plan_s* P, int level, const void* xf, const void* xg, void* out, int64_t B, char* ws,
                  hipStream_t s) {
    const AxisPlan& A = P->ax[level];
    const size_t eb = elem(P);
    if (level == P->ndim - 1) return conv1d(A, xf, xg, out, B, A.d.L, A.d.M, 1, ws, eb, s);
    const bool same = xf == xg;
    const int64_t D = std::min(A.d.D, A.d.q);
    const int64_t inner_in = prod_L(P, level + 1), inner_out = prod_M(P, level + 1);
    const int64_t nbmax = B * D * A.d.m;
    char* Xf = ws;
    char* Xg = ws + (size_t)(nbmax * inner_in) * eb;
    char* Y = Xg + (size_t)(nbmax * inner_in) * eb;
    char* rest = Y + (size_t)(nbmax * inner_out) * eb;
    for (int64_t r0 = 0; r0 < A.d.q; r0 += D) {
        const int64_t Dg = std::min(D, A.d.q - r0);
        const int64_t nb = B * Dg * A.d.m;
        // block sums, m1-point DFTs and four-step twiddles (copies = the inner extent)
        hdc_status st = run_col_fwd(A, xf, Xf, B, A.d.L * inner_in, Dg * A.d.m * inner_in, inner_in, r0, Dg, s);
        if (st == HDC_OK && !same)
            st = run_col_fwd(A, xg, Xg, B, A.d.L * inner_in, Dg * A.d.m * inner_in, inner_in, r0, Dg, s);
        // the remaining m2-point DFTs of a long outer axis, in place
        if (st == HDC_OK && A.d.m2 > 1) {
            st = run_col_plain(A, Xf, B * Dg * A.d.m1, inner_in, +1, s);
            if (st == HDC_OK && !same) st = run_col_plain(A, Xg, B * Dg * A.d.m1, inner_in, +1, s);
        }
        if (st == HDC_OK) st = convnd(P, level + 1, Xf, same ? Xf : Xg, Y, nb, rest, s);
        if (st == HDC_OK && A.d.m2 > 1) st = run_col_plain(A, Y, B * Dg * A.d.m1, inner_out, -1, s);
        if (st == HDC_OK)
            st = run_col_bwd(A, Y, out, B, Dg * A.d.m * inner_out, A.d.M * inner_out, inner_out, r0, Dg, r0 > 0, s);
        if (st != HDC_OK) return st;
    }
    return HDC_OK;
}

// Real f, g of an N-D plan (section 3.6 with z = f + i s g): the outer axis's
// forward column passes read f and s g as z, the inner axes run the complex
// autoconvolution of its residue rows, and the outer backward writes
// h = Im(z * z) / (2 s) (the convolution is bilinear: z * z = f * f - s^2 g * g
// + 2 i s f * g).
hdc_status convnd_real(const hdc_plan_s* P, const void* f, const void* g, void* out, const void* mx, char* ws,
                       hipStream_t s) {
    const AxisPlan& A = P->ax[0];
    const size_t eb = elem(P);
    const int64_t D = std::min(A.d.D, A.d.q);
    const int64_t inner_in = prod_L(P, 1), inner_out = prod_M(P, 1);
    const int64_t nbmax = D * A.d.m;
    char* X = ws;
    char* Y = ws + (size_t)(2 * nbmax * inner_in) * eb;  // the complex plan's layout (its Xg unused)
    char* rest = Y + (size_t)(nbmax * inner_out) * eb;
    for (int64_t r0 = 0; r0 < A.d.q; r0 += D) {
        const int64_t Dg = std::min(D, A.d.q - r0);
        const int64_t nb = Dg * A.d.m;
        hdc_status st = run_col_fwd(A, f, X, 1, A.d.L * inner_in, Dg * A.d.m * inner_in, inner_in, r0, Dg, s, nullptr,
                                    1, 0, g, 0, 0, mx);
        if (st == HDC_OK && A.d.m2 > 1) st = run_col_plain(A, X, Dg * A.d.m1, inner_in, +1, s);
        if (st == HDC_OK) st = convnd(P, 1, X, X, Y, nb, rest, s);
        if (st == HDC_OK && A.d.m2 > 1) st = run_col_plain(A, Y, Dg * A.d.m1, inner_out, -1, s);
        if (st == HDC_OK)
            st = run_col_bwd(A, Y, out, 1, Dg * A.d.m * inner_out, A.d.M * inner_out, inner_out, r0, Dg, r0 > 0, s,
                             nullptr, true, mx);
        if (st != HDC_OK) return st;
    }
    return HDC_OK;
}

// Multi-convolution in N-D (section 6.1 with section 3.6's recursion): the
// outer axis's residue group of every operand, the inner (N-1)-D
// multi-convolution per residue row, the outer backward.
int64_t wsnd_multi(const hdc_plan_s* P, int level, int64_t B) {
    const AxisPlan& A = P->ax[level];
    if (level == P->ndim - 1) return P->nops == 2 ? ws1d(A, B, 1) : ws_multi(A, P->nops, B, 1);
    const int64_t Dg = std::min(A.d.D, A.d.q);
    const int64_t inner_in = prod_L(P, level + 1), inner_out = prod_M(P, level + 1);
    const int64_t nb = B * Dg * A.d.m;
    return (int64_t)P->nops * nb * inner_in + nb * inner_out + wsnd_multi(P, level + 1, nb);
}

hdc_status convnd_multi(const hdc_plan_s* P, int level, const void* const* xs, void* out, int64_t B, char* ws,
                        hipStream_t s) {
    const AxisPlan& A = P->ax[level];
    const size_t eb = elem(P);
    const int nops = P->nops;
    if (level == P->ndim - 1) {
        if (nops == 2) return conv1d(A, xs[0], xs[1], out, B, A.d.L, A.d.M, 1, ws, eb, s);
        return conv1d_multi(A, xs, nops, out, B, A.d.L, A.d.M, 1, ws, eb, s);
    }
    const int64_t D = std::min(A.d.D, A.d.q);
    const int64_t inner_in = prod_L(P, level + 1), inner_out = prod_M(P, level + 1);
    const int64_t nbmax = B * D * A.d.m;
    const void* X[kMaxOps];
    for (int o = 0; o < nops; ++o) X[o] = ws + (size_t)(o * nbmax * inner_in) * eb;
    char* Y = ws + (size_t)(nops * nbmax * inner_in) * eb;
    char* rest = Y + (size_t)(nbmax * inner_out) * eb;
    for (int64_t r0 = 0; r0 < A.d.q; r0 += D) {
        const int64_t Dg = std::min(D, A.d.q - r0);
        const int64_t nb = B * Dg * A.d.m;
        hdc_status st = HDC_OK;
        for (int o = 0; o < nops && st == HDC_OK; ++o) {
            st = run_col_fwd(A, xs[o], (void*)X[o], B, A.d.L * inner_in, Dg * A.d.m * inner_in, inner_in, r0, Dg, s);
            if (st == HDC_OK && A.d.m2 > 1) st = run_col_plain(A, (void*)X[o], B * Dg * A.d.m1, inner_in, +1, s);
        }
        if (st == HDC_OK) st = convnd_multi(P, level + 1, X, Y, nb, rest, s);
        if (st == HDC_OK && A.d.m2 > 1) st = run_col_plain(A, Y, B * Dg * A.d.m1, inner_out, -1, s);
        if (st == HDC_OK)
            st = run_col_bwd(A, Y, out, B, Dg * A.d.m * inner_out, A.d.M * inner_out, inner_out, r0, Dg, r0 > 0, s);
        if (st != HDC_OK) return st;
    }
    return HDC_OK;
}

// Section 3.5: for every residue group of the longer operand, the shorter
// operand's matching residues r_f = q_g lambda + r_g (lambda < Lambda) are
// formed by its own column stage, stored row-interleaved so that the row pass
// multiplies row by row; the backward runs in the longer operand's geometry.
// Section 3.5 along one axis for B batches of C1 interleaved copies: xs is the
// operand that is shorter on this axis (plan F, m-point residues), xl the
// longer one (plan G, Lambda m-point residues), batch strides xs_bs, xl_bs and
// out_bs.  With Lambda = 1 and a transform that fits one workgroup, the single
// fused kernel runs (both operands share m); with the shorter operand's column
// stage trivial (m1f = 1), the row pass forms its rows from the raw input;
// otherwise both column stages run, the shorter one's residues r_f = q_g lambda
// + r_g stored row-interleaved so that the row pass multiplies row by row.
hdc_status conv_uneq(const AxisPlan& G, const AxisPlan& F, int64_t lam, const void* xs, const void* xl, void* out,
                     int64_t B, int64_t xs_bs, int64_t xl_bs, int64_t out_bs, int64_t C1, char* ws, size_t eb,
                     hipStream_t s) {
    if (G.d.variant == 0) {
        RowAddr is{C1, xs_bs, 1, C1}, il{C1, xl_bs, 1, C1}, io{C1, out_bs, 1, C1};
        return run_fused(G, xs, xl, out, B * C1, is, io, nullptr, s, F.d.L, il);
    }
    const int64_t D = std::min(G.d.D, G.d.q);
    const bool raw = F.d.m1 == 1;
    char* Xg = ws;
    char* Xf = ws + (size_t)(B * D * G.d.m * C1) * eb;
    for (int64_t r0 = 0; r0 < G.d.q; r0 += D) {
        const int64_t Dg = std::min(D, G.d.q - r0);
        const int64_t xbs = Dg * G.d.m * C1;
        const int64_t rows = B * Dg * G.d.m1 * C1;
        hdc_status st = run_col_fwd(G, xl, Xg, B, xl_bs, xbs, C1, r0, Dg, s);
        if (st == HDC_OK) {
            if (raw) {
                st = run_rows_raw(G, F, xs, Xg, Xg, rows, C1, r0, Dg, xs_bs, s);
            } else {
                st = run_col_fwd(F, xs, Xf, B, xs_bs, xbs, C1, r0, Dg, s, nullptr, lam, G.d.q);
                if (st == HDC_OK) st = run_rows(G, Xf, Xg, Xg, rows, C1, MODE_CONV, s);
            }
        }
        if (st == HDC_OK) st = run_col_bwd(G, Xg, out, B, xbs, out_bs, C1, r0, Dg, r0 > 0, s);
        if (st != HDC_OK) return st;
    }
    return HDC_OK;
}

// Workspace (elements) of conv_uneq for B batches of C1 copies.
int64_t ws_uneq(const AxisPlan& G, const AxisPlan& F, int64_t B, int64_t C1) {
    if (G.d.variant == 0) return 0;
    const int64_t one = B * std::min(G.d.D, G.d.q) * G.d.m * C1;
    return F.d.m1 == 1 ? one : 2 * one;
}

int64_t prod3(const int64_t* L, int from, int ndim) {
    int64_t v = 1;
    for (int a = from; a < ndim; ++a) v *= L[a];
    return v;
}

// Workspace (elements) of the unequal N-D recursion from `level` with B batches.
int64_t wsnd_uneq(const hdc_plan_s* P, int level, int64_t B) {
    const AxisPlan& G = P->ax[level];
    if (level == P->ndim - 1) return ws_uneq(G, P->fx[level], B, 1);
    const int64_t Dg = std::min(G.d.D, G.d.q);
    const int64_t nb = B * Dg * G.d.m;
    const int64_t inf = prod3(P->Lf, level + 1, P->ndim), ing = prod3(P->Lg, level + 1, P->ndim);
    int64_t inner_out = 1;
    for (int a = level + 1; a < P->ndim; ++a) inner_out *= P->ax[a].d.M;
    return nb * (inf + ing + inner_out) + wsnd_uneq(P, level + 1, nb);
}

// Section 3.6 with section 3.5's lengths: along the outer axis, for each residue
// group of the longer operand, the forward column stages of both operands (the
// shorter one in its matching residue slots), the remaining strided m2-point
// DFTs, the inner (N-1)-D unequal problem for every row pair, and the backward
// along the outer axis in the longer operand's geometry.
hdc_status convnd_uneq(const hdc_plan_s* P, int level, const void* xf, const void* xg, void* out, int64_t B, char* ws,
                       hipStream_t s) {
    const AxisPlan& G = P->ax[level];
    const AxisPlan& F = P->fx[level];
    const bool sw = P->swap[level];
    const size_t eb = elem(P);
    if (level == P->ndim - 1) {
        const int64_t Lf = P->Lf[level], Lg = P->Lg[level];
        return sw ? conv_uneq(G, F, P->lam[level], xg, xf, out, B, Lg, Lf, G.d.M, 1, ws, eb, s)
                  : conv_uneq(G, F, P->lam[level], xf, xg, out, B, Lf, Lg, G.d.M, 1, ws, eb, s);
    }
    const int64_t D = std::min(G.d.D, G.d.q);
    const int64_t inf = prod3(P->Lf, level + 1, P->ndim), ing = prod3(P->Lg, level + 1, P->ndim);
    int64_t inner_out = 1;
    for (int a = level + 1; a < P->ndim; ++a) inner_out *= P->ax[a].d.M;
    const int64_t nbmax = B * D * G.d.m;
    char* Xf = ws;
    char* Xg = Xf + (size_t)(nbmax * inf) * eb;
    char* Y = Xg + (size_t)(nbmax * ing) * eb;
    char* rest = Y + (size_t)(nbmax * inner_out) * eb;
    const AxisPlan& Af = sw ? G : F;  // plan of f on this axis
    const AxisPlan& Ag = sw ? F : G;
    for (int64_t r0 = 0; r0 < G.d.q; r0 += D) {
        const int64_t Dg = std::min(D, G.d.q - r0);
        const int64_t nb = B * Dg * G.d.m;
        hdc_status st = sw ? run_col_fwd(Af, xf, Xf, B, P->Lf[level] * inf, Dg * G.d.m * inf, inf, r0, Dg, s)
                           : run_col_fwd(Af, xf, Xf, B, P->Lf[level] * inf, Dg * G.d.m * inf, inf, r0, Dg, s, nullptr,
                                         P->lam[level], G.d.q);
        if (st == HDC_OK)
            st = sw ? run_col_fwd(Ag, xg, Xg, B, P->Lg[level] * ing, Dg * G.d.m * ing, ing, r0, Dg, s, nullptr,
                                  P->lam[level], G.d.q)
                    : run_col_fwd(Ag, xg, Xg, B, P->Lg[level] * ing, Dg * G.d.m * ing, ing, r0, Dg, s);
        if (st == HDC_OK && G.d.m2 > 1) {
            st = run_col_plain(Af, Xf, B * Dg * G.d.m1, inf, +1, s);
            if (st == HDC_OK) st = run_col_plain(Ag, Xg, B * Dg * G.d.m1, ing, +1, s);
        }
        if (st == HDC_OK) st = convnd_uneq(P, level + 1, Xf, Xg, Y, nb, rest, s);
        if (st == HDC_OK && G.d.m2 > 1) st = run_col_plain(G, Y, B * Dg * G.d.m1, inner_out, -1, s);
        if (st == HDC_OK)
            st = run_col_bwd(G, Y, out, B, Dg * G.d.m * inner_out, G.d.M * inner_out, inner_out, r0, Dg, r0 > 0, s);
        if (st != HDC_OK) return st;
    }
    return HDC_OK;
}

// Derivation and kernel geometry of axis a of an unequal-length plan.
hdc_status uneq_axis(hdc_plan_s* P, int a, int64_t Lf, int64_t Lg, int64_t M, int64_t m, int64_t lam, int64_t C,
                     int64_t D, bool outer, bool many_rows) {
    bool sw = false;
    AxisPlan& G = P->ax[a];
    AxisPlan& F = P->fx[a];
    hdc_status st = derive_uneq(Lf, Lg, M, m, lam, C, D, P->dtype, &F.d, &G.d, &sw, outer, many_rows);
    if (st != HDC_OK) return st;
    P->swap[a] = sw;
    P->lam[a] = G.d.m / F.d.m;
    G.dbl = F.dbl = P->dtype == HDC_C128;
    const int32_t var = G.d.variant;
    st = geometry(G, outer, many_rows, true);
    if (st == HDC_OK) st = geometry(F, outer, false, true);
    // the fused kernel serves Lambda = 1 only; geometry() may have allowed it
    // the whole LDS for the many rows of an innermost N-D axis
    (void)var;
    G.d.variant = (!outer && P->lam[a] == 1 && G.d.variant == 0) ? 0 : 1;
    F.d.variant = 1;
    return st;
}

hdc_status finish_plan(hdc_plan_s* P) {
    std::vector<unsigned char> blob;
    for (int a = 0; a < P->ndim; ++a) stage_tables(P->ax[a], blob);
    if (P->uneq)
        for (int a = 0; a < P->ndim; ++a) stage_tables(P->fx[a], blob);
    void* dev = nullptr;
    hipError_t e = hipMalloc(&dev, std::max<size_t>(blob.size(), 256));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(twiddle tables)");
    e = hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "hipMemcpy(twiddle tables)");
    }
    P->tables = dev;
    for (int a = 0; a < P->ndim; ++a) bind_tables(P->ax[a], (unsigned char*)dev);
    if (P->uneq)
        for (int a = 0; a < P->ndim; ++a) bind_tables(P->fx[a], (unsigned char*)dev);
    if (P->uneq) {
        P->ws_bytes = (size_t)(P->ndim == 1 ? ws_uneq(P->ax[0], P->fx[0], 1, P->ax[0].d.C) : wsnd_uneq(P, 0, 1)) *
                      elem(P);
    } else if (P->real) {
        P->ws_bytes = (size_t)ws_real(P->ax[0], 1, P->ax[0].d.C) * elem(P);
    } else if (P->nops > 2 && P->ndim > 1) {
        P->ws_bytes = (size_t)wsnd_multi(P, 0, 1) * elem(P);
    } else if (P->nops > 2) {
        P->ws_bytes = (size_t)ws_multi(P->ax[0], P->nops, 1, P->ax[0].d.C) * elem(P);
    } else if (P->ndim == 1) {
        P->ws_bytes = (size_t)ws1d(P->ax[0], 1, P->ax[0].d.C) * elem(P);
    } else if (P->real_nd) {
        // the two scale words, then the N-D workspace
        P->ws_bytes = 256 + (size_t)wsnd(P, 0, 1) * elem(P);
    } else {
        P->ws_bytes = (size_t)wsnd(P, 0, 1) * elem(P);
    }
    return HDC_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

// ------------------------------------------------------------------- C-ABI --

extern "C" {

const char* hdc_last_error(void) { return g_err.c_str(); }
const char* hdc_version(void) { return "hdc 0.1 (gfx950)"; }

hdc_status hdc_derive(int64_t L, int64_t M, int64_t m, int64_t p, int64_t q, int64_t C, int64_t D, hdc_dtype dtype,
                      hdc_axis_desc* out) {
    if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
    hdc_axis_desc d{};
    hdc_status st = derive_axis(L, M, m, p, q, C, D, complex_of(dtype), &d);
    if (st != HDC_OK) return st;
    *out = d;
    return HDC_OK;
}

hdc_status hdc_plan(hdc_plan_t* out, int64_t L, int64_t M, int64_t m, int64_t p, int64_t q, int64_t C, int64_t D,
                    hdc_dtype dtype) {
    if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    hdc_plan_s* P = new hdc_plan_s();
    P->ndim = 1;
    P->real = is_real(dtype);
    P->dtype = complex_of(dtype);
    AxisPlan& A = P->ax[0];
    hdc_status st = derive_axis(L, M, m, p, q, C, D, P->dtype, &A.d);
    if (st == HDC_OK && P->real && !is_pow2(A.d.m))
        st = fail(HDC_ERR_UNSUPPORTED, "real-data plans take power-of-two m");
    if (st == HDC_OK) {
        A.dbl = P->dtype == HDC_C128;
        st = geometry(A, false);
    }
    if (st == HDC_OK && !P->real) enable_raw_rows(A);
    if (st == HDC_OK) st = finish_plan(P);
    if (st != HDC_OK) {
        delete P;
        return st;
    }
    *out = P;
    return HDC_OK;
}

static hdc_status check_ptrs(hdc_plan_t P, const void* a, const void* b, const void* c);

hdc_status hdc_plan_multi(hdc_plan_t* out, int A, int64_t L, int64_t M, int64_t m, int64_t p, int64_t q, int64_t C,
                          int64_t D, hdc_dtype dtype) {
    if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (A < 2 || A > kMaxOps) return fail(HDC_ERR_INVALID_ARG, "A = %d operands: must be 2 .. %d", A, kMaxOps);
    if (L < 1) return fail(HDC_ERR_INVALID_ARG, "L = %lld must be >= 1", (long long)L);
    if (L >= (int64_t(1) << 40)) return fail(HDC_ERR_UNSUPPORTED, "sizes of 2^40 and beyond are not supported");
    hdc_plan_s* P = new hdc_plan_s();
    P->ndim = 1;
    P->dtype = dtype;
    P->nops = A;
    AxisPlan& Ax = P->ax[0];
    // the A-fold linear convolution has A (L - 1) + 1 terms: the transform must cover them
    hdc_status st = derive_axis(L, M, m, p, q, C, D, dtype, &Ax.d, (int64_t)A * (L - 1) + 1);
    if (st == HDC_OK && !is_pow2(Ax.d.m))
        st = fail(HDC_ERR_UNSUPPORTED, "multi-convolution plans take power-of-two m");
    if (st == HDC_OK) {
        Ax.dbl = dtype == HDC_C128;
        st = geometry(Ax, false);
    }
    if (st == HDC_OK) st = finish_plan(P);
    if (st != HDC_OK) {
        delete P;
        return st;
    }
    *out = P;
    return HDC_OK;
}

hdc_status hdc_convolve_multi(hdc_plan_t P, const void* const* x, void* h, void* ws, hipStream_t s) {
    if (!P || !x || !h) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (P->uneq || P->real || P->real_nd)
        return fail(HDC_ERR_INVALID_ARG,
                    "hdc_convolve_multi takes a complex plan of hdc_plan_multi, hdc_plan_multi_nd, hdc_plan or "
                    "hdc_plan_nd");
    for (int o = 0; o < P->nops; ++o) {
        if (!x[o]) return fail(HDC_ERR_INVALID_ARG, "operand %d is NULL", o);
        if (x[o] == h) return fail(HDC_ERR_INVALID_ARG, "h must not alias an operand");
        hdc_status st = check_ptrs(P, x[o], nullptr, nullptr);
        if (st != HDC_OK) return st;
    }
    hdc_status st = check_ptrs(P, h, nullptr, nullptr);
    if (st != HDC_OK) return st;
    if (P->ws_bytes > 0 && !ws) return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes required", P->ws_bytes);
    struct CurPlan {
        explicit CurPlan(const void* p) { g_cur_plan = p; }
        ~CurPlan() { g_cur_plan = nullptr; }
    } cur(P);
    if (P->ndim > 1) return convnd_multi(P, 0, x, h, 1, (char*)ws, s);
    const AxisPlan& Ax = P->ax[0];
    if (P->nops == 2) return conv1d(Ax, x[0], x[1], h, 1, 0, 0, Ax.d.C, (char*)ws, elem(P), s);
    return conv1d_multi(Ax, x, P->nops, h, 1, 0, 0, Ax.d.C, (char*)ws, elem(P), s);
}

static hdc_status nd_extents_ok(int ndim, const AxisPlan* ax);

hdc_status hdc_plan_multi_nd(hdc_plan_t* out, int A, int ndim, const int64_t* L, const int64_t* M, const int64_t* m,
                             const int64_t* D, hdc_dtype dtype) {
    if (!out || !L || !m) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (A < 2 || A > kMaxOps) return fail(HDC_ERR_INVALID_ARG, "A = %d operands: must be 2 .. %d", A, kMaxOps);
    if (ndim < 2 || ndim > 3) return fail(HDC_ERR_INVALID_ARG, "ndim = %d must be 2 or 3 (1D: hdc_plan_multi)", ndim);
    if (dtype != HDC_C64 && dtype != HDC_C128)
        return fail(HDC_ERR_UNSUPPORTED, "multi-convolution plans are complex (HDC_C64 / HDC_C128)");
    hdc_plan_s* P = new hdc_plan_s();
    P->ndim = ndim;
    P->dtype = dtype;
    P->nops = A;
    hdc_status st = HDC_OK;
    for (int a = 0; a < ndim && st == HDC_OK; ++a) {
        if (L[a] < 1 || L[a] >= (int64_t(1) << 40)) {
            st = fail(HDC_ERR_INVALID_ARG, "axis %d: L = %lld out of range", a, (long long)L[a]);
            break;
        }
        const int64_t K = (int64_t)A * (L[a] - 1) + 1;  // terms of the A-fold result
        AxisPlan& Ax = P->ax[a];
        st = derive_axis(L[a], M ? M[a] : K, m[a], 0, 0, 1, D ? D[a] : 0, dtype, &Ax.d, K);
        if (st == HDC_OK && !is_pow2(Ax.d.m))
            st = fail(HDC_ERR_UNSUPPORTED, "axis %d: multi-convolution plans take power-of-two m", a);
        if (st == HDC_OK) {
            Ax.dbl = dtype == HDC_C128;
            // the innermost axis keeps the two variants the multi-operand kernels implement
            st = geometry(Ax, a < ndim - 1, false);
        }
    }
    if (st == HDC_OK) st = nd_extents_ok(ndim, P->ax);
    if (st == HDC_OK) st = finish_plan(P);
    if (st != HDC_OK) {
        delete P;
        return st;
    }
    *out = P;
    return HDC_OK;
}

hdc_status hdc_uneq_derive(int64_t Lf, int64_t Lg, int64_t M, int64_t m, int64_t Lambda, int64_t C, int64_t D,
                           hdc_dtype dtype, hdc_axis_desc* short_out, hdc_axis_desc* long_out, int* swapped) {
    bool sw = false;
    hdc_axis_desc f{}, g{};
    hdc_status st = derive_uneq(Lf, Lg, M, m, Lambda, C, D, dtype, &f, &g, &sw);
    if (st != HDC_OK) return st;
    if (short_out) *short_out = f;
    if (long_out) *long_out = g;
    if (swapped) *swapped = sw ? 1 : 0;
    return HDC_OK;
}

hdc_status hdc_plan_uneq(hdc_plan_t* out, int64_t Lf, int64_t Lg, int64_t M, int64_t m, int64_t Lambda, int64_t C,
                         int64_t D, hdc_dtype dtype) {
    if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    hdc_plan_s* P = new hdc_plan_s();
    P->ndim = 1;
    P->dtype = dtype;
    P->uneq = true;
    P->Lf[0] = Lf;
    P->Lg[0] = Lg;
    hdc_status st = uneq_axis(P, 0, Lf, Lg, M, m, Lambda, C, D, false, false);
    if (st == HDC_OK) st = finish_plan(P);
    if (st != HDC_OK) {
        delete P;
        return st;
    }
    *out = P;
    return HDC_OK;
}

// Extents of an N-D problem.  No buffer is longer along an axis than that
// axis' transform length N; the column kernels index m2 x (inner extents)
// columns in 32 bits, and the element count must stay far inside 64 bits.
static hdc_status nd_extents_ok(int ndim, const AxisPlan* ax) {
    int64_t total = 1;
    for (int a = 0; a < ndim; ++a) {
        int64_t inner = 1;
        for (int b = a + 1; b < ndim; ++b) inner *= ax[b].d.N;  // at most two factors below 2^31
        if (inner > ((int64_t(1) << 31) - 1) / std::max<int64_t>(1, ax[a].d.m2))
            return fail(HDC_ERR_UNSUPPORTED, "axis %d: %lld x %lld columns exceed the 32-bit range", a,
                        (long long)ax[a].d.m2, (long long)inner);
        if (total > (int64_t(1) << 40) / ax[a].d.N)
            return fail(HDC_ERR_UNSUPPORTED, "the N-D transform holds more than 2^40 values");
        total *= ax[a].d.N;
    }
    return HDC_OK;
}

static hdc_status uneq_nd_fill(hdc_plan_s* P, int ndim, const int64_t* Lf, const int64_t* Lg, const int64_t* M,
                               const int64_t* m, const int64_t* Lambda, const int64_t* D) {
    if (!Lf || !Lg || !M) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (ndim < 1 || ndim > 3) return fail(HDC_ERR_INVALID_ARG, "ndim = %d must be 1..3", ndim);
    P->ndim = ndim;
    P->uneq = true;
    for (int a = 0; a < ndim; ++a) {
        P->Lf[a] = Lf[a];
        P->Lg[a] = Lg[a];
        hdc_status st = uneq_axis(P, a, Lf[a], Lg[a], M[a], m ? m[a] : 0, Lambda ? Lambda[a] : 0, 1, D ? D[a] : 0,
                                  a < ndim - 1, ndim > 1 && a == ndim - 1);
        if (st != HDC_OK) return st;
    }
    hdc_status st = nd_extents_ok(ndim, P->ax);
    return st == HDC_OK ? nd_extents_ok(ndim, P->fx) : st;
}

hdc_status hdc_uneq_nd_check(int ndim, const int64_t* Lf, const int64_t* Lg, const int64_t* M, const int64_t* m,
                             const int64_t* Lambda, const int64_t* D, hdc_dtype dtype, hdc_axis_desc* short_out,
                             hdc_axis_desc* long_out, int* swapped) {
    hdc_plan_s P;
    P.dtype = dtype;
    hdc_status st = uneq_nd_fill(&P, ndim, Lf, Lg, M, m, Lambda, D);
    if (st != HDC_OK) return st;
    for (int a = 0; a < ndim; ++a) {
        if (short_out) short_out[a] = P.fx[a].d;
        if (long_out) long_out[a] = P.ax[a].d;
        if (swapped) swapped[a] = P.swap[a] ? 1 : 0;
    }
    return HDC_OK;
}

hdc_status hdc_plan_uneq_nd(hdc_plan_t* out, int ndim, const int64_t* Lf, const int64_t* Lg, const int64_t* M,
                            const int64_t* m, const int64_t* Lambda, const int64_t* D, hdc_dtype dtype) {
    if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    hdc_plan_s* P = new hdc_plan_s();
    P->dtype = dtype;
    hdc_status st = uneq_nd_fill(P, ndim, Lf, Lg, M, m, Lambda, D);
    if (st == HDC_OK) st = finish_plan(P);
    if (st != HDC_OK) {
        delete P;
        return st;
    }
    *out = P;
    return HDC_OK;
}

hdc_status hdc_plan_nd(hdc_plan_t* out, int ndim, const int64_t* L, const int64_t* M, const int64_t* m,
                       const int64_t* p, const int64_t* q, const int64_t* D, hdc_dtype dtype) {
    if (!out || !L || !M || !m) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (ndim < 1 || ndim > 3) return fail(HDC_ERR_INVALID_ARG, "ndim = %d must be 1..3", ndim);
    if (is_real(dtype) && ndim == 1)
        return fail(HDC_ERR_UNSUPPORTED, "1D real data take hdc_plan (the Hermitian residue pairing)");
    const bool real_nd = is_real(dtype);
    dtype = complex_of(dtype);
    hdc_plan_s* P = new hdc_plan_s();
    P->ndim = ndim;
    P->dtype = dtype;
    P->real_nd = real_nd;
    hdc_status st = HDC_OK;
    for (int a = 0; a < ndim && st == HDC_OK; ++a) {
        AxisPlan& A = P->ax[a];
        st = derive_axis(L[a], M[a], m[a], p ? p[a] : 0, q ? q[a] : 0, 1, D ? D[a] : 0, dtype, &A.d);
        if (st == HDC_OK) {
            A.dbl = dtype == HDC_C128;
            st = geometry(A, a < ndim - 1, ndim > 1 && a == ndim - 1);
        }
    }
    if (st == HDC_OK) st = hdc_plan_nd_check(ndim, L, M, m, p, q, D, dtype, nullptr);
    if (st == HDC_OK) st = finish_plan(P);
    if (st != HDC_OK) {
        delete P;
        return st;
    }
    *out = P;
    return HDC_OK;
}

hdc_status hdc_plan_nd_check(int ndim, const int64_t* L, const int64_t* M, const int64_t* m, const int64_t* p,
                             const int64_t* q, const int64_t* D, hdc_dtype dtype, hdc_axis_desc* out) {
    if (!L || !M || !m) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (ndim < 1 || ndim > 3) return fail(HDC_ERR_INVALID_ARG, "ndim = %d must be 1..3", ndim);
    AxisPlan ax[3];
    for (int a = 0; a < ndim; ++a) {
        hdc_status st = derive_axis(L[a], M[a], m[a], p ? p[a] : 0, q ? q[a] : 0, 1, D ? D[a] : 0,
                                    complex_of(dtype), &ax[a].d);
        if (st != HDC_OK) return st;
        ax[a].dbl = dtype == HDC_C128;
        st = geometry(ax[a], a < ndim - 1, ndim > 1 && a == ndim - 1);
        if (st != HDC_OK) return st;
        if (out) out[a] = ax[a].d;
    }
    return nd_extents_ok(ndim, ax);
}

// Axes of a tuner parameter set (hdc_tune.h): derivation and geometry of every
// axis with its column tile, the checks of hdc_plan (1D, C = batch copies) or
// hdc_plan_nd (N-D, no copies).
static hdc_status params_axes(const hdc_problem* pr, const hdc_params* pm, AxisPlan* ax) {
    if (!pr || !pm) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    const int nd = pr->ndim;
    if (nd < 1 || nd > 3) return fail(HDC_ERR_INVALID_ARG, "ndim = %d must be 1..3", nd);
    if (pr->dtype != HDC_C64 && pr->dtype != HDC_C128)
        return fail(HDC_ERR_UNSUPPORTED, "tuner problems are complex (HDC_C64 / HDC_C128)");
    if (pr->batch < 1) return fail(HDC_ERR_INVALID_ARG, "batch = %lld must be >= 1", (long long)pr->batch);
    if (nd > 1 && pr->batch != 1) return fail(HDC_ERR_UNSUPPORTED, "batched N-D problems are not implemented");
    for (int a = 0; a < nd; ++a) {
        hdc_status st = derive_axis(pr->L[a], pr->M[a], pm->m[a], pm->p[a], pm->q[a], nd == 1 ? pr->batch : 1,
                                    pm->D[a], pr->dtype, &ax[a].d);
        if (st != HDC_OK) return st;
        ax[a].dbl = pr->dtype == HDC_C128;
        if (pm->tile[a] < 0) return fail(HDC_ERR_INVALID_ARG, "tile %d must be >= 0", (int)pm->tile[a]);
        ax[a].tile_req = pm->tile[a];
        st = geometry(ax[a], a < nd - 1, nd > 1 && a == nd - 1);
        if (st != HDC_OK) return st;
        if (nd == 1) enable_raw_rows(ax[a]);
    }
    return nd > 1 ? nd_extents_ok(nd, ax) : HDC_OK;
}

hdc_status hdc_params_check(const hdc_problem* pr, const hdc_params* pm, hdc_params* out) {
    AxisPlan ax[3];
    hdc_status st = params_axes(pr, pm, ax);
    if (st != HDC_OK || !out) return st;
    hdc_params o{};
    int64_t inner = 1;
    for (int a = pr->ndim - 1; a >= 0; --a) {
        const hdc_axis_desc& d = ax[a].d;
        o.m[a] = d.m;
        o.p[a] = d.p;
        o.q[a] = d.q;
        o.D[a] = d.D;
        o.C[a] = pr->ndim == 1 ? pr->batch : inner;
        o.tile[a] = d.variant == 1 ? ax[a].cf_tile : 0;
        inner *= d.M;
    }
    *out = o;
    return HDC_OK;
}

hdc_status hdc_plan_params(hdc_plan_t* out, const hdc_problem* pr, const hdc_params* pm) {
    if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    hdc_plan_s* P = new hdc_plan_s();
    hdc_status st = params_axes(pr, pm, P->ax);
    if (st == HDC_OK) {
        P->ndim = pr->ndim;
        P->dtype = pr->dtype;
        st = finish_plan(P);
    }
    if (st != HDC_OK) {
        delete P;
        return st;
    }
    *out = P;
    return HDC_OK;
}

hdc_status hdc_plan_destroy(hdc_plan_t P) {
    if (!P) return HDC_OK;
    if (P->tables) (void)hipFree(P->tables);
    delete P;
    return HDC_OK;
}

hdc_status hdc_plan_axis(hdc_plan_t P, int axis, int* ndim, hdc_axis_desc* out) {
    if (!P) return fail(HDC_ERR_INVALID_ARG, "plan is NULL");
    if (ndim) *ndim = P->ndim;
    if (P->uneq && axis >= P->ndim && axis < 2 * P->ndim) {
        if (out) *out = P->fx[axis - P->ndim].d;
        return HDC_OK;
    }
    if (axis < 0 || axis >= P->ndim) return fail(HDC_ERR_INVALID_ARG, "axis %d out of range", axis);
    if (out) *out = P->ax[axis].d;
    return HDC_OK;
}

hdc_status hdc_workspace_size(hdc_plan_t P, size_t* bytes) {
    if (!P || !bytes) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    *bytes = P->ws_bytes;
    return HDC_OK;
}

hdc_status hdc_residue_buffer_size(hdc_plan_t P, size_t* bytes) {
    if (!P || !bytes) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (P->ndim != 1 || P->real)
        return fail(HDC_ERR_UNSUPPORTED, "residue buffers are defined for complex 1D plans");
    const hdc_axis_desc& d = P->ax[0].d;
    *bytes = (size_t)(std::min(d.D, d.q) * d.m * d.C) * elem(P);
    return HDC_OK;
}

static hdc_status check_ptrs(hdc_plan_t P, const void* a, const void* b, const void* c) {
    const size_t al = (elem(P) == 16 ? 16 : 8) / ((P->real || P->real_nd) ? 2 : 1);
    if ((a && !aligned(a, al)) || (b && !aligned(b, al)) || (c && !aligned(c, al)))
        return fail(HDC_ERR_INVALID_ARG, "data pointers must be %zu-byte aligned", al);
    return HDC_OK;
}

hdc_status hdc_convolve(hdc_plan_t P, const void* f, const void* g, void* h, void* ws, hipStream_t s) {
    if (!P || !f || !g || !h) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (h == f || h == g) return fail(HDC_ERR_INVALID_ARG, "h must not alias f or g");
    hdc_status st = check_ptrs(P, f, g, h);
    if (st != HDC_OK) return st;
    if (P->ws_bytes > 0 && !ws) return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes required", P->ws_bytes);
    if (P->nops > 2)
        return fail(HDC_ERR_INVALID_ARG, "a plan of %d operands takes hdc_convolve_multi", P->nops);
    struct CurPlan {
        explicit CurPlan(const void* p) { g_cur_plan = p; }
        ~CurPlan() { g_cur_plan = nullptr; }
    } cur(P);
    if (P->uneq) {
        if (P->ndim > 1) return convnd_uneq(P, 0, f, g, h, 1, (char*)ws, s);
        const AxisPlan& G = P->ax[0];
        const int64_t C = G.d.C;
        return P->swap[0] ? conv_uneq(G, P->fx[0], P->lam[0], g, f, h, 1, 0, 0, 0, C, (char*)ws, elem(P), s)
                          : conv_uneq(G, P->fx[0], P->lam[0], f, g, h, 1, 0, 0, 0, C, (char*)ws, elem(P), s);
    }
    if (P->real) {
        const AxisPlan& A = P->ax[0];
        return conv1d_real(A, f, g, h, 1, 0, 0, A.d.C, (char*)ws, elem(P), s);
    }
    if (P->ndim == 1) {
        const AxisPlan& A = P->ax[0];
        return conv1d(A, f, g, h, 1, 0, 0, A.d.C, (char*)ws, elem(P), s);
    }
    if (P->real_nd) {
        // h = Im(z * z) / (2 s), z = f + i s g: the scale words, then the outer
        // axis's real column passes around the inner autoconvolution
        char* mx = (char*)ws;
        {
            LaunchScope ls(s, 7, (double)prod_L(P, 0) * (double)elem(P));
            hipError_t e = launch_real_scale(P->dtype == HDC_C128, f, g, prod_L(P, 0), mx, s);
            if (e != hipSuccess) return hip_fail(e, "real scale launch");
        }
        return convnd_real(P, f, g, h, mx, mx + 256, s);
    }
    return convnd(P, 0, f, g, h, 1, (char*)ws, s);
}

// Workspace of hdc_convolve_noalloc: a device array of HDC_SCRATCH_BYTES per
// GPU, alive until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device memory: the device address is looked up once per
// device (hipGetSymbolAddress with that device current) and only that address
// is handed to the kernels.
static __device__ __align__(256) unsigned char scratch[HDC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (set up on first use).
hdc_status scratch_address(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HDC_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(HDC_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL on device %d", dev);
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HDC_OK;
}
}  // namespace

hdc_status hdc_convolve_noalloc(hdc_plan_t P, const void* f, const void* g, void* h, hipStream_t s) {
    if (!P) return fail(HDC_ERR_INVALID_ARG, "NULL plan");
    if (P->ws_bytes > HDC_SCRATCH_BYTES)
        return fail(HDC_ERR_WORKSPACE, "the plan needs %zu bytes of workspace; hdc_convolve_noalloc holds %zu",
                    P->ws_bytes, (size_t)HDC_SCRATCH_BYTES);
    void* ws = nullptr;
    if (P->ws_bytes > 0) {
        hdc_status st = scratch_address(&ws);
        if (st != HDC_OK) return st;
    }
    return hdc_convolve(P, f, g, h, ws, s);
}

static hdc_status group_check(hdc_plan_t P, int64_t r0, int64_t* Dg) {
    if (P->real) return fail(HDC_ERR_UNSUPPORTED, "a real-data plan exposes hdc_convolve only");
    if (P->ndim != 1) return fail(HDC_ERR_UNSUPPORTED, "forward/multiply/backward are defined for 1D plans");
    const hdc_axis_desc& d = P->ax[0].d;
    if (!is_pow2(d.m))
        return fail(HDC_ERR_UNSUPPORTED, "m = %lld: the separate stages take power-of-two m (use hdc_convolve)",
                    (long long)d.m);
    const int64_t D = std::min(d.D, d.q);
    if (r0 < 0 || r0 >= d.q || r0 % D != 0)
        return fail(HDC_ERR_INVALID_ARG, "r0 = %lld must be a multiple of D = %lld below q = %lld", (long long)r0,
                    (long long)D, (long long)d.q);
    *Dg = std::min(D, d.q - r0);
    return HDC_OK;
}

hdc_status hdc_forward_operand(hdc_plan_t P, int operand, const void* x, void* F, int64_t r0, void* ws,
                               hipStream_t s) {
    if (!P || !x || !F) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (operand != 0 && operand != 1) return fail(HDC_ERR_INVALID_ARG, "operand = %d must be 0 (f) or 1 (g)", operand);
    if (!P->uneq) return hdc_forward(P, x, F, r0, ws, s);
    int64_t Dg = 0;
    hdc_status st = group_check(P, r0, &Dg);
    if (st == HDC_OK) st = check_ptrs(P, x, F, nullptr);
    if (st != HDC_OK) return st;
    const AxisPlan& G = P->ax[0];
    const int64_t C = G.d.C;
    const bool shorter = (operand == 0) != P->swap[0];
    st = shorter ? run_col_fwd(P->fx[0], x, F, 1, 0, 0, C, r0, Dg, s, nullptr, P->lam[0], G.d.q)
                 : run_col_fwd(G, x, F, 1, 0, 0, C, r0, Dg, s);
    if (st != HDC_OK) return st;
    return run_rows(G, F, F, F, Dg * G.d.m1 * C, C, MODE_FWD, s);
}

hdc_status hdc_forward(hdc_plan_t P, const void* f, void* F, int64_t r0, void* ws, hipStream_t s) {
    (void)ws;
    if (!P || !f || !F) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (P->uneq) return fail(HDC_ERR_INVALID_ARG, "unequal-length plan: use hdc_forward_operand");
    int64_t Dg = 0;
    hdc_status st = group_check(P, r0, &Dg);
    if (st == HDC_OK) st = check_ptrs(P, f, F, nullptr);
    if (st != HDC_OK) return st;
    const AxisPlan& A = P->ax[0];
    const int64_t C = A.d.C;
    st = run_col_fwd(A, f, F, 1, 0, 0, C, r0, Dg, s);
    if (st != HDC_OK) return st;
    return run_rows(A, F, F, F, Dg * A.d.m1 * C, C, MODE_FWD, s);
}

hdc_status hdc_multiply(hdc_plan_t P, void* F, const void* G, int64_t r0, hipStream_t s) {
    if (!P || !F || !G) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    int64_t Dg = 0;
    hdc_status st = group_check(P, r0, &Dg);
    if (st == HDC_OK) st = check_ptrs(P, F, G, nullptr);
    if (st != HDC_OK) return st;
    const hdc_axis_desc& d = P->ax[0].d;
    hipError_t e = launch_mul(P->dtype == HDC_C128, F, G, Dg * d.m * d.C, s);
    if (e != hipSuccess) return hip_fail(e, "multiply launch");
    return HDC_OK;
}

hdc_status hdc_backward(hdc_plan_t P, void* F, void* h, int64_t r0, void* ws, hipStream_t s) {
    (void)ws;
    if (!P || !F || !h) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    int64_t Dg = 0;
    hdc_status st = group_check(P, r0, &Dg);
    if (st == HDC_OK) st = check_ptrs(P, F, h, nullptr);
    if (st != HDC_OK) return st;
    const AxisPlan& A = P->ax[0];
    const int64_t C = A.d.C;
    st = run_rows(A, F, F, F, Dg * A.d.m1 * C, C, MODE_INV, s);
    if (st != HDC_OK) return st;
    return run_col_bwd(A, F, h, 1, 0, 0, C, r0, Dg, r0 > 0, s);
}

hdc_status hdc_residues_natural(hdc_plan_t P, const void* F, int64_t r0, void* out, hipStream_t s) {
    if (!P || !F || !out) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (F == out) return fail(HDC_ERR_INVALID_ARG, "out must not alias F");
    int64_t Dg = 0;
    hdc_status st = group_check(P, r0, &Dg);
    if (st == HDC_OK) st = check_ptrs(P, F, out, nullptr);
    if (st != HDC_OK) return st;
    const hdc_axis_desc& d = P->ax[0].d;
    hipError_t e = launch_natural(P->dtype == HDC_C128, F, out, Dg, d.m1, d.m2, d.C, s);
    if (e != hipSuccess) return hip_fail(e, "natural-order launch");
    return HDC_OK;
}

static thread_local Recorder* t_profile = nullptr;

hdc_status hdc_profile_begin(hdc_plan_t filter) {
    if (t_profile) return fail(HDC_ERR_INVALID_ARG, "profiling already active on this thread");
    t_profile = new Recorder();
    t_profile->filter = filter;
    g_rec = t_profile;
    return HDC_OK;
}

hdc_status hdc_profile_end(int max_launches, int* n_launches, int32_t* kinds, float* ms, double* bytes) {
    if (!t_profile) return fail(HDC_ERR_INVALID_ARG, "profiling not active");
    Recorder* rec = t_profile;
    t_profile = nullptr;
    g_rec = nullptr;
    hipError_t e = hipDeviceSynchronize();
    const int n = (int)rec->kind.size();
    if (n_launches) *n_launches = n;
    for (int i = 0; i < n && i < max_launches; ++i) {
        float t = 0.f;
        (void)hipEventElapsedTime(&t, rec->ev[2 * i], rec->ev[2 * i + 1]);
        if (kinds) kinds[i] = rec->kind[i];
        if (ms) ms[i] = t;
        if (bytes) bytes[i] = rec->bytes[i];
    }
    for (auto& x : rec->ev) (void)hipEventDestroy(x);
    delete rec;
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    return HDC_OK;
}

hdc_status hdc_convolve_profiled(hdc_plan_t P, const void* f, const void* g, void* h, void* ws, hipStream_t s,
                                 int max_launches, int* n_launches, int32_t* kinds, float* ms, double* bytes) {
    if (!n_launches || max_launches < 0) return fail(HDC_ERR_INVALID_ARG, "bad profiling arguments");
    hdc_status st = hdc_profile_begin(nullptr);
    if (st != HDC_OK) return st;
    st = hdc_convolve(P, f, g, h, ws, s);
    hdc_status st2 = hdc_profile_end(max_launches, n_launches, kinds, ms, bytes);
    return st != HDC_OK ? st : st2;
}

hdc_status hdc_time_convolve(hdc_plan_t P, const void* f, const void* g, void* h, void* ws, hipStream_t s, int warmup,
                             int reps, float* ms_out) {
    if (!P || !ms_out || reps < 1 || warmup < 0) return fail(HDC_ERR_INVALID_ARG, "bad timing arguments");
    for (int i = 0; i < warmup; ++i) {
        hdc_status st = hdc_convolve(P, f, g, h, ws, s);
        if (st != HDC_OK) return st;
    }
    std::vector<hipEvent_t> ev(2 * (size_t)reps);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    hdc_status st = HDC_OK;
    for (int i = 0; i < reps && st == HDC_OK; ++i) {
        HIP_TRY(hipEventRecord(ev[2 * i], s));
        st = hdc_convolve(P, f, g, h, ws, s);
        HIP_TRY(hipEventRecord(ev[2 * i + 1], s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < reps; ++i) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
        ms_out[i] = ms;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return st;
}

}  // extern "C"

// ------------------------------------------------------------------ batches --
//
// n independent 1D convolutions of uneven lengths.  Problems that share the
// FFT size m and the derived (p, q) form a bucket with one set of twiddle
// tables; every launch of a bucket covers all of its problems, the kernels
// reading each problem's offsets and lengths from a descriptor array.

namespace {

struct Bucket {
    AxisPlan A;
    int64_t count = 0;
    // concurrency lane of the captured graph and the element offset of the
    // lane's workspace region (buckets of one lane run in turn and share it)
    int lane = 0;
    size_t ws_off = 0;
    // host descriptors, uploaded into the batch's device block
    bool queued = false;              // served by the persistent fused launch
    std::vector<int64_t> fused_desc;  // {f_off, h_off, L, M} per problem
    std::vector<int64_t> fwd_desc;    // {f_off, L} per problem
    std::vector<int64_t> bwd_desc;    // {h_off, M} per problem
    size_t off_fused = 0, off_fwd = 0, off_bwd = 0;
    const int64_t* d_fused = nullptr;
    const int64_t* d_fwd = nullptr;
    const int64_t* d_bwd = nullptr;
};

}  // namespace

// Problems of the raw-row path (residue transforms of one row of m points,
// q <= 32) with the same m: one launch of raw residue rows and one of output
// sums for all of them, problems and rows described by device tables.
struct RawGroup {
    int64_t m = 0;
    size_t rep = 0;  // a bucket of this m: row geometry and pass table
    int64_t nrows = 0, ntiles = 0, count = 0;
    double bytes_rows = 0, bytes_qsum = 0;  // algorithmic bytes of the two launches
    int lane = 0;
    size_t ws_off = 0;
    std::vector<int64_t> members;  // buckets
    size_t off_probs = 0, off_rowmap = 0, off_ybase = 0, off_tilemap = 0;
    const RawProb* d_probs = nullptr;
    const int32_t* d_rowmap = nullptr;
    const int64_t* d_ybase = nullptr;
    const int32_t* d_tilemap = nullptr;
};

// The fused buckets served by one persistent launch (k_fused_queue): their
// argument records and the item queue in the batch's device block.
struct FusedQueue {
    std::vector<size_t> members;  // buckets
    int64_t nitems = 0;
    size_t lds = 0;
    double bytes = 0;
    int lane = 0;
    size_t off_args = 0, off_items = 0, off_counter = 0;
    const FusedArgs* d_args = nullptr;
    const int32_t* d_items = nullptr;
    int* d_counter = nullptr;
};

struct hdc_batch_s {
    hdc_dtype dtype = HDC_C64;
    int64_t n = 0, total_L = 0, total_M = 0;
    std::vector<Bucket> buckets;
    std::vector<RawGroup> raws;
    FusedQueue fq;
    void* block = nullptr;
    size_t ws_bytes = 0;
    int nlanes = 1;
    // captured graph and the arguments it was captured with
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void *g_f = nullptr, *g_g = nullptr;
    void *g_h = nullptr, *g_ws = nullptr;
    // the graph is captured on and replayed from a private stream (default
    // priority), ordered after and before the caller's stream with events
    hipStream_t side = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // lanes 1.. of the graph: streams forked from `side` inside the capture
    // (default priority) and the events that join them back
    std::vector<hipStream_t> lane_streams;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;
};

namespace {

// Default FFT size for a problem of length L: the smallest power of two >= L
// (p = 1, q = 2 for M = 2L-1), i.e. explicit padding to m, implicit to 2m.
constexpr int kBatchLanes = 4;  // concurrent lanes of a batch's captured graph

// The smallest power of two >= L (p = 1), except that lengths in (4096, 8192]
// take m = 4096 (p = 2): one-row residues on the raw-row path, measured faster
// than the column/row/column passes of m = 8192 for such problems.
int64_t default_m(int64_t L) {
    int64_t m = 1;
    while (m < L) m <<= 1;
    if (m == 2 * kMaxRow) m = kMaxRow;
    return m;
}

// Every bucket's launches, on stream lanes[bk.lane] (or all on s when lanes is
// NULL); each bucket uses its lane's workspace region.
hdc_status batch_launch(hdc_batch_s* Bt, const void* f, const void* g, void* h, void* ws, hipStream_t s,
                        const hipStream_t* lanes = nullptr) {
    const size_t eb = elem_bytes(Bt->dtype);
    const bool same = f == g;
    if (Bt->fq.nitems > 0) {
        if (lanes) s = lanes[Bt->fq.lane];
        FusedQueueArgs a{};
        a.f = f;
        a.g = g;
        a.h = h;
        a.same = same ? 1 : 0;
        a.nitems = (int32_t)Bt->fq.nitems;
        a.args = Bt->fq.d_args;
        a.items = Bt->fq.d_items;
        a.counter = Bt->fq.d_counter;
        LaunchScope ls(s, 0, Bt->fq.bytes);
        hipError_t e = launch_fused_queue(Bt->dtype == HDC_C128, a, Bt->fq.nitems, Bt->fq.lds, s);
        if (e != hipSuccess) return hip_fail(e, "persistent fused launch");
    }
    for (const RawGroup& rg : Bt->raws) {
        const AxisPlan& A = Bt->buckets[rg.rep].A;
        if (lanes) s = lanes[rg.lane];
        RawArgs a{};
        a.f = f;
        a.g = g;
        a.Y = (char*)ws + rg.ws_off * eb;
        a.h = h;
        a.nrows = rg.nrows;
        a.m = (int32_t)rg.m;
        a.rpw = A.r_rpw;
        a.C1 = 1;
        a.same = same ? 1 : 0;
        a.probs = rg.d_probs;
        a.rowmap = rg.d_rowmap;
        a.ybase = rg.d_ybase;
        a.tilemap = rg.d_tilemap;
        a.twp = A.tw_p2;
        {
            LaunchScope ls(s, 4, rg.bytes_rows);
            hipError_t e = launch_row_rr(A.dbl, (int)rg.m, a, A.r_threads, ceil_div(rg.nrows, A.r_rpw), A.r_lds, s);
            if (e != hipSuccess) return hip_fail(e, "raw row launch");
        }
        LaunchScope ls(s, 5, rg.bytes_qsum);
        hipError_t e = launch_qsum(A.dbl, a, rg.ntiles, 1, s);
        if (e != hipSuccess) return hip_fail(e, "output sum launch");
    }
    for (size_t b = 0; b < Bt->buckets.size(); ++b) {
        const Bucket& bk = Bt->buckets[b];
        const AxisPlan& A = bk.A;
        if (A.d.variant == 2 || bk.queued) continue;  // in a raw group or the fused queue
        if (lanes) s = lanes[bk.lane];
        if (A.d.variant == 0) {
            RowAddr in{1, 0, 0, 1}, out{1, 0, 0, 1};
            hdc_status st = run_fused(A, f, g, h, bk.count, in, out, bk.d_fused, s);
            if (st != HDC_OK) return st;
            continue;
        }
        const int64_t D = std::min(A.d.D, A.d.q);
        char* Xf = (char*)ws + bk.ws_off * eb;
        char* Xg = same ? Xf : Xf + (size_t)(bk.count * D * A.d.m) * eb;
        for (int64_t r0 = 0; r0 < A.d.q; r0 += D) {
            const int64_t Dg = std::min(D, A.d.q - r0);
            const int64_t xbs = Dg * A.d.m;
            for (int64_t b0 = 0; b0 < bk.count; b0 += 65535) {
                const int64_t nb = std::min<int64_t>(65535, bk.count - b0);
                char* xf = Xf + (size_t)(b0 * xbs) * eb;
                char* xg = Xg + (size_t)(b0 * xbs) * eb;
                hdc_status st = run_col_fwd(A, f, xf, nb, 0, xbs, 1, r0, Dg, s, bk.d_fwd + 2 * b0);
                if (st == HDC_OK && !same) st = run_col_fwd(A, g, xg, nb, 0, xbs, 1, r0, Dg, s, bk.d_fwd + 2 * b0);
                if (st == HDC_OK) st = run_rows(A, xf, xg, xf, nb * Dg * A.d.m1, 1, MODE_CONV, s);
                if (st == HDC_OK)
                    st = run_col_bwd(A, xf, h, nb, xbs, 0, 1, r0, Dg, r0 > 0, s, bk.d_bwd + 2 * b0);
                if (st != HDC_OK) return st;
            }
        }
    }
    return HDC_OK;
}

}  // namespace

extern "C" {

hdc_status hdc_batch_plan(hdc_batch_t* out, int64_t n, const int64_t* L, const int64_t* M, const int64_t* bucket_m,
                          hdc_dtype dtype) {
    if (!out || !L || n < 1) return fail(HDC_ERR_INVALID_ARG, "bad batch arguments");
    *out = nullptr;
    if (is_real(dtype)) return fail(HDC_ERR_UNSUPPORTED, "real data are implemented for 1D plans (hdc_plan) only");
    if (dtype != HDC_C64 && dtype != HDC_C128) return fail(HDC_ERR_INVALID_ARG, "bad dtype");
    hdc_batch_s* Bt = new hdc_batch_s();
    Bt->dtype = dtype;
    Bt->n = n;
    struct Key {
        int64_t m, p, q;
        bool operator==(const Key& o) const { return m == o.m && p == o.p && q == o.q; }
    };
    std::vector<Key> keys;
    std::vector<std::vector<int64_t>> members;
    std::vector<int64_t> foff(n), hoff(n);
    int64_t fo = 0, ho = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t Li = L[i];
        const int64_t Mi = M ? M[i] : 2 * Li - 1;
        const int64_t mi = (bucket_m && bucket_m[i] > 0) ? bucket_m[i] : default_m(Li);
        hdc_axis_desc d{};
        hdc_status st = derive_axis(Li, Mi, mi, 0, 0, 1, 0, dtype, &d);
        if (st != HDC_OK) {
            delete Bt;
            return fail(st, "problem %lld: %s", (long long)i, g_err.c_str());
        }
        foff[i] = fo;
        hoff[i] = ho;
        fo += Li;
        ho += Mi;
        Key k{mi, d.p, d.q};
        size_t b = 0;
        while (b < keys.size() && !(keys[b] == k)) ++b;
        if (b == keys.size()) {
            keys.push_back(k);
            members.emplace_back();
        }
        members[b].push_back(i);
    }
    Bt->total_L = fo;
    Bt->total_M = ho;
    std::vector<unsigned char> blob;
    std::vector<double> cost;       // estimated HBM bytes of each bucket
    std::vector<size_t> bucket_ws;  // workspace elements of each bucket
    for (size_t b = 0; b < keys.size(); ++b) {
        Bucket bk;
        int64_t Lmax = 0, Mmax = 0;
        for (int64_t i : members[b]) {
            Lmax = std::max(Lmax, L[i]);
            Mmax = std::max(Mmax, M ? M[i] : 2 * L[i] - 1);
        }
        hdc_status st = derive_axis(Lmax, Mmax, keys[b].m, keys[b].p, keys[b].q, 1, 0, dtype, &bk.A.d);
        if (st == HDC_OK) {
            bk.A.dbl = dtype == HDC_C128;
            st = geometry(bk.A, false);
        }
        if (st != HDC_OK) {
            delete Bt;
            return st;
        }
        bk.count = (int64_t)members[b].size();
        double bytes = 0;
        for (int64_t i : members[b]) {
            const int64_t Mi = M ? M[i] : 2 * L[i] - 1;
            bytes += (double)(2 * L[i] + Mi) * (double)elem_bytes(dtype);
            bk.fused_desc.insert(bk.fused_desc.end(), {foff[i], hoff[i], L[i], Mi});
            bk.fwd_desc.insert(bk.fwd_desc.end(), {foff[i], L[i]});
            bk.bwd_desc.insert(bk.bwd_desc.end(), {hoff[i], Mi});
        }
        stage_tables(bk.A, blob);
        auto put = [&](const std::vector<int64_t>& v) {
            while (blob.size() % 256) blob.push_back(0);
            size_t off = blob.size();
            blob.insert(blob.end(), (const unsigned char*)v.data(), (const unsigned char*)(v.data() + v.size()));
            return off;
        };
        bk.off_fused = put(bk.fused_desc);
        bk.off_fwd = put(bk.fwd_desc);
        bk.off_bwd = put(bk.bwd_desc);
        // the column/row/column path moves about four times the problem bytes;
        // every launch costs about as much as 64 MB of traffic
        const bool fused = bk.A.d.variant == 0;
        cost.push_back(bytes * (fused ? 1.0 : 4.0) + (fused ? 1.0 : 4.0) * 6.4e7);
        bucket_ws.push_back(fused ? 0 : (size_t)ws1d(bk.A, bk.count, 1));
        Bt->buckets.push_back(std::move(bk));
    }
    // raw groups: buckets whose residue transform is one row (m1 = 1) with
    // q <= 32 run as one raw-row launch and one output-sum launch per m
    for (size_t b = 0; b < Bt->buckets.size(); ++b) {
        Bucket& bk = Bt->buckets[b];
        enable_raw_rows(bk.A);
        if (bk.A.d.variant != 2) continue;
        size_t gi = 0;
        while (gi < Bt->raws.size() && Bt->raws[gi].m != bk.A.d.m) ++gi;
        if (gi == Bt->raws.size()) {
            RawGroup rg;
            rg.m = bk.A.d.m;
            rg.rep = b;
            Bt->raws.push_back(rg);
        }
        Bt->raws[gi].members.push_back((int64_t)b);
    }
    auto put_bytes = [&](const void* p, size_t n) {
        while (blob.size() % 256) blob.push_back(0);
        size_t off = blob.size();
        blob.insert(blob.end(), (const unsigned char*)p, (const unsigned char*)p + n);
        return off;
    };
    // the fused buckets the persistent kernel serves: one queue of (bucket, m,
    // block of rows) items, largest transform first
    {
        const int64_t maxm = dtype == HDC_C128 ? kQueueMaxM128 : kQueueMaxM64;
        FusedQueue& fq = Bt->fq;
        for (size_t b = 0; b < Bt->buckets.size(); ++b)
            if (Bt->buckets[b].A.d.variant == 0 && Bt->buckets[b].A.d.m <= maxm && is_pow2(Bt->buckets[b].A.d.m))
                fq.members.push_back(b);
        std::stable_sort(fq.members.begin(), fq.members.end(), [&](size_t x, size_t y) {
            return Bt->buckets[x].A.d.m > Bt->buckets[y].A.d.m;
        });
        std::vector<int32_t> items;
        for (size_t k = 0; k < fq.members.size(); ++k) {
            Bucket& bk = Bt->buckets[fq.members[k]];
            bk.queued = true;
            const AxisPlan& A = bk.A;
            const int64_t blocks = ceil_div(bk.count, A.f_rpw);
            for (int64_t blk = 0; blk < blocks; ++blk) items.insert(items.end(), {(int32_t)k, (int32_t)A.d.m, (int32_t)blk});
            const int lg = ilog2i(A.d.m);
            const int64_t lo = int64_t(1) << ((lg + 1) / 2), hi = std::max<int64_t>(A.d.m / lo, 1);
            fq.lds = std::max(fq.lds, A.f_lds + (size_t)(lo + hi) * elem_bytes(dtype));
            fq.bytes += cost[fq.members[k]] - 6.4e7;  // the bucket's problem bytes
        }
        fq.nitems = (int64_t)items.size() / 3;
        if (fq.nitems > 0) {
            fq.off_items = put_bytes(items.data(), items.size() * sizeof(int32_t));
            std::vector<FusedArgs> zeros(fq.members.size());
            fq.off_args = put_bytes(zeros.data(), zeros.size() * sizeof(FusedArgs));  // filled below
            const int32_t zero = 0;
            fq.off_counter = put_bytes(&zero, sizeof zero);
        }
    }
    // schedulable units: buckets outside raw groups and the queue, the queue, then raw groups
    struct Unit {
        int kind;  // 0 bucket, 1 raw group, 2 the fused queue
        size_t idx;
        double cost;
        size_t ws;
    };
    std::vector<Unit> units;
    for (size_t b = 0; b < Bt->buckets.size(); ++b)
        if (Bt->buckets[b].A.d.variant != 2 && !Bt->buckets[b].queued) units.push_back({0, b, cost[b], bucket_ws[b]});
    if (Bt->fq.nitems > 0) units.push_back({2, 0, Bt->fq.bytes + 6.4e7, 0});
    for (size_t gi = 0; gi < Bt->raws.size(); ++gi) {
        RawGroup& rg = Bt->raws[gi];
        std::vector<int32_t> rowmap, tilemap;
        std::vector<int64_t> ybase;
        double bytes = 0;
        int32_t pi = 0;
        for (int64_t b : rg.members) {
            const Bucket& bk = Bt->buckets[(size_t)b];
            for (int64_t i : members[(size_t)b]) {
                const int64_t Mi = M ? M[i] : 2 * L[i] - 1;
                bytes += (double)(2 * L[i] + Mi) * (double)elem_bytes(dtype);
                rg.bytes_rows += (double)(2 * L[i] + bk.A.d.q * rg.m) * (double)elem_bytes(dtype);
                rg.bytes_qsum += (double)(bk.A.d.q * rg.m + Mi) * (double)elem_bytes(dtype);
                ybase.push_back(rg.nrows);
                for (int32_t r = 0; r < (int32_t)bk.A.d.q; ++r) rowmap.insert(rowmap.end(), {pi, r});
                rg.nrows += bk.A.d.q;
                for (int64_t c0 = 0; c0 < rg.m; c0 += 256) tilemap.insert(tilemap.end(), {pi, (int32_t)c0});
                ++pi;
            }
        }
        rg.count = pi;
        rg.ntiles = (int64_t)tilemap.size() / 2;
        rg.off_rowmap = put_bytes(rowmap.data(), rowmap.size() * sizeof(int32_t));
        rg.off_tilemap = put_bytes(tilemap.data(), tilemap.size() * sizeof(int32_t));
        rg.off_ybase = put_bytes(ybase.data(), ybase.size() * sizeof(int64_t));
        std::vector<RawProb> zeros((size_t)rg.count);
        rg.off_probs = put_bytes(zeros.data(), zeros.size() * sizeof(RawProb));  // filled once the tables have addresses
        // inputs from L2, the product rows written and read, the outputs written
        units.push_back({1, gi, bytes * 2.0 + 2.0 * 6.4e7, (size_t)(rg.nrows * rg.m)});
    }
    // lanes of the captured graph: units dealt longest first onto the
    // least-loaded lane; each lane owns a workspace region as large as its
    // largest unit needs
    const int nl = (int)std::min<size_t>(kBatchLanes, units.size());
    std::stable_sort(units.begin(), units.end(), [](const Unit& x, const Unit& y) { return x.cost > y.cost; });
    std::vector<double> load(nl, 0.0);
    std::vector<size_t> lane_ws(nl, 0), lane_off(nl, 0);
    std::vector<int> unit_lane(units.size());
    for (size_t u = 0; u < units.size(); ++u) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        unit_lane[u] = k;
        load[k] += units[u].cost;
        lane_ws[k] = std::max(lane_ws[k], units[u].ws);
    }
    size_t ws_elems = 0;
    for (int k = 0; k < nl; ++k) {
        lane_off[k] = ws_elems;
        ws_elems += lane_ws[k];
    }
    for (size_t u = 0; u < units.size(); ++u) {
        if (units[u].kind == 0) {
            Bt->buckets[units[u].idx].lane = unit_lane[u];
            Bt->buckets[units[u].idx].ws_off = lane_off[unit_lane[u]];
        } else if (units[u].kind == 2) {
            Bt->fq.lane = unit_lane[u];
        } else {
            Bt->raws[units[u].idx].lane = unit_lane[u];
            Bt->raws[units[u].idx].ws_off = lane_off[unit_lane[u]];
        }
    }
    Bt->nlanes = std::max(nl, 1);
    void* dev = nullptr;
    hipError_t e = hipMalloc(&dev, std::max<size_t>(blob.size(), 256));
    if (e != hipSuccess) {
        delete Bt;
        return hip_fail(e, "batch tables");
    }
    Bt->block = dev;
    for (Bucket& bk : Bt->buckets) {
        bind_tables(bk.A, (unsigned char*)dev);
        bk.d_fused = (const int64_t*)((unsigned char*)dev + bk.off_fused);
        bk.d_fwd = (const int64_t*)((unsigned char*)dev + bk.off_fwd);
        bk.d_bwd = (const int64_t*)((unsigned char*)dev + bk.off_bwd);
    }
    for (RawGroup& rg : Bt->raws) {
        std::vector<RawProb> probs;
        for (int64_t b : rg.members) {
            const Bucket& bk = Bt->buckets[(size_t)b];
            for (int64_t i : members[(size_t)b]) {
                RawProb pr = raw_prob(bk.A);
                pr.f_off = foff[i];
                pr.h_off = hoff[i];
                pr.L = (int32_t)L[i];
                pr.M = (int32_t)(M ? M[i] : 2 * L[i] - 1);
                pr.qout = (int32_t)ceil_div(pr.M, rg.m);
                probs.push_back(pr);
            }
        }
        std::memcpy(blob.data() + rg.off_probs, probs.data(), probs.size() * sizeof(RawProb));
        rg.d_probs = (const RawProb*)((unsigned char*)dev + rg.off_probs);
        rg.d_rowmap = (const int32_t*)((unsigned char*)dev + rg.off_rowmap);
        rg.d_ybase = (const int64_t*)((unsigned char*)dev + rg.off_ybase);
        rg.d_tilemap = (const int32_t*)((unsigned char*)dev + rg.off_tilemap);
    }
    if (Bt->fq.nitems > 0) {
        FusedQueue& fq = Bt->fq;
        std::vector<FusedArgs> args;
        for (size_t b : fq.members) {
            const Bucket& bk = Bt->buckets[b];
            const AxisPlan& A = bk.A;
            FusedArgs a{};  // f, g, h and same come with each launch
            a.nrows = bk.count;
            a.in = RowAddr{1, 0, 0, 1};
            a.out = RowAddr{1, 0, 0, 1};
            a.desc = bk.d_fused;
            a.L = (int32_t)A.d.L;
            a.M = (int32_t)A.d.M;
            a.p = (int32_t)A.d.p;
            a.q = (int32_t)A.d.q;
            a.qout = (int32_t)A.d.q_out;
            a.N = (int32_t)A.d.N;
            a.Dc = A.Dc;
            a.rpw = A.f_rpw;
            a.hiprec = A.hiprec ? 1 : 0;
            a.tw = A.tw;
            a.twm = A.tw_m;
            a.invN = 1.0 / (double)A.d.N;
            a.nops = 2;
            args.push_back(a);
        }
        std::memcpy(blob.data() + fq.off_args, args.data(), args.size() * sizeof(FusedArgs));
        fq.d_args = (const FusedArgs*)((unsigned char*)dev + fq.off_args);
        fq.d_items = (const int32_t*)((unsigned char*)dev + fq.off_items);
        fq.d_counter = (int*)((unsigned char*)dev + fq.off_counter);
    }
    e = hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hdc_batch_destroy(Bt);
        return hip_fail(e, "batch tables");
    }
    Bt->ws_bytes = ws_elems * elem_bytes(dtype);
    *out = Bt;
    return HDC_OK;
}

hdc_status hdc_batch_default_m(int64_t L, int64_t* m) {
    if (!m || L < 1) return fail(HDC_ERR_INVALID_ARG, "bad arguments");
    *m = default_m(L);
    return HDC_OK;
}

hdc_status hdc_batch_workspace_size(hdc_batch_t Bt, size_t* bytes) {
    if (!Bt || !bytes) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    *bytes = Bt->ws_bytes;
    return HDC_OK;
}

hdc_status hdc_batch_info(hdc_batch_t Bt, int64_t* n_buckets, int64_t* total_L, int64_t* total_M) {
    if (!Bt) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (n_buckets) *n_buckets = (int64_t)Bt->buckets.size();
    if (total_L) *total_L = Bt->total_L;
    if (total_M) *total_M = Bt->total_M;
    return HDC_OK;
}

static hdc_status batch_args(hdc_batch_t Bt, const void* f, const void* g, void* h, void* ws) {
    if (!Bt || !f || !g || !h) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (h == f || h == g) return fail(HDC_ERR_INVALID_ARG, "h must not alias f or g");
    if (Bt->ws_bytes > 0 && !ws) return fail(HDC_ERR_WORKSPACE, "workspace of %zu bytes required", Bt->ws_bytes);
    return HDC_OK;
}

hdc_status hdc_batch_convolve_eager(hdc_batch_t Bt, const void* f, const void* g, void* h, void* ws, hipStream_t s) {
    hdc_status st = batch_args(Bt, f, g, h, ws);
    if (st != HDC_OK) return st;
    return batch_launch(Bt, f, g, h, ws, s);
}

hdc_status hdc_batch_convolve(hdc_batch_t Bt, const void* f, const void* g, void* h, void* ws, hipStream_t s) {
    hdc_status st = batch_args(Bt, f, g, h, ws);
    if (st != HDC_OK) return st;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(HDC_ERR_INVALID_ARG,
                    "the stream is being captured: hdc_batch_convolve replays a graph of its own, "
                    "call hdc_batch_convolve_eager inside a capture");
    if (!Bt->side) {
        HIP_TRY(hipStreamCreateWithFlags(&Bt->side, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&Bt->ev_in, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&Bt->ev_out, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&Bt->ev_fork, hipEventDisableTiming));
    }
    while ((int)Bt->lane_streams.size() + 1 < Bt->nlanes) {
        hipStream_t ls = nullptr;
        hipEvent_t ev = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking));
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(ls);
            return hip_fail(e, "hipEventCreateWithFlags");
        }
        Bt->lane_streams.push_back(ls);
        Bt->ev_join.push_back(ev);
    }
    const bool hit = Bt->exec && Bt->g_f == f && Bt->g_g == g && Bt->g_h == h && Bt->g_ws == ws;
    if (!hit) {
        if (Bt->exec) {
            (void)hipGraphExecDestroy(Bt->exec);
            Bt->exec = nullptr;
        }
        if (Bt->graph) {
            (void)hipGraphDestroy(Bt->graph);
            Bt->graph = nullptr;
        }
        HIP_TRY(hipStreamBeginCapture(Bt->side, hipStreamCaptureModeThreadLocal));
        // fork: lanes 1.. join the capture by waiting on an event of the
        // capturing stream, and are joined back before the capture ends
        std::vector<hipStream_t> lanes{Bt->side};
        hipError_t e = hipEventRecord(Bt->ev_fork, Bt->side);
        for (size_t k = 0; e == hipSuccess && k < Bt->lane_streams.size(); ++k) {
            e = hipStreamWaitEvent(Bt->lane_streams[k], Bt->ev_fork, 0);
            lanes.push_back(Bt->lane_streams[k]);
        }
        st = e == hipSuccess ? batch_launch(Bt, f, g, h, ws, Bt->side, lanes.data()) : hip_fail(e, "graph fork");
        for (size_t k = 0; k + 1 < lanes.size(); ++k) {
            hipError_t ej = hipEventRecord(Bt->ev_join[k], Bt->lane_streams[k]);
            if (ej == hipSuccess) ej = hipStreamWaitEvent(Bt->side, Bt->ev_join[k], 0);
            if (ej != hipSuccess && st == HDC_OK) st = hip_fail(ej, "graph join");
        }
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(Bt->side, &graph);
        if (st != HDC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&Bt->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(e, "hipGraphInstantiate");
        }
        Bt->graph = graph;
        Bt->g_f = f;
        Bt->g_g = g;
        Bt->g_h = h;
        Bt->g_ws = ws;
    }
    HIP_TRY(hipEventRecord(Bt->ev_in, s));
    HIP_TRY(hipStreamWaitEvent(Bt->side, Bt->ev_in, 0));
    HIP_TRY(hipGraphLaunch(Bt->exec, Bt->side));
    HIP_TRY(hipEventRecord(Bt->ev_out, Bt->side));
    HIP_TRY(hipStreamWaitEvent(s, Bt->ev_out, 0));
    return HDC_OK;
}

hdc_status hdc_batch_destroy(hdc_batch_t Bt) {
    if (!Bt) return HDC_OK;
    if (Bt->exec) (void)hipGraphExecDestroy(Bt->exec);
    if (Bt->graph) (void)hipGraphDestroy(Bt->graph);
    if (Bt->side) {
        (void)hipStreamSynchronize(Bt->side);
        (void)hipStreamDestroy(Bt->side);
    }
    for (hipStream_t ls : Bt->lane_streams) {
        (void)hipStreamSynchronize(ls);
        (void)hipStreamDestroy(ls);
    }
    for (hipEvent_t ev : Bt->ev_join) (void)hipEventDestroy(ev);
    if (Bt->ev_fork) (void)hipEventDestroy(Bt->ev_fork);
    if (Bt->ev_in) (void)hipEventDestroy(Bt->ev_in);
    if (Bt->ev_out) (void)hipEventDestroy(Bt->ev_out);
    if (Bt->block) (void)hipFree(Bt->block);
    delete Bt;
    return HDC_OK;
}

}  // extern "C"
