// HIP kernels of the hybrid dealiased convolution, written for gfx950 (CDNA4).
//
// Notation (section 2.2, eqs. (3)-(4)): N = q m, residue r < q, block t < p,
// column s < m, frequency l < m; zeta_n = exp(+2 pi i / n).
//
//   forward   F_{q l + r} = sum_s zeta_m^{l s} [ zeta_N^{r s} sum_t zeta_q^{r t} f_{t m + s} ]
//   backward  h_{t m + s} = (1/N) sum_r zeta_q^{-t r} zeta_N^{-s r} sum_l zeta_m^{-s l} H_{q l + r}
//
// The m-point DFTs are radix-8 Stockham autosort passes (plus one radix-2 or
// radix-4 pass) with every thread owning PPT = 8 points at positions
// lane + v*(n/8).  With that ownership the inputs of every pass and the
// outputs of the last pass sit in the same registers, so
//   * the block sum of eq. (3) is computed straight into the registers of the
//     first radix pass (it never touches LDS or HBM), and
//   * the pointwise product F.G sits between the last forward pass and the
//     first inverse pass in registers (section 2.4, the convolution theorem).
// LDS only carries the exchanges between passes.
//
// Large m is split m = m1 * m2 (the four-step factorisation of the m-point
// DFT): a column kernel does the block sum, the m1-point DFTs down strided
// columns and the twiddle zeta_m^{l1 s2}; a row kernel does the contiguous
// m2-point DFTs, the product and the inverse; a second column kernel does the
// inverse m1-point DFTs and the backward post-processing over residues.  The
// same column kernels serve the outer axes of 2D/3D problems, whose copies
// are the inner extents (section 2.5's C).
#include "hdc_internal.h"

namespace hdc {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> mk(T a, T b) {
    cplx<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cplx<T> scale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// a * (sign * i)
template <int SIGN, typename T>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a) {
    return SIGN > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// zeta_N^e from the two-level FP64 table.
__device__ __forceinline__ double2 tw_n(const TwN& t, uint32_t e) {
    const double2 a = t.lo[e & (uint32_t)t.mask];
    const double2 b = t.hi[e >> t.lgB];
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// v * z (CONJ: v * conj(z)); complex64 data use an FP64 product when hp is set.
template <bool CONJ, typename T>
__device__ __forceinline__ cplx<T> mul_tw(cplx<T> v, double2 z, bool hp);

template <>
__device__ __forceinline__ cplx<double> mul_tw<false, double>(cplx<double> v, double2 z, bool) {
    return mk<double>(v.x * z.x - v.y * z.y, v.x * z.y + v.y * z.x);
}
template <>
__device__ __forceinline__ cplx<double> mul_tw<true, double>(cplx<double> v, double2 z, bool) {
    return mk<double>(v.x * z.x + v.y * z.y, v.y * z.x - v.x * z.y);
}
template <>
__device__ __forceinline__ cplx<float> mul_tw<false, float>(cplx<float> v, double2 z, bool hp) {
    if (hp) {
        const double x = v.x, y = v.y;
        return mk<float>((float)(x * z.x - y * z.y), (float)(x * z.y + y * z.x));
    }
    const float zx = (float)z.x, zy = (float)z.y;
    return mk<float>(v.x * zx - v.y * zy, v.x * zy + v.y * zx);
}
template <>
__device__ __forceinline__ cplx<float> mul_tw<true, float>(cplx<float> v, double2 z, bool hp) {
    if (hp) {
        const double x = v.x, y = v.y;
        return mk<float>((float)(x * z.x + y * z.y), (float)(y * z.x - x * z.y));
    }
    const float zx = (float)z.x, zy = (float)z.y;
    return mk<float>(v.x * zx + v.y * zy, v.y * zx - v.x * zy);
}

// ------------------------------------------------------------ Stockham DFT --

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

template <int NSZ, int PPTW = (NSZ >= 8 ? 8 : NSZ)>
struct FP {
    static constexpr int LG = ilog2c(NSZ);
    static constexpr int PPT = PPTW;  // points per thread (8, or 16 for register-rich kernels)
    static constexpr int TPF = NSZ / PPT;  // threads per transform
    static constexpr int R0 = NSZ < 8 ? NSZ : ((LG % 3) == 0 ? 8 : (1 << (LG % 3)));
    static constexpr int NPASS = NSZ <= 1 ? 0 : (NSZ < 8 ? 1 : ((LG % 3) == 0 ? LG / 3 : LG / 3 + 1));
};

template <int R, int SIGN, typename T>
__device__ __forceinline__ void dft_r(cplx<T>* x) {
    if constexpr (R == 2) {
        const cplx<T> a = x[0];
        x[0] = a + x[1];
        x[1] = a - x[1];
    } else if constexpr (R == 4) {
        const cplx<T> a = x[0] + x[2], b = x[0] - x[2], c = x[1] + x[3];
        const cplx<T> d = mul_i<SIGN>(x[1] - x[3]);
        x[0] = a + c;
        x[2] = a - c;
        x[1] = b + d;
        x[3] = b - d;
    } else if constexpr (R == 8) {
        cplx<T> a[4] = {x[0], x[2], x[4], x[6]};
        cplx<T> b[4] = {x[1], x[3], x[5], x[7]};
        dft_r<4, SIGN>(a);
        dft_r<4, SIGN>(b);
        const T rh = (T)0.70710678118654752440;
        const T s = (T)SIGN;
        b[1] = mk<T>((b[1].x - s * b[1].y) * rh, (s * b[1].x + b[1].y) * rh);
        b[2] = mul_i<SIGN>(b[2]);
        b[3] = mk<T>((-b[3].x - s * b[3].y) * rh, (s * b[3].x - b[3].y) * rh);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = a[k] + b[k];
            x[k + 4] = a[k] - b[k];
        }
    }
}

// LDS layouts of a transform's exchange buffer.  LAY_COL: tile columns side
// by side (position pos of column cc at pos * tile + cc), conflict-free as it
// is.  LAY_PAD: contiguous with one pad slot after every 8 values (the fused
// kernels, whose address arithmetic then folds into instruction offsets).
// LAY_XOR: contiguous, positions permuted inside aligned blocks of 16
// (complex128) or 32 (complex64) values by an XOR of the low bits with
// higher bits, chosen so that the stride-8 writes of the first pass, the
// blocked writes of the later passes and the unit-stride reloads each put the
// lanes that the LDS serves together on distinct banks, whether it serves 128
// or 256 bytes per clock (the row kernels).
enum { LAY_COL = 0, LAY_PAD = 1, LAY_XOR = 2 };

template <int LAY, typename T, int NSZ>
__device__ __forceinline__ int lds_at(int pos, int bstride) {
    constexpr int c = ilog2c(NSZ) % 3;  // the first pass is radix 8, 2 or 4 for c = 0, 1, 2
    if constexpr (LAY == LAY_COL) {
        return pos * bstride;
    } else if constexpr (LAY == LAY_PAD) {
        return pos + (pos >> 3);
    } else if constexpr (sizeof(T) == 8) {  // 16-byte values
        return pos ^ (((pos >> 3) ^ (pos >> (c == 1 ? 4 : 5))) & 15);
    } else if constexpr (c == 1) {  // 8-byte values
        return pos ^ (((pos >> 3) ^ (pos >> 4) ^ (pos >> 5)) & 31);
    } else {
        return pos ^ (((pos >> 3) ^ (pos >> (c == 0 ? 7 : 4))) & 31);
    }
}

// Padded length of a contiguous n-point LDS buffer.
__host__ __device__ constexpr int padded(int n) { return n + (n >> 3); }

// zeta_n^e for the Stockham passes from a two-level table in LDS:
// zeta_n^e = lo[e mod B] * hi[e / B], B = 2^ceil(log2(n)/2).  Keeping the
// per-pass twiddles out of global memory lets a kernel keep prefetched global
// loads in flight across a whole transform (vector loads retire in order).
template <typename T>
struct TwLds {
    const cplx<T>* lo;
    const cplx<T>* hi;
    int mask;
    int lg;
    __device__ __forceinline__ cplx<T> operator[](int e) const { return lo[e & mask] * hi[e >> lg]; }
    // the twiddles zeta^{e1}, zeta^{2 e1}, zeta^{4 e1} of a radix-8 pass
    __device__ __forceinline__ void get3(int, int, int e1, cplx<T>& w1, cplx<T>& w2, cplx<T>& w4) const {
        w1 = (*this)[e1];
        w2 = (*this)[2 * e1];
        w4 = (*this)[4 * e1];
    }
};

// Per-pass twiddle tables in LDS for transforms whose lanes run along the
// transform (rows): the radix-8 pass over sub-transforms of length Ns needs
// zeta_{8 Ns}^{i k}, i = 1, 2, 4, at k = position mod Ns.  Stored as three
// arrays of Ns values per pass, lanes with consecutive k read consecutive
// 16-byte slots, so the reads are free of bank conflicts (the two-level table
// is read at strides of up to 8 slots there) and need no product.  Passes
// follow the first one (radix R0, Ns = 1, no twiddles): Ns = R0 8^j.
template <int NSZ>
struct PassTab {
    static constexpr int R0 = FP<NSZ>::R0;
    static constexpr int NP = FP<NSZ>::NPASS;
    // entries: 3 * (R0 + 8 R0 + ... + 8^(NP-2) R0)
    static constexpr int LEN = NP > 1 ? 3 * R0 * ((1 << (3 * (NP - 1))) - 1) / 7 : 0;
};

template <typename T>
struct TwPass {
    const cplx<T>* t;
    int r0;
    __device__ __forceinline__ void get3(int Ns, int k, int, cplx<T>& w1, cplx<T>& w2, cplx<T>& w4) const {
        const cplx<T>* p = t + 3 * (Ns - r0) / 7;
        w1 = p[k];
        w2 = p[Ns + k];
        w4 = p[2 * Ns + k];
    }
};

// Copy a PassTab<NSZ> table (built by the plan in the same layout) into LDS.
template <typename T, int NSZ>
__device__ __forceinline__ void fill_pass_tab(cplx<T>* t, const void* twp, int tid, int nth) {
    const cplx<T>* src = reinterpret_cast<const cplx<T>*>(twp);
    for (int e = tid; e < PassTab<NSZ>::LEN; e += nth) t[e] = src[e];
}

template <int NSZ>
struct TwSplit {
    static constexpr int LG = (ilog2c(NSZ) + 1) / 2;
    static constexpr int LO = 1 << LG;
    static constexpr int HI = NSZ / LO > 0 ? NSZ / LO : 1;
};

// One radix-R pass over sub-transforms of length Ns -> Ns*R.  Register v[w]
// holds position lane + w*TPF.  Non-final passes write to LDS; the final
// pass leaves its outputs in v.  Twiddles zeta^{i k}: i = 1, 2, 4 from the
// table `tw`, the other four as products.
template <typename T, int NSZ, int R, int SIGN, bool LAST, int PAD, int PPTW = (NSZ >= 8 ? 8 : NSZ), class TW>
__device__ __forceinline__ void stock_pass(cplx<T> (&v)[PPTW], int Ns, cplx<T>* buf, int bstride, int lane,
                                           const TW& tw, bool act) {
    constexpr int PPT = PPTW;
    constexpr int Q = NSZ / PPTW;
    constexpr int NB = PPT / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = lane + u * Q;
        const int k = j & (Ns - 1);
        cplx<T> x[R];
#pragma unroll
        for (int i = 0; i < R; ++i) x[i] = v[u + i * NB];
        // only the radix-8 passes after the first (Ns > 1) carry twiddles
        if (R == 8 && Ns > 1) {
            const int e1 = k * (NSZ / (Ns * R));
            cplx<T> w[8];
            tw.get3(Ns, k, e1, w[1], w[2], w[4]);
            if (SIGN < 0) {
                w[1].y = -w[1].y;
                w[2].y = -w[2].y;
                w[4].y = -w[4].y;
            }
            w[3] = w[1] * w[2];
            w[5] = w[1] * w[4];
            w[6] = w[2] * w[4];
            w[7] = w[3] * w[4];
#pragma unroll
            for (int i = 1; i < R; ++i) x[i] = x[i] * w[i];
        }
        dft_r<R, SIGN>(x);
        if constexpr (LAST) {
#pragma unroll
            for (int a = 0; a < R; ++a) v[u + a * NB] = x[a];
        } else {
            if (act) {
                const int base = (j - k) * R + k;
#pragma unroll
                for (int a = 0; a < R; ++a) buf[lds_at<PAD, T, NSZ>(base + a * Ns, bstride)] = x[a];
            }
        }
    }
}

template <typename T, int NSZ, int PAD, int PPTW = (NSZ >= 8 ? 8 : NSZ)>
__device__ __forceinline__ void lds_reload(cplx<T> (&v)[PPTW], const cplx<T>* buf, int bstride, int lane,
                                           bool act) {
    constexpr int PPT = PPTW;
    constexpr int Q = NSZ / PPTW;
    __syncthreads();
    if (act) {
#pragma unroll
        for (int w = 0; w < PPT; ++w) v[w] = buf[lds_at<PAD, T, NSZ>(lane + w * Q, bstride)];
    }
    __syncthreads();
}

// NSZ-point DFT with zeta_NSZ^{SIGN}, registers in and out (positions lane + w*TPF).
// Every thread of the workgroup must call it (it contains barriers).
template <typename T, int NSZ, int SIGN, int PAD, int PPTW = (NSZ >= 8 ? 8 : NSZ), class TW>
__device__ __forceinline__ void fft_regs(cplx<T> (&v)[PPTW], cplx<T>* buf, int bstride, int lane, const TW& tw,
                                         bool act) {
    using P = FP<NSZ, PPTW>;
    if constexpr (P::NPASS == 1) {
        stock_pass<T, NSZ, P::R0, SIGN, true, PAD, PPTW>(v, 1, buf, bstride, lane, tw, act);
    } else if constexpr (P::NPASS > 1) {
        stock_pass<T, NSZ, P::R0, SIGN, false, PAD, PPTW>(v, 1, buf, bstride, lane, tw, act);
        int Ns = P::R0;
#pragma unroll
        for (int ps = 1; ps < P::NPASS - 1; ++ps) {
            lds_reload<T, NSZ, PAD, PPTW>(v, buf, bstride, lane, act);
            stock_pass<T, NSZ, 8, SIGN, false, PAD, PPTW>(v, Ns, buf, bstride, lane, tw, act);
            Ns *= 8;
        }
        lds_reload<T, NSZ, PAD, PPTW>(v, buf, bstride, lane, act);
        stock_pass<T, NSZ, 8, SIGN, true, PAD, PPTW>(v, Ns, buf, bstride, lane, tw, act);
    }
}

// The same transform for contiguous rows with two exchange buffers used in
// turn (ping-pong): exchange n writes buf[ph], waits at one barrier and reads
// it back, and the next exchange writes the other buffer, so no second
// barrier is needed before the writes (the one barrier in between orders every
// read of a buffer before its next write).  `ph` carries the turn across
// consecutive transforms that share the buffers.
template <typename T, int NSZ, int SIGN, class TW>
__device__ __forceinline__ void fft_rows_pp(cplx<T> (&v)[FP<NSZ>::PPT], cplx<T>* buf0, cplx<T>* buf1, int& ph,
                                            int lane, const TW& tw, bool act) {
    using P = FP<NSZ>;
    constexpr int PPT = P::PPT;
    constexpr int Q = NSZ / PPT;
    if constexpr (P::NPASS == 1) {
        stock_pass<T, NSZ, P::R0, SIGN, true, LAY_XOR>(v, 1, buf0, 1, lane, tw, act);
    } else if constexpr (P::NPASS > 1) {
        int Ns = 1;
#pragma unroll
        for (int ps = 0; ps < P::NPASS - 1; ++ps) {
            cplx<T>* buf = ph ? buf1 : buf0;
            if (ps == 0)
                stock_pass<T, NSZ, P::R0, SIGN, false, LAY_XOR>(v, 1, buf, 1, lane, tw, act);
            else
                stock_pass<T, NSZ, 8, SIGN, false, LAY_XOR>(v, Ns, buf, 1, lane, tw, act);
            Ns = ps == 0 ? P::R0 : Ns * 8;
            __syncthreads();
            if (act) {
#pragma unroll
                for (int w = 0; w < PPT; ++w) v[w] = buf[lds_at<LAY_XOR, T, NSZ>(lane + w * Q, 1)];
            }
            ph ^= 1;
        }
        stock_pass<T, NSZ, 8, SIGN, true, LAY_XOR>(v, Ns, buf0, 1, lane, tw, act);
    }
}

// Workgroup -> task map that keeps consecutive tasks on one XCD: workgroups
// are dealt to the 8 XCDs round-robin, so block b runs on XCD b % 8; XCD x
// takes the contiguous task range [x*per, (x+1)*per).  Neighbouring column
// tiles then share that XCD's L2 (partial cache lines, re-read inputs).
__device__ __forceinline__ int xcd_task(int bid, int nblk) {
    const int per = nblk >> 3;
    return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ int64_t row_base(const RowAddr& a, int64_t row) {
    if (a.inner_cnt == 1) return row * a.outer_stride;  // uniform: plain rows need no division
    const int64_t o = row / a.inner_cnt;
    return o * a.outer_stride + (row - o * a.inner_cnt) * a.inner_stride;
}

// ------------------------------------------------------------- fused kernel --

// Operand o >= 2 of a multi-convolution (constant indices into the kernel
// argument, so the array is never copied to private memory).
__device__ __forceinline__ const void* multi_ptr(const FusedArgs& a, int o) {
    switch (o) {
        case 2: return a.xm[0];
        case 3: return a.xm[1];
        case 4: return a.xm[2];
        case 5: return a.xm[3];
        case 6: return a.xm[4];
        default: return a.xm[5];
    }
}
//
// One row (an independent 1D convolution) per group of TPF*Dc threads; its
// q residues are processed Dc at a time.  Residue r uses LDS region U[r]
// (m values) as its exchange buffer and finally stores
//     u^(r)_s zeta_N^{-r s} / N
// there.  After all residues, the output blocks t < ceil(M/m) are the
// q-point sums over r with zeta_q^{-t r}.  LDS: rows * N values + q twiddles.

// MULTI: more than two operands (section 6.1), a separate instantiation so that
// the two-operand kernel keeps its registers.
//
// The body is a device function over one block of rows `blk` so that the
// persistent batch kernel below can run it for any bucket; threads beyond the
// bucket's rows (a larger workgroup) stay idle but take part in the barriers.
template <typename T, int MSZ, bool MULTI = false>
__device__ __forceinline__ void fused_rows(const FusedArgs& a, const void* fp, const void* gp, void* hp, bool same,
                                           int64_t blk, unsigned char* smem_raw) {
    using P = FP<MSZ>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
    using S = TwSplit<MSZ>;
    double2* twq =
        reinterpret_cast<double2*>(smem_raw + ((size_t)a.rpw * a.q * padded(MSZ) * sizeof(cplx<T>) + 15) / 16 * 16);
    cplx<T>* tlo = reinterpret_cast<cplx<T>*>(twq + a.q);
    cplx<T>* thi = tlo + S::LO;

    constexpr int RS = padded(MSZ);  // LDS slots per residue
    const int rowthreads = TPF * a.Dc;
    const int tid = threadIdx.x;
    const int rloc = tid / rowthreads;
    const int lt = tid - rloc * rowthreads;
    const int grp = lt / TPF;
    const int lane = lt - grp * TPF;
    const int64_t row = blk * a.rpw + rloc;
    const bool rowok = rloc < a.rpw && row < a.nrows;

    // zeta_q^e, e < q, shared by the block sums and the output sums; the
    // two-level table of zeta_m for the transform passes
    for (int e = tid; e < a.q; e += blockDim.x) twq[e] = tw_n(a.tw, (uint32_t)e * (uint32_t)MSZ);
    {
        const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.twm);
        for (int e = tid; e < S::LO; e += blockDim.x) tlo[e] = twg[e];
        for (int e = tid; e < S::HI; e += blockDim.x) thi[e] = twg[e * S::LO];
    }
    __syncthreads();
    const TwLds<T> twm{tlo, thi, S::LO - 1, S::LG};

    int L = a.L, M = a.M;
    int Lg = a.Lg > 0 ? a.Lg : a.L;
    int64_t fbase, hbase;
    if (a.desc != nullptr) {
        const int64_t* d = a.desc + 4 * (rowok ? row : 0);
        fbase = d[0];
        hbase = d[1];
        L = (int)d[2];
        M = (int)d[3];
        Lg = L;
    } else {
        fbase = row_base(a.in, rowok ? row : 0);
        hbase = row_base(a.out, rowok ? row : 0);
    }
    const int64_t gbase = (a.Lg > 0 && a.desc == nullptr) ? row_base(a.ing, rowok ? row : 0) : fbase;
    const int64_t ies = a.in.es, oes = a.out.es;
    const cplx<T>* f = reinterpret_cast<const cplx<T>*>(fp) + fbase;
    const cplx<T>* g = reinterpret_cast<const cplx<T>*>(gp) + gbase;
    cplx<T>* h = reinterpret_cast<cplx<T>*>(hp) + hbase;
    cplx<T>* U = smem + (size_t)(rowok ? rloc : 0) * a.q * RS;
    const T invN = (T)a.invN;

    for (int rb = 0; rb < a.q; rb += a.Dc) {
        const int r = rb + grp;
        const bool act = rowok && r < a.q;
        cplx<T>* buf = U + (size_t)(act ? r : 0) * RS;

        // block sums of eq. (3) for f and g, straight into the first radix pass
        cplx<T> F[PPT], G[PPT];
#pragma unroll
        for (int v = 0; v < PPT; ++v) {
            F[v] = mk<T>(0, 0);
            G[v] = mk<T>(0, 0);
        }
        if (act) {
            int e = 0;  // (r t) mod q
            for (int t = 0; t < a.p; ++t) {
                const double2 z = twq[e];
                e += r;
                if (e >= a.q) e -= a.q;
#pragma unroll
                for (int v = 0; v < PPT; ++v) {
                    const int j = t * MSZ + lane + v * TPF;
                    if (j < L) F[v] = F[v] + mul_tw<false>(f[(int64_t)j * ies], z, false);
                    if (!same && j < Lg) G[v] = G[v] + mul_tw<false>(g[(int64_t)j * ies], z, false);
                }
            }
        }
        const uint32_t ru = (uint32_t)(act ? r : 0);
        // zeta_N^{r s} for s = lane + v TPF, as z0 zs^v
        const double2 z0 = tw_n(a.tw, ru * (uint32_t)lane);
        const double2 zs = tw_n(a.tw, ru * (uint32_t)TPF);
        {
            double2 z = z0;
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                F[v] = mul_tw<false>(F[v], z, a.hiprec);
                if (!same) G[v] = mul_tw<false>(G[v], z, a.hiprec);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
        fft_regs<T, MSZ, +1, LAY_PAD>(F, buf, 1, lane, twm, act);
        if (!same) {
            fft_regs<T, MSZ, +1, LAY_PAD>(G, buf, 1, lane, twm, act);
#pragma unroll
            for (int v = 0; v < PPT; ++v) F[v] = F[v] * G[v];
        } else {
#pragma unroll
            for (int v = 0; v < PPT; ++v) F[v] = F[v] * F[v];
        }
        // further operands of a multi-convolution (section 6.1): the residue of
        // each is formed like f's and multiplies into the product
        for (int o = 2; MULTI && o < a.nops; ++o) {
            const cplx<T>* x = reinterpret_cast<const cplx<T>*>(multi_ptr(a, o)) + fbase;
#pragma unroll
            for (int v = 0; v < PPT; ++v) G[v] = mk<T>(0, 0);
            if (act) {
                int e = 0;
                for (int t = 0; t < a.p; ++t) {
                    const double2 z = twq[e];
                    e += r;
                    if (e >= a.q) e -= a.q;
#pragma unroll
                    for (int v = 0; v < PPT; ++v) {
                        const int j = t * MSZ + lane + v * TPF;
                        if (j < L) G[v] = G[v] + mul_tw<false>(x[(int64_t)j * ies], z, false);
                    }
                }
            }
            double2 z = z0;
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                G[v] = mul_tw<false>(G[v], z, a.hiprec);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
            fft_regs<T, MSZ, +1, LAY_PAD>(G, buf, 1, lane, twm, act);
#pragma unroll
            for (int v = 0; v < PPT; ++v) F[v] = F[v] * G[v];
        }
        fft_regs<T, MSZ, -1, LAY_PAD>(F, buf, 1, lane, twm, act);
        if (act) {
            double2 z = z0;
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                const int s = lane + v * TPF;
                buf[lds_at<LAY_PAD, T, MSZ>(s, 1)] = scale(mul_tw<true>(F[v], z, a.hiprec), invN);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
    }
    __syncthreads();
    if (!rowok) return;
    // h_{t m + s} = sum_r zeta_q^{-t r} U[r][s]
    for (int k = lt; k < M; k += rowthreads) {
        const int t = k / MSZ;
        const int s = k - t * MSZ;
        cplx<T> acc = mk<T>(0, 0);
        int e = 0;  // (t r) mod q
        for (int r = 0; r < a.q; ++r) {
            acc = acc + mul_tw<true>(U[(size_t)r * RS + lds_at<LAY_PAD, T, MSZ>(s, 1)], twq[e], false);
            e += t;
            if (e >= a.q) e -= a.q;
        }
        h[(int64_t)k * oes] = acc;
    }
}

// Mixed-radix fused kernel: m = R MSZ with R odd (3, 5, 7, 9, 15, ... <= 63),
// section 3.1's FFT-friendly sizes.  The m-point DFT of a residue is split by
// decimation in time, s = rho + R s': R sub-transforms of MSZ points (one
// thread group each, the radix-8 engine above) and a direct R-point stage
//     F_{l' + MSZ k} = sum_rho zeta_R^{rho k} zeta_m^{rho l'} X_rho[l'],
// exchanged through LDS; the inverse runs the two stages in the opposite order,
//     u_{rho + R s'} = sum_{l'} zeta_MSZ^{-s' l'} zeta_m^{-rho l'} sum_k zeta_R^{-rho k} H_{l' + MSZ k}.
// Everything else (block sums, product, output sums) is the fused kernel's.
template <typename T, int MSZ>
__device__ __forceinline__ void fused_rows_mixed(const FusedArgs& a, const void* fp, const void* gp, void* hp,
                                                 bool same, int64_t blk, unsigned char* smem_raw) {
    using P = FP<MSZ>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    constexpr int SUB = padded(MSZ);  // LDS slots of one sub-transform
    cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
    using S = TwSplit<MSZ>;
    const int R = a.R;
    const int m = R * MSZ;
    const int RSm = m + (m >> 3);  // LDS slots per residue (holds R sub-buffers)
    double2* twq =
        reinterpret_cast<double2*>(smem_raw + ((size_t)a.rpw * a.q * RSm * sizeof(cplx<T>) + 15) / 16 * 16);
    cplx<T>* tlo = reinterpret_cast<cplx<T>*>(twq + a.q);
    cplx<T>* thi = tlo + S::LO;

    const int rowthreads = TPF * R * a.Dc;  // Dc residues of R units each
    const int tid = threadIdx.x;
    const int rloc = tid / rowthreads;
    const int lt = tid - rloc * rowthreads;
    const int unit = lt / TPF;  // (residue in the round, rho)
    const int lane = lt - unit * TPF;
    const int rr = unit / R;
    const int rho = unit - rr * R;
    const int64_t row = blk * a.rpw + rloc;
    const bool rowok = rloc < a.rpw && row < a.nrows;

    const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.twm);  // zeta_m^e, e < m
    for (int e = tid; e < a.q; e += blockDim.x) twq[e] = tw_n(a.tw, (uint32_t)e * (uint32_t)m);
    // zeta_MSZ^e = zeta_m^{R e} for the sub-transforms' passes
    for (int e = tid; e < S::LO; e += blockDim.x) tlo[e] = twg[R * e];
    for (int e = tid; e < S::HI; e += blockDim.x) thi[e] = twg[R * e * S::LO];
    __syncthreads();
    const TwLds<T> twm{tlo, thi, S::LO - 1, S::LG};

    int L = a.L, M = a.M;
    int64_t fbase, hbase;
    if (a.desc != nullptr) {
        const int64_t* d = a.desc + 4 * (rowok ? row : 0);
        fbase = d[0];
        hbase = d[1];
        L = (int)d[2];
        M = (int)d[3];
    } else {
        fbase = row_base(a.in, rowok ? row : 0);
        hbase = row_base(a.out, rowok ? row : 0);
    }
    const int64_t ies = a.in.es, oes = a.out.es;
    const cplx<T>* f = reinterpret_cast<const cplx<T>*>(fp) + fbase;
    const cplx<T>* g = reinterpret_cast<const cplx<T>*>(gp) + fbase;
    cplx<T>* h = reinterpret_cast<cplx<T>*>(hp) + hbase;
    cplx<T>* U = smem + (size_t)(rowok ? rloc : 0) * a.q * RSm;
    const T invN = (T)a.invN;

    for (int rb = 0; rb < a.q; rb += a.Dc) {
        const int r = rb + rr;
        const bool act = rowok && r < a.q;
        cplx<T>* res = U + (size_t)(act ? r : 0) * RSm;  // this residue's region
        cplx<T>* buf = res + rho * SUB;                  // this unit's sub-buffer

        // block sums of eq. (3) at the points s = rho + R (lane + v TPF)
        cplx<T> F[PPT], G[PPT];
#pragma unroll
        for (int v = 0; v < PPT; ++v) {
            F[v] = mk<T>(0, 0);
            G[v] = mk<T>(0, 0);
        }
        if (act) {
            int e = 0;  // (r t) mod q
            for (int t = 0; t < a.p; ++t) {
                const double2 z = twq[e];
                e += r;
                if (e >= a.q) e -= a.q;
#pragma unroll
                for (int v = 0; v < PPT; ++v) {
                    const int j = t * m + rho + R * (lane + v * TPF);
                    if (j < L) {
                        F[v] = F[v] + mul_tw<false>(f[(int64_t)j * ies], z, false);
                        if (!same) G[v] = G[v] + mul_tw<false>(g[(int64_t)j * ies], z, false);
                    }
                }
            }
        }
        const uint32_t ru = (uint32_t)(act ? r : 0);
        // zeta_N^{r s}, s = rho + R lane + R TPF v, as z0 zs^v (r s < q m = N)
        const double2 z0 = tw_n(a.tw, ru * (uint32_t)(rho + R * lane));
        const double2 zs = tw_n(a.tw, ru * (uint32_t)(R * TPF));
        {
            double2 z = z0;
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                F[v] = mul_tw<false>(F[v], z, a.hiprec);
                if (!same) G[v] = mul_tw<false>(G[v], z, a.hiprec);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
        // forward: MSZ-point sub-transform, then the R-point stage through LDS;
        // afterwards unit rho holds F_{l' + MSZ rho} at l' = lane + v TPF
        auto forward = [&](cplx<T>(&X)[PPT]) {
            fft_regs<T, MSZ, +1, LAY_PAD>(X, buf, 1, lane, twm, act);
            if (act) {
#pragma unroll
                for (int v = 0; v < PPT; ++v) {
                    const int l = lane + v * TPF;
                    buf[lds_at<LAY_PAD, T, MSZ>(l, 1)] = X[v] * twg[rho * l];  // zeta_m^{rho l'}
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int v = 0; v < PPT; ++v) {
                    const int l = lane + v * TPF;
                    cplx<T> acc = mk<T>(0, 0);
                    int e = 0;  // (rho2 rho) mod R
                    for (int rho2 = 0; rho2 < R; ++rho2) {
                        acc = acc + res[rho2 * SUB + lds_at<LAY_PAD, T, MSZ>(l, 1)] * twg[e * MSZ];
                        e += rho;
                        if (e >= R) e -= R;
                    }
                    X[v] = acc;
                }
            }
            __syncthreads();
        };
        forward(F);
        if (!same) {
            forward(G);
#pragma unroll
            for (int v = 0; v < PPT; ++v) F[v] = F[v] * G[v];
        } else {
#pragma unroll
            for (int v = 0; v < PPT; ++v) F[v] = F[v] * F[v];
        }
        // inverse: the R-point stage (unit rho gathers H_{l' + MSZ k}, k < R), then
        // the MSZ-point inverse sub-transform
        if (act) {
#pragma unroll
            for (int v = 0; v < PPT; ++v) buf[lds_at<LAY_PAD, T, MSZ>(lane + v * TPF, 1)] = F[v];
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                const int l = lane + v * TPF;
                cplx<T> acc = mk<T>(0, 0);
                int e = 0;  // (rho k) mod R, conjugated below
                for (int k = 0; k < R; ++k) {
                    const cplx<T> w = twg[e * MSZ];
                    acc = acc + res[k * SUB + lds_at<LAY_PAD, T, MSZ>(l, 1)] * mk<T>(w.x, -w.y);
                    e += rho;
                    if (e >= R) e -= R;
                }
                const cplx<T> w = twg[rho * l];
                F[v] = acc * mk<T>(w.x, -w.y);  // zeta_m^{-rho l'}
            }
        }
        __syncthreads();
        fft_regs<T, MSZ, -1, LAY_PAD>(F, buf, 1, lane, twm, act);
        // every unit of the residue has read its sub-buffer for the last time (the
        // transform's final barrier, or the one above when it has a single pass):
        // the residue's region now takes u^(r)_s zeta_N^{-r s} / N in natural order
        if (act) {
            double2 z = z0;
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                const int s = rho + R * (lane + v * TPF);
                res[lds_at<LAY_PAD, T, MSZ>(s, 1)] = scale(mul_tw<true>(F[v], z, a.hiprec), invN);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
        __syncthreads();
    }
    if (!rowok) return;
    // h_{t m + s} = sum_r zeta_q^{-t r} U[r][s]
    for (int k = lt; k < M; k += rowthreads) {
        const int t = k / m;
        const int s = k - t * m;
        cplx<T> acc = mk<T>(0, 0);
        int e = 0;  // (t r) mod q
        for (int r = 0; r < a.q; ++r) {
            acc = acc + mul_tw<true>(U[(size_t)r * RSm + lds_at<LAY_PAD, T, MSZ>(s, 1)], twq[e], false);
            e += t;
            if (e >= a.q) e -= a.q;
        }
        h[(int64_t)k * oes] = acc;
    }
}

template <typename T, int MSZ>
__global__ void __launch_bounds__(512) k_fused_mixed(FusedArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fused_rows_mixed<T, MSZ>(a, a.f, a.g, a.h, a.same != 0, blockIdx.x, smem_raw);
}

// Whole-row convolution for the many rows of an innermost N-D axis: one group
// of TPF = m / 8 threads per row runs the row's q residues in turn (block sums
// of eq. (3), forward transforms of f and g, product, inverse, the
// zeta_N^{-rs} / N twiddle) and accumulates eq. (4)'s output sums
//     h_{t m + s} += zeta_q^{-t r} y^(r)_s,   t < ceil(M/m) <= QO,
// in registers: thread lane holds the same points s = lane + v TPF of every
// residue, so no residue is kept in LDS or HBM.  The transforms are the row
// kernels' (two exchange buffers per row, per-pass twiddle tables in LDS).
// Persistent: the workgroup walks rows base, base + stride, ...; every residue
// sums the row's p input blocks again (from L2 after the first).
template <typename T, int MSZ, int QO>
__global__ void __launch_bounds__(512) k_rowconv(FusedArgs a) {
    using P = FP<MSZ>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* tpt = smem + (size_t)a.rpw * 2 * MSZ;
    double2* twq = reinterpret_cast<double2*>(
        smem_raw + (((size_t)a.rpw * 2 * MSZ + PassTab<MSZ>::LEN) * sizeof(cplx<T>) + 15) / 16 * 16);
    const int tid = threadIdx.x;
    fill_pass_tab<T, MSZ>(tpt, a.twm, tid, blockDim.x);
    for (int e = tid; e < a.q; e += blockDim.x) twq[e] = tw_n(a.tw, (uint32_t)e * (uint32_t)MSZ);
    __syncthreads();
    const TwPass<T> tw{tpt, PassTab<MSZ>::R0};

    const int rloc = tid / TPF;
    const int lane = tid - rloc * TPF;
    cplx<T>* buf0 = smem + (size_t)rloc * 2 * MSZ;
    cplx<T>* buf1 = buf0 + MSZ;
    int ph = 0;
    const int L = a.L, M = a.M;
    const int64_t ies = a.in.es, oes = a.out.es;
    const bool same = a.same != 0;
    const T invN = (T)a.invN;
    const cplx<T>* fg = reinterpret_cast<const cplx<T>*>(a.f);
    const cplx<T>* gg = reinterpret_cast<const cplx<T>*>(a.g);
    cplx<T>* hg = reinterpret_cast<cplx<T>*>(a.h);
    const int64_t stride = (int64_t)gridDim.x * a.rpw;

    for (int64_t base = (int64_t)blockIdx.x * a.rpw; base < a.nrows; base += stride) {  // uniform
        const int64_t row = base + rloc;
        const bool ok = row < a.nrows;
        const int64_t fb = row_base(a.in, ok ? row : 0);
        cplx<T> acc[QO][PPT];
#pragma unroll
        for (int t = 0; t < QO; ++t)
#pragma unroll
            for (int v = 0; v < PPT; ++v) acc[t][v] = mk<T>(0, 0);
        for (int r = 0; r < a.q; ++r) {
            cplx<T> F[PPT], G[PPT];
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                F[v] = mk<T>(0, 0);
                G[v] = mk<T>(0, 0);
            }
            if (ok) {
                int e = 0;  // (r t) mod q
                for (int t = 0; t < a.p; ++t) {
                    const double2 z = twq[e];
                    e += r;
                    if (e >= a.q) e -= a.q;
#pragma unroll
                    for (int v = 0; v < PPT; ++v) {
                        const int j = t * MSZ + lane + v * TPF;
                        if (j < L) {
                            F[v] = F[v] + mul_tw<false>(fg[fb + (int64_t)j * ies], z, false);
                            if (!same) G[v] = G[v] + mul_tw<false>(gg[fb + (int64_t)j * ies], z, false);
                        }
                    }
                }
            }
            // zeta_N^{r s} for s = lane + v TPF, as z0 zs^v (1 for r = 0)
            const double2 z0 = tw_n(a.tw, (uint32_t)r * (uint32_t)lane);
            const double2 zs = tw_n(a.tw, (uint32_t)r * (uint32_t)TPF);
            if (r > 0) {
                double2 z = z0;
#pragma unroll
                for (int v = 0; v < PPT; ++v) {
                    F[v] = mul_tw<false>(F[v], z, a.hiprec);
                    if (!same) G[v] = mul_tw<false>(G[v], z, a.hiprec);
                    z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
                }
            }
            fft_rows_pp<T, MSZ, +1>(F, buf0, buf1, ph, lane, tw, ok);
            if (!same) {
                fft_rows_pp<T, MSZ, +1>(G, buf0, buf1, ph, lane, tw, ok);
#pragma unroll
                for (int v = 0; v < PPT; ++v) F[v] = F[v] * G[v];
            } else {
#pragma unroll
                for (int v = 0; v < PPT; ++v) F[v] = F[v] * F[v];
            }
            fft_rows_pp<T, MSZ, -1>(F, buf0, buf1, ph, lane, tw, ok);
            {
                double2 z = z0;
#pragma unroll
                for (int v = 0; v < PPT; ++v) {
                    F[v] = scale(r > 0 ? mul_tw<true>(F[v], z, a.hiprec) : F[v], invN);
                    z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
                }
            }
            int e = 0;  // (t r) mod q
#pragma unroll
            for (int t = 0; t < QO; ++t) {
                if (t < a.qout) {
                    const double2 w = twq[e];
#pragma unroll
                    for (int v = 0; v < PPT; ++v)
                        acc[t][v] = acc[t][v] + (t == 0 ? F[v] : mul_tw<true>(F[v], w, false));
                }
                e += r;
                if (e >= a.q) e -= a.q;
            }
        }
        if (ok) {
            cplx<T>* h = hg + row_base(a.out, row);
#pragma unroll
            for (int t = 0; t < QO; ++t) {
                if (t < a.qout) {
#pragma unroll
                    for (int v = 0; v < PPT; ++v) {
                        const int k = t * MSZ + lane + v * TPF;
                        if (k < M) h[(int64_t)k * oes] = acc[t][v];
                    }
                }
            }
        }
    }
}

template <typename T, int MSZ, bool MULTI = false>
__global__ void __launch_bounds__(512) k_fused(FusedArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    fused_rows<T, MSZ, MULTI>(a, a.f, a.g, a.h, a.same != 0, blockIdx.x, smem_raw);
}

// Persistent fused kernel of a batch: every workgroup takes items (bucket,
// FFT size, block of rows) from a queue with an integer atomic counter (zeroed
// by the launch before it) until the queue is empty, and runs the fused body
// for the item's bucket; items are queued largest transform first.  No
// workgroup waits for another, so every wave reaches the end of the queue.
// Sizes: m <= 4096 (complex64), m <= 512 (complex128; see kQueueMaxM128).
template <typename T>
__global__ void __launch_bounds__(512) k_fused_queue(FusedQueueArgs q) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(q.counter, 1);
        __syncthreads();
        const int it = item_s;
        __syncthreads();
        if (it >= q.nitems) break;
        const FusedArgs& a = q.args[q.items[3 * it]];
        const int m = q.items[3 * it + 1];
        const int64_t blk = q.items[3 * it + 2];
        switch (m) {
#define HDC_QCASE(n) \
    case n: fused_rows<T, n>(a, q.f, q.g, q.h, q.same != 0, blk, smem_raw); break;
            HDC_QCASE(1) HDC_QCASE(2) HDC_QCASE(4) HDC_QCASE(8) HDC_QCASE(16) HDC_QCASE(32) HDC_QCASE(64)
            HDC_QCASE(128) HDC_QCASE(256) HDC_QCASE(512)
#undef HDC_QCASE
            // the complex128 bodies above 512 points need 234-244 VGPRs: with
            // the queue around them the kernel would spill, so such buckets run
            // their own launches
            case 1024:
                if constexpr (sizeof(T) == 4) fused_rows<T, 1024>(a, q.f, q.g, q.h, q.same != 0, blk, smem_raw);
                break;
            case 2048:
                if constexpr (sizeof(T) == 4) fused_rows<T, 2048>(a, q.f, q.g, q.h, q.same != 0, blk, smem_raw);
                break;
            case 4096:
                if constexpr (sizeof(T) == 4) fused_rows<T, 4096>(a, q.f, q.g, q.h, q.same != 0, blk, smem_raw);
                break;
            default: break;
        }
    }
}

__global__ void k_zero_counter(int* c) { *c = 0; }

// Real N-D data: f * g = Im(z * z) / (2 s) for z = f + i s g (the convolution is
// bilinear: z * z = f * f - s^2 g * g + 2 i s f * g), one complex
// autoconvolution instead of two forward transforms.  s = max|f| / max|g|
// balances the two terms' scales; the maxima are exact and order-independent
// (integer maxima of the non-negative values' bit patterns).
template <typename T>
struct AbsBits;
template <>
struct AbsBits<float> {
    using U = unsigned int;
    static __device__ U bits(float x) { return __float_as_uint(fabsf(x)); }
    static __device__ float value(U u) { return __uint_as_float(u); }
};
template <>
struct AbsBits<double> {
    using U = unsigned long long;
    static __device__ U bits(double x) { return (U)__double_as_longlong(fabs(x)); }
    static __device__ double value(U u) { return __longlong_as_double((long long)u); }
};

template <typename T>
__global__ void k_real_clear(typename AbsBits<T>::U* mx) {
    if (threadIdx.x < 2) mx[threadIdx.x] = 0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_real_absmax(const T* x, int64_t n, typename AbsBits<T>::U* mx) {
    using U = typename AbsBits<T>::U;
    __shared__ U red[256];
    U v = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const U b = AbsBits<T>::bits(x[i]);
        v = b > v ? b : v;
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && red[threadIdx.x + w] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(mx, red[0]);
}

template <typename T>
__device__ __forceinline__ T real_scale(const typename AbsBits<T>::U* mx) {
    const T a = AbsBits<T>::value(mx[0]), b = AbsBits<T>::value(mx[1]);
    return (a > 0 && b > 0) ? a / b : (T)1;
}

// ------------------------------------------------------- column kernels --
//
// A workgroup owns `tile` adjacent columns c' (coalesced) and all m1 rows of
// one residue (forward) or all residues of a group (backward).  LDS holds an
// m1 x tile block, element (pos, cc) at pos*tile + cc.
//
// Column c' = s2*C1 + c1 (s2 < m2 the four-step column, c1 < C1 the copy);
// axis index j = t*m + s1*m2 + s2 lives at element (t*m1 + s1)*Ccols + c'.

// REAL: the input is two real arrays x (f) and x2 (g), transformed together as
// z = f + i g (the real case, whose product stage pairs residue r with q - r).
// (the real variant reads two arrays of half-size values: its threads own 16
// points each, so that 8 columns, 64-byte segments of each array, take at most
// 512 threads and the registers fit without spilling)
template <int M1, bool REAL>
constexpr int colf_ppt() {
    return (REAL && M1 >= 16) ? 16 : (M1 >= 8 ? 8 : M1);
}

// SC (with REAL): real N-D data, g read as s g (the scale words in a.gs).
template <typename T, int M1, bool REAL = false, bool SC = false>
__global__ void __launch_bounds__(REAL ? 512 : 1024) k_col_fwd(ColFwdArgs a) {
    using P = FP<M1, colf_ppt<M1, REAL>()>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* tpt = lds + (size_t)M1 * a.tile;
    fill_pass_tab<T, M1>(tpt, a.tw1, threadIdx.x, blockDim.x);
    __syncthreads();
    const TwPass<T> tw1{tpt, PassTab<M1>::R0};

    // task = (tile, residue) with the residue fastest: the Dg residues of a
    // tile run back to back on one XCD and re-read its input from that L2
    const int task = xcd_task(blockIdx.x, gridDim.x);
    if (task >= a.ntiles * a.Dg) return;
    const int tl = task / a.Dg;
    const int dd = task - tl * a.Dg;
    // residue slot dd = d lam + li holds r = r0 + d + li rstride, stored at row
    // block (d m1 + l1) lam + li (section 3.5's matching when lam > 1)
    const int d = dd / a.lam;
    const int li = dd - d * a.lam;
    // the last nsec slots hold the descending residues r2, r2 - 1, ...
    const int dg1 = a.Dg - a.nsec;
    const bool second = dd >= dg1;
    const int tile = a.tile;
    const int tid = threadIdx.x;
    const int cc = tid % tile;
    const int lane = tid / tile;
    const int64_t b = blockIdx.y;
    const int cp = tl * tile + cc;
    const bool ok = cp < a.Ccols;
    const int s2 = ok ? cp / a.C1 : 0;
    int64_t xoff = b * a.in_bs;
    int64_t L = a.L;
    if (a.desc != nullptr) {
        xoff = a.desc[2 * b];
        L = a.desc[2 * b + 1];
    }
    const cplx<T>* x = reinterpret_cast<const cplx<T>*>(a.x) + xoff;
    const T* xr = reinterpret_cast<const T*>(a.x) + xoff;
    const T* xi = reinterpret_cast<const T*>(a.x2) + xoff;
    // real N-D data: g enters as s g
    T gsc = (T)1;
    if constexpr (SC) gsc = real_scale<T>(reinterpret_cast<const typename AbsBits<T>::U*>(a.gs));
    cplx<T>* X = reinterpret_cast<cplx<T>*>(a.X) + b * a.out_bs;

    // block t, point v of this thread: x[(t*m1 + s1)*Ccols + cp] with s1 = lane + v TPF,
    // axis index j = t m + s1 m2 + s2, zero for j >= L.  Per-thread bases plus uniform
    // strides, so the per-point offsets are scalar products.
    const int64_t ibase = (int64_t)lane * a.Ccols + cp, istep_v = (int64_t)TPF * a.Ccols,
                  istep_t = (int64_t)M1 * a.Ccols;
    const int64_t jbase = (int64_t)lane * a.m2 + s2, jstep_v = (int64_t)TPF * a.m2,
                  jstep_t = (int64_t)M1 * a.m2;
#define HDC_IDX(t, v) ((t) * istep_t + ibase + (v) * istep_v)
#define HDC_LOAD(t, v)                                                                        \
    ((ok && (t) * jstep_t + jbase + (v) * jstep_v < L)                                        \
         ? (REAL ? mk<T>(xr[HDC_IDX(t, v)], SC ? gsc * xi[HDC_IDX(t, v)] : xi[HDC_IDX(t, v)])  \
                 : x[HDC_IDX(t, v)])                                                          \
         : mk<T>(0, 0))

    {
        const int r = second ? a.r2 - (dd - dg1) : a.r0 + d + li * a.rstride;
        cplx<T> w[PPT];
#pragma unroll
        for (int v = 0; v < PPT; ++v) w[v] = HDC_LOAD(0, v);
        int e = r;  // (r t) mod q for t = 1
        if (e >= a.q) e -= a.q;
        for (int t = 1; t < a.p; ++t) {
            const double2 z = tw_n(a.tw, (uint32_t)e * (uint32_t)a.m);
            e += r;
            if (e >= a.q) e -= a.q;
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                w[v] = w[v] + mul_tw<false>(HDC_LOAD(t, v), z, a.hiprec);
            }
        }
        if (r != 0) {
            // zeta_N^{r s}, s = (lane + v TPF) m2 + s2: z0 zs^v (r < q and s < m, so
            // r s < q m = N needs no reduction)
            double2 z = tw_n(a.tw, (uint32_t)r * (uint32_t)jbase);
            const double2 zs = tw_n(a.tw, (uint32_t)r * (uint32_t)jstep_v);
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                w[v] = mul_tw<false>(w[v], z, a.hiprec);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
        fft_regs<T, M1, +1, LAY_COL, PPT>(w, lds + cc, tile, lane, tw1, true);
        if (a.m2 > 1 && s2 != 0) {
            // four-step twiddle zeta_m^{l1 s2}, l1 = lane + v TPF: z0 zs^v
            double2 z = tw_n(a.tw, (uint32_t)lane * (uint32_t)s2 * (uint32_t)a.q);
            const double2 zs = tw_n(a.tw, (uint32_t)TPF * (uint32_t)s2 * (uint32_t)a.q);
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                w[v] = mul_tw<false>(w[v], z, a.hiprec);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
        // X[((d m1 + l1) lam + li) Ccols + cp], l1 = lane + v TPF
        const int64_t obase = (((int64_t)d * M1 + lane) * a.lam + li) * a.Ccols + cp;
        const int64_t ostep = (int64_t)TPF * a.lam * a.Ccols;
#pragma unroll
        for (int v = 0; v < PPT; ++v) {
            if (ok) X[obase + v * ostep] = w[v];
        }
    }
#undef HDC_LOAD
#undef HDC_IDX
}

// REAL: the residues are those of a Hermitian product (real output, the real
// case of section 7): only r <= q/2 are given, each counted twice except r = 0
// and r = q/2, and the real part is written to a real h.
// IM (with REAL): real N-D data, h = Im(...) / (2 s) (the scale words in a.gs)
// instead of the Hermitian residues' weighted real part.
template <typename T, int M1, int DMAX, bool REAL = false, bool IM = false>
__global__ void __launch_bounds__(512) k_col_bwd(ColBwdArgs a) {
    using P = FP<M1>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* tpt = lds + (size_t)M1 * a.tile;
    fill_pass_tab<T, M1>(tpt, a.tw1, threadIdx.x, blockDim.x);
    __syncthreads();
    const TwPass<T> tw1{tpt, PassTab<M1>::R0};

    const int tl = xcd_task(blockIdx.x, gridDim.x);
    if (tl >= a.ntiles) return;
    const int tile = a.tile;
    const int tid = threadIdx.x;
    const int cc = tid % tile;
    const int lane = tid / tile;
    const int64_t b = blockIdx.y;
    const int cp = tl * tile + cc;
    const bool ok = cp < a.Ccols;
    const int s2 = ok ? cp / a.C1 : 0;
    int64_t hoff = b * a.out_bs;
    int64_t M = a.M;
    if (a.desc != nullptr) {
        hoff = a.desc[2 * b];
        M = a.desc[2 * b + 1];
    }
    const cplx<T>* Y = reinterpret_cast<const cplx<T>*>(a.Y) + b * a.in_bs;
    cplx<T>* h = reinterpret_cast<cplx<T>*>(a.h) + hoff;
    T* hr = reinterpret_cast<T*>(a.h) + hoff;
    T wim = (T)0;
    if constexpr (IM) wim = (T)0.5 / real_scale<T>(reinterpret_cast<const typename AbsBits<T>::U*>(a.gs));
    const T invN = (T)a.invN;
    // four-step twiddle conj(zeta_m^{l1 s2}), l1 = lane + v TPF, as z0 zs^v
    const bool fs = a.m2 > 1 && s2 != 0;
    const double2 fz0 = fs ? tw_n(a.tw, (uint32_t)lane * (uint32_t)s2 * (uint32_t)a.q) : make_double2(1.0, 0.0);
    const double2 fzs = fs ? tw_n(a.tw, (uint32_t)TPF * (uint32_t)s2 * (uint32_t)a.q) : make_double2(1.0, 0.0);

    // per-thread bases and uniform strides of the residue reads Y[(d m1 + l1) Ccols + cp],
    // l1 = lane + v TPF, and of the output h[(t m1 + s1) Ccols + cp] at axis index
    // k = t m + s1 m2 + s2, s1 = lane + v TPF
    const int64_t ibase = (int64_t)lane * a.Ccols + cp, istep_v = (int64_t)TPF * a.Ccols,
                  istep_t = (int64_t)M1 * a.Ccols;
    // (k < qout m <= N fits 32 bits; the output offsets stay 64-bit from a per-block base)
    const int kbase = lane * a.m2 + s2, kstep_v = TPF * a.m2, kstep_t = M1 * a.m2;

    for (int db = 0; db < a.Dg; db += DMAX) {
        const int nd = min(DMAX, a.Dg - db);
        cplx<T> V[DMAX][PPT];
        // every residue's reads are issued first, so that those of the later
        // residues stay in flight behind the first transforms
#pragma unroll
        for (int dd = 0; dd < DMAX; ++dd) {
            const int64_t rb = (int64_t)(db + dd) * istep_t + ibase;
#pragma unroll
            for (int v = 0; v < PPT; ++v) V[dd][v] = (ok && dd < nd) ? Y[rb + v * istep_v] : mk<T>(0, 0);
        }
#pragma unroll
        for (int dd = 0; dd < DMAX; ++dd) {
            if (dd < nd) {
                if (fs) {
                    double2 z = fz0;
#pragma unroll
                    for (int v = 0; v < PPT; ++v) {
                        V[dd][v] = mul_tw<true>(V[dd][v], z, a.hiprec);
                        z = make_double2(z.x * fzs.x - z.y * fzs.y, z.x * fzs.y + z.y * fzs.x);
                    }
                }
                fft_regs<T, M1, -1, LAY_COL>(V[dd], lds + cc, tile, lane, tw1, true);
                const int r = a.r0 + db + dd;
                // conj(zeta_N^{r s}), s = (lane + v TPF) m2 + s2, as z0 zs^v (r < q and
                // s < m, so r s < q m = N needs no reduction)
                double2 z = tw_n(a.tw, (uint32_t)r * (uint32_t)kbase);
                const double2 zs = tw_n(a.tw, (uint32_t)r * (uint32_t)kstep_v);
#pragma unroll
                for (int v = 0; v < PPT; ++v) {
                    V[dd][v] = scale(mul_tw<true>(V[dd][v], z, a.hiprec), invN);
                    z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
                }
            }
        }
        const bool add = a.accumulate || db > 0;
        // (t r) mod q for residue r = r0 + db + dd, advanced by r per block t (r < q, so
        // one subtraction keeps it below q; unused slots dd >= nd stay at 0)
        int e[DMAX], rs[DMAX];
#pragma unroll
        for (int dd = 0; dd < DMAX; ++dd) {
            e[dd] = 0;
            rs[dd] = dd < nd ? a.r0 + db + dd : 0;
        }
        for (int t = 0; t < a.qout; ++t) {
            cplx<T>* ht = h + t * istep_t + ibase;
            T* hrt = hr + t * istep_t + ibase;
            const int kt = t * kstep_t + kbase;
            double2 z[DMAX];
#pragma unroll
            for (int dd = 0; dd < DMAX; ++dd) {
                z[dd] = tw_n(a.tw, (uint32_t)e[dd] * (uint32_t)a.m);
                e[dd] += rs[dd];
                if (e[dd] >= a.q) e[dd] -= a.q;
            }
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                const int k = kt + v * kstep_v;
                if (!ok || k >= M) continue;
                const int64_t idx = v * istep_v;
                if constexpr (REAL) {
                    T acc = 0;
#pragma unroll
                    for (int dd = 0; dd < DMAX; ++dd) {
                        if (dd < nd) {
                            const cplx<T> u = mul_tw<true>(V[dd][v], z[dd], false);
                            if constexpr (IM) {  // real N-D: Im(z * z) / (2 s)
                                acc += wim * u.y;
                            } else {  // Hermitian residues: weight 2 but for r = 0 and r = q/2
                                const int r = a.r0 + db + dd;
                                acc += ((r == 0 || 2 * r == a.q) ? (T)1 : (T)2) * u.x;
                            }
                        }
                    }
                    if (add) acc += hrt[idx];
                    hrt[idx] = acc;
                } else {
                    cplx<T> acc = mk<T>(0, 0);
#pragma unroll
                    for (int dd = 0; dd < DMAX; ++dd)
                        if (dd < nd) acc = acc + mul_tw<true>(V[dd][v], z[dd], false);
                    if (add) acc = acc + ht[idx];
                    ht[idx] = acc;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- rows --

// Operand a's row formed from the raw shorter operand (section 3.5, its column
// stage trivial): row (d m1g + l1g) C1 + c1 holds residue r = r0 + d + l1g qg,
//   w_s = zeta_N^{r s} sum_{t < pf} zeta_qf^{r t} f_{(t m2 + s) C1 + c1},  s < m2.
template <typename T, int MSZ>
__device__ __forceinline__ void raw_row(const RowArgs& a, int64_t row, bool ok, int lane, cplx<T>* v) {
    constexpr int PPT = FP<MSZ>::PPT;
    constexpr int TPF = FP<MSZ>::TPF;
#pragma unroll
    for (int w = 0; w < PPT; ++w) v[w] = mk<T>(0, 0);
    if (!ok) return;
    // the host keeps nrows below 2^31 for this mode
    const uint32_t C1 = (uint32_t)a.addr.inner_cnt;
    const uint32_t rw = (uint32_t)row;
    const uint32_t c1 = rw % C1;
    const uint32_t t1 = rw / C1;
    const uint32_t l1 = t1 % (uint32_t)a.m1g;
    const uint32_t t2 = t1 / (uint32_t)a.m1g;
    const uint32_t b = t2 / (uint32_t)a.Dg;
    const uint32_t r = (uint32_t)a.r0 + (t2 - b * (uint32_t)a.Dg) + l1 * (uint32_t)a.qg;
    const cplx<T>* f = reinterpret_cast<const cplx<T>*>(a.fraw) + (int64_t)b * a.fbs + c1;
#pragma unroll
    for (int w = 0; w < PPT; ++w) {
        const int j = lane + w * TPF;
        if (j < a.Lf) v[w] = f[(int64_t)j * C1];
    }
    uint32_t e = r;  // (r t) mod qf for t = 1
    for (int t = 1; t < a.pf; ++t) {
        const double2 z = tw_n(a.twN, e * (uint32_t)MSZ);
        e += r;
        if (e >= (uint32_t)a.qf) e -= (uint32_t)a.qf;
#pragma unroll
        for (int w = 0; w < PPT; ++w) {
            const int j = t * MSZ + lane + w * TPF;
            if (j < a.Lf) v[w] = v[w] + mul_tw<false>(f[(int64_t)j * C1], z, a.hiprec);
        }
    }
    if (r != 0) {
        // r < qf and lane < TPF = m2 / PPT, so r lane and r TPF stay below N
        double2 z = tw_n(a.twN, r * (uint32_t)lane);
        const double2 zs = tw_n(a.twN, r * (uint32_t)TPF);
#pragma unroll
        for (int w = 0; w < PPT; ++w) {
            v[w] = mul_tw<false>(v[w], z, a.hiprec);
            z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
        }
    }
}

// Persistent row kernel: the workgroup walks rows base, base + stride, ...
// with a skewed software pipeline: the g row of iteration i is loaded when
// the iteration starts (hidden behind the f transform), and the f row of
// iteration i+1 is loaded before the g transform (hidden behind the g
// transform, the product and the inverse), so HBM traffic overlaps the LDS
// passes while only three rows of registers are live.
template <typename T, int MSZ, int MODE, bool TWO, bool FRAW>
__global__ void __launch_bounds__(512) k_row(RowArgs a) {
    using P = FP<MSZ>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* tpt = smem + (size_t)a.rpw * 2 * MSZ;
    const int tid = threadIdx.x;
    fill_pass_tab<T, MSZ>(tpt, a.twp, tid, blockDim.x);
    __syncthreads();
    const TwPass<T> tw{tpt, PassTab<MSZ>::R0};

    const int rloc = tid / TPF;
    const int lane = tid - rloc * TPF;
    // two exchange buffers per row, used in turn
    cplx<T>* buf0 = smem + (size_t)rloc * 2 * MSZ;
    cplx<T>* buf1 = buf0 + MSZ;
    int ph = 0;
    const int64_t es = a.addr.es;
    // point w of this thread sits at row base + lane es + w (TPF es)
    const int64_t lbase = (int64_t)lane * es, wstep = (int64_t)TPF * es;
    const int64_t stride = (int64_t)gridDim.x * a.rpw;
    constexpr bool conv = MODE == MODE_CONV;
    constexpr bool two = conv && TWO;
    const cplx<T>* Ag = reinterpret_cast<const cplx<T>*>(a.a);
    const cplx<T>* Bg = reinterpret_cast<const cplx<T>*>(a.b);
    cplx<T>* Og = reinterpret_cast<cplx<T>*>(a.out);

    int64_t base = (int64_t)blockIdx.x * a.rpw;  // uniform over the workgroup
    cplx<T> v[PPT];
    if constexpr (!FRAW) {
        const int64_t row = base + rloc;
        const bool ok = row < a.nrows;
        const int64_t rb = row_base(a.addr, ok ? row : 0);
#pragma unroll
        for (int w = 0; w < PPT; ++w) v[w] = ok ? Ag[rb + lbase + w * wstep] : mk<T>(0, 0);
    }
    for (; base < a.nrows; base += stride) {
        const int64_t row = base + rloc;
        const bool ok = row < a.nrows;
        const int64_t rb = row_base(a.addr, ok ? row : 0);
        const int64_t nrow = row + stride;
        const bool nok = nrow < a.nrows;
        const int64_t nrb = row_base(a.addr, nok ? nrow : 0);
        cplx<T> u[PPT], pv[PPT];
        if constexpr (two) {
#pragma unroll
            for (int w = 0; w < PPT; ++w) u[w] = ok ? Bg[rb + lbase + w * wstep] : mk<T>(0, 0);
        }
        // a raw operand row is formed from L2-resident input while the b row
        // is in flight, so it needs no prefetch
        if constexpr (FRAW) raw_row<T, MSZ>(a, row, ok, lane, v);
        if constexpr (MODE == MODE_INV) {
#pragma unroll
            for (int w = 0; w < PPT; ++w) pv[w] = nok ? Ag[nrb + lbase + w * wstep] : mk<T>(0, 0);
            fft_rows_pp<T, MSZ, -1>(v, buf0, buf1, ph, lane, tw, ok);
        } else {
            fft_rows_pp<T, MSZ, +1>(v, buf0, buf1, ph, lane, tw, ok);
            if constexpr (!FRAW) {
#pragma unroll
                for (int w = 0; w < PPT; ++w) pv[w] = nok ? Ag[nrb + lbase + w * wstep] : mk<T>(0, 0);
            }
            if constexpr (conv) {
                if constexpr (two) {
                    fft_rows_pp<T, MSZ, +1>(u, buf0, buf1, ph, lane, tw, ok);
#pragma unroll
                    for (int w = 0; w < PPT; ++w) v[w] = v[w] * u[w];
                } else {
#pragma unroll
                    for (int w = 0; w < PPT; ++w) v[w] = v[w] * v[w];
                }
                fft_rows_pp<T, MSZ, -1>(v, buf0, buf1, ph, lane, tw, ok);
            }
        }
        if (ok) {
#pragma unroll
            for (int w = 0; w < PPT; ++w) Og[rb + lbase + w * wstep] = v[w];
        }
        if constexpr (!FRAW) {
#pragma unroll
            for (int w = 0; w < PPT; ++w) v[w] = pv[w];
        }
    }
}

// Multi-convolution rows (section 6.1): operand o's row of the group sits at
// a + o ostride; the row DFTs of all nops operands multiply into one product,
// whose inverse overwrites operand 0's row.
template <typename T, int MSZ>
__global__ void __launch_bounds__(512) k_row_multi(RowArgs a) {
    using P = FP<MSZ>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* tpt = smem + (size_t)a.rpw * 2 * MSZ;
    const int tid = threadIdx.x;
    fill_pass_tab<T, MSZ>(tpt, a.twp, tid, blockDim.x);
    __syncthreads();
    const TwPass<T> tw{tpt, PassTab<MSZ>::R0};
    const int rloc = tid / TPF;
    const int lane = tid - rloc * TPF;
    cplx<T>* buf0 = smem + (size_t)rloc * 2 * MSZ;
    cplx<T>* buf1 = buf0 + MSZ;
    int ph = 0;
    const int64_t es = a.addr.es;
    const int64_t lbase = (int64_t)lane * es, wstep = (int64_t)TPF * es;  // point w at lbase + w wstep
    const int64_t stride = (int64_t)gridDim.x * a.rpw;
    const cplx<T>* X = reinterpret_cast<const cplx<T>*>(a.a);
    cplx<T>* Og = reinterpret_cast<cplx<T>*>(a.out);
    for (int64_t base = (int64_t)blockIdx.x * a.rpw; base < a.nrows; base += stride) {
        const int64_t row = base + rloc;
        const bool ok = row < a.nrows;
        const int64_t rb = row_base(a.addr, ok ? row : 0);
        cplx<T> v[PPT], u[PPT];
#pragma unroll
        for (int w = 0; w < PPT; ++w) v[w] = ok ? X[rb + lbase + w * wstep] : mk<T>(0, 0);
        fft_rows_pp<T, MSZ, +1>(v, buf0, buf1, ph, lane, tw, ok);
        for (int o = 1; o < a.nops; ++o) {
            const cplx<T>* Xo = X + o * a.ostride;
#pragma unroll
            for (int w = 0; w < PPT; ++w) u[w] = ok ? Xo[rb + lbase + w * wstep] : mk<T>(0, 0);
            fft_rows_pp<T, MSZ, +1>(u, buf0, buf1, ph, lane, tw, ok);
#pragma unroll
            for (int w = 0; w < PPT; ++w) v[w] = v[w] * u[w];
        }
        fft_rows_pp<T, MSZ, -1>(v, buf0, buf1, ph, lane, tw, ok);
        if (ok) {
#pragma unroll
            for (int w = 0; w < PPT; ++w) Og[rb + lbase + w * wstep] = v[w];
        }
    }
}

// --------------------------------------------------------------- real case --
//
// Real f and g are transformed together as z = f + i g, so Z_k = F_k + i G_k
// with F, G Hermitian: F_k = (Z_k + conj Z_{N-k}) / 2, G_k = (Z_k - conj Z_{N-k}) / (2i)
// and H_k = F_k G_k = (Z_k^2 - (conj Z_{N-k})^2) / (4i).  With k = q l + r,
// N - k lies in residue q - r at l' = m - 1 - l (residue 0: l' = -l mod m); in
// the four-step order l = l1 + m1 l2 that is row m1 - 1 - l1, point m2 - 1 - l2
// (residue 0, l1 > 0: row m1 - l1, point m2 - 1 - l2; residue 0, l1 = 0: row 0,
// point -l2 mod m2).  A row DFT turns a conjugated row pre-multiplied by
// zeta_m2^{s} into conj X_{m2-1-l2} (unmultiplied: conj X_{-l2}), so the partner
// arrives in the right registers without a permutation.  H is Hermitian too,
// so only residues r <= q/2 are formed and inverted.

// Work items of a group's product rows.  A residue j other than 0 and q/2
// pairs with residue q - j (stored in slot Dg + j - pfirst): each of its m1
// rows is one item, its row l1 against the partner's row m1 - 1 - l1.  The
// residues 0 and q/2 pair with themselves, row l1 with row l1' (m1 - l1 mod m1
// for 0, m1 - 1 - l1 for q/2): H is Hermitian, so the inverse of row l1' is
// zeta_m2^s conj(inverse of row l1) and one item (l1 < l1') gives both rows;
// a row that is its own partner is an item of its own.  Per batch and copy
// the items run residue 0 (m1/2 + 1 of them, or 1 when m1 = 1), the other
// residues (m1 each), residue q/2 (m1/2, or 1), which is always last in its
// group.  Z holds S slots per batch (slot d < Dg: residue r0 + d).
struct RealItem {
    int64_t ab, pb, ob, ob2;  // Z row, partner Z row, output row, mirrored output row (-1: none)
    bool rev;                 // partner points run m2 - 1 - l2 (else -l2)
};

__device__ __forceinline__ RealItem real_item(const RowArgs& a, int64_t item) {
    const int64_t C1 = a.addr.inner_cnt;
    const int64_t m1 = a.m1g;
    const int64_t n0 = m1 == 1 ? 1 : m1 / 2 + 1;
    const int64_t nh = m1 == 1 ? 1 : m1 / 2;
    const bool has0 = a.r0 == 0;
    const bool hash = (a.qg % 2 == 0) && (a.r0 + a.Dg - 1 == a.qg / 2) && a.qg / 2 != 0;
    const int64_t W = a.Dg * m1 - (has0 ? m1 - n0 : 0) - (hash ? m1 - nh : 0);
    const int64_t c1 = item % C1;
    const int64_t t1 = item / C1;
    const int64_t b = t1 / W;
    int64_t t = t1 - b * W;
    int64_t d, l1;
    if (has0 && t < n0) {
        d = 0;
        l1 = t;
    } else {
        if (has0) t -= n0;
        const int64_t d0 = has0 ? 1 : 0;
        d = d0 + t / m1;
        l1 = t - (d - d0) * m1;
    }
    const int64_t j = a.r0 + d;
    int64_t ps, pl;
    RealItem it;
    bool self = false;
    if (j == 0) {
        ps = d;
        pl = l1 == 0 ? 0 : m1 - l1;
        it.rev = l1 != 0;
        self = true;
    } else {
        self = 2 * j == a.qg;
        ps = self ? d : a.Dg + (j - a.pfirst);
        pl = m1 - 1 - l1;
        it.rev = true;
    }
    const int64_t os = a.addr.outer_stride;  // m2 C1
    it.ab = ((b * a.S + d) * m1 + l1) * os + c1;
    it.pb = ((b * a.S + ps) * m1 + pl) * os + c1;
    it.ob = ((b * a.Dg + d) * m1 + l1) * os + c1;
    it.ob2 = (self && pl != l1) ? ((b * a.Dg + d) * m1 + pl) * os + c1 : -1;
    return it;
}

template <typename T, int MSZ>
__global__ void __launch_bounds__(512) k_row_real(RowArgs a) {
    using P = FP<MSZ>;
    using S = TwSplit<MSZ>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* tlo = smem + (size_t)a.rpw * 2 * MSZ;
    cplx<T>* thi = tlo + S::LO;
    cplx<T>* tpt = thi + S::HI;
    const int tid = threadIdx.x;
    const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.tw);
    for (int e = tid; e < S::LO; e += blockDim.x) tlo[e] = twg[e];
    for (int e = tid; e < S::HI; e += blockDim.x) thi[e] = twg[e * S::LO];
    fill_pass_tab<T, MSZ>(tpt, a.twp, tid, blockDim.x);
    __syncthreads();
    const TwLds<T> twl{tlo, thi, S::LO - 1, S::LG};  // zeta_m2^s for the partner rows
    const TwPass<T> tw{tpt, PassTab<MSZ>::R0};
    const int rloc = tid / TPF;
    const int lane = tid - rloc * TPF;
    cplx<T>* buf0 = smem + (size_t)rloc * 2 * MSZ;  // two exchange buffers, used in turn
    cplx<T>* buf1 = buf0 + MSZ;
    int ph = 0;
    const int64_t es = a.addr.es;
    const int64_t stride = (int64_t)gridDim.x * a.rpw;
    const cplx<T>* Z = reinterpret_cast<const cplx<T>*>(a.a);
    cplx<T>* Og = reinterpret_cast<cplx<T>*>(a.out);
    for (int64_t base = (int64_t)blockIdx.x * a.rpw; base < a.nrows; base += stride) {
        const int64_t row = base + rloc;
        const bool ok = row < a.nrows;
        const RealItem it = real_item(a, ok ? row : 0);
        cplx<T> v[PPT], u[PPT];
#pragma unroll
        for (int w = 0; w < PPT; ++w) {
            const int s = lane + w * TPF;
            v[w] = ok ? Z[it.ab + (int64_t)s * es] : mk<T>(0, 0);
            cplx<T> x = ok ? Z[it.pb + (int64_t)s * es] : mk<T>(0, 0);
            x.y = -x.y;
            u[w] = it.rev ? x * twl[s] : x;
        }
        fft_rows_pp<T, MSZ, +1>(v, buf0, buf1, ph, lane, tw, ok);
        fft_rows_pp<T, MSZ, +1>(u, buf0, buf1, ph, lane, tw, ok);
        // H = (Z^2 - W^2) / (4i), W = conj Z_{N-k}
#pragma unroll
        for (int w = 0; w < PPT; ++w) v[w] = scale(mul_i<-1>(v[w] * v[w] - u[w] * u[w]), (T)0.25);
        fft_rows_pp<T, MSZ, -1>(v, buf0, buf1, ph, lane, tw, ok);
        if (ok) {
#pragma unroll
            for (int w = 0; w < PPT; ++w) Og[it.ob + (int64_t)(lane + w * TPF) * es] = v[w];
            if (it.ob2 >= 0) {
                // the mirrored row of a self-paired residue: zeta_m2^s conj(v_s)
#pragma unroll
                for (int w = 0; w < PPT; ++w) {
                    const int s = lane + w * TPF;
                    cplx<T> x = v[w];
                    x.y = -x.y;
                    Og[it.ob2 + (int64_t)s * es] = x * twl[s];
                }
            }
        }
    }
}

// Fused real case: every residue of one row in LDS.  Pass 1 forms Z for all q
// residues; pass 2 forms H for r <= q/2 from Z_r and the mirrored Z_{q-r},
// inverts it and stores u^(r)_s zeta_N^{-r s} / N; the output is the real part
// of the weighted residue sum.  f, g and h are real.
template <typename T, int MSZ>
__global__ void __launch_bounds__(512) k_fused_real(FusedArgs a) {
    using P = FP<MSZ>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
    using S = TwSplit<MSZ>;
    double2* twq =
        reinterpret_cast<double2*>(smem_raw + ((size_t)a.rpw * a.q * padded(MSZ) * sizeof(cplx<T>) + 15) / 16 * 16);
    cplx<T>* tlo = reinterpret_cast<cplx<T>*>(twq + a.q);
    cplx<T>* thi = tlo + S::LO;
    constexpr int RS = padded(MSZ);
    const int rowthreads = TPF * a.Dc;
    const int tid = threadIdx.x;
    const int rloc = tid / rowthreads;
    const int lt = tid - rloc * rowthreads;
    const int grp = lt / TPF;
    const int lane = lt - grp * TPF;
    const int64_t row = (int64_t)blockIdx.x * a.rpw + rloc;
    const bool rowok = row < a.nrows;
    for (int e = tid; e < a.q; e += blockDim.x) twq[e] = tw_n(a.tw, (uint32_t)e * (uint32_t)MSZ);
    {
        const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.twm);
        for (int e = tid; e < S::LO; e += blockDim.x) tlo[e] = twg[e];
        for (int e = tid; e < S::HI; e += blockDim.x) thi[e] = twg[e * S::LO];
    }
    __syncthreads();
    const TwLds<T> twm{tlo, thi, S::LO - 1, S::LG};
    const int L = a.L, M = a.M, q = a.q;
    const int qh = q / 2 + 1;
    const int64_t fbase = row_base(a.in, rowok ? row : 0);
    const int64_t hbase = row_base(a.out, rowok ? row : 0);
    const int64_t ies = a.in.es, oes = a.out.es;
    const T* f = reinterpret_cast<const T*>(a.f) + fbase;
    const T* g = reinterpret_cast<const T*>(a.g) + fbase;
    T* h = reinterpret_cast<T*>(a.h) + hbase;
    cplx<T>* U = smem + (size_t)rloc * q * RS;
    const T invN = (T)a.invN;

    // pass 1: Z_r for every residue
    for (int rb = 0; rb < q; rb += a.Dc) {
        const int r = rb + grp;
        const bool act = rowok && r < q;
        cplx<T>* buf = U + (size_t)(act ? r : 0) * RS;
        cplx<T> Zr[PPT];
#pragma unroll
        for (int v = 0; v < PPT; ++v) Zr[v] = mk<T>(0, 0);
        if (act) {
            int e = 0;
            for (int t = 0; t < a.p; ++t) {
                const double2 z = twq[e];
                e += r;
                if (e >= q) e -= q;
#pragma unroll
                for (int v = 0; v < PPT; ++v) {
                    const int j = t * MSZ + lane + v * TPF;
                    if (j < L) Zr[v] = Zr[v] + mul_tw<false>(mk<T>(f[(int64_t)j * ies], g[(int64_t)j * ies]), z, false);
                }
            }
        }
        const uint32_t ru = (uint32_t)(act ? r : 0);
        {
            double2 z = tw_n(a.tw, ru * (uint32_t)lane);
            const double2 zs = tw_n(a.tw, ru * (uint32_t)TPF);
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                Zr[v] = mul_tw<false>(Zr[v], z, a.hiprec);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
        fft_regs<T, MSZ, +1, LAY_PAD>(Zr, buf, 1, lane, twm, act);
        if (act) {
#pragma unroll
            for (int v = 0; v < PPT; ++v) buf[lds_at<LAY_PAD, T, MSZ>(lane + v * TPF, 1)] = Zr[v];
        }
        __syncthreads();
    }
    // pass 2: H_r, r <= q/2, inverted in place
    for (int rb = 0; rb < qh; rb += a.Dc) {
        const int r = rb + grp;
        const bool act = rowok && r < qh;
        const int ru = act ? r : 0;
        cplx<T>* buf = U + (size_t)ru * RS;
        const cplx<T>* pbuf = U + (size_t)(ru == 0 ? 0 : q - ru) * RS;
        cplx<T> Hr[PPT];
#pragma unroll
        for (int v = 0; v < PPT; ++v) {
            const int l = lane + v * TPF;
            const int lp = ru == 0 ? (l == 0 ? 0 : MSZ - l) : MSZ - 1 - l;
            const cplx<T> z = act ? buf[lds_at<LAY_PAD, T, MSZ>(l, 1)] : mk<T>(0, 0);
            cplx<T> w = act ? pbuf[lds_at<LAY_PAD, T, MSZ>(lp, 1)] : mk<T>(0, 0);
            w.y = -w.y;
            Hr[v] = scale(mul_i<-1>(z * z - w * w), (T)0.25);
        }
        __syncthreads();  // every partner read before the transforms reuse the buffers
        fft_regs<T, MSZ, -1, LAY_PAD>(Hr, buf, 1, lane, twm, act);
        if (act) {
            double2 z = tw_n(a.tw, (uint32_t)ru * (uint32_t)lane);
            const double2 zs = tw_n(a.tw, (uint32_t)ru * (uint32_t)TPF);
#pragma unroll
            for (int v = 0; v < PPT; ++v) {
                buf[lds_at<LAY_PAD, T, MSZ>(lane + v * TPF, 1)] = scale(mul_tw<true>(Hr[v], z, a.hiprec), invN);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
        __syncthreads();
    }
    if (!rowok) return;
    // h_{t m + s} = Re sum_{r <= q/2} w_r zeta_q^{-t r} U[r][s]
    for (int k = lt; k < M; k += rowthreads) {
        const int t = k / MSZ;
        const int s2 = k - t * MSZ;
        T acc = 0;
        int e = 0;
        for (int r = 0; r < qh; ++r) {
            const T wgt = (r == 0 || 2 * r == q) ? (T)1 : (T)2;
            acc += wgt * mul_tw<true>(U[(size_t)r * RS + lds_at<LAY_PAD, T, MSZ>(s2, 1)], twq[e], false).x;
            e += t;
            if (e >= q) e -= q;
        }
        h[(int64_t)k * oes] = acc;
    }
}

// ------------------------------------------- raw residue rows (m1 = 1) --
//
// When a residue transform is a single row (m <= 4096, no column stage), a
// workgroup forms residue r of both operands straight from their inputs: the
// block sum of eq. (3), sum_{t<p} zeta_q^{r t} x_{t m + s}, times zeta_N^{r s},
// transforms the two rows, multiplies them, inverts the product and stores
//     y^(r)_s = zeta_N^{-r s} u^(r)_s / N,
// residue r's term of eq. (4) before the sum over r.  Each residue reads the
// inputs again; the problems this path serves (q <= 32, so L <= 16 m) keep
// them in L2, and the residues never pass through HBM before the product.
// k_qsum then forms h_{t m + s} = sum_r zeta_q^{-t r} y^(r)_s.

// Block sum of residue r of x (length L, p blocks, copy stride C1) into the
// points s = lane + w TPF of a row, times zeta_N^{r s}.
template <typename T, int MSZ>
__device__ __forceinline__ void rr_blocksum(const cplx<T>* x, int32_t L, int32_t p, int32_t q, int32_t C1,
                                            uint32_t r, const TwN& tw, bool hp, int lane, cplx<T>* v) {
    constexpr int PPT = FP<MSZ>::PPT;
    constexpr int TPF = FP<MSZ>::TPF;
#pragma unroll
    for (int w = 0; w < PPT; ++w) {
        const int j = lane + w * TPF;
        v[w] = j < L ? x[(int64_t)j * C1] : mk<T>(0, 0);
    }
    uint32_t e = r;  // (r t) mod q for t = 1
    if (e >= (uint32_t)q) e -= (uint32_t)q;
    for (int t = 1; t < p; ++t) {
        const double2 z = tw_n(tw, e * (uint32_t)MSZ);
        e += r;
        if (e >= (uint32_t)q) e -= (uint32_t)q;
#pragma unroll
        for (int w = 0; w < PPT; ++w) {
            const int j = t * MSZ + lane + w * TPF;
            if (j < L) v[w] = v[w] + mul_tw<false>(x[(int64_t)j * C1], z, false);
        }
    }
    if (r != 0) {
        // r < q and s < m, so r s < q m = N needs no reduction
        double2 z = tw_n(tw, r * (uint32_t)lane);
        const double2 zs = tw_n(tw, r * (uint32_t)TPF);
#pragma unroll
        for (int w = 0; w < PPT; ++w) {
            v[w] = mul_tw<false>(v[w], z, hp);
            z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
        }
    }
}

template <typename T, int MSZ>
__global__ void __launch_bounds__(512) k_row_rr(RawArgs a) {
    using P = FP<MSZ>;
    constexpr int PPT = P::PPT;
    constexpr int TPF = P::TPF;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
    cplx<T>* tpt = smem + (size_t)a.rpw * 2 * MSZ;
    const int tid = threadIdx.x;
    fill_pass_tab<T, MSZ>(tpt, a.twp, tid, blockDim.x);
    __syncthreads();
    const TwPass<T> tw{tpt, PassTab<MSZ>::R0};

    const int rloc = tid / TPF;
    const int lane = tid - rloc * TPF;
    cplx<T>* buf0 = smem + (size_t)rloc * 2 * MSZ;
    cplx<T>* buf1 = buf0 + MSZ;
    int ph = 0;
    const int64_t stride = (int64_t)gridDim.x * a.rpw;
    const cplx<T>* F = reinterpret_cast<const cplx<T>*>(a.f);
    const cplx<T>* G = reinterpret_cast<const cplx<T>*>(a.g);
    cplx<T>* Y = reinterpret_cast<cplx<T>*>(a.Y);
    // neighbouring row blocks (the residues of one problem) on one XCD, which
    // then reads the problem's inputs into its L2 once: block b runs on XCD b % 8
    const int64_t lb = (gridDim.x % 8 == 0) ? (int64_t)(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8
                                            : (int64_t)blockIdx.x;
    for (int64_t base = lb * a.rpw; base < a.nrows; base += stride) {
        const int64_t row = base + rloc;
        const bool ok = row < a.nrows;
        const int64_t rw = ok ? row : 0;
        RawProb pr;
        uint32_t r;
        int64_t xoff, yoff;
        int C1 = 1;
        if (a.rowmap != nullptr) {
            const int i = a.rowmap[2 * rw];
            r = (uint32_t)a.rowmap[2 * rw + 1];
            pr = a.probs[i];
            xoff = pr.f_off;
            yoff = rw * MSZ;
        } else {
            pr = a.p0;
            C1 = a.C1;
            const int64_t t1 = rw / C1;
            const int c1 = (int)(rw - t1 * C1);
            const int64_t b = t1 / a.Dg;
            const int d = (int)(t1 - b * a.Dg);
            r = (uint32_t)(a.r0 + d);
            xoff = b * a.fbs + c1;
            yoff = b * a.ybs + (int64_t)d * MSZ * C1 + c1;
        }
        const bool hp = pr.hiprec != 0;
        cplx<T> v[PPT], u[PPT];
        if (ok) {
            rr_blocksum<T, MSZ>(F + xoff, pr.L, pr.p, pr.q, C1, r, pr.tw, hp, lane, v);
            if (!a.same) rr_blocksum<T, MSZ>(G + xoff, pr.L, pr.p, pr.q, C1, r, pr.tw, hp, lane, u);
        } else {
#pragma unroll
            for (int w = 0; w < PPT; ++w) v[w] = u[w] = mk<T>(0, 0);
        }
        fft_rows_pp<T, MSZ, +1>(v, buf0, buf1, ph, lane, tw, ok);
        if (!a.same) {
            fft_rows_pp<T, MSZ, +1>(u, buf0, buf1, ph, lane, tw, ok);
#pragma unroll
            for (int w = 0; w < PPT; ++w) v[w] = v[w] * u[w];
        } else {
#pragma unroll
            for (int w = 0; w < PPT; ++w) v[w] = v[w] * v[w];
        }
        fft_rows_pp<T, MSZ, -1>(v, buf0, buf1, ph, lane, tw, ok);
        if (ok) {
            const T invN = (T)pr.invN;
            double2 z = tw_n(pr.tw, r * (uint32_t)lane);
            const double2 zs = tw_n(pr.tw, r * (uint32_t)TPF);
#pragma unroll
            for (int w = 0; w < PPT; ++w) {
                Y[yoff + (int64_t)(lane + w * TPF) * C1] = scale(mul_tw<true>(v[w], z, hp), invN);
                z = make_double2(z.x * zs.x - z.y * zs.y, z.x * zs.y + z.y * zs.x);
            }
        }
    }
}

// The output sums of eq. (4) over a residue group [r0, r0 + Dg) of the raw
// rows: h_{t m + s} = sum_d zeta_q^{-t (r0 + d)} y^(r0 + d)_s for t m + s < M,
// one column (s, copy) per thread, the group's values held in registers;
// accumulate adds to h (later groups).  Plain mode: grid (column tiles, B);
// batch mode: one workgroup per tilemap entry, every residue of its problem.
template <typename T>
__global__ void __launch_bounds__(256) k_qsum(RawArgs a) {
    __shared__ double2 twq[kMaxQsum];
    const int tid = threadIdx.x;
    RawProb pr;
    int64_t col, ncols, yb, ystride, hb;
    int C1 = 1, Dg, r0;
    if (a.tilemap != nullptr) {
        const int i = a.tilemap[2 * blockIdx.x];
        pr = a.probs[i];
        col = (int64_t)a.tilemap[2 * blockIdx.x + 1] + tid;
        ncols = a.m;
        yb = a.ybase[i] * a.m;
        ystride = a.m;
        hb = pr.h_off;
        Dg = pr.q;
        r0 = 0;
    } else {
        pr = a.p0;
        C1 = a.C1;
        col = (int64_t)blockIdx.x * blockDim.x + tid;
        ncols = (int64_t)a.m * C1;
        yb = (int64_t)blockIdx.y * a.ybs;
        ystride = (int64_t)a.m * C1;
        hb = (int64_t)blockIdx.y * a.hbs;
        Dg = a.Dg;
        r0 = a.r0;
    }
    // zeta_q^e, e < q (exact: zeta_N^{e m})
    if (tid < pr.q) twq[tid] = tw_n(pr.tw, (uint32_t)tid * (uint32_t)a.m);
    __syncthreads();
    if (col >= ncols) return;
    const cplx<T>* Y = reinterpret_cast<const cplx<T>*>(a.Y) + yb + col;
    cplx<T>* h = reinterpret_cast<cplx<T>*>(a.h) + hb + col;
    cplx<T> V[kMaxQsum];
#pragma unroll
    for (int d = 0; d < kMaxQsum; ++d) V[d] = d < Dg ? Y[(int64_t)d * ystride] : mk<T>(0, 0);
    const int64_t s = col / C1;
    const int64_t ostep = (int64_t)a.m * C1;
    for (int t = 0; t < pr.qout; ++t) {
        if ((int64_t)t * a.m + s >= pr.M) break;
        // exponent t (r0 + d) mod q, advanced by t per residue (t < q)
        int e = (int)(((int64_t)t * r0) % pr.q);
        cplx<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int d = 0; d < kMaxQsum; ++d) {
            if (d < Dg) {
                acc = acc + mul_tw<true>(V[d], twq[e], false);
                e += t;
                if (e >= pr.q) e -= pr.q;
            }
        }
        cplx<T>* o = h + (int64_t)t * ostep;
        if (a.accumulate) acc = acc + *o;
        *o = acc;
    }
}

// ------------------------------------------------------------ elementwise --

template <typename T>
__global__ void k_mul(cplx<T>* F, const cplx<T>* G, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) F[i] = F[i] * G[i];
}

// out[((d m) + l) C + c] = F[((d m1 + l1) m2 + l2) C + c] with l = l1 + m1 l2.
template <typename T>
__global__ void k_natural(const cplx<T>* F, cplx<T>* out, int64_t Dg, int64_t m1, int64_t m2, int64_t C) {
    const int64_t m = m1 * m2;
    const int64_t n = Dg * m * C;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t c = i % C;
        const int64_t l = (i / C) % m;
        const int64_t d = i / (C * m);
        const int64_t l1 = l % m1, l2 = l / m1;
        out[i] = F[((d * m1 + l1) * m2 + l2) * C + c];
    }
}

// --------------------------------------------------------------- launchers --

// Compute units of the current device (256 on gfx950 when the query fails).
int cu_count() {
    static int n = 0;
    if (n == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            n = v;
        else
            n = 256;
    }
    return n;
}

namespace {


template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template <typename T, int MSZ, bool MULTI>
hipError_t fused_m(const FusedArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    lds += (size_t)(TwSplit<MSZ>::LO + TwSplit<MSZ>::HI) * sizeof(cplx<T>);
    hipError_t e = allow_lds(k_fused<T, MSZ, MULTI>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fused<T, MSZ, MULTI>), dim3((unsigned)blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T, int MSZ>
hipError_t fused_t(const FusedArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    return a.nops > 2 ? fused_m<T, MSZ, true>(a, threads, blocks, lds, s)
                      : fused_m<T, MSZ, false>(a, threads, blocks, lds, s);
}

template <typename T, int M1, bool REAL>
hipError_t colf_r(const ColFwdArgs& a, int threads, int64_t gx, int64_t gy, size_t lds, hipStream_t s) {
    lds += (size_t)PassTab<M1>::LEN * sizeof(cplx<T>);
    auto kern = (REAL && a.gs != nullptr) ? k_col_fwd<T, M1, REAL, true> : k_col_fwd<T, M1, REAL, false>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)gx, (unsigned)gy), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T, int M1>
hipError_t colf_t(const ColFwdArgs& a, int threads, int64_t gx, int64_t gy, size_t lds, hipStream_t s, bool real) {
    return real ? colf_r<T, M1, true>(a, threads, gx, gy, lds, s) : colf_r<T, M1, false>(a, threads, gx, gy, lds, s);
}

template <typename T, int M1, int DMAX, bool REAL>
hipError_t colb_d(const ColBwdArgs& a, int threads, int64_t gx, int64_t gy, size_t lds, hipStream_t s) {
    lds += (size_t)PassTab<M1>::LEN * sizeof(cplx<T>);
    auto kern = (REAL && a.gs != nullptr) ? k_col_bwd<T, M1, DMAX, REAL, true> : k_col_bwd<T, M1, DMAX, REAL, false>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)gx, (unsigned)gy), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// DMAX: residues held in registers per pass over h (more passes read-modify-write
// h).  complex64 at m1 = 1024 holds 2 when a group has at most 2 (fewer registers
// live through the transforms: 168 VGPRs instead of 214, backward columns 4-8 %
// faster), else 4.
template <typename T, int M1, bool REAL>
hipError_t colb_r(const ColBwdArgs& a, int threads, int64_t gx, int64_t gy, size_t lds, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        return colb_d<T, M1, (M1 >= 1024 ? 2 : 3), REAL>(a, threads, gx, gy, lds, s);
    } else if constexpr (M1 >= 1024) {
        return a.Dg <= 2 ? colb_d<T, M1, 2, REAL>(a, threads, gx, gy, lds, s)
                         : colb_d<T, M1, 4, REAL>(a, threads, gx, gy, lds, s);
    } else {
        return colb_d<T, M1, 4, REAL>(a, threads, gx, gy, lds, s);
    }
}

template <typename T, int M1>
hipError_t colb_t(const ColBwdArgs& a, int threads, int64_t gx, int64_t gy, size_t lds, hipStream_t s, bool real) {
    return real ? colb_r<T, M1, true>(a, threads, gx, gy, lds, s) : colb_r<T, M1, false>(a, threads, gx, gy, lds, s);
}

template <typename T, int MSZ>
hipError_t row_real_t(const RowArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    lds += (size_t)(TwSplit<MSZ>::LO + TwSplit<MSZ>::HI + PassTab<MSZ>::LEN) * sizeof(cplx<T>);
    auto kern = k_row_real<T, MSZ>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, lds) != hipSuccess || occ < 1) occ = 1;
    const int64_t resident = (int64_t)occ * cu_count();
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T, int MSZ>
hipError_t row_multi_t(const RowArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    lds += (size_t)PassTab<MSZ>::LEN * sizeof(cplx<T>);
    auto kern = k_row_multi<T, MSZ>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, lds) != hipSuccess || occ < 1) occ = 1;
    const int64_t resident = (int64_t)occ * cu_count();
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T, int MSZ>
hipError_t fused_real_t(const FusedArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    lds += (size_t)(TwSplit<MSZ>::LO + TwSplit<MSZ>::HI) * sizeof(cplx<T>);
    hipError_t e = allow_lds(k_fused_real<T, MSZ>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fused_real<T, MSZ>), dim3((unsigned)blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}


template <typename T, int MSZ, int MODE, bool TWO, bool FRAW = false>
hipError_t row_mode(const RowArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    auto kern = k_row<T, MSZ, MODE, TWO, FRAW>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, lds) != hipSuccess || occ < 1) occ = 1;
    const int64_t resident = (int64_t)occ * cu_count();
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T, int MSZ>
hipError_t row_t(const RowArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    lds += (size_t)PassTab<MSZ>::LEN * sizeof(cplx<T>);
    switch (a.mode) {
        case MODE_FWD: return row_mode<T, MSZ, MODE_FWD, false>(a, threads, blocks, lds, s);
        case MODE_INV: return row_mode<T, MSZ, MODE_INV, false>(a, threads, blocks, lds, s);
        default:
            if (a.fraw != nullptr) return row_mode<T, MSZ, MODE_CONV, true, true>(a, threads, blocks, lds, s);
            return a.same ? row_mode<T, MSZ, MODE_CONV, false>(a, threads, blocks, lds, s)
                          : row_mode<T, MSZ, MODE_CONV, true>(a, threads, blocks, lds, s);
    }
}

}  // namespace

#define HDC_POW2_CASES(F, ...)             \
    case 1: return F<T, 1>(__VA_ARGS__);       \
    case 2: return F<T, 2>(__VA_ARGS__);       \
    case 4: return F<T, 4>(__VA_ARGS__);       \
    case 8: return F<T, 8>(__VA_ARGS__);       \
    case 16: return F<T, 16>(__VA_ARGS__);     \
    case 32: return F<T, 32>(__VA_ARGS__);     \
    case 64: return F<T, 64>(__VA_ARGS__);     \
    case 128: return F<T, 128>(__VA_ARGS__);   \
    case 256: return F<T, 256>(__VA_ARGS__);   \
    case 512: return F<T, 512>(__VA_ARGS__);   \
    case 1024: return F<T, 1024>(__VA_ARGS__);

template <typename T, int MSZ>
hipError_t fused_mixed_t(const FusedArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    lds += (size_t)(TwSplit<MSZ>::LO + TwSplit<MSZ>::HI) * sizeof(cplx<T>);
    hipError_t e = allow_lds(k_fused_mixed<T, MSZ>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fused_mixed<T, MSZ>), dim3((unsigned)blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T, int MSZ, int QO>
hipError_t rowconv_t(const FusedArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    auto kern = k_rowconv<T, MSZ, QO>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, lds) != hipSuccess || occ < 1) occ = 1;
    const int64_t resident = (int64_t)occ * cu_count();
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// Row-convolution instances (complex64; complex128 rows would spill
// registers): m = 1024 .. 4096, QO = 2 or 4 output blocks.
template <typename T, int MSZ>
static hipError_t rowconv_q(const FusedArgs& a, int th, int64_t bl, size_t lds, hipStream_t s) {
    if (a.qout <= 2) return rowconv_t<T, MSZ, 2>(a, th, bl, lds, s);
    if (a.qout <= 4) return rowconv_t<T, MSZ, 4>(a, th, bl, lds, s);
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t rowconv_disp(int m, const FusedArgs& a, int th, int64_t bl, size_t lds, hipStream_t s) {
    switch (m) {
        case 1024: return rowconv_q<T, 1024>(a, th, bl, lds, s);
        case 2048: return rowconv_q<T, 2048>(a, th, bl, lds, s);
        case 4096: return rowconv_q<T, 4096>(a, th, bl, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t fused_disp(int m, const FusedArgs& a, int th, int64_t bl, size_t lds, hipStream_t s) {
    if (a.R > 1) {  // m = R 2^k: dispatch on the power-of-two part
        switch (m / a.R) {
            HDC_POW2_CASES(fused_mixed_t, a, th, bl, lds, s)
            default: return hipErrorInvalidValue;
        }
    }
    switch (m) {
        HDC_POW2_CASES(fused_t, a, th, bl, lds, s)
        case 2048: return fused_t<T, 2048>(a, th, bl, lds, s);
        case 4096: return fused_t<T, 4096>(a, th, bl, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t row_disp(int m, const RowArgs& a, int th, int64_t bl, size_t lds, hipStream_t s) {
    switch (m) {
        HDC_POW2_CASES(row_t, a, th, bl, lds, s)
        case 2048: return row_t<T, 2048>(a, th, bl, lds, s);
        case 4096: return row_t<T, 4096>(a, th, bl, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t colf_disp(int m1, const ColFwdArgs& a, int th, int64_t gx, int64_t gy, size_t lds, hipStream_t s,
                            bool real) {
    switch (m1) {
        HDC_POW2_CASES(colf_t, a, th, gx, gy, lds, s, real)
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t colb_disp(int m1, const ColBwdArgs& a, int th, int64_t gx, int64_t gy, size_t lds, hipStream_t s,
                            bool real) {
    switch (m1) {
        HDC_POW2_CASES(colb_t, a, th, gx, gy, lds, s, real)
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t row_real_disp(int m, const RowArgs& a, int th, int64_t bl, size_t lds, hipStream_t s) {
    switch (m) {
        HDC_POW2_CASES(row_real_t, a, th, bl, lds, s)
        case 2048: return row_real_t<T, 2048>(a, th, bl, lds, s);
        case 4096: return row_real_t<T, 4096>(a, th, bl, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t row_multi_disp(int m, const RowArgs& a, int th, int64_t bl, size_t lds, hipStream_t s) {
    switch (m) {
        HDC_POW2_CASES(row_multi_t, a, th, bl, lds, s)
        case 2048: return row_multi_t<T, 2048>(a, th, bl, lds, s);
        case 4096: return row_multi_t<T, 4096>(a, th, bl, lds, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t fused_real_disp(int m, const FusedArgs& a, int th, int64_t bl, size_t lds, hipStream_t s) {
    switch (m) {
        HDC_POW2_CASES(fused_real_t, a, th, bl, lds, s)
        case 2048: return fused_real_t<T, 2048>(a, th, bl, lds, s);
        case 4096: return fused_real_t<T, 4096>(a, th, bl, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fused(bool dbl, int m, const FusedArgs& a, int threads, int64_t blocks, size_t lds,
                        hipStream_t s) {
    return dbl ? fused_disp<double>(m, a, threads, blocks, lds, s) : fused_disp<float>(m, a, threads, blocks, lds, s);
}

hipError_t launch_row(bool dbl, int m2, const RowArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    return dbl ? row_disp<double>(m2, a, threads, blocks, lds, s) : row_disp<float>(m2, a, threads, blocks, lds, s);
}

hipError_t launch_col_fwd(bool dbl, int m1, const ColFwdArgs& a, int threads, int64_t gx, int64_t gy, size_t lds,
                          hipStream_t s, bool real) {
    return dbl ? colf_disp<double>(m1, a, threads, gx, gy, lds, s, real)
               : colf_disp<float>(m1, a, threads, gx, gy, lds, s, real);
}

hipError_t launch_col_bwd(bool dbl, int m1, const ColBwdArgs& a, int threads, int64_t gx, int64_t gy, size_t lds,
                          hipStream_t s, bool real) {
    return dbl ? colb_disp<double>(m1, a, threads, gx, gy, lds, s, real)
               : colb_disp<float>(m1, a, threads, gx, gy, lds, s, real);
}

hipError_t launch_row_real(bool dbl, int m2, const RowArgs& a, int threads, int64_t blocks, size_t lds,
                           hipStream_t s) {
    return dbl ? row_real_disp<double>(m2, a, threads, blocks, lds, s)
               : row_real_disp<float>(m2, a, threads, blocks, lds, s);
}

hipError_t launch_row_multi(bool dbl, int m2, const RowArgs& a, int threads, int64_t blocks, size_t lds,
                            hipStream_t s) {
    return dbl ? row_multi_disp<double>(m2, a, threads, blocks, lds, s)
               : row_multi_disp<float>(m2, a, threads, blocks, lds, s);
}

hipError_t launch_rowconv(bool dbl, int m, const FusedArgs& a, int threads, int64_t blocks, size_t lds,
                          hipStream_t s) {
    return dbl ? hipErrorInvalidValue : rowconv_disp<float>(m, a, threads, blocks, lds, s);
}

hipError_t launch_fused_real(bool dbl, int m, const FusedArgs& a, int threads, int64_t blocks, size_t lds,
                             hipStream_t s) {
    return dbl ? fused_real_disp<double>(m, a, threads, blocks, lds, s)
               : fused_real_disp<float>(m, a, threads, blocks, lds, s);
}

template <typename T, int MSZ>
hipError_t row_rr_t(const RawArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    lds += (size_t)PassTab<MSZ>::LEN * sizeof(cplx<T>);
    auto kern = k_row_rr<T, MSZ>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, threads, lds) != hipSuccess || occ < 1) occ = 1;
    const int64_t resident = (int64_t)occ * cu_count();
    int64_t grid = blocks < resident ? blocks : resident;
    if (grid >= 8) grid = (grid + 7) / 8 * 8;  // whole XCD rounds (spare blocks find no rows)
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t row_rr_disp(int m, const RawArgs& a, int th, int64_t bl, size_t lds, hipStream_t s) {
    switch (m) {
        HDC_POW2_CASES(row_rr_t, a, th, bl, lds, s)
        case 2048: return row_rr_t<T, 2048>(a, th, bl, lds, s);
        case 4096: return row_rr_t<T, 4096>(a, th, bl, lds, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_row_rr(bool dbl, int m, const RawArgs& a, int threads, int64_t blocks, size_t lds, hipStream_t s) {
    return dbl ? row_rr_disp<double>(m, a, threads, blocks, lds, s) : row_rr_disp<float>(m, a, threads, blocks, lds, s);
}

hipError_t launch_qsum(bool dbl, const RawArgs& a, int64_t gx, int64_t gy, hipStream_t s) {
    if (gx <= 0 || gy <= 0) return hipSuccess;
    if (dbl)
        hipLaunchKernelGGL(k_qsum<double>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_qsum<float>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
static hipError_t fused_queue_t(const FusedQueueArgs& a, int64_t nitems, size_t lds, hipStream_t s) {
    auto kern = k_fused_queue<T>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 512, lds) != hipSuccess || occ < 1) occ = 1;
    const int64_t resident = (int64_t)occ * cu_count();
    const int64_t grid = nitems < resident ? nitems : resident;
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, a.counter);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(512), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_fused_queue(bool dbl, const FusedQueueArgs& a, int64_t nitems, size_t lds, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    return dbl ? fused_queue_t<double>(a, nitems, lds, s) : fused_queue_t<float>(a, nitems, lds, s);
}

hipError_t launch_mul(bool dbl, void* F, const void* G, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    if (dbl)
        hipLaunchKernelGGL(k_mul<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<cplx<double>*>(F), reinterpret_cast<const cplx<double>*>(G), n);
    else
        hipLaunchKernelGGL(k_mul<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<cplx<float>*>(F), reinterpret_cast<const cplx<float>*>(G), n);
    return hipGetLastError();
}

template <typename T>
static hipError_t real_scale_t(const void* f, const void* g, int64_t n, void* mx, hipStream_t s) {
    using U = typename AbsBits<T>::U;
    U* m = reinterpret_cast<U*>(mx);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_real_clear<T>, dim3(1), dim3(64), 0, s, m);
    hipLaunchKernelGGL(k_real_absmax<T>, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const T*>(f), n, m);
    hipLaunchKernelGGL(k_real_absmax<T>, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const T*>(g), n,
                       m + 1);
    return hipGetLastError();
}

hipError_t launch_real_scale(bool dbl, const void* f, const void* g, int64_t n, void* mx, hipStream_t s) {
    return dbl ? real_scale_t<double>(f, g, n, mx, s) : real_scale_t<float>(f, g, n, mx, s);
}

hipError_t launch_natural(bool dbl, const void* F, void* out, int64_t Dg, int64_t m1, int64_t m2, int64_t C,
                          hipStream_t s) {
    const int64_t n = Dg * m1 * m2 * C;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    if (dbl)
        hipLaunchKernelGGL(k_natural<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const cplx<double>*>(F), reinterpret_cast<cplx<double>*>(out), Dg, m1,
                           m2, C);
    else
        hipLaunchKernelGGL(k_natural<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           reinterpret_cast<const cplx<float>*>(F), reinterpret_cast<cplx<float>*>(out), Dg, m1, m2,
                           C);
    return hipGetLastError();
}

}  // namespace hdc
