// Device building blocks of the gfx950 RPM-FFT path: complex arithmetic,
// radix-2/3/4/8/16 butterflies, an LDS-resident Stockham FFT stage shared by all
// pencil passes, and deterministic workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpm {

constexpr int kThreads = 256;     // every pass kernel runs 4 waves of 64
constexpr int kWaves = kThreads / 64;
constexpr int kMaxStages = 10;
constexpr int kMaxP = 64;         // basis cap

template <typename T>
struct __align__(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
// multiply by s*i, s = +1 or -1
template <typename T, int S>
__device__ __forceinline__ cx<T> cmul_si(cx<T> a) { return S > 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x}; }

// Division by a launch-invariant divisor d >= 1 as a multiply-high and a
// shift (Granlund-Montgomery): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, n / d = (mulhi(n, m) + n) >> l for
// 0 <= n < 2^31.  Index arithmetic in the pencil kernels uses it in place of
// the integer division sequence.
struct FDiv {
    uint32_t d, m;
    int l;
    __host__ __device__ __forceinline__ int div(int n) const
    {
        const uint32_t t = (uint32_t)(((uint64_t)(uint32_t)n * m) >> 32);
        return (int)((t + (uint32_t)n) >> l);
    }
};

inline FDiv make_fdiv(int d)
{
    FDiv f;
    f.d = (uint32_t)d;
    f.l = 0;
    while ((1ull << f.l) < (unsigned long long)d) ++f.l;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << f.l) - (unsigned long long)d)) / (unsigned long long)d + 1);
    return f;
}

// Transform lengths are products of the radices of one plan.
struct Plan {
    int n;
    int nst;
    int rad[kMaxStages];
};

// ---------------------------------------------------------------------------
// In-register DFTs of length R with kernel exp(D * 2 pi i j k / R), D = -1
// (forward) or +1 (inverse).
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void dft2(cx<T>* v)
{
    cx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <typename T, int D>
__device__ __forceinline__ void dft3(cx<T>* v)
{
    const T half = T(0.5);
    const T s3 = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
    cx<T> t1 = cadd(v[1], v[2]);
    cx<T> t2 = csub(v[1], v[2]);
    cx<T> m = {v[0].x - half * t1.x, v[0].y - half * t1.y};
    // D * i * s3 * t2
    cx<T> r = cmul_si<T, D>(cscale(t2, s3));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

template <typename T, int D>
__device__ __forceinline__ void dft4(cx<T>* v)
{
    cx<T> y0 = cadd(v[0], v[2]);
    cx<T> y1 = csub(v[0], v[2]);
    cx<T> y2 = cadd(v[1], v[3]);
    cx<T> y3 = cmul_si<T, D>(csub(v[1], v[3]));
    v[0] = cadd(y0, y2);
    v[2] = csub(y0, y2);
    v[1] = cadd(y1, y3);
    v[3] = csub(y1, y3);
}

template <typename T, int D>
__device__ __forceinline__ void dft8(cx<T>* v)
{
    const T r2 = T(0.70710678118654752440084436210485);
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T, D>(e);
    dft4<T, D>(o);
    // w8^k = exp(D 2 pi i k / 8)
    cx<T> o1 = {r2 * (o[1].x - D * o[1].y), r2 * (o[1].y + D * o[1].x)};
    cx<T> o2 = cmul_si<T, D>(o[2]);
    cx<T> o3 = {r2 * (-o[3].x - D * o[3].y), r2 * (-o[3].y + D * o[3].x)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

// Length 16 as 4 x 4: DFT-4 over the stride-4 subsequences, twiddles
// w16^(n2 k1), DFT-4 across them; output index k1 + 4 k2.
template <typename T, int D>
__device__ __forceinline__ void dft16(cx<T>* v)
{
    // cos and sin of 2 pi m / 16, m = 0..3
    const T c1 = T(0.92387953251128675612818318939679), s1 = T(0.38268343236508977172845998403040);
    const T r2 = T(0.70710678118654752440084436210485);
    cx<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        cx<T> t[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
        dft4<T, D>(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
    }
    // twiddles exp(D 2 pi i m / 16) for m = n2 * k1
    auto tw = [&](cx<T> a, int m) -> cx<T> {
        T c, s;
        switch (m) {
            case 1: c = c1; s = s1; break;
            case 2: c = r2; s = r2; break;
            case 3: c = s1; s = c1; break;
            case 4: c = T(0); s = T(1); break;
            case 6: c = -r2; s = r2; break;
            case 9: c = -c1; s = -s1; break;
            default: c = T(1); s = T(0); break;
        }
        s = D * s;
        return cx<T>{a.x * c - a.y * s, a.x * s + a.y * c};
    };
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) y[n2][k1] = tw(y[n2][k1], n2 * k1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cx<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        dft4<T, D>(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
}

template <typename T, int R, int D>
__device__ __forceinline__ void dftR(cx<T>* v)
{
    if constexpr (R == 2) dft2<T, D>(v);
    else if constexpr (R == 3) dft3<T, D>(v);
    else if constexpr (R == 4) dft4<T, D>(v);
    else if constexpr (R == 8) dft8<T, D>(v);
    else dft16<T, D>(v);
}

// LDS layout of the pencils: element i of a sequence sits at lpad(i) (one
// spare slot after every 16 elements) and sequences are lrow(n) slots apart.
// The spare slots break the power-of-two strides of the Stockham writes
// (16 j + q in the first radix-16 stage) and of column-wise fills (runs of
// four voxels per lane), which otherwise land on a few LDS banks.
__host__ __device__ constexpr int lpad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lrow(int n) { return n + (n >> 4) + 1; }

// One Stockham stage over nseq sequences of length n held in LDS with row
// stride ss.  Ns = product of the radices already applied.
// tw[e] = exp(-2 pi i e / n), e in [0, n).
template <typename T, int R, int D, int NT = kThreads>
__device__ __forceinline__ void fft_stage(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int n, int Ns,
                                          int nseq, int ss, const cx<T>* __restrict__ tw)
{
    const int nb = n / R;
    const int total = nb * nseq;
    const int tws = n / (Ns * R);
    for (int g = threadIdx.x; g < total; g += NT) {
        const int s = g / nb;
        const int j = g - s * nb;
        const cx<T>* in = src + s * ss;
        cx<T>* out = dst + s * ss;
        cx<T> v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = in[lpad(j + q * nb)];
        const int k = j % Ns;
        if (Ns > 1) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                cx<T> w = tw[q * k * tws];
                if (D > 0) w.y = -w.y;
                v[q] = cmul(v[q], w);
            }
        }
        dftR<T, R, D>(v);
        const int o = (j - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) out[lpad(o + q * Ns)] = v[q];
    }
}

// The same stage with the length and the stage position fixed at compile time
// (power-of-two lengths): index arithmetic reduces to shifts and masks.
template <typename T, int R, int D, int N, int NS, int NT>
__device__ __forceinline__ void fft_stage_ct(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int nseq,
                                             int ss, const cx<T>* __restrict__ tw, int tid)
{
    constexpr int nb = N / R;
    constexpr int tws = N / (NS * R);
    const int total = nb * nseq;
    for (int g = tid; g < total; g += NT) {
        const int s = g / nb;
        const int j = g & (nb - 1);
        const cx<T>* in = src + s * ss;
        cx<T>* out = dst + s * ss;
        cx<T> v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = in[lpad(j + q * nb)];
        const int k = j & (NS - 1);
        if constexpr (NS > 1) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                cx<T> w = tw[q * k * tws];
                if (D > 0) w.y = -w.y;
                v[q] = cmul(v[q], w);
            }
        }
        dftR<T, R, D>(v);
        const int o = (j - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) out[lpad(o + q * NS)] = v[q];
    }
}

// Radix sequence of a power-of-two length: radix 16 while possible, then one
// stage of 8, 4 or 2 (the host plan builds the same sequence).
constexpr int ct_log2(int n) { return n <= 1 ? 0 : 1 + ct_log2(n / 2); }
constexpr int ct_nst(int n) { return ct_log2(n) / 4 + (ct_log2(n) % 4 ? 1 : 0); }
constexpr int ct_rad(int n, int st) { return st < ct_log2(n) / 4 ? 16 : (1 << (ct_log2(n) % 4)); }

template <typename T, int D, int N, int ST, int NS, int NT>
__device__ __forceinline__ cx<T>* ct_stages(cx<T>* src, cx<T>* dst, int nseq, int ss, const cx<T>* tw, int tid)
{
    if constexpr (ST == ct_nst(N)) {
        return src;
    } else {
        constexpr int R = ct_rad(N, ST);
        fft_stage_ct<T, R, D, N, NS, NT>(src, dst, nseq, ss, tw, tid);
        __syncthreads();
        return ct_stages<T, D, N, ST + 1, NS * R, NT>(dst, src, nseq, ss, tw, tid);
    }
}

// In-place variant of the compile-time stages for at most one butterfly per
// thread (nseq * N / R <= NT at every stage): each thread reads its inputs,
// the block synchronises, then every thread writes its outputs into the same
// rows.  Half the LDS of the ping-pong form (more resident blocks).
template <typename T, int D, int N, int ST, int NS, int NT>
__device__ __forceinline__ void ct_stages_ip(cx<T>* buf, int nseq, int ss, const cx<T>* tw, int tid)
{
    if constexpr (ST < ct_nst(N)) {
        constexpr int R = ct_rad(N, ST);
        constexpr int nb = N / R;
        constexpr int tws = N / (NS * R);
        const bool act = tid < nb * nseq;
        const int s = tid / nb;
        const int j = tid & (nb - 1);
        cx<T> v[R];
        if (act) {
            const cx<T>* in = buf + s * ss;
#pragma unroll
            for (int q = 0; q < R; ++q) v[q] = in[lpad(j + q * nb)];
            const int k = j & (NS - 1);
            if constexpr (NS > 1) {
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    cx<T> w = tw[q * k * tws];
                    if (D > 0) w.y = -w.y;
                    v[q] = cmul(v[q], w);
                }
            }
            dftR<T, R, D>(v);
        }
        __syncthreads();
        if (act) {
            const int k = j & (NS - 1);
            const int o = (j - k) * R + k;
            cx<T>* out = buf + s * ss;
#pragma unroll
            for (int q = 0; q < R; ++q) out[lpad(o + q * NS)] = v[q];
        }
        __syncthreads();
        ct_stages_ip<T, D, N, ST + 1, NS * R, NT>(buf, nseq, ss, tw, tid);
    }
}

// Full LDS FFT of nseq sequences (data in a; b is the ping-pong buffer).
// Caller must __syncthreads() after filling a.  Returns the buffer that holds
// the natural-order result; all threads are synchronised on return.
template <typename T, int D, int NT = kThreads>
__device__ cx<T>* lds_fft(cx<T>* a, cx<T>* b, const Plan& pl, int nseq, int ss, const cx<T>* tw,
                         int tid = threadIdx.x)
{
    if (pl.n == 128) return ct_stages<T, D, 128, 0, 1, NT>(a, b, nseq, ss, tw, tid);
    int Ns = 1;
    cx<T>* src = a;
    cx<T>* dst = b;
    for (int st = 0; st < pl.nst; ++st) {
        const int R = pl.rad[st];
        if (R == 16) fft_stage<T, 16, D, NT>(src, dst, pl.n, Ns, nseq, ss, tw);
        else if (R == 8) fft_stage<T, 8, D, NT>(src, dst, pl.n, Ns, nseq, ss, tw);
        else if (R == 4) fft_stage<T, 4, D, NT>(src, dst, pl.n, Ns, nseq, ss, tw);
        else if (R == 2) fft_stage<T, 2, D, NT>(src, dst, pl.n, Ns, nseq, ss, tw);
        else fft_stage<T, 3, D, NT>(src, dst, pl.n, Ns, nseq, ss, tw);
        __syncthreads();
        Ns *= R;
        cx<T>* t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// ---------------------------------------------------------------------------
// Deterministic workgroup reductions (fixed shuffle tree, fixed wave order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sums M per-thread values over the workgroup of NT threads; thread m < M
// writes the m-th total to dst[m].  lds needs (NT / 64) * M doubles.
template <int M, int NT = kThreads>
__device__ __forceinline__ void wg_sum_store(double (&v)[M], double* __restrict__ dst, double* lds)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double s = wave_sum(v[m]);
        if (lane == 0) lds[wave * M + m] = s;
    }
    __syncthreads();
    if (threadIdx.x < M) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += lds[w * M + threadIdx.x];
        dst[threadIdx.x] = s;
    }
    __syncthreads();
}

// Frobenius weight of stored tensor component c (shear components count twice).
__device__ __forceinline__ double frob_w(int c) { return c < 3 ? 1.0 : 2.0; }

}  // namespace rpm
