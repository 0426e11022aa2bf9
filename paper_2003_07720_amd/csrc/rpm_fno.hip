// Learned warm start for the RPM-FFT solver: a Fourier-neural-operator-style
// network that maps the stiffness field of a cell to the strain fluctuation of
// the six unit load cases (the localization tensor), so that a solve for a
// mean strain E can start from E plus the predicted fluctuation instead of the
// uniform E of Algorithm 2's initialization.  The network and its training
// are not in the paper; they sit in front of the method, whose own equilibrium
// error still decides when the result is accepted.
//
// Network (per voxel features x, C hidden channels, L spectral layers):
//   h_0     = W_lift x + b_lift
//   h_{l+1} = gelu(W_l h_l + b_l + K_l h_l)          l = 0 .. L-1
//   y       = W_proj h_L + b_proj
//   K_l h   = (1/N) Re sum_{k in M} exp(+2 pi i k.x/n) R_l(k) sum_x' exp(-2 pi i k.x'/n) h(x')
// with M the m^3 signed frequencies {-m/2 .. m/2-1}^3 and R_l(k) a complex
// C x C matrix per retained frequency.
//
// Every contraction -- the truncated DFTs axis by axis, the per-frequency
// channel mixing, the pointwise channel maps and all their adjoints -- is one
// batched strided GEMM on the matrix cores: v_mfma_f32_16x16x16_bf16, operands
// rounded to bfloat16 as they are loaded (weights and activations), products
// accumulated in FP32.  Complex products are four real GEMMs on planar
// real/imaginary arrays.  Elementwise work (bias, GELU and its derivative,
// loss, Adam) runs in small FP32 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "rpmfno.h"

namespace {

// ---------------------------------------------------------------------------
// Batched strided GEMM on the matrix cores
// ---------------------------------------------------------------------------
// C[b](i, j) = alpha sum_k A[b](i, k) B[b](k, j) + beta C[b](i, j), element
// (i, k) of A[b] at A + b sAb + i sAi + k sAk (likewise B, C); transposes and
// complex planes are strides.  Operands are FP32 in memory, rounded to
// bfloat16 (nearest even) on load; FP32 accumulation.
struct GemmDesc {
    const float* A;
    const float* B;
    float* C;
    int M, N, K;
    long long sAb, sAi, sAk, sBb, sBk, sBj, sCb, sCi, sCj;
    float alpha, beta;
};

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)(u >> 16);  // inf / nan kept
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// 256 threads = 4 waves; a block owns a 32 x 32 tile of C[b] (waves in 2 x 2
// tiles of 16 x 16), b = blockIdx.y.  Per 16-deep step lane l loads
// A(i0 + l % 16, k0 + 4 (l / 16) + q) and B(k0 + 4 (l / 16) + q, j0 + l % 16),
// q < 4, and receives C(i0 + 4 (l / 16) + q, j0 + l % 16).  Out-of-range
// elements read as zero and are not written.
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmDesc d)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tilesN = (d.N + 31) >> 5;
    const int bm = blockIdx.x / tilesN, bn = blockIdx.x - (blockIdx.x / tilesN) * tilesN;
    const int i0 = bm * 32 + (wave >> 1) * 16, j0 = bn * 32 + (wave & 1) * 16;
    const long long b = blockIdx.y;
    const float* A = d.A + b * d.sAb;
    const float* B = d.B + b * d.sBb;
    const int li = lane & 15, lk = 4 * (lane >> 4);
    const int ia = i0 + li, jb = j0 + li;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < d.K; k0 += 16) {
        bf16x4 a, bb;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + lk + q;
            const float av = (ia < d.M && k < d.K) ? A[ia * d.sAi + k * d.sAk] : 0.f;
            const float bv = (k < d.K && jb < d.N) ? B[k * d.sBk + jb * d.sBj] : 0.f;
            a[q] = to_bf16(av);
            bb[q] = to_bf16(bv);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc, 0, 0, 0);
    }
    float* C = d.C + b * d.sCb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + lk + q, j = j0 + li;
        if (i < d.M && j < d.N) {
            float* c = C + i * d.sCi + j * d.sCj;
            *c = d.beta != 0.f ? d.alpha * acc[q] + d.beta * *c : d.alpha * acc[q];
        }
    }
}

bool gemm(hipStream_t s, const GemmDesc& d, int batch)
{
    if (d.M <= 0 || d.N <= 0 || batch <= 0) return true;
    const long long tiles = (long long)((d.M + 31) / 32) * ((d.N + 31) / 32);
    if (tiles > 0x7fffffffLL || batch > 65535) return false;
    k_gemm_bf16<<<dim3((unsigned)tiles, (unsigned)batch), 256, 0, s>>>(d);
    return true;
}

// row-major helpers: X (rows x cols) with leading dimension ld
GemmDesc gd(const float* A, long long sAb, long long sAi, long long sAk, const float* B, long long sBb,
            long long sBk, long long sBj, float* C, long long sCb, long long sCi, long long sCj, int M, int N, int K,
            float alpha, float beta)
{
    GemmDesc d;
    d.A = A;
    d.B = B;
    d.C = C;
    d.M = M;
    d.N = N;
    d.K = K;
    d.sAb = sAb;
    d.sAi = sAi;
    d.sAk = sAk;
    d.sBb = sBb;
    d.sBk = sBk;
    d.sBj = sBj;
    d.sCb = sCb;
    d.sCi = sCi;
    d.sCj = sCj;
    d.alpha = alpha;
    d.beta = beta;
    return d;
}

// ---------------------------------------------------------------------------
// Elementwise kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ float gelu(float x)
{
    return 0.5f * x * (1.f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x)
{
    const float cdf = 0.5f * (1.f + erff(x * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
    return cdf + x * pdf;
}

// pre = acc + bias[c]; out = gelu(pre) (act) or pre; layout [B][C][N]
__global__ void k_bias_act(float* __restrict__ acc, const float* __restrict__ bias, float* __restrict__ out, int C,
                           long long N, long long total, int act)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)((i / N) % C);
    const float p = acc[i] + bias[c];
    acc[i] = p;
    out[i] = act ? gelu(p) : p;
}

// dpre = dout * gelu'(pre)
__global__ void k_gelu_back(const float* __restrict__ pre, const float* __restrict__ dout, float* __restrict__ dpre,
                            long long total)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) dpre[i] = dout[i] * gelu_grad(pre[i]);
}

// db[c] = sum_{b, v} d[b][c][v]; one block per channel, fixed order
__global__ __launch_bounds__(256) void k_bias_grad(const float* __restrict__ d, float* __restrict__ db, int B, int C,
                                                   long long N)
{
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int b = 0; b < B; ++b) {
        const float* p = d + ((long long)b * C + c) * N;
        for (long long v = threadIdx.x; v < N; v += 256) s += p[v];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = red[0];
}

__global__ void k_add(float* __restrict__ a, const float* __restrict__ b, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += b[i];
}

// weighted mean squared error over the n = B cout N outputs:
// L = sum w (y - t)^2 / n with w the voxel's stiffness relative to the
// stiffest phase, 10^(3 x0) from the first feature (1 without features), so
// the strain inside pores -- which carries no stress -- hardly counts;
// dy = 2 w (y - t) / n; per-block partial sums of w (y - t)^2
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             const float* __restrict__ x, int cin, int cout, long long N,
                                             float* __restrict__ dy, double* __restrict__ part, long long n)
{
    __shared__ double red[256];
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const long long v = i % N, b = i / (N * cout);
        const float w = x ? expf(6.90775527898f * x[b * cin * N + v]) : 1.f;
        const float e = y[i] - t[i];
        if (dy) dy[i] = 2.f * w * e / (float)n;
        s += (double)w * e * e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// input features of a cell: x[0] = max(log10(E / E_max), -3) / 3 with E the
// Young modulus of the voxel's phase and E_max the stiffest phase of the table
// (pores softer than 1e-3 of it look alike), x[1] = nu - 0.3
struct FeatTab {
    float v[512];
};
__global__ void k_features(const uint8_t* __restrict__ phase, FeatTab t, float* __restrict__ x, long long N)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int p = phase[v];
    x[v] = t.v[2 * p];
    x[N + v] = t.v[2 * p + 1];
}

// eps0[c][v] = E[c] + sum_j g_j y[j * 6 + c][v]: y holds the predicted strain
// fluctuation of the six unit load cases (Voigt order, engineering shear), so
// a tensor shear component E_j enters as g_j = 2 E_j
struct E6 {
    double e[6];
};
template <typename T>
__global__ void k_assemble(const float* __restrict__ y, E6 E, T* __restrict__ eps, long long N)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    for (int c = 0; c < 6; ++c) {
        double s = E.e[c];
        for (int j = 0; j < 6; ++j) {
            const double gj = j < 3 ? E.e[j] : 2.0 * E.e[j];
            s += gj * (double)y[((long long)j * 6 + c) * N + v];
        }
        eps[(long long)c * N + v] = (T)s;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
inline int blocks(long long n) { return (int)((n + 255) / 256); }

struct Net {
    int cin, cout, C, L, m, m3;
    // parameter offsets (floats)
    long long lift_w, lift_b, proj_w, proj_b, total;
    std::vector<long long> pw_w, pw_b, r_re, r_im;
    bool ok;
};

Net make_net(const rpm_fno_config* c)
{
    Net n{};
    n.ok = c && c->c_in >= 1 && c->c_out >= 1 && c->width >= 1 && c->width <= 256 && c->layers >= 0 &&
           c->layers <= 16 && c->modes >= 1 && c->modes <= 32;
    if (!n.ok) return n;
    n.cin = c->c_in;
    n.cout = c->c_out;
    n.C = c->width;
    n.L = c->layers;
    n.m = c->modes;
    n.m3 = n.m * n.m * n.m;
    long long off = 0;
    n.lift_w = off;
    off += (long long)n.C * n.cin;
    n.lift_b = off;
    off += n.C;
    for (int l = 0; l < n.L; ++l) {
        n.pw_w.push_back(off);
        off += (long long)n.C * n.C;
        n.pw_b.push_back(off);
        off += n.C;
        n.r_re.push_back(off);
        off += (long long)n.m3 * n.C * n.C;
        n.r_im.push_back(off);
        off += (long long)n.m3 * n.C * n.C;
    }
    n.proj_w = off;
    off += (long long)n.cout * n.C;
    n.proj_b = off;
    off += n.cout;
    n.total = off;
    return n;
}

// Workspace: twiddles, activations kept for the backward pass, spectral
// temporaries.  All offsets in floats.
struct FWs {
    long long tw[3];                  // per axis: cos then sin tables, m x n each
    long long h;                      // h_0 .. h_L: (L + 1) x [B][C][N]
    long long pre;                    // pre-activations of the L layers: L x [B][C][N]
    long long xhat;                   // DFT of each layer input: L x 2 x [B][C][m3]
    long long s1, s2, s3, s4;         // spectral temporaries (2 planes each)
    long long acc, dh, dh2, dpre;     // [B][C][N] scratch
    long long y;                      // output [B][cout][N]
    long long feat;                   // input features of a warm start [cin][N]
    long long part;                   // loss partial sums (double, 1024)
    long long total;
    long long N;
    int n[3];
};

FWs make_fws(const Net& net, const int32_t n[3], int B)
{
    FWs w{};
    const long long N = (long long)n[0] * n[1] * n[2];
    w.N = N;
    for (int a = 0; a < 3; ++a) w.n[a] = n[a];
    const long long C = net.C, m = net.m;
    long long off = 0;
    auto take = [&](long long f) {
        const long long at = off;
        off += (f + 63) / 64 * 64;
        return at;
    };
    for (int a = 0; a < 3; ++a) w.tw[a] = take(2 * m * n[a]);
    w.h = take((long long)(net.L + 1) * B * C * N);
    w.pre = take((long long)std::max(net.L, 1) * B * C * N);
    w.xhat = take((long long)std::max(net.L, 1) * 2 * B * C * net.m3);
    // stage sizes: x: B C nz ny m; y: B C nz m m; z: B C m m m; inverse z: B C nz m m; inverse y: B C nz ny m
    const long long sx = (long long)B * C * n[2] * n[1] * m;
    const long long sy = (long long)B * C * n[2] * m * m;
    const long long sz = (long long)B * C * net.m3;
    const long long smax = std::max(std::max(sx, sy), sz);
    w.s1 = take(2 * smax);
    w.s2 = take(2 * smax);
    w.s3 = take(2 * smax);
    w.s4 = take(2 * smax);
    w.acc = take((long long)B * std::max<long long>(C, net.cout) * N);
    w.dh = take((long long)B * std::max<long long>(C, net.cin) * N);
    w.dh2 = take((long long)B * C * N);
    w.dpre = take((long long)B * std::max<long long>(C, net.cout) * N);
    w.y = take((long long)B * net.cout * N);
    w.feat = take((long long)net.cin * N);
    w.part = take(2 * 1024);
    w.total = off;
    return w;
}

struct Fno {
    Net net;
    FWs w;
    float* ws;
    hipStream_t s;
    int B;
    bool ok = true;
    float* at(long long off) { return ws + off; }
    void G(const GemmDesc& d, int batch)
    {
        if (!gemm(s, d, batch)) ok = false;
    }
};

// Twiddle tables of axis a: cos(2 pi k x / n) and sin(2 pi k x / n), k the
// signed frequency index kk - m/2, row-major [kk][x].
bool upload_twiddles(Fno& f)
{
    const int m = f.net.m;
    for (int a = 0; a < 3; ++a) {
        const int n = f.w.n[a];
        std::vector<float> t(2 * (size_t)m * n);
        for (int kk = 0; kk < m; ++kk) {
            const long long k = kk - m / 2;
            for (int x = 0; x < n; ++x) {
                const long long r = ((k * x) % n + n) % n;
                const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)r / n;
                t[(size_t)kk * n + x] = (float)std::cos(ang);
                t[(size_t)m * n + (size_t)kk * n + x] = (float)std::sin(ang);
            }
        }
        if (hipMemcpyAsync(f.at(f.w.tw[a]), t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice, f.s) !=
            hipSuccess)
            return false;
        if (hipStreamSynchronize(f.s) != hipSuccess) return false;
    }
    return true;
}

// Truncated forward DFT of real fields v [P][n2][n1][n0] (P = B C) into the
// planar spectrum X (re at X, im at X + plane) laid out [P][kz][ky][kx]:
// x, then y, then z, each a batched GEMM with the m x n twiddle table
// (temporaries s1, s2).
void dft_forward(Fno& f, const float* v, float* X, long long plane)
{
    const int m = f.net.m;
    const long long P = (long long)f.B * f.net.C;
    const int n0 = f.w.n[0], n1 = f.w.n[1], n2 = f.w.n[2];
    const float* cx = f.at(f.w.tw[0]);
    const float* sx = cx + (long long)m * n0;
    const float* cy = f.at(f.w.tw[1]);
    const float* sy = cy + (long long)m * n1;
    const float* cz = f.at(f.w.tw[2]);
    const float* sz = cz + (long long)m * n2;
    float* T1 = f.at(f.w.s1);
    const long long sx1 = P * n2 * n1 * m;  // stage-1 plane size
    // stage x: T1[(p,z,y)][kx] = sum_x v[(p,z,y)][x] (cos - i sin)
    const int Mx = (int)(P * n2 * n1);
    f.G(gd(v, 0, n0, 1, cx, 0, 1, n0, T1, 0, m, 1, Mx, m, n0, 1.f, 0.f), 1);
    f.G(gd(v, 0, n0, 1, sx, 0, 1, n0, T1 + sx1, 0, m, 1, Mx, m, n0, -1.f, 0.f), 1);
    // stage y: T2[(p,z)][ky][kx] = sum_y F[ky][y] T1[(p,z)][y][kx], F = cos - i sin
    float* T2 = f.at(f.w.s2);
    const long long sy2 = P * n2 * m * m;
    const int By = (int)(P * n2);
    const long long sAy = 0, sBy = (long long)n1 * m, sCy = (long long)m * m;
    // re = C T1re + S T1im ; im = C T1im - S T1re
    f.G(gd(cy, sAy, n1, 1, T1, sBy, m, 1, T2, sCy, m, 1, m, m, n1, 1.f, 0.f), By);
    f.G(gd(sy, sAy, n1, 1, T1 + sx1, sBy, m, 1, T2, sCy, m, 1, m, m, n1, 1.f, 1.f), By);
    f.G(gd(cy, sAy, n1, 1, T1 + sx1, sBy, m, 1, T2 + sy2, sCy, m, 1, m, m, n1, 1.f, 0.f), By);
    f.G(gd(sy, sAy, n1, 1, T1, sBy, m, 1, T2 + sy2, sCy, m, 1, m, m, n1, -1.f, 1.f), By);
    // stage z: X[p][kz][(ky,kx)] = sum_z F[kz][z] T2[p][z][(ky,kx)]
    const int Bz = (int)P;
    const long long mm = (long long)m * m;
    const long long sBz = (long long)n2 * mm, sCz = (long long)m * mm;
    f.G(gd(cz, 0, n2, 1, T2, sBz, mm, 1, X, sCz, mm, 1, m, (int)mm, n2, 1.f, 0.f), Bz);
    f.G(gd(sz, 0, n2, 1, T2 + sy2, sBz, mm, 1, X, sCz, mm, 1, m, (int)mm, n2, 1.f, 1.f), Bz);
    f.G(gd(cz, 0, n2, 1, T2 + sy2, sBz, mm, 1, X + plane, sCz, mm, 1, m, (int)mm, n2, 1.f, 0.f), Bz);
    f.G(gd(sz, 0, n2, 1, T2, sBz, mm, 1, X + plane, sCz, mm, 1, m, (int)mm, n2, -1.f, 1.f), Bz);
}

// out (real, [P][n2][n1][n0]) = alpha Re sum_k exp(+2 pi i k.x/n) Y[p][k]
// (planar Y, [P][kz][ky][kx]; temporaries s3, s4); beta accumulates into out.
void dft_inverse(Fno& f, const float* Y, long long plane, float* out, float alpha, float beta)
{
    const int m = f.net.m;
    const long long P = (long long)f.B * f.net.C;
    const int n0 = f.w.n[0], n1 = f.w.n[1], n2 = f.w.n[2];
    const float* cx = f.at(f.w.tw[0]);
    const float* sx = cx + (long long)m * n0;
    const float* cy = f.at(f.w.tw[1]);
    const float* sy = cy + (long long)m * n1;
    const float* cz = f.at(f.w.tw[2]);
    const float* sz = cz + (long long)m * n2;
    const long long mm = (long long)m * m;
    // inverse z: U[p][z][(ky,kx)] = sum_kz G[z][kz] Y[p][kz][(ky,kx)], G = cos + i sin (tables read transposed)
    float* U = f.at(f.w.s3);
    const long long su = P * n2 * mm;
    const int Bz = (int)P;
    const long long sBz = (long long)m * mm, sCz = (long long)n2 * mm;
    // re = C Yre - S Yim ; im = C Yim + S Yre
    f.G(gd(cz, 0, 1, n2, Y, sBz, mm, 1, U, sCz, mm, 1, n2, (int)mm, m, 1.f, 0.f), Bz);
    f.G(gd(sz, 0, 1, n2, Y + plane, sBz, mm, 1, U, sCz, mm, 1, n2, (int)mm, m, -1.f, 1.f), Bz);
    f.G(gd(cz, 0, 1, n2, Y + plane, sBz, mm, 1, U + su, sCz, mm, 1, n2, (int)mm, m, 1.f, 0.f), Bz);
    f.G(gd(sz, 0, 1, n2, Y, sBz, mm, 1, U + su, sCz, mm, 1, n2, (int)mm, m, 1.f, 1.f), Bz);
    // inverse y: V[(p,z)][y][kx] = sum_ky G[y][ky] U[(p,z)][ky][kx]
    float* V = f.at(f.w.s4);
    const long long sv = P * n2 * n1 * m;
    const int By = (int)(P * n2);
    const long long sBy = mm, sCy = (long long)n1 * m;
    f.G(gd(cy, 0, 1, n1, U, sBy, m, 1, V, sCy, m, 1, n1, m, m, 1.f, 0.f), By);
    f.G(gd(sy, 0, 1, n1, U + su, sBy, m, 1, V, sCy, m, 1, n1, m, m, -1.f, 1.f), By);
    f.G(gd(cy, 0, 1, n1, U + su, sBy, m, 1, V + sv, sCy, m, 1, n1, m, m, 1.f, 0.f), By);
    f.G(gd(sy, 0, 1, n1, U, sBy, m, 1, V + sv, sCy, m, 1, n1, m, m, 1.f, 1.f), By);
    // inverse x, real part: out[(p,z,y)][x] = alpha (Vre C^T - Vim S^T) + beta out
    const int Mx = (int)(P * n2 * n1);
    f.G(gd(V, 0, m, 1, cx, 0, n0, 1, out, 0, n0, 1, Mx, n0, m, alpha, beta), 1);
    f.G(gd(V + sv, 0, m, 1, sx, 0, n0, 1, out, 0, n0, 1, Mx, n0, m, -alpha, 1.f), 1);
}

// Y[b][o][k] = sum_i R(k)[o][i] X[b][i][k] (conj = 0) or sum_i conj(R(k)[i][o]) X[b][i][k]
// (conj = 1, the adjoint); planar complex, R (re, im) [k][o][i].
void mix(Fno& f, const float* Rre, const float* Rim, const float* X, long long xplane, float* Y, long long yplane,
         int conj)
{
    const int C = f.net.C, m3 = f.net.m3, B = f.B;
    // batch over k: A = R(k) (C x C): stride C*C per k; conj: transposed
    const long long sAb = (long long)C * C;
    const long long sAi = conj ? 1 : C, sAk = conj ? C : 1;
    // B(k)[i][b] = X[b][i][k]: strides i -> m3, b -> C m3, k -> 1
    const long long sBb = 1, sBk = m3, sBj = (long long)C * m3;
    const long long sCb = 1, sCi = m3, sCj = (long long)C * m3;
    const float si = conj ? -1.f : 1.f;  // conj(R) = Rre - i Rim
    // re = Rre Xre - si Rim Xim ; im = Rre Xim + si Rim Xre
    f.G(gd(Rre, sAb, sAi, sAk, X, sBb, sBk, sBj, Y, sCb, sCi, sCj, C, B, C, 1.f, 0.f), m3);
    f.G(gd(Rim, sAb, sAi, sAk, X + xplane, sBb, sBk, sBj, Y, sCb, sCi, sCj, C, B, C, -si, 1.f), m3);
    f.G(gd(Rre, sAb, sAi, sAk, X + xplane, sBb, sBk, sBj, Y + yplane, sCb, sCi, sCj, C, B, C, 1.f, 0.f), m3);
    f.G(gd(Rim, sAb, sAi, sAk, X, sBb, sBk, sBj, Y + yplane, sCb, sCi, sCj, C, B, C, si, 1.f), m3);
}

// out[b][o][v] = alpha sum_i W[o][i] in[b][i][v] + beta out (W row-major [co][ci];
// trans: W^T)
void pointwise(Fno& f, const float* W, int co, int ci, const float* in, float* out, float alpha, float beta,
               int trans)
{
    const long long N = f.w.N;
    const long long sAi = trans ? 1 : ci, sAk = trans ? ci : 1;  // W[o][i] at o ci + i
    const int M = trans ? ci : co, K = trans ? co : ci;
    f.G(gd(W, 0, sAi, sAk, in, (long long)K * N, N, 1, out, (long long)M * N, N, 1, M, (int)N, K, alpha, beta), f.B);
}

// dW[o][i] = sum_b sum_v d[b][o][v] in[b][i][v]
void pointwise_wgrad(Fno& f, const float* d, int co, const float* in, int ci, float* dW)
{
    const long long N = f.w.N;
    for (int b = 0; b < f.B; ++b)
        f.G(gd(d + (long long)b * co * N, 0, N, 1, in + (long long)b * ci * N, 0, 1, N, dW, 0, ci, 1, co, ci, (int)N,
               1.f, b == 0 ? 0.f : 1.f),
            1);
}

void forward(Fno& f, const float* P, const float* x)
{
    const Net& net = f.net;
    const long long N = f.w.N, B = f.B, C = net.C;
    const long long act = B * C * N;
    const long long xplane = B * C * net.m3;
    float* h0 = f.at(f.w.h);
    // lift
    pointwise(f, P + net.lift_w, (int)C, net.cin, x, f.at(f.w.acc), 1.f, 0.f, 0);
    k_bias_act<<<blocks(act), 256, 0, f.s>>>(f.at(f.w.acc), P + net.lift_b, h0, (int)C, N, act, 0);
    for (int l = 0; l < net.L; ++l) {
        const float* h = h0 + l * act;
        float* hn = h0 + (l + 1) * act;
        float* pre = f.at(f.w.pre) + l * act;
        float* X = f.at(f.w.xhat) + 2 * l * xplane;
        dft_forward(f, h, X, xplane);
        float* Y = f.at(f.w.s1);  // stage buffers are free again
        mix(f, P + net.r_re[l], P + net.r_im[l], X, xplane, Y, xplane, 0);
        dft_inverse(f, Y, xplane, pre, 1.f / (float)N, 0.f);
        pointwise(f, P + net.pw_w[l], (int)C, (int)C, h, pre, 1.f, 1.f, 0);
        k_bias_act<<<blocks(act), 256, 0, f.s>>>(pre, P + net.pw_b[l], hn, (int)C, N, act, 1);
    }
    // projection
    const long long outn = B * net.cout * N;
    pointwise(f, P + net.proj_w, net.cout, (int)C, h0 + net.L * act, f.at(f.w.y), 1.f, 0.f, 0);
    k_bias_act<<<blocks(outn), 256, 0, f.s>>>(f.at(f.w.y), P + net.proj_b, f.at(f.w.y), net.cout, N, outn, 0);
}

// gradient of the parameters (and of the input, dx nullable) for the output
// gradient dy; the activations of the preceding forward call are in the workspace
void backward(Fno& f, const float* P, const float* x, const float* dy, float* g, float* dx)
{
    const Net& net = f.net;
    const long long N = f.w.N, B = f.B, C = net.C;
    const long long act = B * C * N;
    const long long xplane = B * C * net.m3;
    float* h0 = f.at(f.w.h);
    float* dh = f.at(f.w.dh);
    float* dh2 = f.at(f.w.dh2);
    float* dpre = f.at(f.w.dpre);
    // projection
    pointwise_wgrad(f, dy, net.cout, h0 + net.L * act, (int)C, g + net.proj_w);
    k_bias_grad<<<net.cout, 256, 0, f.s>>>(dy, g + net.proj_b, f.B, net.cout, N);
    pointwise(f, P + net.proj_w, net.cout, (int)C, dy, dh, 1.f, 0.f, 1);
    for (int l = net.L - 1; l >= 0; --l) {
        const float* h = h0 + l * act;
        const float* pre = f.at(f.w.pre) + l * act;
        const float* X = f.at(f.w.xhat) + 2 * l * xplane;
        k_gelu_back<<<blocks(act), 256, 0, f.s>>>(pre, dh, dpre, act);
        // pointwise weight and bias
        pointwise_wgrad(f, dpre, (int)C, h, (int)C, g + net.pw_w[l]);
        k_bias_grad<<<(int)C, 256, 0, f.s>>>(dpre, g + net.pw_b[l], f.B, (int)C, N);
        // spectral: D = F dpre (into s3; the transform's stages use s1, s2);
        // dR(k) = (1/N) sum_b D X^H; dh = W^T dpre + (1/N) Re F^H R^H D
        float* Dk = f.at(f.w.s3);
        dft_forward(f, dpre, Dk, xplane);
        // dRre = (Dre Xre^T + Dim Xim^T)/N ; dRim = (Dim Xre^T - Dre Xim^T)/N, batched over k:
        // A(k)[o][b] = D[b][o][k], B(k)[b][i] = X[b][i][k]
        const int m3 = net.m3;
        const float invN = 1.f / (float)N;
        const long long sAb = 1, sAi = m3, sAk = C * m3;
        const long long sBb = 1, sBk = C * m3, sBj = m3;
        const long long sCb = C * C, sCi = C, sCj = 1;
        float* gre = g + net.r_re[l];
        float* gim = g + net.r_im[l];
        f.G(gd(Dk, sAb, sAi, sAk, X, sBb, sBk, sBj, gre, sCb, sCi, sCj, (int)C, (int)C, f.B, invN, 0.f), m3);
        f.G(gd(Dk + xplane, sAb, sAi, sAk, X + xplane, sBb, sBk, sBj, gre, sCb, sCi, sCj, (int)C, (int)C, f.B, invN,
               1.f),
            m3);
        f.G(gd(Dk + xplane, sAb, sAi, sAk, X, sBb, sBk, sBj, gim, sCb, sCi, sCj, (int)C, (int)C, f.B, invN, 0.f), m3);
        f.G(gd(Dk, sAb, sAi, sAk, X + xplane, sBb, sBk, sBj, gim, sCb, sCi, sCj, (int)C, (int)C, f.B, -invN, 1.f),
            m3);
        // R^H D into s1 (free after the transform; the inverse stages use s3, s4)
        float* RD = f.at(f.w.s1);
        mix(f, P + net.r_re[l], P + net.r_im[l], Dk, xplane, RD, xplane, 1);
        dft_inverse(f, RD, xplane, dh2, 1.f / (float)N, 0.f);
        pointwise(f, P + net.pw_w[l], (int)C, (int)C, dpre, dh2, 1.f, 1.f, 1);
        std::swap(dh, dh2);
    }
    // lift
    pointwise_wgrad(f, dh, (int)C, x, net.cin, g + net.lift_w);
    k_bias_grad<<<(int)C, 256, 0, f.s>>>(dh, g + net.lift_b, f.B, (int)C, N);
    if (dx) pointwise(f, P + net.lift_w, (int)C, net.cin, dh, dx, 1.f, 0.f, 1);
}

bool valid_grid(const int32_t n[3])
{
    if (!n) return false;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] > 1024) return false;
    return true;
}

rpm_status fno_open(Fno& f, const rpm_fno_config* cfg, const int32_t n[3], int32_t batch, void* ws, size_t ws_bytes,
                    void* stream)
{
    f.net = make_net(cfg);
    if (!f.net.ok || !valid_grid(n) || batch < 1 || batch > 4096) return RPM_E_INVALID;
    f.w = make_fws(f.net, n, batch);
    if (!ws || ws_bytes < (size_t)f.w.total * sizeof(float)) return RPM_E_WORKSPACE;
    f.ws = (float*)ws;
    f.s = (hipStream_t)stream;
    f.B = batch;
    if (!upload_twiddles(f)) return RPM_E_HIP;
    return RPM_OK;
}

}  // namespace

extern "C" {

rpm_status rpm_gemm_bf16(int32_t M, int32_t N, int32_t K, int32_t batch, const float* A, const int64_t sA[3],
                         const float* B, const int64_t sB[3], float* C, const int64_t sC[3], float alpha, float beta,
                         void* hip_stream)
{
    if (M < 1 || N < 1 || K < 1 || batch < 1 || batch > 65535 || !A || !B || !C || !sA || !sB || !sC)
        return RPM_E_INVALID;
    hipStream_t s = (hipStream_t)hip_stream;
    if (!gemm(s, gd(A, sA[0], sA[1], sA[2], B, sB[0], sB[1], sB[2], C, sC[0], sC[1], sC[2], M, N, K, alpha, beta),
              batch))
        return RPM_E_INVALID;
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return RPM_E_HIP;
    return RPM_OK;
}

rpm_status rpm_fno_param_count(const rpm_fno_config* cfg, int64_t* count)
{
    const Net n = make_net(cfg);
    if (!n.ok || !count) return RPM_E_INVALID;
    *count = n.total;
    return RPM_OK;
}

rpm_status rpm_fno_workspace_size(const rpm_fno_config* cfg, const int32_t n[3], int32_t batch, size_t* bytes)
{
    const Net net = make_net(cfg);
    if (!net.ok || !valid_grid(n) || batch < 1 || batch > 4096 || !bytes) return RPM_E_INVALID;
    *bytes = (size_t)make_fws(net, n, batch).total * sizeof(float);
    return RPM_OK;
}

rpm_status rpm_fno_init(const rpm_fno_config* cfg, uint64_t seed, float* params, void* hip_stream)
{
    const Net net = make_net(cfg);
    if (!net.ok || !params) return RPM_E_INVALID;
    // splitmix64 counter-based stream: uniform in [0, 1) from the top 24 bits
    std::vector<float> p((size_t)net.total, 0.f);
    uint64_t ctr = seed;
    auto uni = [&]() {
        uint64_t z = (ctr += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        return (float)((z >> 40) * (1.0 / 16777216.0));
    };
    auto fill = [&](long long off, long long count, float lo, float hi) {
        for (long long i = 0; i < count; ++i) p[(size_t)(off + i)] = lo + (hi - lo) * uni();
    };
    const float al = 1.f / std::sqrt((float)net.cin), ac = 1.f / std::sqrt((float)net.C);
    fill(net.lift_w, (long long)net.C * net.cin, -al, al);
    for (int l = 0; l < net.L; ++l) {
        fill(net.pw_w[l], (long long)net.C * net.C, -ac, ac);
        const float sr = 1.f / ((float)net.C * net.C);
        fill(net.r_re[l], (long long)net.m3 * net.C * net.C, 0.f, sr);
        fill(net.r_im[l], (long long)net.m3 * net.C * net.C, 0.f, sr);
    }
    fill(net.proj_w, (long long)net.cout * net.C, -ac, ac);
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipMemcpyAsync(params, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess)
        return RPM_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RPM_E_HIP;
    return RPM_OK;
}

rpm_status rpm_fno_forward(const rpm_fno_config* cfg, const float* params, const int32_t n[3], int32_t batch,
                           const float* x, float* y, void* workspace, size_t ws_bytes, void* hip_stream)
{
    if (!params || !x) return RPM_E_INVALID;
    Fno f;
    rpm_status rs = fno_open(f, cfg, n, batch, workspace, ws_bytes, hip_stream);
    if (rs != RPM_OK) return rs;
    forward(f, params, x);
    if (y && hipMemcpyAsync(y, f.at(f.w.y), sizeof(float) * (size_t)batch * f.net.cout * f.w.N,
                            hipMemcpyDeviceToDevice, f.s) != hipSuccess)
        return RPM_E_HIP;
    if (!f.ok || hipGetLastError() != hipSuccess || hipStreamSynchronize(f.s) != hipSuccess) return RPM_E_HIP;
    return RPM_OK;
}

rpm_status rpm_fno_backward(const rpm_fno_config* cfg, const float* params, const int32_t n[3], int32_t batch,
                            const float* x, const float* dy, float* grad, float* dx, void* workspace, size_t ws_bytes,
                            void* hip_stream)
{
    if (!params || !x || !dy || !grad) return RPM_E_INVALID;
    Fno f;
    rpm_status rs = fno_open(f, cfg, n, batch, workspace, ws_bytes, hip_stream);
    if (rs != RPM_OK) return rs;
    backward(f, params, x, dy, grad, dx);
    if (!f.ok || hipGetLastError() != hipSuccess || hipStreamSynchronize(f.s) != hipSuccess) return RPM_E_HIP;
    return RPM_OK;
}

rpm_status rpm_fno_train_step(const rpm_fno_config* cfg, float* params, float* grad, float* adam_m, float* adam_v,
                              int32_t step, float lr, const int32_t n[3], int32_t batch, const float* x,
                              const float* target, double* loss, void* workspace, size_t ws_bytes, void* hip_stream)
{
    if (!params || !grad || !adam_m || !adam_v || !x || !target || step < 1 || !(lr > 0.f)) return RPM_E_INVALID;
    Fno f;
    rpm_status rs = fno_open(f, cfg, n, batch, workspace, ws_bytes, hip_stream);
    if (rs != RPM_OK) return rs;
    forward(f, params, x);
    const long long ny = (long long)batch * f.net.cout * f.w.N;
    // the output gradient in the accumulator slot (backward does not use it)
    float* dy = f.at(f.w.acc);
    const int nb = (int)std::min<long long>(1024, (ny + 255) / 256);
    double* part = reinterpret_cast<double*>(f.at(f.w.part));
    k_mse<<<nb, 256, 0, f.s>>>(f.at(f.w.y), target, x, f.net.cin, f.net.cout, f.w.N, dy, part, ny);
    backward(f, params, x, dy, grad, nullptr);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    k_adam<<<blocks(f.net.total), 256, 0, f.s>>>(params, grad, adam_m, adam_v, f.net.total, lr, b1, b2, eps, c1, c2);
    if (loss) {
        std::vector<double> hp((size_t)nb);
        if (hipMemcpyAsync(hp.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, f.s) != hipSuccess)
            return RPM_E_HIP;
        if (hipStreamSynchronize(f.s) != hipSuccess) return RPM_E_HIP;
        double s = 0.0;
        for (double v : hp) s += v;
        *loss = s / (double)ny;
    }
    if (!f.ok || hipGetLastError() != hipSuccess || hipStreamSynchronize(f.s) != hipSuccess) return RPM_E_HIP;
    return RPM_OK;
}

// Feature table of a phase table (host).
bool feature_table(const rpm_problem* pr, float* tab)
{
    double emax = 0.0;
    std::vector<double> E((size_t)pr->n_phases), nu((size_t)pr->n_phases);
    for (int i = 0; i < pr->n_phases; ++i) {
        const double l = pr->lame[2 * i], m = pr->lame[2 * i + 1];
        if (!(m > 0.0) || !std::isfinite(l) || !(l + m > 0.0)) return false;
        E[(size_t)i] = m * (3.0 * l + 2.0 * m) / (l + m);
        nu[(size_t)i] = l / (2.0 * (l + m));
        emax = std::max(emax, E[(size_t)i]);
    }
    for (int i = 0; i < 512; ++i) tab[i] = 0.f;
    for (int i = 0; i < pr->n_phases; ++i) {
        tab[2 * i] = (float)(std::max(std::log10(E[(size_t)i] / emax), -3.0) / 3.0);
        tab[2 * i + 1] = (float)(nu[(size_t)i] - 0.3);
    }
    return true;
}

rpm_status rpm_fno_features(const rpm_problem* pr, float* x, void* hip_stream)
{
    if (!pr || !pr->phase || !pr->lame || !x || pr->n_phases < 1 || pr->n_phases > 256) return RPM_E_INVALID;
    for (int a = 0; a < 3; ++a)
        if (pr->n[a] < 1) return RPM_E_INVALID;
    FeatTab t;
    if (!feature_table(pr, t.v)) return RPM_E_INVALID;
    const long long N = (long long)pr->n[0] * pr->n[1] * pr->n[2];
    hipStream_t s = (hipStream_t)hip_stream;
    k_features<<<blocks(N), 256, 0, s>>>(pr->phase, t, x, N);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return RPM_E_HIP;
    return RPM_OK;
}

rpm_status rpm_fno_warm_start(const rpm_fno_config* cfg, const float* params, const rpm_problem* pr,
                              const double E[6], int32_t precision, void* eps0, void* workspace, size_t ws_bytes,
                              void* hip_stream)
{
    if (!cfg || !params || !pr || !pr->phase || !pr->lame || !E || !eps0) return RPM_E_INVALID;
    if (cfg->c_in != 2 || cfg->c_out != 36) return RPM_E_INVALID;
    if (precision != RPM_FP64 && precision != RPM_FP32) return RPM_E_INVALID;
    if (pr->n_phases < 1 || pr->n_phases > 256) return RPM_E_INVALID;
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(E[i])) return RPM_E_INVALID;
    FeatTab t;
    if (!feature_table(pr, t.v)) return RPM_E_INVALID;
    Fno f;
    rpm_status rs = fno_open(f, cfg, pr->n, 1, workspace, ws_bytes, hip_stream);
    if (rs != RPM_OK) return rs;
    const long long N = f.w.N;
    k_features<<<blocks(N), 256, 0, f.s>>>(pr->phase, t, f.at(f.w.feat), N);
    forward(f, params, f.at(f.w.feat));
    E6 e;
    for (int i = 0; i < 6; ++i) e.e[i] = E[i];
    if (precision == RPM_FP64) k_assemble<double><<<blocks(N), 256, 0, f.s>>>(f.at(f.w.y), e, (double*)eps0, N);
    else k_assemble<float><<<blocks(N), 256, 0, f.s>>>(f.at(f.w.y), e, (float*)eps0, N);
    if (!f.ok || hipGetLastError() != hipSuccess || hipStreamSynchronize(f.s) != hipSuccess) return RPM_E_HIP;
    return RPM_OK;
}

}  // extern "C"
