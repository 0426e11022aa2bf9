// Pass kernels of the gfx950 RPM-FFT path.
//
// One application of the Lippmann-Schwinger map (the iteration body of
// Algorithm 1; the operator F of Sec. 3) is five pencil passes over an FFT pipeline whose
// spectrum is transposed as it goes, so that every pass reads or writes whole
// contiguous rows and the other side in 128-byte (or longer) segments:
//
//   xfwd   strain tile -> sigma = C(x):eps in registers, real-to-complex
//          FFT along x (two components packed per complex FFT), spectrum
//          written as S1[c][kx][z][y]
//   yfwd   S1 rows along y -> FFT -> S2[c][ky][kx][z]
//   gamma  S2 rows along z -> FFT -> per frequency t = Gamma0(k):sigma_hat,
//          equilibrium-error partial sums, <sigma> -> inverse FFT in place
//   yinv   S2 -> inverse FFT along y -> S1
//   xinv   S1 -> complex-to-real inverse FFT along x -> xi = eps - t
//
// and, in an RPM iteration, two streams over the basis Z: the recombination
// eps = xi_prev + Z d before the map (k_recombine_split for FP32 fields; for
// FP64 fields on 128-point rows inside xfwd, else k_recombine) and the
// projections Z^T xi after it (k_gdots_split / k_gdots, FP64 accumulation).
//
// In 2-D (nz == 1) the y passes are skipped and gamma runs along y on S1.
// The k = 0 term of t is N(<eps> - E), so xi = eps - F^-1[Gamma sigma_hat]
// + (E - <eps>), which is exactly the paper's update with xi_hat(0) = N E.
#pragma once

#include <type_traits>

#include "rpm_device.h"

namespace rpm {

// 16-byte non-temporal loads: the per-step basis streams read 50 MB per column
// and would otherwise push the fields the FFT passes re-read out of the caches
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 nt_load(const float4* p)
{
    const nt_f4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    return make_float4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ double2 nt_load(const double2* p)
{
    const nt_d2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    return make_double2(t.x, t.y);
}

// waves per SIMD the compiler budgets registers for: the in-place gamma pass
// (five resident blocks per CU), and the x pass that recombines eps = xi + Z d
// on the way in (four; with 8 basis columns in flight per lane it needs ~114
// VGPRs, and 16 columns spill at four waves and drop to three); RC_GROUP is
// the basis columns in flight per lane there
#ifndef RPM_GIP_WPE
#define RPM_GIP_WPE 5
#endif
#ifndef RPM_RC_GROUP
#define RPM_RC_GROUP 8
#endif
#ifndef RPM_RC_WPE
#define RPM_RC_WPE 4
#endif

struct Geo {
    int nx, ny, nz, nh;    // nh = nx/2 + 1 (half spectrum along x)
    long long N;           // voxels
    long long nspec;       // complex entries per component of the half spectrum
    int ty;                // y rows per x-pass tile
    int tz;                // z columns per y-pass tile
    int np;                // pencils per gamma tile
    int two_d;
    int ncomp;             // spectral components of the forward passes (6, or 12 with eps)
    FDiv fnx, fny, fnh, fty, ftz, frow;  // divisions by nx, ny, nh, ty, tz and the gamma row length
    double kh[3];          // 2 pi / n per axis (wave number of index 1)
};

// Basis storage: Z (and W = F_u Z) in tiles of kZTile consecutive elements of
// the 6N-vector; tile t holds its slice of all P column slots contiguously, so
// element e of column j sits at zix(e, j, P).  Per-voxel recombination and the
// basis products then read contiguous kilobyte slices.
constexpr int kZTile = 256;
constexpr int kMaxTy = 128;  // x-pass tiles hold at most this many rows
__host__ __device__ __forceinline__ long long zix(long long e, int j, int P)
{
    return ((e / kZTile) * (long long)P + j) * kZTile + (e % kZTile);
}

// Device-resident solver state (one per workspace).
struct DevState {
    int magic;         // kStateMagic once the workspace has been initialised
    int cfg[6];        // nx, ny, nz, precision, p_max, map the basis was built for
    int done;          // 1 once the iteration stopped (any reason)
    int status;        // 0 converged, 1 not converged, 2 diverged, 3 singular, 4 stalled
    int iters;         // main-loop F applications so far
    int p;             // basis dimension
    int singular;      // LU of I - H hit a tiny pivot
    int max_iter;
    int pad1;
    double tol;
    double err0;       // error of the starting iterate
    double err;        // error of the latest iterate
    double sig_hat0[6];// sigma_hat(0) of the latest F application
    double mean_eps[6];
    double E[6];       // prescribed mean strain of the current solve
    double Ezero[6];   // zeros (mean strain of Jacobian-vector products)
    double gnorm;      // norm of the shift field of a correction solve
    double best_err;   // lowest error below 0.9 x the previous lowest (stall test)
    int best_it;       // iteration at which best_err was reached
    int stall_window;  // stop (status 4) after this many iterations without a new best_err; 0 = off
    double medium[8];  // lambda0, mu0, alpha, beta, a hash of the phase table and a checksum of the phase map
                       // the basis was built for
    double z[kMaxP], zeta[kMaxP], d[kMaxP];
    double zeta_ring[4][kMaxP];
    double H[kMaxP * kMaxP];
    double LU[kMaxP * kMaxP];
    double G[kMaxP * kMaxP];     // Gram matrix <Z_i, Z_j> of the stored columns
    double AinvT[kMaxP * kMaxP]; // (I - H)^{-1}, transposed: AinvT[j * kMaxP + i] = inv[i][j]
    int piv[kMaxP];
};

constexpr int kStateMagic = 0x52504d31;

enum { DC_MEAN = 0, DC_ZERO = 1 };   // t_hat(0) = N(<eps> - E) or 0
enum { OUT_XI = 0, OUT_T = 1 };      // xinv writes eps - t or t

// 16-byte vector type of an element type
template <typename TZ>
struct Vec4;
template <>
struct Vec4<float> {
    using type = float4;
};
template <>
struct Vec4<double> {
    using type = double2;  // 16-byte loads for double columns
};

template <typename T>
struct MaxV;
template <>
struct MaxV<float> { static constexpr int v = 8; };
template <>
struct MaxV<double> { static constexpr int v = 4; };

// ---------------------------------------------------------------------------
// x-forward: constitutive law + R2C FFT along x (two real components per
// complex transform), per-block <eps> partial sums.  POL: eps is transformed
// too (components 6..11 of S1), for the polarization iteration.
// RC (RPM iterations, VEC only): the strain is recombined on the way in,
// eps = xin + sum_{j < p} d_j Z_j, in the order and rounding of k_recombine,
// and stored to eps_out (the x-inverse pass reads it); the tile's basis
// slices stream through eight columns at a time.
// grid: nz * (ny / ty) blocks.  LDS: 2 * ty * lrow(nx) + nx complex + reduction.
// ---------------------------------------------------------------------------
template <typename T, bool VEC, bool POL, int NT, bool IP, bool RC = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (RC ? RPM_RC_WPE : 4) : 2))) void k_xfwd(const T* __restrict__ xin, const uint8_t* __restrict__ phase,
                                                   const double* __restrict__ lame, int use_ref, double lam0,
                                                   double mu0, cx<T>* __restrict__ S1,
                                                   double* __restrict__ part_mean, Geo g, Plan px,
                                                   const cx<T>* __restrict__ twx, const int* __restrict__ done,
                                                   const T* __restrict__ Z = nullptr, int p = 0, int zP = 0,
                                                   const double* __restrict__ dco = nullptr,
                                                   T* __restrict__ eps_out = nullptr)
{
    static_assert(!RC || VEC, "recombination on the way in needs 16-byte runs");
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int MV = MaxV<T>::v * kThreads / NT;  // voxels per thread
    const int nx = g.nx, ty = g.ty, ss = lrow(nx);
    cx<T>* A = reinterpret_cast<cx<T>*>(smem);
    cx<T>* B = A + ty * ss;
    cx<T>* tw = IP ? B : B + ty * ss;  // IP: one buffer, transforms in place
    double* red = reinterpret_cast<double*>(tw + nx);
    constexpr int RG = RPM_RC_GROUP;  // basis columns in flight per thread
    __shared__ T dj[RC ? kMaxP + RG : 1];
    if constexpr (RC) {
        for (int j = threadIdx.x; j < kMaxP + RG; j += NT) dj[j] = j < p ? (T)dco[j] : T(0);
        __syncthreads();
    }

    const int nyt = g.ny / ty;
    const int z = blockIdx.x / nyt;
    const int y0 = (blockIdx.x - z * nyt) * ty;
    const long long base = ((long long)z * g.ny + y0) * nx;  // tile = contiguous rows
    const int nvox = ty * nx;
    const long long N = g.N;

    for (int i = threadIdx.x; i < nx; i += NT) tw[i] = twx[i];

    // VEC: each thread takes runs of VL consecutive voxels (16-byte accesses).
    // All strain loads are issued up front, the three components of the first
    // transform's inputs first: the later components are only needed by the
    // later transforms and stay in flight meanwhile.
    constexpr int VL = VEC ? (int)(16 / sizeof(T)) : 1;
    constexpr int NI = MV / VL;
    using V = typename Vec4<T>::type;
    T e[MV][6];
    T lamv[MV], muv[MV];
    auto load_comp = [&](int c) {
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int v0 = (threadIdx.x + i * NT) * VL;
            const long long gi = base + v0;
            if (v0 < nvox) {
                if constexpr (RC) {
                    // a wave's run covers contiguous elements of one basis tile per column
                    const long long el = c * N + gi;
                    V acc = *reinterpret_cast<const V*>(xin + el);
                    T* a = reinterpret_cast<T*>(&acc);
                    const T* zt = Z + zix(el, 0, zP);
                    for (int gq = 0; gq < p; gq += RG) {
                        V zv[RG];
#pragma unroll
                        for (int u = 0; u < RG; ++u)
                            zv[u] = nt_load(reinterpret_cast<const V*>(zt + (long long)min(gq + u, p - 1) * kZTile));
#pragma unroll
                        for (int u = 0; u < RG; ++u) {
                            const T* zs = reinterpret_cast<const T*>(&zv[u]);
                            const T cf = dj[gq + u];
#pragma unroll
                            for (int q = 0; q < VL; ++q) a[q] += cf * zs[q];
                        }
                    }
                    *reinterpret_cast<V*>(eps_out + el) = acc;
#pragma unroll
                    for (int u = 0; u < VL; ++u) e[i * VL + u][c] = a[u];
                } else if constexpr (VEC) {
                    const V t = *reinterpret_cast<const V*>(xin + c * N + gi);
                    const T* ts = reinterpret_cast<const T*>(&t);
#pragma unroll
                    for (int u = 0; u < VL; ++u) e[i * VL + u][c] = ts[u];
                } else {
                    e[i][c] = xin[c * N + gi];
                }
            } else {
#pragma unroll
                for (int u = 0; u < VL; ++u) e[i * VL + u][c] = T(0);
            }
        }
    };
#pragma unroll
    for (int c = 0; c < 3; ++c) load_comp(c);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int v0 = (threadIdx.x + i * NT) * VL;
#pragma unroll
        for (int u = 0; u < VL; ++u) {
            if (use_ref || v0 >= nvox) {
                lamv[i * VL + u] = (T)lam0;
                muv[i * VL + u] = (T)mu0;
            } else {
                const int ph = phase[base + v0 + u];
                lamv[i * VL + u] = (T)lame[2 * ph];
                muv[i * VL + u] = (T)lame[2 * ph + 1];
            }
        }
    }
#pragma unroll
    for (int c = 3; c < 6; ++c) load_comp(c);

    // sigma = C(x):eps of components 2q, 2q+1 (the trace term on the normal ones)
    auto sig = [&](int v, int c) -> T {
        const T s = (muv[v] + muv[v]) * e[v][c];
        return c < 3 ? s + lamv[v] * (e[v][0] + e[v][1] + e[v][2]) : s;
    };
    double msum[6] = {0, 0, 0, 0, 0, 0};
    const int nh = g.nh;
#pragma unroll
    for (int q = 0; q < (POL ? 6 : 3); ++q) {  // unrolled: the register arrays take constant indices
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int v0 = (threadIdx.x + i * NT) * VL;
            if (v0 < nvox) {
                const int r = g.fnx.div(v0);
                const int x = v0 - r * nx;
#pragma unroll
                for (int u = 0; u < VL; ++u) {
                    const int v = i * VL + u;
                    cx<T> val;
                    if (q < 3) {
                        val = cx<T>{sig(v, 2 * q), sig(v, 2 * q + 1)};
                        msum[2 * q] += (double)e[v][2 * q];
                        msum[2 * q + 1] += (double)e[v][2 * q + 1];
                    } else {
                        val = cx<T>{e[v][2 * q - 6], e[v][2 * q - 5]};
                    }
                    A[r * ss + lpad(x + u)] = val;
                }
            }
        }
        __syncthreads();
        const cx<T>* R;
        if constexpr (IP) {
            ct_stages_ip<T, -1, 128, 0, 1, NT>(A, ty, ss, tw, threadIdx.x);
            R = A;
        } else {
            R = lds_fft<T, -1, NT>(A, B, px, ty, ss, tw);
        }
        // split the packed transform into the two real-input spectra
        cx<T>* outa = S1 + (long long)(2 * q) * g.nspec;
        cx<T>* outb = S1 + (long long)(2 * q + 1) * g.nspec;
        for (int t = threadIdx.x; t < nh * ty; t += NT) {
            const int k = g.fty.div(t);
            const int r = t - k * ty;
            const cx<T> X = R[r * ss + lpad(k)];
            const cx<T> Yc = cconj(R[r * ss + lpad(k == 0 ? 0 : nx - k)]);
            const cx<T> s = cadd(X, Yc);
            const cx<T> d = csub(X, Yc);
            const long long o = ((long long)k * g.nz + z) * g.ny + y0 + r;
            outa[o] = cx<T>{T(0.5) * s.x, T(0.5) * s.y};
            outb[o] = cx<T>{T(0.5) * d.y, T(-0.5) * d.x};
        }
    }
    if (part_mean) {
        __syncthreads();
        wg_sum_store<6, NT>(msum, part_mean + (long long)blockIdx.x * 6, red);
    }
}

// ---------------------------------------------------------------------------
// y-forward (FFT along y): S1[c][kx][z][y] -> S2[c][ky][kx][z].
// grid: 6 * nh * (nz / tz) blocks.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_yfwd(const cx<T>* __restrict__ S1, cx<T>* __restrict__ S2, Geo g,
                                                   Plan py, const cx<T>* __restrict__ twy,
                                                   const int* __restrict__ done)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int ny = g.ny, tz = g.tz, ss = lrow(ny);
    cx<T>* A = reinterpret_cast<cx<T>*>(smem);
    cx<T>* B = A + tz * ss;
    cx<T>* tw = B + tz * ss;
    const int nzt = g.nz / tz;
    int b = blockIdx.x;
    const int zt = b % nzt;
    b /= nzt;
    const int kx = b % g.nh;
    const int c = b / g.nh;
    const int z0 = zt * tz;
    for (int i = threadIdx.x; i < ny; i += kThreads) tw[i] = twy[i];
    const cx<T>* src = S1 + (long long)c * g.nspec + ((long long)kx * g.nz + z0) * ny;
    for (int t = threadIdx.x; t < tz * ny; t += kThreads) {
        const int r = g.fny.div(t);
        const int y = t - r * ny;
        A[r * ss + lpad(y)] = src[t];
    }
    __syncthreads();
    const cx<T>* R = lds_fft<T, -1>(A, B, py, tz, ss, tw);
    cx<T>* dst = S2 + (long long)c * g.nspec;
    for (int t = threadIdx.x; t < tz * ny; t += kThreads) {
        const int ky = g.ftz.div(t);
        const int r = t - ky * tz;
        dst[((long long)ky * g.nh + kx) * g.nz + z0 + r] = R[r * ss + lpad(ky)];
    }
}

// Software-pipelined y passes: a persistent grid walks the tiles; each thread
// keeps its share of the next tile in registers (loads in flight during the
// current tile's LDS transform and stores).  PT bounds tz * ny / kThreads.
template <typename T, int D, int PT, bool IP>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (IP ? 5 : 4) : 2))) void k_ypipe(const cx<T>* __restrict__ Sin, cx<T>* __restrict__ Sout, Geo g,
                                                    Plan py, const cx<T>* __restrict__ twy, int ntiles,
                                                    const int* __restrict__ done)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int ny = g.ny, tz = g.tz, ss = lrow(ny);
    cx<T>* A = reinterpret_cast<cx<T>*>(smem);
    cx<T>* B = A + tz * ss;
    cx<T>* tw = IP ? B : B + tz * ss;  // IP: one buffer, transforms in place
    const int nzt = g.nz / tz;
    const int nel = tz * ny;
    for (int i = threadIdx.x; i < ny; i += kThreads) tw[i] = twy[i];
    cx<T> pre[PT];
    // forward (D < 0): tile rows are contiguous in S1; inverse: TZ-segments of S2
    auto load = [&](int t) {
        int b = t;
        const int zt = b % nzt;
        b /= nzt;
        const int kx = b % g.nh;
        const int c = b / g.nh;
        const int z0 = zt * tz;
        // per-element offsets are recomputed per tile, not kept in registers
        // across the loop (the inverse pass would spill them)
        int opq = 0;
        asm volatile("" : "+s"(opq));
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int e = threadIdx.x + opq + u * kThreads;
            if (e < nel) {
                if (D < 0) {
                    pre[u] = Sin[(long long)c * g.nspec + ((long long)kx * g.nz + z0) * ny + e];
                } else {
                    const int ky = g.ftz.div(e), r = e - ky * tz;
                    pre[u] = Sin[(long long)c * g.nspec + ((long long)ky * g.nh + kx) * g.nz + z0 + r];
                }
            }
        }
    };
    int t = blockIdx.x;
    if (t < ntiles) load(t);
    for (; t < ntiles; t += gridDim.x) {
        __syncthreads();  // the previous tile's stores have read A/B
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int e = threadIdx.x + u * kThreads;
            if (e < nel) {
                if (D < 0) {
                    const int r = g.fny.div(e), y = e - r * ny;
                    A[r * ss + lpad(y)] = pre[u];
                } else {
                    const int ky = g.ftz.div(e), r = e - ky * tz;
                    A[r * ss + lpad(ky)] = pre[u];
                }
            }
        }
        __syncthreads();
        const int tn = t + gridDim.x;
        if (tn < ntiles) load(tn);  // next tile in flight during the transform
        const cx<T>* R;
        if constexpr (IP) {
            ct_stages_ip<T, D, 128, 0, 1, kThreads>(A, tz, ss, tw, threadIdx.x);
            R = A;
        } else {
            R = lds_fft<T, D>(A, B, py, tz, ss, tw);
        }
        int b = t;
        const int zt = b % nzt;
        b /= nzt;
        const int kx = b % g.nh;
        const int c = b / g.nh;
        const int z0 = zt * tz;
        if (D < 0) {
            cx<T>* dst = Sout + (long long)c * g.nspec;
            for (int e = threadIdx.x; e < nel; e += kThreads) {
                const int ky = g.ftz.div(e), r = e - ky * tz;
                dst[((long long)ky * g.nh + kx) * g.nz + z0 + r] = R[r * ss + lpad(ky)];
            }
        } else {
            cx<T>* dst = Sout + (long long)c * g.nspec + ((long long)kx * g.nz + z0) * ny;
            for (int e = threadIdx.x; e < nel; e += kThreads) {
                const int r = g.fny.div(e), y = e - r * ny;
                dst[e] = R[r * ss + lpad(y)];
            }
        }
    }
}

// Cross-lane exchange within rows of 16 lanes through the data-parallel
// primitives (DPP) of the vector ALU: the value of lane l ^ H (H = 1, 2, 4, 8).
// H = 4 takes two moves (lanes 4..7 of each 8 from the right, 0..3 from the
// left, selected by bank masks).
template <int H>
__device__ __forceinline__ float lane_xor(float v)
{
    const int i = __float_as_int(v);
    int r;
    if constexpr (H == 1) r = __builtin_amdgcn_update_dpp(i, i, 0xB1, 0xF, 0xF, false);        // quad_perm 1,0,3,2
    else if constexpr (H == 2) r = __builtin_amdgcn_update_dpp(i, i, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    else if constexpr (H == 8) r = __builtin_amdgcn_update_dpp(i, i, 0x128, 0xF, 0xF, false);  // row_ror 8
    else {
        r = __builtin_amdgcn_update_dpp(i, i, 0x104, 0xF, 0x5, false);  // row_shl 4 into banks 0, 2
        r = __builtin_amdgcn_update_dpp(r, i, 0x114, 0xF, 0xA, false);  // row_shr 4 into banks 1, 3
    }
    return __int_as_float(r);
}

// y passes with the 128-point transforms in registers (FP32, ny = 128, tiles
// of 16 z rows, nz % 16 == 0): a wave takes four rows of a tile at a time, one
// row per 16-lane group; lane j of a group holds elements 8j .. 8j+7 of its
// row.  With n = 8j + m and k = k2 + 16 k1: a 16-point DFT over j
// across the group's lanes (four radix-2 stages, partners exchanged by DPP,
// output k2 at lane bitrev(k2)), twiddles w128^(m k2), and an 8-point DFT over
// m in registers give X[k2 + 16 k1] in register k1 — for each k1 the group
// holds 16 consecutive outputs.  No LDS and no barriers: rows along y are read
// (forward) or written (inverse) as 64-byte runs per lane or 128-byte runs per
// group, the transposed side S2[c][ky][kx][z] as 32-byte runs of the four rows
// of a wave (the four tasks of a tile complete each 128-byte line).  A
// persistent grid of waves walks the tasks (four rows of a tile each) with the
// next task's loads in flight.
template <int D>
__global__ __launch_bounds__(kThreads) void k_ywave(const cx<float>* __restrict__ Sin, cx<float>* __restrict__ Sout,
                                                    Geo g, const cx<float>* __restrict__ twy, int ntasks,
                                                    const int* __restrict__ done)
{
    if (done && *done) return;
    const int lane = threadIdx.x & 63;
    const int j = lane & 15;
    const int nzt = g.nz / 16;
    // per-lane twiddles: of the three span-h stages (upper lanes; 1 below)
    // and w128^(m k2) of the lane's output index k2 = bitrev(j)
    const int k2 = (int)(__builtin_bitreverse32((unsigned)j) >> 28);
    cx<float> ws[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int H = 8 >> s;
        ws[s] = cx<float>{1.f, 0.f};
        if (j & H) {
            ws[s] = twy[(j & (H - 1)) * (64 / H)];  // w_2h^e = w_128^(64 e / h)
            if (D > 0) ws[s].y = -ws[s].y;
        }
    }
    cx<float> wm[8];
#pragma unroll
    for (int m = 1; m < 8; ++m) {
        wm[m] = twy[(m * k2) & 127];
        if (D > 0) wm[m].y = -wm[m].y;
    }
    // a task is four rows of a 16-row tile: rows 4 (t & 3) .. 4 (t & 3) + 3
    // of tile t >> 2, one row per 16-lane group
    auto row_of = [&](int t, int& kx, int& z, long long& cb) {
        int b = t >> 2;
        const int zt = b % nzt;
        b /= nzt;
        kx = b % g.nh;
        cb = (long long)(b / g.nh) * g.nspec;
        z = zt * 16 + 4 * (t & 3) + (lane >> 4);
    };
    cx<float> v[8];
    auto load = [&](int t) {
        int kx, z;
        long long cb;
        row_of(t, kx, z, cb);
        if constexpr (D < 0) {
            // row (c, kx, z) of S1, elements 8j .. 8j+7
            const float4* src = reinterpret_cast<const float4*>(Sin + cb + ((long long)kx * g.nz + z) * 128 + 8 * j);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 u = src[q];
                v[2 * q] = cx<float>{u.x, u.y};
                v[2 * q + 1] = cx<float>{u.z, u.w};
            }
        } else {
            // S2[c][ky][kx][z] for ky = 8j + m
#pragma unroll
            for (int m = 0; m < 8; ++m) v[m] = Sin[cb + ((long long)(8 * j + m) * g.nh + kx) * g.nz + z];
        }
    };
    const int gw = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int nw = gridDim.x * (kThreads / 64);
    int t = gw;
    if (t < ntasks) load(t);
    for (; t < ntasks; t += nw) {
        cx<float> a[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) a[m] = v[m];
        if (t + nw < ntasks) load(t + nw);  // the next task's loads in flight
        // 16-point DIF over j: span h, lower lanes a + b, upper (a - b) w_2h^(j mod h)
        auto stage = [&](auto hc, const cx<float>& w) {
            constexpr int H = decltype(hc)::value;
            const float sg = (j & H) ? -1.f : 1.f;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const float px = lane_xor<H>(a[m].x), py = lane_xor<H>(a[m].y);
                cx<float> u = {px + sg * a[m].x, py + sg * a[m].y};
                if constexpr (H > 1) u = cmul(u, w);
                a[m] = u;
            }
        };
        stage(std::integral_constant<int, 8>{}, ws[0]);
        stage(std::integral_constant<int, 4>{}, ws[1]);
        stage(std::integral_constant<int, 2>{}, ws[2]);
        stage(std::integral_constant<int, 1>{}, ws[2]);
#pragma unroll
        for (int m = 1; m < 8; ++m) a[m] = cmul(a[m], wm[m]);
        dftR<float, 8, D>(a);
        int kx, z;
        long long cb;
        row_of(t, kx, z, cb);
        if constexpr (D < 0) {
            // X[ky], ky = k2 + 16 k1, to S2[c][ky][kx][z]
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1) Sout[cb + ((long long)(k2 + 16 * k1) * g.nh + kx) * g.nz + z] = a[k1];
        } else {
            cx<float>* dst = Sout + cb + ((long long)kx * g.nz + z) * 128;
#pragma unroll
            for (int k1 = 0; k1 < 8; ++k1) dst[k2 + 16 * k1] = a[k1];
        }
    }
}

// ---------------------------------------------------------------------------
// y-inverse: S2[c][ky][kx][z] -> inverse FFT along y -> S1[c][kx][z][y].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_yinv(const cx<T>* __restrict__ S2, cx<T>* __restrict__ S1, Geo g,
                                                   Plan py, const cx<T>* __restrict__ twy,
                                                   const int* __restrict__ done)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int ny = g.ny, tz = g.tz, ss = lrow(ny);
    cx<T>* A = reinterpret_cast<cx<T>*>(smem);
    cx<T>* B = A + tz * ss;
    cx<T>* tw = B + tz * ss;
    const int nzt = g.nz / tz;
    int b = blockIdx.x;
    const int zt = b % nzt;
    b /= nzt;
    const int kx = b % g.nh;
    const int c = b / g.nh;
    const int z0 = zt * tz;
    for (int i = threadIdx.x; i < ny; i += kThreads) tw[i] = twy[i];
    const cx<T>* src = S2 + (long long)c * g.nspec;
    for (int t = threadIdx.x; t < tz * ny; t += kThreads) {
        const int ky = g.ftz.div(t);
        const int r = t - ky * tz;
        A[r * ss + lpad(ky)] = src[((long long)ky * g.nh + kx) * g.nz + z0 + r];
    }
    __syncthreads();
    const cx<T>* R = lds_fft<T, +1>(A, B, py, tz, ss, tw);
    cx<T>* dst = S1 + (long long)c * g.nspec + ((long long)kx * g.nz + z0) * ny;
    for (int t = threadIdx.x; t < tz * ny; t += kThreads) {
        const int r = g.fny.div(t);
        const int y = t - r * ny;
        dst[t] = R[r * ss + lpad(y)];
    }
}

// Wave vector (radians per voxel) of half-spectrum index (kx, ky, kz): signed
// index in [-n/2, n/2); a Nyquist component takes -pi times the sign of the
// first non-Nyquist non-zero component in the order z, y, x (+1 if none), so
// that k(-m) = -k(m) and the inverse transform of Gamma sigma_hat stays real.
__device__ __forceinline__ void wave_vector(int kx, int ky, int kz, const Geo& g, double* k)
{
    const int m[3] = {kx, ky, kz};
    const int n[3] = {g.nx, g.ny, g.nz};
    bool nyq[3];
    int sv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nyq[a] = ((n[a] & 1) == 0) && (2 * m[a] == n[a]);
        sv[a] = (2 * m[a] <= n[a]) ? m[a] : m[a] - n[a];
    }
    // later axes override earlier ones: z decides first, then y, then x
    int sgn = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (!nyq[a] && sv[a] != 0) sgn = sv[a] > 0 ? 1 : -1;
    const double pi = 3.14159265358979323846;
#pragma unroll
    for (int a = 0; a < 3; ++a) k[a] = nyq[a] ? -pi * sgn : (double)sv[a] * g.kh[a];
}

// ---------------------------------------------------------------------------
// gamma: FFT along the last axis, t_hat = Gamma0(k):sigma_hat per frequency
// (isotropic reference medium: t = sym(n (x) s)/mu0 - c0 (n.s) n (x) n with
// s = sigma_hat n, c0 = (lam0 + mu0)/(mu0 (lam0 + 2 mu0))), the equilibrium
// error sum_m |k . sigma_hat|^2 = |k|^2 |s|^2 (half-spectrum weights), the
// k = 0 term, and the inverse FFT, in place.
// POL (polarization iteration, Algorithm 3): the pencils also carry eps_hat
// (components 6..11); the Green operator acts on s_b = alpha sigma_hat -
// beta C0:eps_hat, the k = 0 entry is -N beta E, and only the six components
// of the result go back (the error still measures sigma_hat).
// 3-D: rows along z of S2 (pencil = ky * nh + kx).  2-D: rows along y of S1
// (pencil = kx, kz = 0).  grid: ceil(npencils / np).
// ---------------------------------------------------------------------------
// Green operator at one frequency of a gamma tile: component c of the pencil
// sits in row c * nrs + r of R (element i).  Overwrites components 0..5 with
// t_hat (the k = 0 entry as described above) and returns the frequency's share
// of the equilibrium error.
template <typename T, bool POL>
__device__ __forceinline__ double gamma_point(cx<T>* R, int ss, int nrs, int r, int i, int kx, int ky, int kz,
                                              const Geo& g, double lam0, double mu0, double alpha, double beta,
                                              int dc_mode, const double* __restrict__ E, const double* dc_mean,
                                              DevState* __restrict__ st)
{
    cx<T> s[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) s[c] = R[(c * nrs + r) * ss + lpad(i)];
    // the field the Green operator acts on: sigma_hat, or s_b (POL)
    cx<T> sg[6];
    if constexpr (POL) {
        cx<T> e[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) e[c] = R[((6 + c) * nrs + r) * ss + lpad(i)];
        const cx<T> tr = cadd(cadd(e[0], e[1]), e[2]);
        const T al = (T)alpha, bl = (T)(beta * lam0), b2m = (T)(2.0 * beta * mu0);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            cx<T> v = csub(cscale(s[c], al), cscale(e[c], b2m));
            if (c < 3) v = csub(v, cscale(tr, bl));
            sg[c] = v;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) sg[c] = s[c];
    }
    double esum = 0.0;
    cx<T> o[6];
    if (kx == 0 && ky == 0 && kz == 0) {
        const double Nd = (double)g.N;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            st->sig_hat0[c] = (double)s[c].x;
            st->mean_eps[c] = dc_mean[c] / Nd;
            double v;
            if constexpr (POL) v = (dc_mode == DC_MEAN) ? -Nd * beta * E[c] : 0.0;
            else v = (dc_mode == DC_MEAN) ? (dc_mean[c] - Nd * E[c]) : 0.0;
            o[c] = cx<T>{(T)v, T(0)};
        }
    } else {
        const double c0 = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0));
        const double imu = 1.0 / mu0;
        double k[3];
        wave_vector(kx, ky, kz, g, k);
        const double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        T n0, n1, n2;
        if constexpr (sizeof(T) == 4) {
            // FP32 fields: the unit direction to FP32 accuracy is all the filter uses
            const float ik = rsqrtf((float)kk);
            n0 = (float)k[0] * ik;
            n1 = (float)k[1] * ik;
            n2 = (float)k[2] * ik;
        } else {
            const double ik = 1.0 / sqrt(kk);
            n0 = k[0] * ik;
            n1 = k[1] * ik;
            n2 = k[2] * ik;
        }
        // s = sigma_hat n with components xx,yy,zz,yz,xz,xy = 0..5
        cx<T> sx = cadd(cadd(cscale(s[0], n0), cscale(s[5], n1)), cscale(s[4], n2));
        cx<T> sy = cadd(cadd(cscale(s[5], n0), cscale(s[1], n1)), cscale(s[3], n2));
        cx<T> sz = cadd(cadd(cscale(s[4], n0), cscale(s[3], n1)), cscale(s[2], n2));
        const double w = (kx == 0 || 2 * kx == g.nx) ? 1.0 : 2.0;
        const T s2 = sx.x * sx.x + sx.y * sx.y + sy.x * sy.x + sy.y * sy.y + sz.x * sz.x + sz.y * sz.y;
        esum = w * kk * (double)s2;
        if constexpr (POL) {
            sx = cadd(cadd(cscale(sg[0], n0), cscale(sg[5], n1)), cscale(sg[4], n2));
            sy = cadd(cadd(cscale(sg[5], n0), cscale(sg[1], n1)), cscale(sg[3], n2));
            sz = cadd(cadd(cscale(sg[4], n0), cscale(sg[3], n1)), cscale(sg[2], n2));
        }
        const cx<T> a = cadd(cadd(cscale(sx, n0), cscale(sy, n1)), cscale(sz, n2));
        const T m1 = (T)imu, cc = (T)c0, hm = T(0.5) * (T)imu;
        o[0] = csub(cscale(sx, m1 * n0), cscale(a, cc * n0 * n0));
        o[1] = csub(cscale(sy, m1 * n1), cscale(a, cc * n1 * n1));
        o[2] = csub(cscale(sz, m1 * n2), cscale(a, cc * n2 * n2));
        o[3] = csub(cadd(cscale(sz, hm * n1), cscale(sy, hm * n2)), cscale(a, cc * n1 * n2));
        o[4] = csub(cadd(cscale(sz, hm * n0), cscale(sx, hm * n2)), cscale(a, cc * n0 * n2));
        o[5] = csub(cadd(cscale(sy, hm * n0), cscale(sx, hm * n1)), cscale(a, cc * n0 * n1));
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) R[(c * nrs + r) * ss + lpad(i)] = o[c];
    return esum;
}

// Frequency indices of element i of gamma pencil pen.
__device__ __forceinline__ void gamma_freq(const Geo& g, int pen, int i, int& kx, int& ky, int& kz)
{
    if (g.two_d) {
        kx = pen;
        ky = i;
        kz = 0;
    } else {
        ky = g.fnh.div(pen);
        kx = pen - ky * g.nh;
        kz = i;
    }
}

// <eps> from the x-pass partial sums (block 0 of a gamma launch holds k = 0).
__device__ __forceinline__ void gamma_dc_mean(int dc_mode, const double* __restrict__ part_mean, int n_mean,
                                              double* dc_mean, double* red)
{
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (dc_mode == DC_MEAN) {
        for (int b = threadIdx.x; b < n_mean; b += kThreads) {
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[c] += part_mean[(long long)b * 6 + c];
        }
    }
    wg_sum_store<6>(acc, dc_mean, red);
}

template <typename T, bool POL>
__global__ __launch_bounds__(kThreads) void k_gamma(cx<T>* __restrict__ S, Geo g, Plan pr,
                                                    const cx<T>* __restrict__ twr, double lam0, double mu0,
                                                    double alpha, double beta, int dc_mode,
                                                    const double* __restrict__ E,
                                                    const double* __restrict__ part_mean, int n_mean,
                                                    double* __restrict__ part_err, DevState* __restrict__ st,
                                                    const int* __restrict__ done)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NC = POL ? 12 : 6;
    const int nrow = g.two_d ? g.ny : g.nz;
    const int npen = g.two_d ? g.nh : g.ny * g.nh;
    const int ss = lrow(nrow);
    const int p0 = blockIdx.x * g.np;
    const int npl = min(g.np, npen - p0);
    const int nseq = 6 * npl;
    cx<T>* A = reinterpret_cast<cx<T>*>(smem);
    cx<T>* B = A + NC * g.np * ss;
    cx<T>* tw = B + NC * g.np * ss;
    double* red = reinterpret_cast<double*>(tw + nrow);

    for (int i = threadIdx.x; i < nrow; i += kThreads) tw[i] = twr[i];
    for (int c = 0; c < NC; ++c) {
        const cx<T>* src = S + (long long)c * g.nspec + (long long)p0 * nrow;
        for (int t = threadIdx.x; t < npl * nrow; t += kThreads) {
            const int pl = g.frow.div(t);
            const int i = t - pl * nrow;
            A[(c * npl + pl) * ss + lpad(i)] = src[t];
        }
    }
    __shared__ double dc_mean[6];
    if (blockIdx.x == 0) gamma_dc_mean(dc_mode, part_mean, n_mean, dc_mean, red);
    __syncthreads();
    cx<T>* R = lds_fft<T, -1>(A, B, pr, NC * npl, ss, tw);

    double esum = 0.0;
    for (int t = threadIdx.x; t < npl * nrow; t += kThreads) {
        const int pl = g.frow.div(t);
        const int i = t - pl * nrow;
        int kx, ky, kz;
        gamma_freq(g, p0 + pl, i, kx, ky, kz);
        esum += gamma_point<T, POL>(R, ss, npl, pl, i, kx, ky, kz, g, lam0, mu0, alpha, beta, dc_mode, E, dc_mean,
                                    st);
    }
    __syncthreads();
    const cx<T>* Q = lds_fft<T, +1>(R, R == A ? B : A, pr, nseq, ss, tw);
    for (int c = 0; c < 6; ++c) {
        cx<T>* dst = S + (long long)c * g.nspec + (long long)p0 * nrow;
        for (int t = threadIdx.x; t < npl * nrow; t += kThreads) {
            const int pl = g.frow.div(t);
            const int i = t - pl * nrow;
            dst[t] = Q[(c * npl + pl) * ss + lpad(i)];
        }
    }
    double ev[1] = {esum};
    if (part_err) wg_sum_store<1>(ev, part_err + blockIdx.x, red);
}

// Software-pipelined gamma pass for tiles of exactly kThreads elements per
// component (g.np pencils of nrow = kThreads / g.np): a persistent grid walks
// the tiles; each thread holds its element of every component of the next
// tile in registers, in flight while the current tile is transformed,
// filtered and stored.  Pencils past the last one are zero and never stored.
// part_err gets one sum per block.
template <typename T, bool POL, bool IP>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && IP && !POL ? RPM_GIP_WPE : 1))) void k_gpipe(cx<T>* __restrict__ S, Geo g, Plan pr,
                                                    const cx<T>* __restrict__ twr, double lam0, double mu0,
                                                    double alpha, double beta, int dc_mode,
                                                    const double* __restrict__ E,
                                                    const double* __restrict__ part_mean, int n_mean,
                                                    double* __restrict__ part_err, DevState* __restrict__ st,
                                                    int ntiles, const int* __restrict__ done)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NC = POL ? 12 : 6;
    const int np = g.np;
    const int nrow = g.two_d ? g.ny : g.nz;
    const long long nlast = (long long)(g.two_d ? g.nh : g.ny * g.nh) * nrow;  // elements per component
    const int ss = lrow(nrow);
    cx<T>* A0 = reinterpret_cast<cx<T>*>(smem);
    cx<T>* B0 = A0 + NC * np * ss;
    cx<T>* tw0 = IP ? B0 : B0 + NC * np * ss;  // IP: one buffer, transforms in place
    double* red = reinterpret_cast<double*>(tw0 + nrow);

    for (int i = threadIdx.x; i < nrow; i += kThreads) tw0[i] = twr[i];
    __shared__ double dc_mean[6];
    if (blockIdx.x == 0) gamma_dc_mean(dc_mode, part_mean, n_mean, dc_mean, red);
    // this thread's element of a tile: pencil pl, row element i
    const int pl = g.frow.div(threadIdx.x);
    const int i = threadIdx.x - pl * nrow;
    const int la = pl * ss + lpad(i);
    cx<T> pre[NC];
    auto load = [&](int t) {
        const long long o = (long long)t * kThreads + threadIdx.x;
        const bool in = o < nlast;
#pragma unroll
        for (int c = 0; c < NC; ++c) pre[c] = in ? S[c * g.nspec + o] : cx<T>{T(0), T(0)};
    };
    double esum = 0.0;
    int t = blockIdx.x;
    if (t < ntiles) load(t);
    for (; t < ntiles; t += gridDim.x) {
        // LDS addresses are recomputed per tile rather than kept in registers
        // across the loop (which would cost the occupancy the pipeline needs)
        int opq = 0;
        asm volatile("" : "+s"(opq));
        cx<T>* const A = A0 + opq;
        cx<T>* const B = B0 + opq;
        const cx<T>* const tw = tw0 + opq;
        __syncthreads();  // the previous tile's stores have read A/B
#pragma unroll
        for (int c = 0; c < NC; ++c) A[c * np * ss + la] = pre[c];
        __syncthreads();
        const int tn = t + gridDim.x;
        if (tn < ntiles) load(tn);  // next tile in flight during this one
        cx<T>* R;
        if constexpr (IP) {
            ct_stages_ip<T, -1, 128, 0, 1, kThreads>(A, NC * np, ss, tw, threadIdx.x + opq);
            R = A;
        } else {
            R = lds_fft<T, -1>(A, B, pr, NC * np, ss, tw, threadIdx.x + opq);
        }
        const long long o = (long long)t * kThreads + threadIdx.x;
        const bool in = o < nlast;
        if (in) {
            int kx, ky, kz;
            gamma_freq(g, t * np + pl, i, kx, ky, kz);
            esum += gamma_point<T, POL>(R, ss, np, pl, i, kx, ky, kz, g, lam0, mu0, alpha, beta, dc_mode, E,
                                        dc_mean, st);
        }
        __syncthreads();
        const cx<T>* Q;
        if constexpr (IP) {
            ct_stages_ip<T, +1, 128, 0, 1, kThreads>(A, 6 * np, ss, tw, threadIdx.x + opq);
            Q = A;
        } else {
            Q = lds_fft<T, +1>(R, R == A ? B : A, pr, 6 * np, ss, tw, threadIdx.x + opq);
        }
        if (in) {
#pragma unroll
            for (int c = 0; c < 6; ++c) S[c * g.nspec + o] = Q[c * np * ss + la];
        }
    }
    double ev[1] = {esum};
    if (part_err) wg_sum_store<1>(ev, part_err + blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// x-inverse: complex-to-real FFT along x, out = eps - t (OUT_XI) or t (OUT_T).
// POL (polarization iteration, Algorithm 3, OUT_XI only): t is Gamma0 s_b -
// beta E, eps_b = -t, and out = (C(x) + C0)^{-1} (sigma + (1 - beta) C0 eps +
// C0 eps_b) with sigma = C(x) eps, voxel by voxel once all six components of t
// are back.
// grid: nz * (ny / ty).
// ---------------------------------------------------------------------------
template <typename T, bool POL, int NT, bool IP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) void k_xinv(const cx<T>* __restrict__ S1, const T* __restrict__ eps,
                                                   T* __restrict__ out, int out_mode, const T* __restrict__ shift,
                                                   double* __restrict__ part_inc, Geo g, Plan px,
                                                   const cx<T>* __restrict__ twx, const uint8_t* __restrict__ phase,
                                                   const double* __restrict__ lame, double lam0, double mu0,
                                                   double beta, const int* __restrict__ done)
{
    if (done && *done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int MV = MaxV<T>::v * kThreads / NT;  // voxels per thread
    const int nx = g.nx, ty = g.ty, ss = lrow(nx), nh = g.nh;
    cx<T>* A = reinterpret_cast<cx<T>*>(smem);
    cx<T>* B = A + ty * ss;
    cx<T>* tw = IP ? B : B + ty * ss;  // IP: one buffer, transforms in place
    const int nyt = g.ny / ty;
    const int z = blockIdx.x / nyt;
    const int y0 = (blockIdx.x - z * nyt) * ty;
    const long long base = ((long long)z * g.ny + y0) * nx;
    const int nvox = ty * nx;
    const long long N = g.N;
    const T invN = T(1.0 / (double)N);

    for (int i = threadIdx.x; i < nx; i += NT) tw[i] = twx[i];
    double inc = 0.0;  // sum of w (out - eps)^2 over the tile (correction solves)
    T tb[POL ? MV : 1][6];  // POL: t of this thread's voxels, all components
    // Software pipeline over the three packed transforms: the spectra of the
    // next pair and the strains of the current pair are loaded while the
    // current pair is transformed.  KS bounds nh * ty / NT.
    constexpr int KS = (MV * NT / 2 + kMaxTy + NT - 1) / NT;
    const int nspt = nh * ty;
    cx<T> pa[KS], pb[KS];
    auto load_spec = [&](int q) {
        const cx<T>* ina = S1 + (long long)(2 * q) * g.nspec;
        const cx<T>* inb = S1 + (long long)(2 * q + 1) * g.nspec;
        int opq = 0;  // offsets recomputed per pair rather than held in registers
        asm volatile("" : "+s"(opq));
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const int t = threadIdx.x + opq + u * NT;
            if (t < nspt) {
                const int k = g.fty.div(t);
                const int r = t - k * ty;
                const long long o = ((long long)k * g.nz + z) * g.ny + y0 + r;
                pa[u] = ina[o];
                pb[u] = inb[o];
            }
        }
    };
    load_spec(0);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            const int t = threadIdx.x + u * NT;
            if (t < nspt) {
                const int k = g.fty.div(t);
                const int r = t - k * ty;
                cx<T> a = pa[u];
                cx<T> b = pb[u];
                const bool selfc = (k == 0) || (2 * k == nx);
                if (selfc) {
                    a.y = T(0);
                    b.y = T(0);
                }
                A[r * ss + lpad(k)] = cx<T>{a.x - b.y, a.y + b.x};
                if (!selfc) A[r * ss + lpad(nx - k)] = cx<T>{a.x + b.y, b.x - a.y};
            }
        }
        __syncthreads();
        if (q < 2) load_spec(q + 1);
        const int ca = 2 * q, cb = 2 * q + 1;
        T ea[POL ? 1 : MV], eb[POL ? 1 : MV];
        if constexpr (!POL) {
            if (out_mode == OUT_XI) {
#pragma unroll
                for (int i = 0; i < MV; ++i) {
                    const int v = threadIdx.x + i * NT;
                    if (v < nvox) {
                        ea[i] = eps[ca * N + base + v];
                        eb[i] = eps[cb * N + base + v];
                    }
                }
            }
        }
        const cx<T>* R;
        if constexpr (IP) {
            ct_stages_ip<T, +1, 128, 0, 1, NT>(A, ty, ss, tw, threadIdx.x);
            R = A;
        } else {
            R = lds_fft<T, +1, NT>(A, B, px, ty, ss, tw);
        }
#pragma unroll
        for (int i = 0; i < MV; ++i) {
            const int v = threadIdx.x + i * NT;
            if (v < nvox) {
                const int r = g.fnx.div(v);
                const int x = v - r * nx;
                const cx<T> val = R[r * ss + lpad(x)];
                const long long gi = base + v;
                const T ta = val.x * invN, tb_ = val.y * invN;
                if constexpr (POL) {
                    tb[i][2 * q] = ta;
                    tb[i][2 * q + 1] = tb_;
                } else if (out_mode == OUT_XI) {
                    T oa = ea[i] - ta, ob = eb[i] - tb_;
                    if (shift) {
                        oa += shift[ca * N + gi];
                        ob += shift[cb * N + gi];
                    }
                    out[ca * N + gi] = oa;
                    out[cb * N + gi] = ob;
                    if (part_inc) {
                        const double da = (double)oa - (double)ea[i], db = (double)ob - (double)eb[i];
                        inc += frob_w(ca) * da * da + frob_w(cb) * db * db;
                    }
                } else {
                    out[ca * N + gi] = ta;
                    out[cb * N + gi] = tb_;
                }
            }
        }
    }
    if constexpr (POL) {
        const T l0 = (T)lam0, m0 = (T)mu0, omb = (T)(1.0 - beta);
#pragma unroll
        for (int i = 0; i < MV; ++i) {
            const int v = threadIdx.x + i * NT;
            if (v < nvox) {
                const long long gi = base + v;
                T e[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) e[c] = eps[c * N + gi];
                const int ph = phase[gi];
                const T lam = (T)lame[2 * ph], mu = (T)lame[2 * ph + 1];
                const T tre = e[0] + e[1] + e[2];
                const T tru = tb[i][0] + tb[i][1] + tb[i][2];
                // X = sigma + (1 - beta) C0 eps - C0 t
                T X[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    X[c] = T(2) * (mu + omb * m0) * e[c] - T(2) * m0 * tb[i][c];
                    if (c < 3) X[c] += (lam + omb * l0) * tre - l0 * tru;
                }
                // (C + C0)^{-1} X for the isotropic sum (lam + lam0, mu + mu0)
                const T lp = lam + l0, mp = mu + m0;
                const T trX = X[0] + X[1] + X[2];
                const T kap = lp / (T(3) * lp + T(2) * mp);
                const T inv2m = T(1) / (T(2) * mp);
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    T o = (c < 3 ? X[c] - kap * trX : X[c]) * inv2m;
                    if (shift) o += shift[c * N + gi];
                    out[c * N + gi] = o;
                    if (part_inc) {
                        const double dd = (double)o - (double)e[c];
                        inc += frob_w(c) * dd * dd;
                    }
                }
            }
        }
    }
    if (part_inc) {
        __syncthreads();
        double* red = reinterpret_cast<double*>(tw + nx);
        double v[1] = {inc};
        wg_sum_store<1, NT>(v, part_inc + blockIdx.x, red);
    }
}

// ---------------------------------------------------------------------------
// Products with the tiled basis Z (Frobenius weights: 1 on the normal
// components e < 3N, 2 on the shear ones).
// ---------------------------------------------------------------------------
// Four consecutive elements as raw 16- or 32-byte loads, converted on use.
template <typename T>
struct Raw4;
template <>
struct Raw4<float> {
    float4 v;
    __device__ __forceinline__ void load(const float* __restrict__ p) { v = *reinterpret_cast<const float4*>(p); }
    // NT: non-temporal (a basis stream that would only evict the fields from the caches)
    template <bool NT>
    __device__ __forceinline__ void load_s(const float* __restrict__ p)
    {
        if constexpr (NT) v = nt_load(reinterpret_cast<const float4*>(p));
        else v = *reinterpret_cast<const float4*>(p);
    }
    __device__ __forceinline__ void load_tail(const float* __restrict__ p, long long e0, long long L6)
    {
        v.x = e0 < L6 ? p[0] : 0.f;
        v.y = e0 + 1 < L6 ? p[1] : 0.f;
        v.z = e0 + 2 < L6 ? p[2] : 0.f;
        v.w = e0 + 3 < L6 ? p[3] : 0.f;
    }
    __device__ __forceinline__ void get(double (&o)[4]) const
    {
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};
template <>
struct Raw4<double> {
    double2 a, b;
    __device__ __forceinline__ void load(const double* __restrict__ p)
    {
        a = *reinterpret_cast<const double2*>(p);
        b = *reinterpret_cast<const double2*>(p + 2);
    }
    template <bool NT>
    __device__ __forceinline__ void load_s(const double* __restrict__ p)
    {
        if constexpr (NT) {
            a = nt_load(reinterpret_cast<const double2*>(p));
            b = nt_load(reinterpret_cast<const double2*>(p + 2));
        } else {
            load(p);
        }
    }
    __device__ __forceinline__ void load_tail(const double* __restrict__ p, long long e0, long long L6)
    {
        a.x = e0 < L6 ? p[0] : 0.0;
        a.y = e0 + 1 < L6 ? p[1] : 0.0;
        b.x = e0 + 2 < L6 ? p[2] : 0.0;
        b.y = e0 + 3 < L6 ? p[3] : 0.0;
    }
    __device__ __forceinline__ void get(double (&o)[4]) const
    {
        o[0] = a.x;
        o[1] = a.y;
        o[2] = b.x;
        o[3] = b.y;
    }
};

// Up to four field pointers of a product kernel (unused slots null).
template <typename TA>
struct Fields {
    const TA* f[6];
};

// Column-group products (no update): wave g of a block of 64 * ceil(p / 8)
// threads owns columns 8g .. 8g+7 and streams their slices of every tile the
// block visits (tiles b, b + G, ...), so a wave keeps only 8 accumulators per
// field and issues its 8 column loads together; the waves of a block read the
// same field slice (one HBM read, the rest from cache).  Slices are addressed
// as a wave-uniform base plus the lane offset.  Partial sums are
// column-major: part[(f * ld + j) * G + b], G = gridDim.x.
template <bool FULL, typename TA, typename TZ, int NF, bool NT, int C = 8>
__device__ __forceinline__ void gdots_tile(const Fields<TA>& a, long long t0, const TZ* __restrict__ zt, int lo,
                                           int nj, long long e0, long long L6, long long N3,
                                           double (&acc)[NF][C])
{
    double w[4], fv[NF][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = (FULL || e0 + u < L6) ? (e0 + u < N3 ? 1.0 : 2.0) : 0.0;
    Raw4<TA> ra[NF];
    Raw4<TZ> raw[C];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (FULL) ra[f].load(a.f[f] + t0 + lo);
        else ra[f].load_tail(a.f[f] + t0 + lo, e0, L6);
    }
    // slots past the group's last column repeat it (valid memory); their sums
    // are never stored
#pragma unroll
    for (int u = 0; u < C; ++u) {
        const TZ* zc = zt + (long long)min(u, nj - 1) * kZTile;
        if (FULL) raw[u].template load_s<NT>(zc + lo);
        else raw[u].load_tail(zc + lo, e0, L6);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        ra[f].get(fv[f]);
#pragma unroll
        for (int q = 0; q < 4; ++q) fv[f][q] *= w[q];
    }
#pragma unroll
    for (int u = 0; u < C; ++u) {
        double z[4];
        raw[u].get(z);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f][u] += z[q] * fv[f][q];
    }
}

// SITE separates the call sites in profiles (0: the per-step projections, 1:
// basis growth); both read the basis with non-temporal loads.
template <typename TA, typename TZ, int NF, int SITE>
__global__ __launch_bounds__(512) void k_gdots(Fields<TA> a, const TZ* __restrict__ Z, int p, int zP, long long N,
                                               double* __restrict__ part, int ld)
{
    const int lane = threadIdx.x & 63;
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int j0 = 8 * g;
    const int nj = min(8, p - j0);  // >= 1: the block has ceil(p / 8) waves
    const int lo = 4 * lane;
    const long long L6 = 6 * N, N3 = 3 * N;
    const long long nfull = L6 / kZTile;
    double acc[NF][8];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[f][u] = 0.0;
    long long tile = blockIdx.x;
    for (; tile < nfull; tile += gridDim.x)
        gdots_tile<true, TA, TZ, NF, true>(a, tile * kZTile, Z + (tile * zP + j0) * (long long)kZTile, lo, nj,
                                     tile * kZTile + lo, L6, N3, acc);
    if (tile == nfull && nfull * kZTile < L6)  // the last, partial tile
        gdots_tile<false, TA, TZ, NF, true>(a, tile * kZTile, Z + (tile * zP + j0) * (long long)kZTile, lo, nj,
                                      tile * kZTile + lo, L6, N3, acc);
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double sum = wave_sum(acc[f][u]);
            if (lane == 0 && u < nj) part[(long long)(f * ld + j0 + u) * gridDim.x + blockIdx.x] = sum;
        }
}

// The per-step products with the columns split finer: a wave owns C columns
// (the block has ceil(p / C) <= 16 waves) and streams their slices of TB
// consecutive tiles per round (C * TB loads issued together), so the block's
// waves read each group of tiles' slices of all columns, one contiguous
// region, together (FP32: C = 2, TB = 8 for p <= 32 and C = 4, TB = 4 for
// p <= 64 stream 2-5 % faster than eight columns per wave; FP64, two 16-byte
// loads per column slice: TB = 1, 6-9 % faster).  Same partial-sum layout as
// k_gdots.
template <typename TA, typename TZ, int NF, int SITE, int C, int TB>
__global__ __launch_bounds__(1024) void k_gdots_split(Fields<TA> a, const TZ* __restrict__ Z, int p, int zP,
                                                      long long N, double* __restrict__ part, int ld)
{
    const int lane = threadIdx.x & 63;
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int j0 = C * g;
    const int nj = min(C, p - j0);  // >= 1: the block has ceil(p / C) waves
    const int lo = 4 * lane;
    const long long L6 = 6 * N, N3 = 3 * N;
    const long long nfull = L6 / kZTile;
    const long long ngrp = nfull / TB;
    double acc[NF][C];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int u = 0; u < C; ++u) acc[f][u] = 0.0;
    for (long long grp = blockIdx.x; grp < ngrp; grp += gridDim.x) {
        const long long t0 = grp * TB;
        Raw4<TA> ra[TB][NF];
        Raw4<TZ> raw[TB][C];
#pragma unroll
        for (int t = 0; t < TB; ++t)
#pragma unroll
            for (int f = 0; f < NF; ++f) ra[t][f].load(a.f[f] + (t0 + t) * kZTile + lo);
#pragma unroll
        for (int t = 0; t < TB; ++t)
#pragma unroll
            for (int u = 0; u < C; ++u)
                raw[t][u].template load_s<true>(Z + ((t0 + t) * zP + j0 + min(u, nj - 1)) * (long long)kZTile + lo);
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            const long long e0 = (t0 + t) * kZTile + lo;
            double fv[NF][4];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                ra[t][f].get(fv[f]);
#pragma unroll
                for (int q = 0; q < 4; ++q) fv[f][q] *= (e0 + q < N3 ? 1.0 : 2.0);
            }
#pragma unroll
            for (int u = 0; u < C; ++u) {
                double z[4];
                raw[t][u].get(z);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int f = 0; f < NF; ++f) acc[f][u] += z[q] * fv[f][q];
            }
        }
    }
    // tiles past the last whole group, then the last, partial tile
    for (long long tile = ngrp * TB + blockIdx.x; tile <= nfull; tile += gridDim.x) {
        if (tile < nfull)
            gdots_tile<true, TA, TZ, NF, true, C>(a, tile * kZTile, Z + (tile * zP + j0) * (long long)kZTile, lo, nj,
                                                  tile * kZTile + lo, L6, N3, acc);
        else if (nfull * kZTile < L6)
            gdots_tile<false, TA, TZ, NF, true, C>(a, tile * kZTile, Z + (tile * zP + j0) * (long long)kZTile, lo,
                                                   nj, tile * kZTile + lo, L6, N3, acc);
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int u = 0; u < C; ++u) {
            const double sum = wave_sum(acc[f][u]);
            if (lane == 0 && u < nj) part[(long long)(f * ld + j0 + u) * gridDim.x + blockIdx.x] = sum;
        }
}

// Update-and-project (Gram-Schmidt step) k_tdots: a wave owns whole tiles;
// lane l holds elements 4l .. 4l+3 of its tile and all p columns of it, so
// the update a_f <- a_f - sum_j coef[f * ld + j] Z_j (UPD, every field,
// written back) is complete in registers before the products
//   part[b * rs + f * ld + j] = sum_e w(e) Z_j[e] a_f[e]      (j < p, f < NF)
// and, NRM, the Gram entries of the fields after the update at
// part[b * rs + NF * ld + m]: <a_0, a_0> (NF = 1), or <a_0, a_0>, <a_1, a_1>,
// <a_0, a_1> (NF = 2).
// PC bounds p at compile time (one FP64 accumulator per column and field in
// registers).  Block b takes tiles b * kWaves + wave + k * gridDim.x * kWaves.
template <int NF>
constexpr int tdots_nrm() { return NF == 1 ? 1 : 3; }

// One tile of k_tdots for one lane: elements e0 .. e0+3 (FULL: all inside the
// vector, no guards).
template <bool FULL, typename TA, typename TZ, int NF, int PC, bool UPD, bool NRM>
__device__ __forceinline__ void tdots_tile(TA* __restrict__ a0, TA* __restrict__ a1, const TZ* __restrict__ zt,
                                           long long e0, long long L6, long long N3, int p,
                                           const double (*cf)[PC], double (&acc)[NF][PC],
                                           double (&nrm)[tdots_nrm<NF>()])
{
    constexpr int CG = 8;  // columns whose loads are issued together
    TA* const af[2] = {a0, a1};
    double w[4], fv[NF][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = (FULL || e0 + u < L6) ? (e0 + u < N3 ? 1.0 : 2.0) : 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (FULL) {
            Raw4<TA> r;
            r.load(af[f] + e0);
            r.get(fv[f]);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) fv[f][u] = e0 + u < L6 ? (double)af[f][e0 + u] : 0.0;
        }
    }
    // columns past p in a load group are clamped to column p - 1 (valid memory)
    // and carry weight zero; values stay in their storage type until used
    auto load_group = [&](int g, Raw4<TZ> (&raw)[CG]) {
#pragma unroll
        for (int u = 0; u < CG; ++u) {
            const TZ* zc = zt + (long long)min(g * CG + u, p - 1) * kZTile;
            if (FULL) raw[u].template load_s<false>(zc);
            else raw[u].load_tail(zc, e0, L6);
        }
    };
    if (UPD) {
#pragma unroll
        for (int g = 0; g < PC / CG; ++g) {
            if (g * CG < p) {
                Raw4<TZ> raw[CG];
                load_group(g, raw);
#pragma unroll
                for (int u = 0; u < CG; ++u) {
                    double z[4];
                    raw[u].get(z);
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        const double c = cf[f][g * CG + u];  // zero past p
#pragma unroll
                        for (int q = 0; q < 4; ++q) fv[f][q] -= c * z[q];
                    }
                }
            }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (FULL || e0 + q < L6) af[f][e0 + q] = (TA)fv[f][q];
    }
    if (NRM) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            nrm[0] += w[q] * fv[0][q] * fv[0][q];
            if constexpr (NF == 2) {
                nrm[1] += w[q] * fv[1][q] * fv[1][q];
                nrm[2] += w[q] * fv[0][q] * fv[1][q];
            }
        }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < 4; ++q) fv[f][q] *= w[q];
#pragma unroll
    for (int g = 0; g < PC / CG; ++g) {
        if (g * CG < p) {
            Raw4<TZ> raw[CG];
            load_group(g, raw);
#pragma unroll
            for (int u = 0; u < CG; ++u) {
                const double m = g * CG + u < p ? 1.0 : 0.0;
                double z[4];
                raw[u].get(z);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    double sf = 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) sf += z[q] * fv[f][q];
                    acc[f][g * CG + u] += m * sf;
                }
            }
        }
    }
}

template <typename TA, typename TZ, int NF, int PC, bool UPD, bool NRM>
__global__ __launch_bounds__(kThreads) void k_tdots(TA* __restrict__ a0, TA* __restrict__ a1,
                                                    const TZ* __restrict__ Z, int p, int zP,
                                                    const double* __restrict__ coef, long long N,
                                                    double* __restrict__ part, int ld, int rs)
{
    static_assert(NF == 1 || NF == 2, "one or two fields");
    constexpr int NM = tdots_nrm<NF>();
    constexpr int NA = NF * PC + (NRM ? NM : 0);
    static_assert(PC % 8 == 0, "column capacity is a multiple of the load group");
    __shared__ double red[kWaves][NA];
    __shared__ double cf[UPD ? NF : 1][PC];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (UPD) {
        for (int i = threadIdx.x; i < NF * PC; i += kThreads) {
            const int f = i / PC, j = i - f * PC;
            cf[f][j] = j < p ? coef[f * ld + j] : 0.0;
        }
        __syncthreads();
    }
    const long long L6 = 6 * N, N3 = 3 * N;
    const long long nfull = L6 / kZTile;
    double acc[NF][PC];
    double nrm[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) nrm[m] = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int j = 0; j < PC; ++j) acc[f][j] = 0.0;
    const long long stride = (long long)gridDim.x * kWaves;
    const long long first = (long long)blockIdx.x * kWaves + wave;
    long long tile = first;
    for (; tile < nfull; tile += stride)
        tdots_tile<true, TA, TZ, NF, PC, UPD, NRM>(a0, a1, Z + tile * (long long)zP * kZTile + 4 * lane,
                                                   tile * kZTile + 4 * lane, L6, N3, p, cf, acc, nrm);
    if (tile == nfull && nfull * kZTile < L6)  // the last, partial tile
        tdots_tile<false, TA, TZ, NF, PC, UPD, NRM>(a0, a1, Z + tile * (long long)zP * kZTile + 4 * lane,
                                                    tile * kZTile + 4 * lane, L6, N3, p, cf, acc, nrm);
    // fixed-order reductions: across the wave, then across the waves
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int j = 0; j < PC; ++j) {
            if (j < p) {
                const double s = wave_sum(acc[f][j]);
                if (lane == 0) red[wave][f * PC + j] = s;
            }
        }
    if (NRM) {
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const double s = wave_sum(nrm[m]);
            if (lane == 0) red[wave][NF * PC + m] = s;
        }
    }
    __syncthreads();
    double* out = part + (long long)blockIdx.x * rs;
    for (int i = threadIdx.x; i < NA; i += kThreads) {
        const int f = i / PC, j = i - f * PC;
        if (f < NF && j >= p) continue;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) s += red[q][i];
        out[f < NF ? f * ld + j : NF * ld + (i - NF * PC)] = s;
    }
}

// ---------------------------------------------------------------------------
// Reductions of per-block partial sums (fixed order: deterministic).
// ---------------------------------------------------------------------------
// out[j] = sum_b part[b * bs + j * cs], j < m.  grid: m.
__global__ __launch_bounds__(kThreads) void k_reduce_cols(const double* __restrict__ part, int G, long long bs,
                                                          long long cs, double* __restrict__ out)
{
    __shared__ double red[kWaves];
    __shared__ double tot[1];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < G; b += kThreads) acc += part[(long long)b * bs + j * cs];
    double v[1] = {acc};
    wg_sum_store<1>(v, tot, red);
    if (threadIdx.x == 0) out[j] = tot[0];
}

// ---------------------------------------------------------------------------
// Reductions at the end of a step, one block per output: out[0] = sum of the
// error partials (part_err, G_err entries); out[1 + q] for q < nf * p = sum of
// partial column map(q) of the basis products (column-major part_dots, G_dots
// per column: zeta_j at column j and, nf = 2, z_j at column ld + j).  Fixed
// order: deterministic.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_reduce_main(const double* __restrict__ part_err, int G_err,
                                                          const double* __restrict__ part_dots, int G_dots, int ld,
                                                          int p, double* __restrict__ out,
                                                          const int* __restrict__ done)
{
    if (done && *done) return;
    __shared__ double red[kWaves];
    __shared__ double tot[1];
    const int o = blockIdx.x;
    double acc = 0.0;
    if (o == 0) {
        if (part_err)
            for (int b = threadIdx.x; b < G_err; b += kThreads) acc += part_err[b];
    } else {
        const int q = o - 1;
        const double* src = part_dots + (long long)(q < p ? q : ld + (q - p)) * G_dots;
        for (int b = threadIdx.x; b < G_dots; b += kThreads) acc += src[b];
    }
    double v[1] = {acc};
    wg_sum_store<1>(v, tot, red);
    if (threadIdx.x == 0) out[o] = tot[0];
}

// ---------------------------------------------------------------------------
// End of a step (one block of kThreads) on the reduced sums: the equilibrium
// error of the iterate that went through F, the convergence / divergence /
// budget tests, and the Newton step on the unstable subspace
// z' = z + (I - H)^{-1}(zeta - z), applied as a product with the inverse kept
// by k_factor, giving the recombination coefficients d = z' - zeta for the
// next iterate eps_next = xi + Z d.
// direct: z = Z^T eps was reduced into sums (after a basis change or at the
// start of a solve); otherwise eps = xi_prev + Z d_prev was built from the
// stored pair, so z = zeta_prev + G d_prev with the Gram matrix G = Z^T Z
// (the same numbers without a second pass over the basis).
// newton_only: skip the error bookkeeping (used after basis growth).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_step_end(DevState* __restrict__ st, const double* __restrict__ sums,
                                                       int p, int slot, int two_d, int newton_only, int err_mode,
                                                       int direct, double* __restrict__ hist, int hist_cap)
{
    __shared__ int sdone, snow, ssing;
    __shared__ double dprev[kMaxP], r[kMaxP];
    __shared__ double Gs[kMaxP * kMaxP], Ai[kMaxP * kMaxP];
    const int t = threadIdx.x;
    // thread 0 reads every state scalar of the step at once (independent
    // loads, one memory round trip) before any decision
    int done0 = 0, sing0 = 0, it0 = 0, maxit = 0, win = 0, bit = 0;
    double err00 = 0.0, tol = 0.0, gnorm = 1.0, best = 0.0, num = 0.0, s[6] = {0, 0, 0, 0, 0, 0};
    if (t == 0) {
        done0 = st->done;
        sing0 = st->singular;
        it0 = st->iters;
        maxit = st->max_iter;
        win = st->stall_window;
        bit = st->best_it;
        err00 = st->err0;
        tol = st->tol;
        gnorm = st->gnorm;
        best = st->best_err;
#pragma unroll
        for (int c = 0; c < 6; ++c) s[c] = st->sig_hat0[c];
        num = sums[0];
        sdone = done0;
        ssing = sing0;
    }
    __syncthreads();
    if (sdone) return;  // uniform
    // stage the small matrices while thread 0 does the bookkeeping
    for (int e = t; e < p * p; e += kThreads) {
        const int i = e / p, j = e - (e / p) * p;
        if (!direct) Gs[i * kMaxP + j] = st->G[i * kMaxP + j];
        Ai[i * kMaxP + j] = st->AinvT[i * kMaxP + j];
    }
    for (int j = t; j < p; j += kThreads) dprev[j] = st->d[j];
    // this thread's basis coordinate (t < p): loads issued with the others
    double ze = 0.0, zz = 0.0;
    if (t < p) {
        ze = sums[1 + t];
        zz = direct ? sums[1 + p + t] : st->zeta[t];
    }
    if (t == 0) {
        int done = 0;
        if (!newton_only) {
            const double den = two_d ? (s[0] * s[0] + s[1] * s[1] + 2.0 * s[5] * s[5])
                                     : (s[0] * s[0] + s[1] * s[1] + s[2] * s[2] +
                                        2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
            const double nm = num > 0.0 ? num : 0.0;
            // err_mode 0: equilibrium error of the iterate; 1: fixed-point increment
            // |G(d) - d| / |g| of a correction solve
            const double err = err_mode == 0 ? sqrt(nm) / sqrt(den) : sqrt(nm) / gnorm;
            const int it = it0 + 1;
            st->iters = it;
            if (hist && it - 1 < hist_cap) hist[it - 1] = err;
            if (it == 1) {
                st->err0 = err;
                err00 = err;
            }
            st->err = err;
            int status = -1;
            if (!(err == err) || isinf(err) || err > 1e6 * err00) {
                status = 2;
            } else if (err <= tol) {
                status = 0;
            } else if (it >= maxit) {
                status = 1;
            } else if (win > 0) {
                // stalled: no error below 0.9 x the lowest one for stall_window iterations
                if (err < 0.9 * best) {
                    st->best_err = err;
                    st->best_it = it;
                } else if (it - bit >= win) {
                    status = 4;
                }
            }
            if (status >= 0) {
                st->status = status;
                st->done = 1;
                done = 1;
            }
        }
        snow = done;
    }
    __syncthreads();
    if (t < p) {
        const int i = t;
        if (!direct)
            for (int j = 0; j < p; ++j) zz += Gs[j * kMaxP + i] * dprev[j];
        st->zeta[i] = ze;
        st->z[i] = zz;
        st->zeta_ring[slot][i] = ze;
        r[i] = ze - zz;
    }
    __syncthreads();
    if (snow) return;  // uniform
    if (ssing) {
        if (t == 0) {
            st->status = 3;
            st->done = 1;
        }
        return;
    }
    if (t < p) {
        const int i = t;
        double y = 0.0;
        for (int j = 0; j < p; ++j) y += Ai[j * kMaxP + i] * r[j];
        st->d[i] = y - r[i];  // z' - zeta = (z + y) - zeta
    }
}

// Checksum of the phase map (part of the basis reuse key): per-block wrapping
// sums of (phase + 1) * splitmix64(voxel index); integer sums, so the order
// does not matter.
__global__ __launch_bounds__(kThreads) void k_phase_sum(const uint8_t* __restrict__ phase, long long N,
                                                        unsigned long long* __restrict__ part)
{
    __shared__ unsigned long long red[kThreads];
    unsigned long long s = 0;
    for (long long v = (long long)blockIdx.x * kThreads + threadIdx.x; v < N; v += (long long)gridDim.x * kThreads) {
        unsigned long long z = (unsigned long long)v + 0x9e3779b97f4a7c15ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        s += (unsigned long long)(phase[v] + 1) * z;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Clear the stop flags and the step counter (a fresh map evaluation).
__global__ void k_reset_state(DevState* __restrict__ st)
{
    if (threadIdx.x == 0) {
        st->done = 0;
        st->status = 1;
        st->iters = 0;
    }
}

// H gains row and column p: H[i][p] = col[i] (i <= p), H[p][j] = row[j] (j < p);
// the Gram matrix gains gram[j] = <Z_p, Z_j> (j <= p) in row and column p.
__global__ void k_border(DevState* __restrict__ st, const double* __restrict__ col, const double* __restrict__ row,
                         const double* __restrict__ gram, int p)
{
    if (threadIdx.x != 0) return;
    for (int i = 0; i <= p; ++i) st->H[i * kMaxP + p] = col[i];
    for (int j = 0; j < p; ++j) st->H[p * kMaxP + j] = row[j];
    for (int j = 0; j <= p; ++j) {
        st->G[p * kMaxP + j] = gram[j];
        st->G[j * kMaxP + p] = gram[j];
    }
}

// LU factorisation with partial pivoting of I - H, one wave of 64 threads on
// an LDS copy (row stride kMaxP + 1 keeps the row-parallel updates free of
// bank conflicts).  Thread t eliminates row c + 1 + t at step c.
__global__ __launch_bounds__(64) void k_factor(DevState* __restrict__ st, int p)
{
    constexpr int LD = kMaxP + 1;
    __shared__ double A[kMaxP * LD];
    __shared__ double amax_s;
    __shared__ int piv_s, sing_s;
    const int t = threadIdx.x;
    double amax = 0.0;
    for (int i = 0; i < p; ++i)
        for (int j = t; j < p; j += 64) {
            const double a = (i == j ? 1.0 : 0.0) - st->H[i * kMaxP + j];
            A[i * LD + j] = a;
            amax = fmax(amax, fabs(a));
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_down(amax, off, 64));
    if (t == 0) {
        amax_s = amax;
        sing_s = 0;
    }
    __syncthreads();
    for (int c = 0; c < p; ++c) {
        if (t == 0) {
            int q = c;
            for (int r = c + 1; r < p; ++r)
                if (fabs(A[r * LD + c]) > fabs(A[q * LD + c])) q = r;
            piv_s = q;
            st->piv[c] = q;
            if (!(fabs(A[q * LD + c]) > 1e-14 * amax_s)) sing_s = 1;
        }
        __syncthreads();
        if (sing_s) break;
        const int q = piv_s;
        if (q != c)
            for (int j = t; j < p; j += 64) {
                const double tmp = A[c * LD + j];
                A[c * LD + j] = A[q * LD + j];
                A[q * LD + j] = tmp;
            }
        __syncthreads();
        const int r = c + 1 + t;
        if (r < p) {
            const double f = A[r * LD + c] / A[c * LD + c];
            A[r * LD + c] = f;
            for (int j = c + 1; j < p; ++j) A[r * LD + j] -= f * A[c * LD + j];
        }
        __syncthreads();
    }
    for (int i = 0; i < p; ++i)
        for (int j = t; j < p; j += 64) st->LU[i * kMaxP + j] = A[i * LD + j];
    if (t == 0) {
        st->singular = sing_s;
        st->p = p;
    }
    if (sing_s) return;
    // explicit inverse, one column per thread: L U x = P e_t.  perm[i] is the
    // original row that the pivoting moved to position i.
    __shared__ int perm[kMaxP];
    __shared__ double X[kMaxP * kMaxP];
    if (t == 0) {
        for (int i = 0; i < p; ++i) perm[i] = i;
        for (int c = 0; c < p; ++c) {
            const int q = st->piv[c];
            const int tmp = perm[c];
            perm[c] = perm[q];
            perm[q] = tmp;
        }
    }
    __syncthreads();
    if (t < p) {
        for (int i = 0; i < p; ++i) {  // unit lower triangle
            double v = perm[i] == t ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= A[i * LD + k] * X[k * kMaxP + t];
            X[i * kMaxP + t] = v;
        }
        for (int i = p - 1; i >= 0; --i) {  // upper triangle
            double v = X[i * kMaxP + t];
            for (int k = i + 1; k < p; ++k) v -= A[i * LD + k] * X[k * kMaxP + t];
            X[i * kMaxP + t] = v / A[i * LD + i];
        }
        // column t of the inverse is row t of the transposed store
        for (int i = 0; i < p; ++i) st->AinvT[t * kMaxP + i] = X[i * kMaxP + t];
    }
}

// ---------------------------------------------------------------------------
// Voxel-parallel tall-skinny kernels (basis growth, re-projection).
// Each block covers kChunk voxels; partial sums are per block.
// ---------------------------------------------------------------------------
constexpr int kChunk = kThreads * 8;
constexpr int kVecBlock = 16384;  // elements of the 6N-vector per block (element-parallel sums)

// D1 = (xa - xb) - Z (za - zb);  D0 = (xb - xc) - Z (zb - zc) when xc != 0.
// part[b][0..2] = D1.D1, D1.D0, D0.D0 (Frobenius).  Each thread takes 4
// consecutive elements of the 6N-vector (one tile slice) and the columns in
// groups of 8 whose loads are issued together (slots past p repeat column
// p - 1 with coefficient zero).  grid: ceil(6N / (4 kThreads)).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_growth_diff(const T* __restrict__ xa, const T* __restrict__ xb,
                                                          const T* __restrict__ xc, const T* __restrict__ Z, int p,
                                                          int zP,
                                                          const double* __restrict__ za,
                                                          const double* __restrict__ zb,
                                                          const double* __restrict__ zc, double* __restrict__ D1,
                                                          double* __restrict__ D0, long long N,
                                                          double* __restrict__ part)
{
    __shared__ double red[kWaves * 3 + 3];
    __shared__ double c1[kMaxP + 8], c0[kMaxP + 8];
    for (int j = threadIdx.x; j < kMaxP + 8; j += kThreads) {
        c1[j] = j < p ? za[j] - zb[j] : 0.0;
        c0[j] = (j < p && xc) ? (zb[j] - zc[j]) : 0.0;
    }
    __syncthreads();
    double acc[3] = {0.0, 0.0, 0.0};
    const long long L6 = 6 * N, N3 = 3 * N;
    const long long e0 = ((long long)blockIdx.x * kThreads + threadIdx.x) * 4;
    if (e0 < L6) {
        const bool full = e0 + 4 <= L6;
        double d1[4], d0[4], t[4];
        Raw4<T> r;
        if (full) r.load(xa + e0);
        else r.load_tail(xa + e0, e0, L6);
        r.get(d1);
        if (full) r.load(xb + e0);
        else r.load_tail(xb + e0, e0, L6);
        r.get(t);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            d1[q] -= t[q];
            d0[q] = t[q];
        }
        if (xc) {
            if (full) r.load(xc + e0);
            else r.load_tail(xc + e0, e0, L6);
            r.get(t);
#pragma unroll
            for (int q = 0; q < 4; ++q) d0[q] -= t[q];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) d0[q] = 0.0;
        }
        const T* zt = Z + zix(e0, 0, zP);  // column j at zt + j * kZTile
        for (int g = 0; g < p; g += 8) {
            Raw4<T> raw[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const T* zc_ = zt + (long long)min(g + u, p - 1) * kZTile;
                if (full) raw[u].template load_s<true>(zc_);
                else raw[u].load_tail(zc_, e0, L6);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                double z[4];
                raw[u].get(z);
                const double a1 = c1[g + u], a0 = c0[g + u];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    d1[q] -= a1 * z[q];
                    d0[q] -= a0 * z[q];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!full && e0 + q >= L6) continue;
            D1[e0 + q] = d1[q];
            if (xc) D0[e0 + q] = d0[q];
            const double w = e0 + q < N3 ? 1.0 : 2.0;
            acc[0] += w * d1[q] * d1[q];
            acc[1] += w * d1[q] * d0[q];
            acc[2] += w * d0[q] * d0[q];
        }
    }
    wg_sum_store<3>(acc, part + (long long)blockIdx.x * 3, red);
}

// RPM recombination eps = xi + sum_j d_j Z_j as a streaming pass: each thread
// handles runs of VL consecutive elements; for a column, a wave reads one
// contiguous kilobyte of its tile.  Columns go in groups of 8 whose loads are
// issued together (non-temporal); slots past p repeat column p - 1 with
// coefficient zero.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_recombine(const T* __restrict__ xi, const T* __restrict__ Z, int p,
                                                        int zP, const double* __restrict__ dco,
                                                        T* __restrict__ eps, long long n,
                                                        const int* __restrict__ done)
{
    if (done && *done) return;
    constexpr int VL = 16 / sizeof(T);
    using V = typename Vec4<T>::type;
    __shared__ T dj[kMaxP + 8];
    for (int j = threadIdx.x; j < kMaxP + 8; j += kThreads) dj[j] = j < p ? (T)dco[j] : T(0);
    __syncthreads();
    const long long e = ((long long)blockIdx.x * kThreads + threadIdx.x) * VL;
    if (e >= n) return;
    if (e + VL <= n) {
        V acc = *reinterpret_cast<const V*>(xi + e);
        T* a = reinterpret_cast<T*>(&acc);
        const T* zt = Z + zix(e, 0, zP);  // column j at zt + j * kZTile
        for (int g = 0; g < p; g += 8) {
            V z[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                z[u] = nt_load(reinterpret_cast<const V*>(zt + (long long)min(g + u, p - 1) * kZTile));
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const T* zs = reinterpret_cast<const T*>(&z[u]);
                const T c = dj[g + u];
#pragma unroll
                for (int q = 0; q < VL; ++q) a[q] += c * zs[q];
            }
        }
        *reinterpret_cast<V*>(eps + e) = acc;
    } else {
        for (long long i = e; i < n; ++i) {
            T v = xi[i];
            for (int j = 0; j < p; ++j) v += dj[j] * Z[zix(i, j, zP)];
            eps[i] = v;
        }
    }
}

// The same recombination with the columns split over the waves of a block:
// block b takes the TB basis tiles TB b .. TB b + TB - 1 (kZTile elements,
// four per lane, FP32); wave w sums columns C w .. C w + C - 1 (then the same
// plus 16 C, ...) of them, issuing its C * TB loads together, and wave 0 adds
// the other waves' partial sums from LDS and xi.  The block's waves read the
// group's slices of all columns, one contiguous region, together: a wave
// streaming all columns of its own tile reaches ~10 % less of the HBM rate.
// The grid covers whole groups only (the host takes the remaining tiles).
#ifndef RPM_RS_CPW
#define RPM_RS_CPW 2
#endif
#ifndef RPM_RS_TPB
#define RPM_RS_TPB 4
#endif
constexpr int kRsWaves = 16;
template <typename T, int C = RPM_RS_CPW, int TB = RPM_RS_TPB>
__global__ __launch_bounds__(64 * kRsWaves) void k_recombine_split(const T* __restrict__ xi, const T* __restrict__ Z,
                                                                   int p, int zP, const double* __restrict__ dco,
                                                                   T* __restrict__ eps, const int* __restrict__ done)
{
    static_assert(sizeof(T) == 4 && kZTile == 64 * 4, "FP32 tiles of four elements per lane");
    if (done && *done) return;
    using V = typename Vec4<T>::type;
    constexpr int CS = kRsWaves * C;  // columns per round of the waves
    __shared__ T dj[kMaxP + CS];
    __shared__ V prt[kRsWaves - 1][TB][64];
    for (int j = threadIdx.x; j < kMaxP + CS; j += 64 * kRsWaves) dj[j] = j < p ? (T)dco[j] : T(0);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    V acc[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const long long e = ((long long)blockIdx.x * TB + t) * kZTile + lane * 4;
        acc[t] = w == 0 ? *reinterpret_cast<const V*>(xi + e) : V{T(0), T(0), T(0), T(0)};
    }
    const T* zt0 = Z + zix((long long)blockIdx.x * TB * kZTile, 0, zP) + lane * 4;
    for (int g = C * w; g < p; g += CS) {
        V z[TB][C];
#pragma unroll
        for (int t = 0; t < TB; ++t)
#pragma unroll
            for (int u = 0; u < C; ++u)
                z[t][u] = nt_load(reinterpret_cast<const V*>(zt0 + (long long)t * zP * kZTile +
                                                             (long long)min(g + u, p - 1) * kZTile));
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            T* a = reinterpret_cast<T*>(&acc[t]);
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const T* zs = reinterpret_cast<const T*>(&z[t][u]);
                const T c = dj[g + u];
#pragma unroll
                for (int q = 0; q < 4; ++q) a[q] += c * zs[q];
            }
        }
    }
    if (w > 0)
#pragma unroll
        for (int t = 0; t < TB; ++t) prt[w - 1][t][lane] = acc[t];
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            T* a = reinterpret_cast<T*>(&acc[t]);
#pragma unroll
            for (int k = 0; k < kRsWaves - 1; ++k) {
                const T* b = reinterpret_cast<const T*>(&prt[k][t][lane]);
#pragma unroll
                for (int q = 0; q < 4; ++q) a[q] += b[q];
            }
            const long long e = ((long long)blockIdx.x * TB + t) * kZTile + lane * 4;
            *reinterpret_cast<V*>(eps + e) = acc[t];
        }
    }
}

// Load cases of a batched solve (the unit mean strains of the effective
// tensor): per case the previous xi, the recombined eps, the Newton
// coefficients d and the stop flag.
constexpr int kMaxCases = 6;
template <typename T>
struct CasePtrs {
    const T* xi[kMaxCases];
    T* eps[kMaxCases];
    const double* d[kMaxCases];
    const int* done[kMaxCases];
};

// Batched recombination eps_f = xi_f + sum_j d_f[j] Z_j for the NB load cases,
// one pass over the basis for all of them (each column slice is loaded once
// and applied to every case still iterating); layout and load pattern as
// k_recombine.
template <typename T, int NB>
__global__ __launch_bounds__(kThreads) void k_recombine_multi(CasePtrs<T> cp, const T* __restrict__ Z, int p, int zP,
                                                              long long n)
{
    constexpr int VL = 16 / sizeof(T);
    using V = typename Vec4<T>::type;
    __shared__ T dj[NB][kMaxP + 8];
    __shared__ int act[NB];
    for (int f = 0; f < NB; ++f)
        for (int j = threadIdx.x; j < kMaxP + 8; j += kThreads) dj[f][j] = j < p ? (T)cp.d[f][j] : T(0);
    if (threadIdx.x < NB) act[threadIdx.x] = *cp.done[threadIdx.x] ? 0 : 1;
    __syncthreads();
    const long long e = ((long long)blockIdx.x * kThreads + threadIdx.x) * VL;
    if (e >= n) return;
    if (e + VL <= n) {
        V acc[NB];
#pragma unroll
        for (int f = 0; f < NB; ++f) {
            if (act[f]) acc[f] = *reinterpret_cast<const V*>(cp.xi[f] + e);
            else {
                T* a = reinterpret_cast<T*>(&acc[f]);
#pragma unroll
                for (int q = 0; q < VL; ++q) a[q] = T(0);
            }
        }
        const T* zt = Z + zix(e, 0, zP);
        for (int g = 0; g < p; g += 8) {
            V z[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                z[u] = nt_load(reinterpret_cast<const V*>(zt + (long long)min(g + u, p - 1) * kZTile));
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const T* zs = reinterpret_cast<const T*>(&z[u]);
#pragma unroll
                for (int f = 0; f < NB; ++f) {
                    T* a = reinterpret_cast<T*>(&acc[f]);
                    const T c = dj[f][g + u];
#pragma unroll
                    for (int q = 0; q < VL; ++q) a[q] += c * zs[q];
                }
            }
        }
#pragma unroll
        for (int f = 0; f < NB; ++f)
            if (act[f]) *reinterpret_cast<V*>(cp.eps[f] + e) = acc[f];
    } else {
        for (int f = 0; f < NB; ++f) {
            if (!act[f]) continue;
            for (long long i = e; i < n; ++i) {
                T v = cp.xi[f][i];
                for (int j = 0; j < p; ++j) v += dj[f][j] * Z[zix(i, j, zP)];
                cp.eps[f][i] = v;
            }
        }
    }
}

// The basis part of the solver state (p, H, its factorisation and inverse, the
// Gram matrix) copied from one load case's state to another's after the
// shared basis grew.
__global__ __launch_bounds__(kThreads) void k_copy_basis_state(DevState* __restrict__ dst,
                                                               const DevState* __restrict__ src)
{
    for (int e = threadIdx.x; e < kMaxP * kMaxP; e += kThreads) {
        dst->H[e] = src->H[e];
        dst->LU[e] = src->LU[e];
        dst->G[e] = src->G[e];
        dst->AinvT[e] = src->AinvT[e];
    }
    for (int e = threadIdx.x; e < kMaxP; e += kThreads) dst->piv[e] = src->piv[e];
    if (threadIdx.x == 0) {
        dst->p = src->p;
        dst->singular = src->singular;
    }
}

// Column j of the tiled basis from a contiguous 6N-vector (times scale), and
// optionally the stored values again as a contiguous vector (copy).
template <typename TI, typename T>
__global__ void k_col_put(const TI* __restrict__ in, double scale, T* __restrict__ Z, int j, int zP,
                          T* __restrict__ copy, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const T v = (T)((double)in[i] * scale);
        Z[zix(i, j, zP)] = v;
        if (copy) copy[i] = v;
    }
}

// The new basis columns of a growth step from the two re-orthogonalised
// candidates v0, v1 (FP64): z0 = s0 v0 and z1 = s1 (v1 - c01 z0), the second
// made orthogonal to the first with c01 = <z0, v1>.  Each kept column goes to
// Z (slots j0, j0 + 1; only z1 when the first is dropped, then at j0) and to
// a contiguous copy (out0, out1) for its Jacobian-vector product.
// keep: bit 0 first kept, bit 1 second kept.
template <typename T>
__global__ void k_col_put2(const double* __restrict__ v0, const double* __restrict__ v1, double s0, double c01,
                           double s1, int keep, T* __restrict__ Z, int j0, int zP, T* __restrict__ out0,
                           T* __restrict__ out1, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double z0 = 0.0;
    int j = j0;
    if (keep & 1) {
        z0 = v0[i] * s0;
        const T t = (T)z0;
        Z[zix(i, j, zP)] = t;
        out0[i] = t;
        ++j;
    }
    if (keep & 2) {
        const T t = (T)((v1[i] - c01 * z0) * s1);
        Z[zix(i, j, zP)] = t;
        out1[i] = t;
    }
}

// out = (in - a x) * scale in the output type (the second growth candidate:
// its difference made orthogonal to the first, normalised, to working precision).
template <typename TO>
__global__ void k_convert_sub(const double* __restrict__ in, const double* __restrict__ x, double a, double scale,
                              TO* __restrict__ out, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (TO)((in[i] - a * x[i]) * scale);
}

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, double scale, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (TO)((double)in[i] * scale);
}

// Refinement helpers: g = xi - eps in the working precision of the correction
// solve with part[b] = <xi - eps, xi - eps> (FP64); eps64 += d.
template <typename TG>
__global__ __launch_bounds__(kThreads) void k_residual_shift(const double* __restrict__ xi,
                                                             const double* __restrict__ eps, TG* __restrict__ g,
                                                             long long N, double* __restrict__ part)
{
    __shared__ double red[kWaves + 1];
    double acc[1] = {0.0};
    const long long L6 = 6 * N, N3 = 3 * N;
    const long long e0 = (long long)blockIdx.x * kVecBlock;
    for (int i = threadIdx.x; i < kVecBlock; i += kThreads) {
        const long long e = e0 + i;
        if (e >= L6) break;
        const double d = xi[e] - eps[e];
        g[e] = (TG)d;
        acc[0] += (e < N3 ? 1.0 : 2.0) * d * d;
    }
    wg_sum_store<1>(acc, part + blockIdx.x, red);
}

template <typename TD>
__global__ void k_add_correction(double* __restrict__ eps, const TD* __restrict__ d, double s, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) eps[i] += s * (double)d[i];
}

template <typename T>
__global__ void k_fill_uniform(T* __restrict__ f, const double* __restrict__ E, long long N)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 6 * N) f[i] = (T)E[i / N];
}

// sigma = C(x):eps voxel by voxel.
template <typename T>
__global__ void k_stress(const T* __restrict__ eps, const uint8_t* __restrict__ phase,
                         const double* __restrict__ lame, T* __restrict__ sig, long long N)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    const int ph = phase[x];
    const T lam = (T)lame[2 * ph], mu = (T)lame[2 * ph + 1];
    const T tr = eps[x] + eps[N + x] + eps[2 * N + x];
#pragma unroll
    for (int c = 0; c < 6; ++c) sig[c * N + x] = (mu + mu) * eps[c * N + x] + (c < 3 ? lam * tr : T(0));
}

}  // namespace rpm
