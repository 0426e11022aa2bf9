// Host orchestration and C ABI of the gfx950 RPM-FFT solver.
//
// The hot loop follows Algorithm 2 of the paper (Algorithm 1 when no basis is
// kept): every iteration is one application of F (five pencil passes, see
// rpm_kernels.h) plus one deterministic reduction and one single-workgroup
// finalize that evaluates the equilibrium error, tests convergence and takes
// the Newton step on the unstable subspace.  Everything stays on the device;
// the host reads a 'done' flag every check_every iterations and at the basis
// growth points (every n_max + 1 iterations), where it needs the QR decision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include "rpm_kernels.h"
#include "rpmfft.h"

using namespace rpm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kLdsCap = 60 * 1024;  // leaves room for static shared arrays
constexpr int kMaxN = 512;
constexpr double kFp32Stage = 1e-5;  // FP32 stage target before FP64 refinement
#ifndef RPM_YPIPE
#define RPM_YPIPE 1
#endif
#ifndef RPM_YPIPE_BLOCKS
#define RPM_YPIPE_BLOCKS 1024
#endif
constexpr bool kYPipe = RPM_YPIPE != 0;        // software-pipelined y passes
#ifndef RPM_Y_INPLACE
#define RPM_Y_INPLACE 1
#endif
#ifndef RPM_YIP_BLOCKS
#define RPM_YIP_BLOCKS 1280
#endif
constexpr bool kYInPlace = RPM_Y_INPLACE != 0;  // in-place y transforms (half the LDS)
// persistent grid of the pipelined y passes (four, or with in-place transforms five, resident blocks per CU)
constexpr int kYPipeBlocks = RPM_YPIPE_BLOCKS;
constexpr int kYipBlocks = RPM_YIP_BLOCKS;
#ifndef RPM_TDOTS_BLOCKS
#define RPM_TDOTS_BLOCKS 1024
#endif
constexpr int kTdotsBlocks = RPM_TDOTS_BLOCKS;  // grid cap of the basis products
#ifndef RPM_GPIPE
#define RPM_GPIPE 1
#endif
#ifndef RPM_GPIPE_BLOCKS
#define RPM_GPIPE_BLOCKS 1280
#endif
constexpr bool kGPipe = RPM_GPIPE != 0;        // software-pipelined gamma pass
#ifndef RPM_G_INPLACE
#define RPM_G_INPLACE 1
#endif
#ifndef RPM_GIP_BLOCKS
#define RPM_GIP_BLOCKS 1280
#endif
constexpr bool kGInPlace = RPM_G_INPLACE != 0;  // in-place gamma transforms
#ifndef RPM_X_INPLACE
#define RPM_X_INPLACE 1
#endif
constexpr bool kXInPlace = RPM_X_INPLACE != 0;  // in-place x transforms
#ifndef RPM_FUSE_RECOMBINE
#define RPM_FUSE_RECOMBINE 1
#endif
// RPM recombination inside the x-forward pass (in-place 128-point x
// transforms, not the polarization map; FP64 fields, or FP32 ones when the
// split-column pass below is switched off)
constexpr bool kFuseRecombine = RPM_FUSE_RECOMBINE != 0;
#ifndef RPM_SPLIT_RECOMBINE
#define RPM_SPLIT_RECOMBINE 1
#endif
// FP32 recombination as its own pass with the basis columns split over the
// waves of a block (k_recombine_split) instead of inside the x-forward pass
constexpr bool kSplitRecombine = RPM_SPLIT_RECOMBINE != 0;
#ifndef RPM_SPLIT_DOTS
#define RPM_SPLIT_DOTS 1
#endif
// per-step basis products with two or four columns per wave (k_gdots_split)
constexpr bool kSplitDots = RPM_SPLIT_DOTS != 0;
constexpr int kGipBlocks = RPM_GIP_BLOCKS;      // persistent grid with in-place transforms
constexpr int kGPipeBlocks = RPM_GPIPE_BLOCKS;  // its persistent grid
#ifndef RPM_X_NT
#define RPM_X_NT 256
#endif
// threads of an FP32 x-pass block (the tile size does not change with it)
template <typename T>
constexpr int x_threads() { return sizeof(T) == 4 ? RPM_X_NT : kThreads; }

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool smooth23(int n)
{
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

Plan make_plan(int n)
{
    Plan p{};
    p.n = n;
    p.nst = 0;
    int m = n, twos = 0, threes = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++twos;
    }
    while (m % 3 == 0) {
        m /= 3;
        ++threes;
    }
    while (twos >= 4) {
        p.rad[p.nst++] = 16;
        twos -= 4;
    }
    while (twos >= 3) {
        p.rad[p.nst++] = 8;
        twos -= 3;
    }
    if (twos == 2) p.rad[p.nst++] = 4;
    if (twos == 1) p.rad[p.nst++] = 2;
    for (int i = 0; i < threes; ++i) p.rad[p.nst++] = 3;
    return p;
}

int largest_divisor_leq(int n, int cap)
{
    for (int d = std::min(n, std::max(cap, 1)); d >= 1; --d)
        if (n % d == 0) return d;
    return 1;
}

// Tile shapes and LDS bytes of each pass for element type T.
template <typename T>
struct Shapes {
    Geo g;
    Plan px, py, pr;
    size_t lds_x, lds_y, lds_g;
    int G1, Gy, Gyf, G3, Gg, Gp, Gq;  // Gyf: forward y-pass tiles (all spectral components)
    int Gt;                           // gamma tiles
    bool gpipe;                       // pipelined gamma pass (tiles of kThreads elements per component)
    bool yip;                         // y passes transform in place (one LDS buffer)
    bool gip;                         // gamma pass transforms in place
    bool xip;                         // x passes transform in place
    int Yb;                           // workgroups of the persistent y passes
    bool ok;
    bool tune_ok;                     // the launch-shape overrides (rpm_tuning) apply to this grid
    bool yregs;                       // y transforms in registers (k_ywave)
};

template <typename T>
Shapes<T> make_shapes(const int32_t n[3], int ncomp, const rpm_tuning* tn = nullptr)
{
    Shapes<T> s{};
    s.tune_ok = true;
    const int wsz = (int)sizeof(cx<T>);
    const int MV = MaxV<T>::v;
    Geo& g = s.g;
    g.nx = n[0];
    g.ny = n[1];
    g.nz = n[2];
    g.nh = g.nx / 2 + 1;
    g.N = (long long)g.nx * g.ny * g.nz;
    g.nspec = (long long)g.nh * g.ny * g.nz;
    g.two_d = g.nz == 1 ? 1 : 0;
    g.ncomp = ncomp;
    s.ok = true;
    // x passes: ty rows of nx, at most MV voxels per thread, 128-byte segments
    int tycap = std::min(128 / wsz, MV * kThreads / g.nx);
    if (tycap < 1) s.ok = false;
    g.ty = largest_divisor_leq(g.ny, std::max(tycap, 1));
    while (g.ty > 1 && (size_t)(2 * g.ty * lrow(g.nx) + g.nx) * wsz + 80 * 8 > (size_t)kLdsCap)
        g.ty = largest_divisor_leq(g.ny, g.ty - 1);
    s.lds_x = (size_t)(2 * g.ty * lrow(g.nx) + g.nx) * wsz + 80 * 8;
    // 128-point x transforms of at most one butterfly per thread run in place
    s.xip = kXInPlace && g.nx == 128 && g.ty * 128 / 8 <= kThreads;
    if (s.xip) s.lds_x = (size_t)(g.ty * lrow(g.nx) + g.nx) * wsz + 80 * 8;
    // y passes: tz columns of ny (128-byte segments; FP64 128-point rows,
    // transformed in place in one LDS buffer, take 16: 92 / 66 us against
    // 98 / 71 us for the forward / inverse pass at 128^3)
    g.tz = largest_divisor_leq(g.nz, 128 / wsz);
    while (g.tz > 1 && (size_t)(2 * g.tz * lrow(g.ny) + g.ny) * wsz > (size_t)kLdsCap)
        g.tz = largest_divisor_leq(g.nz, g.tz - 1);
    if (wsz == 16 && kYInPlace && g.ny == 128) {
        const int t = largest_divisor_leq(g.nz, 16);
        if ((size_t)(t * lrow(g.ny) + g.ny) * wsz <= (size_t)kLdsCap) g.tz = t;
    }
    if (tn && tn->y_cols > 0) {
        const int t = tn->y_cols;
        if (g.nz % t != 0 || t > 128 / wsz || t * g.ny > 8 * kThreads ||
            (size_t)(2 * t * lrow(g.ny) + g.ny) * wsz > (size_t)kLdsCap)
            s.tune_ok = false;
        else
            g.tz = t;
    }
    // 128-point y transforms of at most one butterfly per thread run in place
    s.yip = kYInPlace && g.ny == 128 && g.tz * 128 / 8 <= kThreads;
    s.lds_y = (size_t)((s.yip ? 1 : 2) * g.tz * lrow(g.ny) + g.ny) * wsz;
    // gamma pass: np pencils x ncomp components along the last axis
    const int nrow = g.two_d ? g.ny : g.nz;
    const int npen = g.two_d ? g.nh : g.ny * g.nh;
    // pipelined gamma pass: np pencils of exactly kThreads elements per component
    int np = (kGPipe && kThreads % nrow == 0) ? kThreads / nrow : 2;
    if ((size_t)(2 * ncomp * np * lrow(nrow) + nrow) * wsz + 80 * 8 > (size_t)kLdsCap) np = 2;
    while (np > 1 && (size_t)(2 * ncomp * np * lrow(nrow) + nrow) * wsz + 80 * 8 > (size_t)kLdsCap) --np;
    g.np = np;
    s.lds_g = (size_t)(2 * ncomp * np * lrow(nrow) + nrow) * wsz + 80 * 8;
    if (s.lds_x > (size_t)kLdsCap || s.lds_y > (size_t)kLdsCap || s.lds_g > (size_t)kLdsCap) s.ok = false;
    if (g.ty * g.nx > MV * kThreads) s.ok = false;
    if ((long long)g.nh * g.ty > (long long)((MV * kThreads / 2 + kMaxTy + kThreads - 1) / kThreads) * kThreads ||
        g.ty > kMaxTy)
        s.ok = false;  // spectrum slots of the x-inverse prefetch
    g.fnx = make_fdiv(g.nx);
    for (int a = 0; a < 3; ++a) g.kh[a] = 2.0 * 3.14159265358979323846 / (double)n[a];
    g.fny = make_fdiv(g.ny);
    g.fnh = make_fdiv(g.nh);
    g.fty = make_fdiv(g.ty);
    g.ftz = make_fdiv(g.tz);
    g.frow = make_fdiv(nrow);
    s.px = make_plan(g.nx);
    s.py = make_plan(g.ny);
    s.pr = make_plan(nrow);
    s.G1 = g.nz * (g.ny / g.ty);
    s.Gy = 6 * g.nh * (g.nz / g.tz);
    s.Gyf = ncomp * g.nh * (g.nz / g.tz);
    s.Gt = (npen + g.np - 1) / g.np;
    s.gpipe = kGPipe && g.np * nrow == kThreads;
    // 128-point gamma transforms of at most one butterfly per thread run in place
    s.gip = s.gpipe && kGInPlace && nrow == 128 && ncomp * g.np * 128 / 8 <= kThreads;
    if (s.gip) s.lds_g = (size_t)(ncomp * np * lrow(nrow) + nrow) * wsz + 80 * 8;
    s.G3 = s.gpipe ? std::min(s.Gt, s.gip ? kGipBlocks : kGPipeBlocks) : s.Gt;  // gamma blocks (one error partial each)
    s.Yb = s.yip ? kYipBlocks : kYPipeBlocks;
    if (tn && tn->y_blocks > 0) s.Yb = tn->y_blocks;
    s.yregs = tn && tn->y_regs > 0;
    if (s.yregs && !(sizeof(T) == 4 && !g.two_d && g.ny == 128 && g.tz == 16 && tn->y_blocks == 0))
        s.tune_ok = false;
    if (tn && tn->gamma_blocks > 0 && s.gpipe) s.G3 = std::min(s.Gt, tn->gamma_blocks);
    s.Gg = (int)((g.N + kChunk - 1) / kChunk);
    s.Gp = (int)((6 * g.N + kVecBlock - 1) / kVecBlock);
    const long long ntile = (6 * g.N + kZTile - 1) / kZTile;
    s.Gq = (int)std::min<long long>(ntile, kTdotsBlocks);
    return s;
}

// Per-load-case state of a batched solve (case 0 uses the base offsets).
struct CaseOff {
    size_t st, pmean, perr, pinc, pdots, sums, gsum, ring[4], eps, hist;
};

struct Layout {
    size_t st, twx, twy, twr, lame, hist, pmean, perr, pinc, pdots, pg, sums, gsum, gx, ring[4], eps, tmp, tmp2, S1, S2,
        Z, W, D1, D0, shift, sub64, total;
    int ld;
    long long hist_cap;
    int nb = 0;          // load cases of a batched solve (0: not batched)
    size_t bpd = 0;      // basis products of the batched projection (nb x kMaxP columns of Gq partials)
    CaseOff cs[kMaxCases];
};

rpm_options basic_fp64_options(const rpm_options* o)
{
    rpm_options b = *o;
    b.scheme = RPM_SCHEME_BASIC;
    b.p_max = 0;
    b.max_iter = 1;
    b.precision = RPM_FP64;
    return b;
}


// Spectral components carried by the forward passes: sigma, and eps too for
// the polarization iteration.
int spectral_comps(const rpm_options* o) { return o->map == RPM_MAP_POLARIZATION ? 12 : 6; }

template <typename T>
Layout make_layout(const Shapes<T>& s, const rpm_options* o, bool map_only = false);

// Workspace layout.  map_only: what one map application needs (state, tables,
// partial sums, spectra), no fields, basis or FP64 sub-pipeline.
template <typename T>
Layout make_layout(const Shapes<T>& s, const rpm_options* o, bool map_only)
{
    Layout L{};
    const Geo& g = s.g;
    const size_t fT = map_only ? 0 : (size_t)6 * g.N * sizeof(T);
    const size_t fD = (size_t)6 * g.N * sizeof(double);
    const size_t spec = (size_t)g.ncomp * g.nspec * sizeof(cx<T>);
    const int pmax = (o->scheme == RPM_SCHEME_RPM && !map_only) ? o->p_max : 0;
    L.ld = kMaxP;
    L.hist_cap = map_only ? 2 : (long long)o->max_iter + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.st = take(sizeof(DevState));
    L.twx = take(sizeof(cx<T>) * kMaxN);
    L.twy = take(sizeof(cx<T>) * kMaxN);
    L.twr = take(sizeof(cx<T>) * kMaxN);
    L.lame = take(sizeof(double) * 512);
    L.pmean = take(sizeof(double) * 6 * s.G1);
    L.perr = take(sizeof(double) * std::max(s.G3, s.Gt));  // any gamma grid (tuned or not) fits
    L.pinc = take(sizeof(double) * s.G1);
    L.pdots = take(sizeof(double) * 2 * L.ld * std::max(std::max(s.G1, s.Gp), s.Gq));
    const long long Gd = (6 * g.N + 4 * kThreads - 1) / (4 * kThreads);  // k_growth_diff blocks (3 partials each)
    L.pg = take(sizeof(double) * std::max((size_t)(4 * kMaxP + 4) * std::max(std::max(s.Gg, s.Gp), s.Gq),
                                          (size_t)(3 * Gd)));
    L.sums = take(sizeof(double) * (2 * kMaxP + 8));
    L.gsum = take(sizeof(double) * (kMaxP + 8));
    L.gx = take(sizeof(double) * (10 * kMaxP + 16));
    for (int i = 0; i < 4; ++i) L.ring[i] = take(fT);
    L.eps = take(fT);
    L.tmp = take(pmax > 0 ? fT : 0);
    L.tmp2 = take(pmax > 0 ? fT : 0);
    L.S1 = take(spec);
    L.S2 = take(g.two_d ? 0 : spec);
    // tiled basis: ceil(6N / kZTile) tiles of kZTile x p_max elements
    const size_t zT = (size_t)((6 * g.N + kZTile - 1) / kZTile) * kZTile * sizeof(T);
    L.Z = take(zT * pmax);
    L.W = take(zT * pmax);
    L.D1 = take(pmax > 0 ? fD : 0);
    L.D0 = take(pmax > 0 ? fD : 0);
    // FP32 fields: shift field of the correction solves and an FP64 pipeline
    // for certification and refinement
    const bool fp32 = sizeof(T) == 4 && !map_only;
    L.shift = take(fp32 ? fT : 0);
    L.sub64 = off;
    if (fp32) {
        const int32_t n[3] = {g.nx, g.ny, g.nz};
        const rpm_options b = basic_fp64_options(o);
        off = align_up(off + make_layout<double>(make_shapes<double>(n, spectral_comps(&b)), &b).total);
    }
    // batched load cases: their own state, partial sums and fields behind
    // everything a single solve uses (the basis stays where a single solve
    // keeps it, so the two share a carried basis)
    if (o->batch_cases && pmax > 0 && !map_only) {
        L.nb = g.two_d ? 3 : 6;
        L.bpd = take(sizeof(double) * (size_t)L.nb * kMaxP * s.Gq);
        for (int f = 1; f < L.nb; ++f) {
            CaseOff& c = L.cs[f];
            c.st = take(sizeof(DevState));
            c.pmean = take(sizeof(double) * 6 * s.G1);
            c.perr = take(sizeof(double) * std::max(s.G3, s.Gt));
            c.pinc = take(sizeof(double) * s.G1);
            c.pdots = take(sizeof(double) * 2 * L.ld * std::max(std::max(s.G1, s.Gp), s.Gq));
            c.sums = take(sizeof(double) * (2 * kMaxP + 8));
            c.gsum = take(sizeof(double) * (kMaxP + 8));
            for (int i = 0; i < 4; ++i) c.ring[i] = take(fT);
            c.eps = take(fT);
        }
    }
    // last: its size follows max_iter, which may differ between calls that
    // carry the basis, so nothing the workspace keeps may sit behind it
    L.hist = take(sizeof(double) * L.hist_cap);
    for (int f = 1; f < L.nb; ++f) L.cs[f].hist = take(sizeof(double) * L.hist_cap);
    CaseOff& c0 = L.cs[0];
    c0.st = L.st;
    c0.pmean = L.pmean;
    c0.perr = L.perr;
    c0.pinc = L.pinc;
    c0.pdots = L.pdots;
    c0.sums = L.sums;
    c0.gsum = L.gsum;
    for (int i = 0; i < 4; ++i) c0.ring[i] = L.ring[i];
    c0.eps = L.eps;
    c0.hist = L.hist;
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// per-call context
// ---------------------------------------------------------------------------
struct Prof {
    bool on = false;
    uint32_t mask = ~0u;  // kernel classes recorded
    int every = 1;        // one launch in every this many of a class
    int seen[RPM_NKERNEL] = {0};
    std::vector<hipEvent_t> pool;
    struct Rec {
        hipEvent_t a, b;
        int k;
        double bytes;
    };
    std::vector<Rec> recs;
    double ms[RPM_NKERNEL] = {0};
    int n[RPM_NKERNEL] = {0};
    double bytes[RPM_NKERNEL] = {0};
    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void harvest()
    {
        for (auto& r : recs) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                ms[r.k] += t;
                n[r.k] += 1;
                bytes[r.k] += r.bytes;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
    void reset()
    {
        harvest();
        for (int k = 0; k < RPM_NKERNEL; ++k) {
            ms[k] = 0.0;
            n[k] = 0;
            bytes[k] = 0.0;
            seen[k] = 0;
        }
    }
    ~Prof()
    {
        for (auto& r : recs) {
            hipEventDestroy(r.a);
            hipEventDestroy(r.b);
        }
        for (auto e : pool) hipEventDestroy(e);
    }
};

template <typename T>
struct Ctx {
    Shapes<T> sh;
    Layout L;
    hipStream_t s;
    char* ws;
    DevState* st;
    const uint8_t* phase;
    double lam0, mu0;
    int pmax;
    bool pol = false;             // polarization iteration in place of F
    double alpha = 2.0, beta = 2.0;
    Prof prof;
    bool hip_error = false;
    // FP32 fields: the FP64 pipeline in the same workspace, which evaluates
    // the Jacobian-vector products of H and the compatible projection of new
    // basis columns (null for FP64 fields)
    Ctx<double>* sub = nullptr;

    template <typename P>
    P* at(size_t off) { return reinterpret_cast<P*>(ws + off); }
    cx<T>* twx() { return at<cx<T>>(L.twx); }
    cx<T>* twy() { return at<cx<T>>(L.twy); }
    cx<T>* twr() { return at<cx<T>>(L.twr); }
    double* lame() { return at<double>(L.lame); }
    T* ring(int i) { return at<T>(L.ring[i & 3]); }
    T* eps() { return at<T>(L.eps); }
    T* Zb() { return at<T>(L.Z); }  // tiled basis Z (column slots: pmax)
    T* Wb() { return at<T>(L.W); }  // tiled W = F_u Z
    double* sums() { return at<double>(L.sums); }
    double* gsum() { return at<double>(L.gsum); }
    double* gx() { return at<double>(L.gx); }
    double* pdots() { return at<double>(L.pdots); }
    double* pg() { return at<double>(L.pg); }

    void mark_begin(int k, hipEvent_t& a)
    {
        a = nullptr;
        if (!prof.on || !((prof.mask >> k) & 1u)) return;
        if (prof.seen[k]++ % prof.every != prof.every - 1) return;  // the every-th, 2 every-th, ... launch
        a = prof.get();
        if (a) hipEventRecord(a, s);
    }
    void mark_end(int k, hipEvent_t a, double bytes = 0.0)
    {
        if (!prof.on || !a) return;
        hipEvent_t b = prof.get();
        if (!b) return;
        hipEventRecord(b, s);
        prof.recs.push_back({a, b, k, bytes});
    }
    void check_launch()
    {
        if (hipGetLastError() != hipSuccess) hip_error = true;
    }
};

// y passes with register-resident transforms (rpm_tuning.y_regs; FP32 only):
// a persistent grid of RPM_YWAVE_BLOCKS workgroups
#ifndef RPM_YWAVE_BLOCKS
#define RPM_YWAVE_BLOCKS 1024
#endif
constexpr int kYWaveBlocks = RPM_YWAVE_BLOCKS;
template <typename T, int D>
void launch_ywave(hipStream_t s, int tiles, const cx<T>* Sin, cx<T>* Sout, const Geo& g, const cx<T>* tw,
                  const int* done)
{
    if constexpr (sizeof(T) == 4)
        k_ywave<D><<<std::min(tiles, kYWaveBlocks), kThreads, 0, s>>>(Sin, Sout, g, tw, 4 * tiles, done);
}

// One application of the fixed-point map on field xin (optionally corrected
// by Z d), leaving partial sums for the error and the projections.
template <typename T>
void run_F(Ctx<T>& c, const T* xin, int p_corr, T* eps_store, const T* eps_for_inv, T* out, int out_mode,
           int use_ref, int dc_mode, const double* Edev, const int* done, const T* shift = nullptr,
           double* part_inc = nullptr)
{
    const Shapes<T>& sh = c.sh;
    const Geo& g = sh.g;
    cx<T>* S1 = c.template at<cx<T>>(c.L.S1);
    cx<T>* S2 = c.template at<cx<T>>(c.L.S2);
    double* pmean = c.template at<double>(c.L.pmean);
    double* perr = c.template at<double>(c.L.perr);
    // algorithmic bytes of each pass: inputs read once, outputs written once
    const double fieldB = 6.0 * (double)g.N * sizeof(T);
    const double specB = 6.0 * (double)g.nspec * sizeof(cx<T>);
    const double bi = specB + fieldB * (2 + (shift ? 1 : 0));
    hipEvent_t ev;
    const bool pol = c.pol && out_mode == OUT_XI;
    const bool vec = g.nx % (16 / (int)sizeof(T)) == 0;
    constexpr int XT = x_threads<T>();
    const double cf = (double)g.ncomp / 6.0;  // spectral components carried forward, over 6
    const double bx = fieldB + (use_ref ? 0.0 : (double)g.N) + cf * specB;
    // FP32 with whole basis tiles: the split-column streaming pass plus the
    // plain x pass beat the fused pass (its one resident round of blocks
    // cannot overlap their transforms with the stream)
    const bool split = sizeof(T) == 4 && kSplitRecombine && (6 * g.N) % kZTile == 0;
    const bool fuse = eps_store && kFuseRecombine && sh.xip && vec && !pol && !split;
    if (fuse) {
        // eps = xin + Z d recombined inside the x pass (stored for the x-inverse)
        c.mark_begin(RPM_K_XFWD, ev);
        k_xfwd<T, true, false, XT, true, true><<<sh.G1, XT, sh.lds_x, c.s>>>(
            xin, c.phase, c.lame(), use_ref, c.lam0, c.mu0, S1, pmean, g, sh.px, c.twx(), done, c.Zb(), p_corr,
            c.pmax, c.st->d, eps_store);
        c.mark_end(RPM_K_XFWD, ev, bx + fieldB * (1 + p_corr));
    }
    if (eps_store && !fuse) {
        // eps = xin + Z d (a copy while p = 0) as its own streaming pass; the x
        // pass then reads eps
        const long long nel = 6 * g.N;
        const int VL = 16 / (int)sizeof(T);
        const int gb = (int)((nel / VL + kThreads - 1) / kThreads) + 1;
        c.mark_begin(RPM_K_RECOMBINE, ev);
        if constexpr (sizeof(T) == 4) {
            if (split && p_corr > 0) {
                // whole groups of RPM_RS_TPB tiles, then the remaining tiles
                // (addressed from their first tile) one run per thread
                const long long ngrp = nel / kZTile / RPM_RS_TPB;
                const long long off = ngrp * RPM_RS_TPB * kZTile;
                if (ngrp > 0)
                    k_recombine_split<T><<<(int)ngrp, 64 * kRsWaves, 0, c.s>>>(xin, c.Zb(), p_corr, c.pmax, c.st->d,
                                                                               eps_store, done);
                if (off < nel)
                    k_recombine<T><<<(int)((nel - off) / VL + kThreads - 1) / kThreads + 1, kThreads, 0, c.s>>>(
                        xin + off, c.Zb() + off * c.pmax, p_corr, c.pmax, c.st->d, eps_store + off, nel - off, done);
            } else {
                k_recombine<T><<<gb, kThreads, 0, c.s>>>(xin, c.Zb(), p_corr, c.pmax, c.st->d, eps_store, nel, done);
            }
        } else {
            k_recombine<T><<<gb, kThreads, 0, c.s>>>(xin, c.Zb(), p_corr, c.pmax, c.st->d, eps_store, nel, done);
        }
        c.mark_end(RPM_K_RECOMBINE, ev, fieldB * (2 + p_corr));
        xin = eps_store;
    }
    if (!fuse) c.mark_begin(RPM_K_XFWD, ev);
#define RPM_XFWD(V, P, I)                                                                                      \
    k_xfwd<T, V, P, XT, I><<<sh.G1, XT, sh.lds_x, c.s>>>(xin, c.phase, c.lame(), use_ref, c.lam0, c.mu0, S1, pmean, \
                                                         g, sh.px, c.twx(), done)
    if (fuse) {
    } else if (sh.xip) {
        if (pol) {
            if (vec) RPM_XFWD(true, true, true);
            else RPM_XFWD(false, true, true);
        } else {
            if (vec) RPM_XFWD(true, false, true);
            else RPM_XFWD(false, false, true);
        }
    } else {
        if (pol) {
            if (vec) RPM_XFWD(true, true, false);
            else RPM_XFWD(false, true, false);
        } else {
            if (vec) RPM_XFWD(true, false, false);
            else RPM_XFWD(false, false, false);
        }
    }
#undef RPM_XFWD
    if (!fuse) c.mark_end(RPM_K_XFWD, ev, bx);
    if (!g.two_d) {
        const int tiles = pol ? sh.Gyf : sh.Gy;
        c.mark_begin(RPM_K_YFWD, ev);
        if (sh.yregs)
            launch_ywave<T, -1>(c.s, tiles, S1, S2, g, c.twy(), done);
        else if (kYPipe && sh.yip)
            k_ypipe<T, -1, 8, true><<<std::min(tiles, sh.Yb), kThreads, sh.lds_y, c.s>>>(S1, S2, g, sh.py,
                                                                                             c.twy(), tiles, done);
        else if (kYPipe && g.tz * g.ny <= 8 * kThreads)
            k_ypipe<T, -1, 8, false><<<std::min(tiles, sh.Yb), kThreads, sh.lds_y, c.s>>>(S1, S2, g, sh.py,
                                                                                                c.twy(), tiles, done);
        else
            k_yfwd<T><<<tiles, kThreads, sh.lds_y, c.s>>>(S1, S2, g, sh.py, c.twy(), done);
        c.mark_end(RPM_K_YFWD, ev, 2.0 * (pol ? cf : 1.0) * specB);
    }
    c.mark_begin(RPM_K_GAMMA, ev);
    cx<T>* Sg = g.two_d ? S1 : S2;
#define RPM_GAMMA_ARGS                                                                                    \
    Sg, g, sh.pr, c.twr(), c.lam0, c.mu0, c.alpha, c.beta, dc_mode, Edev, pmean, sh.G1, perr, c.st
    if (sh.gip) {
        if (pol) k_gpipe<T, true, true><<<sh.G3, kThreads, sh.lds_g, c.s>>>(RPM_GAMMA_ARGS, sh.Gt, done);
        else k_gpipe<T, false, true><<<sh.G3, kThreads, sh.lds_g, c.s>>>(RPM_GAMMA_ARGS, sh.Gt, done);
    } else if (sh.gpipe) {
        if (pol) k_gpipe<T, true, false><<<sh.G3, kThreads, sh.lds_g, c.s>>>(RPM_GAMMA_ARGS, sh.Gt, done);
        else k_gpipe<T, false, false><<<sh.G3, kThreads, sh.lds_g, c.s>>>(RPM_GAMMA_ARGS, sh.Gt, done);
    } else {
        if (pol) k_gamma<T, true><<<sh.G3, kThreads, sh.lds_g, c.s>>>(RPM_GAMMA_ARGS, done);
        else k_gamma<T, false><<<sh.G3, kThreads, sh.lds_g, c.s>>>(RPM_GAMMA_ARGS, done);
    }
#undef RPM_GAMMA_ARGS
    c.mark_end(RPM_K_GAMMA, ev, ((pol ? cf : 1.0) + 1.0) * specB);
    if (!g.two_d) {
        c.mark_begin(RPM_K_YINV, ev);
        if (sh.yregs)
            launch_ywave<T, 1>(c.s, sh.Gy, S2, S1, g, c.twy(), done);
        else if (kYPipe && sh.yip)
            k_ypipe<T, 1, 8, true><<<std::min(sh.Gy, sh.Yb), kThreads, sh.lds_y, c.s>>>(S2, S1, g, sh.py,
                                                                                            c.twy(), sh.Gy, done);
        else if (kYPipe && g.tz * g.ny <= 8 * kThreads)
            k_ypipe<T, 1, 8, false><<<std::min(sh.Gy, sh.Yb), kThreads, sh.lds_y, c.s>>>(S2, S1, g, sh.py,
                                                                                               c.twy(), sh.Gy, done);
        else
            k_yinv<T><<<sh.Gy, kThreads, sh.lds_y, c.s>>>(S2, S1, g, sh.py, c.twy(), done);
        c.mark_end(RPM_K_YINV, ev, 2.0 * specB);
    }
    c.mark_begin(RPM_K_XINV, ev);
#define RPM_XINV(P, I)                                                                                         \
    k_xinv<T, P, XT, I><<<sh.G1, XT, sh.lds_x, c.s>>>(S1, eps_for_inv, out, out_mode, shift, part_inc, g, sh.px,     \
                                                      c.twx(), c.phase, c.lame(), c.lam0, c.mu0, c.beta, done)
    if (sh.xip) {
        if (pol) RPM_XINV(true, true);
        else RPM_XINV(false, true);
    } else {
        if (pol) RPM_XINV(true, false);
        else RPM_XINV(false, false);
    }
#undef RPM_XINV
    c.mark_end(RPM_K_XINV, ev, bi + (pol ? (double)g.N : 0.0));
    c.check_launch();
}

// Products <Z_j, a_f> (j < p) with the tiled basis: column-major partials
// part[(f * ld + j) * G + b], one wave per group of 8 columns.
template <typename TA, typename TZ, int NF, int SITE>
void launch_gdots(hipStream_t s, int G, Fields<TA> a, const TZ* Z, int p, int zP, long long N, double* part, int ld)
{
    const int ng = (p + 7) / 8;
    k_gdots<TA, TZ, NF, SITE><<<G, 64 * ng, 0, s>>>(a, Z, p, zP, N, part, ld);
}

// v_f <- v_f - sum_j coef[f * kMaxP + j] Z_j (f < NF), then the products
// <Z_j, v_f> (and, NRM, the Gram entries of the v_f): row-major partials
// part[b * rs + f * kMaxP + j], Gram entries from part[b * rs + NF * kMaxP].
template <typename TZ, int NF, bool NRM>
void launch_update(hipStream_t s, int G, double* v0, double* v1, const TZ* Z, int p, int zP, const double* coef,
                   long long N, double* part, int rs)
{
    if (p <= 8)
        k_tdots<double, TZ, NF, 8, true, NRM><<<G, kThreads, 0, s>>>(v0, v1, Z, p, zP, coef, N, part, kMaxP, rs);
    else if (p <= 16)
        k_tdots<double, TZ, NF, 16, true, NRM><<<G, kThreads, 0, s>>>(v0, v1, Z, p, zP, coef, N, part, kMaxP, rs);
    else if (p <= 32)
        k_tdots<double, TZ, NF, 32, true, NRM><<<G, kThreads, 0, s>>>(v0, v1, Z, p, zP, coef, N, part, kMaxP, rs);
    else if constexpr (NF == 1)
        k_tdots<double, TZ, 1, 64, true, NRM><<<G, kThreads, 0, s>>>(v0, v1, Z, p, zP, coef, N, part, kMaxP, rs);
}

// zeta_j = <Z_j, xi> (and, direct, z_j = <Z_j, eps>) partial sums for the Newton step.
template <typename T>
void project(Ctx<T>& c, const T* xi, const T* eps, int p, bool direct)
{
    if (p == 0) return;
    hipEvent_t ev;
    c.mark_begin(RPM_K_PROJECT, ev);
    if (direct)
        launch_gdots<T, T, 2, 0>(c.s, c.sh.Gq, Fields<T>{{xi, eps}}, c.Zb(), p, c.pmax, c.sh.g.N, c.pdots(),
                                 c.L.ld);
    else if constexpr (sizeof(T) == 4) {
        if (kSplitDots && p <= 32)
            k_gdots_split<T, T, 1, 0, 2, 8><<<c.sh.Gq, 64 * ((p + 1) / 2), 0, c.s>>>(Fields<T>{{xi}}, c.Zb(), p, c.pmax,
                                                                                    c.sh.g.N, c.pdots(), c.L.ld);
        else if (kSplitDots && p <= 64)
            k_gdots_split<T, T, 1, 0, 4, 4><<<c.sh.Gq, 64 * ((p + 3) / 4), 0, c.s>>>(Fields<T>{{xi}}, c.Zb(), p, c.pmax,
                                                                                    c.sh.g.N, c.pdots(), c.L.ld);
        else
            launch_gdots<T, T, 1, 0>(c.s, c.sh.Gq, Fields<T>{{xi}}, c.Zb(), p, c.pmax, c.sh.g.N, c.pdots(), c.L.ld);
    } else {
        // FP64 fields: fewer loads in flight per lane (two or four columns of
        // one tile per wave) stream faster than eight columns (759 -> 693 us
        // at p = 32, 1391 -> 1308 us at p = 64 on 128^3)
        if (kSplitDots && p <= 32)
            k_gdots_split<T, T, 1, 0, 2, 1><<<c.sh.Gq, 64 * ((p + 1) / 2), 0, c.s>>>(Fields<T>{{xi}}, c.Zb(), p, c.pmax,
                                                                                    c.sh.g.N, c.pdots(), c.L.ld);
        else if (kSplitDots && p <= 64)
            k_gdots_split<T, T, 1, 0, 4, 1><<<c.sh.Gq, 64 * ((p + 3) / 4), 0, c.s>>>(Fields<T>{{xi}}, c.Zb(), p, c.pmax,
                                                                                    c.sh.g.N, c.pdots(), c.L.ld);
        else
            launch_gdots<T, T, 1, 0>(c.s, c.sh.Gq, Fields<T>{{xi}}, c.Zb(), p, c.pmax, c.sh.g.N, c.pdots(), c.L.ld);
    }
    c.mark_end(RPM_K_PROJECT, ev, 6.0 * (double)c.sh.g.N * sizeof(T) * ((direct ? 2 : 1) + p));
}

// Reductions and the step bookkeeping after one F application (plus projections).
template <typename T>
void reduce_and_finalize(Ctx<T>& c, int p, int slot, int newton_only, bool direct, const int* done,
                         int err_mode = 0)
{
    hipEvent_t ev;
    c.mark_begin(RPM_K_REDUCE, ev);
    const double* perr = newton_only ? nullptr
                                     : (err_mode == 0 ? c.template at<double>(c.L.perr)
                                                      : c.template at<double>(c.L.pinc));
    const int nf = direct ? 2 : 1;
    k_reduce_main<<<1 + nf * p, kThreads, 0, c.s>>>(perr, err_mode == 0 ? c.sh.G3 : c.sh.G1, c.pdots(), c.sh.Gq,
                                                    c.L.ld, p, c.sums(), done);
    c.mark_end(RPM_K_REDUCE, ev);
    c.mark_begin(RPM_K_FINAL, ev);
    k_step_end<<<1, kThreads, 0, c.s>>>(c.st, c.sums(), p, slot & 3, c.sh.g.two_d, newton_only, err_mode,
                                        direct ? 1 : 0, c.template at<double>(c.L.hist), (int)c.L.hist_cap);
    c.mark_end(RPM_K_FINAL, ev);
    c.check_launch();
}

template <typename T>
bool sync_read(Ctx<T>& c, void* host, const void* dev, size_t bytes)
{
    if (hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c.s) != hipSuccess) return false;
    if (hipStreamSynchronize(c.s) != hipSuccess) return false;
    if (c.prof.on) c.prof.harvest();
    return !c.hip_error;
}

template <typename T>
void reduce_cols(Ctx<T>& c, const double* part, int G, long long bs, long long cs, int m, double* out)
{
    k_reduce_cols<<<m, kThreads, 0, c.s>>>(part, G, bs, cs, out);
}

// Initialise or re-validate the workspace header; uploads the tables.
template <typename T>
rpm_status prepare(Ctx<T>& c, const rpm_problem* pr, const rpm_options* o, bool want_reuse, int* p_io,
                   double tol, double gnorm = 1.0, int stall = 0)
{
    const Geo& g = c.sh.g;
    DevState hs;
    if (hipMemcpyAsync(&hs, c.st, sizeof(DevState), hipMemcpyDeviceToHost, c.s) != hipSuccess) return RPM_E_HIP;
    if (hipStreamSynchronize(c.s) != hipSuccess) return RPM_E_HIP;
    const int cfg[6] = {g.nx, g.ny, g.nz, o->precision, c.pmax, o->map};
    // the basis holds the linear part of the map: it depends on the reference
    // medium, the polarization parameters and the phase table (FNV-1a over
    // the table's bytes, kept as two 32-bit halves)
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < 2 * pr->n_phases; ++i) {
        uint64_t b;
        std::memcpy(&b, &pr->lame[i], sizeof(b));
        for (int k = 0; k < 8; ++k) {
            h ^= (b >> (8 * k)) & 0xffu;
            h *= 1099511628211ull;
        }
    }
    const bool pol = o->map == RPM_MAP_POLARIZATION;
    // and on the phase map: a device checksum (wrapping integer sums)
    constexpr int kSumBlocks = 64;
    unsigned long long* psum = reinterpret_cast<unsigned long long*>(c.pg());
    k_phase_sum<<<kSumBlocks, kThreads, 0, c.s>>>(c.phase, g.N, psum);
    unsigned long long parts[kSumBlocks];
    if (hipMemcpyAsync(parts, psum, sizeof(parts), hipMemcpyDeviceToHost, c.s) != hipSuccess) return RPM_E_HIP;
    if (hipStreamSynchronize(c.s) != hipSuccess) return RPM_E_HIP;
    unsigned long long pk = 0;
    for (int b = 0; b < kSumBlocks; ++b) pk += parts[b];
    const double medium[8] = {c.lam0, c.mu0, pol ? o->alpha : 0.0, pol ? o->beta : 0.0,
                              (double)(uint32_t)(h >> 32), (double)(uint32_t)h, (double)(uint32_t)(pk >> 32),
                              (double)(uint32_t)pk};
    bool same = hs.magic == kStateMagic && std::memcmp(hs.cfg, cfg, sizeof(cfg)) == 0 &&
                std::memcmp(hs.medium, medium, sizeof(medium)) == 0;
    if (!(same && want_reuse)) {
        std::memset(&hs, 0, sizeof(hs));
        hs.magic = kStateMagic;
        std::memcpy(hs.cfg, cfg, sizeof(cfg));
        std::memcpy(hs.medium, medium, sizeof(medium));
        hs.p = 0;
    }
    hs.done = 0;
    hs.status = 1;
    hs.iters = 0;
    hs.max_iter = o->max_iter;
    hs.tol = tol;
    hs.gnorm = gnorm;
    hs.err0 = 0.0;
    hs.err = 0.0;
    hs.best_err = 1e300;
    hs.best_it = 0;
    hs.stall_window = stall;
    for (int i = 0; i < 6; ++i) hs.Ezero[i] = 0.0;
    *p_io = hs.p;
    // twiddles exp(-2 pi i e / n) computed in long double on the host; the
    // host buffers stay alive until the stream synchronisation below
    std::vector<cx<T>> tabs[3];
    auto tw = [&](int slot, int n, size_t off) -> bool {
        std::vector<cx<T>>& t = tabs[slot];
        t.resize(n);
        for (int e = 0; e < n; ++e) {
            const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)e / (long double)n;
            t[e] = cx<T>{(T)std::cos(ang), (T)std::sin(ang)};
        }
        return hipMemcpyAsync(c.ws + off, t.data(), sizeof(cx<T>) * n, hipMemcpyHostToDevice, c.s) == hipSuccess;
    };
    if (!tw(0, g.nx, c.L.twx) || !tw(1, g.ny, c.L.twy) || !tw(2, g.two_d ? g.ny : g.nz, c.L.twr)) return RPM_E_HIP;
    std::vector<double> lt(512, 0.0);
    for (int i = 0; i < pr->n_phases; ++i) {
        lt[2 * i] = pr->lame[2 * i];
        lt[2 * i + 1] = pr->lame[2 * i + 1];
    }
    if (hipMemcpyAsync(c.lame(), lt.data(), sizeof(double) * 512, hipMemcpyHostToDevice, c.s) != hipSuccess)
        return RPM_E_HIP;
    if (hipMemcpyAsync(c.st, &hs, sizeof(DevState), hipMemcpyHostToDevice, c.s) != hipSuccess) return RPM_E_HIP;
    if (hipStreamSynchronize(c.s) != hipSuccess) return RPM_E_HIP;
    return RPM_OK;
}

template <typename T>
void set_E(Ctx<T>& c, const double E[6])
{
    hipMemcpyAsync(c.st->E, E, sizeof(double) * 6, hipMemcpyHostToDevice, c.s);
    hipStreamSynchronize(c.s);
}

// Compatible projection of a T field in place: v <- Gamma0 * (C0 : v), k != 0.
template <typename T>
void project_compatible(Ctx<T>& c, T* v, T* out)
{
    run_F<T>(c, v, 0, nullptr, v, out, OUT_T, 1, DC_ZERO, c.st->Ezero, nullptr);
}

// Adds NV (1 or 2) candidate columns v (FP64, overwritten) to the basis:
// two classical Gram-Schmidt passes against Z for both at once (coefficients;
// the update fused with the second coefficients; the second update fused with
// the Gram entries of the results), then the second made orthogonal to the
// first and both normalised as they are stored; a candidate whose norm after
// the projections is not above 1e-10 is dropped.  One Jacobian-vector
// product per kept column, then the new columns of H and of the Gram matrix
// in one pass over Z and the new rows of H in one pass over W.  NV = 2 needs
// p <= 32 and two free slots.  Returns the number of columns added, -1 on a
// HIP error.
template <typename T, int NV>
int add_columns(Ctx<T>& c, int& p, double* const* v, int* jvps)
{
    const long long N = c.sh.g.N;
    const long long nel = 6 * N;
    const int gb = (int)((nel + 255) / 256);
    const int Gq = c.sh.Gq;
    const int rs = 2 * kMaxP + 3;
    constexpr int NM = NV == 1 ? 1 : 3;
    T* tmp = c.template at<T>(c.L.tmp);
    T* tmp2 = c.template at<T>(c.L.tmp2);
    // the candidates' FP64 storage is free once the columns are stored: it
    // takes the Jacobian-vector products
    T* wout[2] = {reinterpret_cast<T*>(c.template at<double>(c.L.D1)),
                  reinterpret_cast<T*>(c.template at<double>(c.L.D0))};
    double* X = c.gx();
    double* C1 = X;                      // NV x kMaxP
    double* C2 = X + 2 * kMaxP;          // NV x kMaxP
    double* nr = X + 4 * kMaxP;          // Gram entries of the projected candidates
    double* HZ = X + 4 * kMaxP + 4;      // per new column: H column, Gram column (kMaxP + 2 each)
    double* RW = HZ + 4 * (kMaxP + 2);   // per new column: H row
    double* v1 = NV == 2 ? v[1] : nullptr;
    Fields<double> fv{{v[0], v1}};
    if (p > 0) {
        launch_gdots<double, T, NV, 1>(c.s, Gq, fv, c.Zb(), p, c.pmax, N, c.pg(), kMaxP);
        for (int f = 0; f < NV; ++f) reduce_cols(c, c.pg() + (long long)f * kMaxP * Gq, Gq, 1, Gq, p, C1 + f * kMaxP);
        launch_update<T, NV, false>(c.s, Gq, v[0], v1, c.Zb(), p, c.pmax, C1, N, c.pg(), rs);
        for (int f = 0; f < NV; ++f) reduce_cols(c, c.pg() + f * kMaxP, Gq, rs, 1, p, C2 + f * kMaxP);
    }
    launch_update<T, NV, true>(c.s, Gq, v[0], v1, c.Zb(), p, c.pmax, C2, N, c.pg(), rs);
    reduce_cols(c, c.pg() + NV * kMaxP, Gq, rs, 1, NM, nr);
    double g[3] = {0.0, 0.0, 0.0};
    if (!sync_read(c, g, nr, sizeof(double) * NM)) return -1;
    const double vn0 = std::sqrt(std::max(g[0], 0.0));
    const bool keep0 = vn0 > 1e-10;
    double c01 = 0.0, vn1 = 0.0;
    bool keep1 = false;
    if (NV == 2) {
        // |v1 - <z0, v1> z0|^2 = |v1|^2 - <z0, v1>^2 with z0 = v0 / |v0|
        c01 = keep0 ? g[2] / vn0 : 0.0;
        vn1 = std::sqrt(std::max(g[1] - c01 * c01, 0.0));
        keep1 = vn1 > 1e-10;
    }
    const int nacc = (keep0 ? 1 : 0) + (keep1 ? 1 : 0);
    if (nacc == 0) return 0;
    T* zc[2] = {tmp, tmp2};
    k_col_put2<T><<<gb, 256, 0, c.s>>>(v[0], v1, keep0 ? 1.0 / vn0 : 0.0, c01, keep1 ? 1.0 / vn1 : 0.0,
                                       (keep0 ? 1 : 0) | (keep1 ? 2 : 0), c.Zb(), p, c.pmax, tmp,
                                       keep0 ? tmp2 : tmp, nel);
    // Jacobian-vector products w = F(z; E = 0) of the stored columns; with FP32
    // fields they run in the FP64 pipeline on the exact FP64 values of the
    // stored columns, and the H columns are formed from the FP64 products (W
    // itself is stored rounded)
    double* z64[2] = {nullptr, nullptr};
    double* w64[2] = {nullptr, nullptr};
    for (int a = 0; a < nacc; ++a) {
        if (c.sub) {
            Ctx<double>& sd = *c.sub;
            z64[a] = sd.ring(a);
            w64[a] = reinterpret_cast<double*>(wout[a]);
            k_convert<T, double><<<gb, 256, 0, c.s>>>(zc[a], z64[a], 1.0, nel);
            run_F<double>(sd, z64[a], 0, nullptr, z64[a], w64[a], OUT_XI, 0, DC_MEAN, sd.st->Ezero, nullptr);
            k_col_put<double, T><<<gb, 256, 0, c.s>>>(w64[a], 1.0, c.Wb(), p + a, c.pmax, nullptr, nel);
        } else {
            run_F<T>(c, zc[a], 0, nullptr, zc[a], wout[a], OUT_XI, 0, DC_MEAN, c.st->Ezero, nullptr);
            k_col_put<T, T><<<gb, 256, 0, c.s>>>(wout[a], 1.0, c.Wb(), p + a, c.pmax, nullptr, nel);
        }
        ++*jvps;
    }
    // H columns <z_i, w_a> and Gram columns <z_i, z_a>, i <= p + a, in one pass
    const int ld = kMaxP + 2;
    if (c.sub) {
        if (nacc == 1)
            launch_gdots<double, T, 2, 1>(c.s, Gq, Fields<double>{{w64[0], z64[0]}}, c.Zb(), p + 1, c.pmax, N,
                                          c.pg(), kMaxP);
        else
            launch_gdots<double, T, 4, 1>(c.s, Gq, Fields<double>{{w64[0], z64[0], w64[1], z64[1]}}, c.Zb(), p + 2,
                                          c.pmax, N, c.pg(), kMaxP);
    } else if (nacc == 1)
        launch_gdots<T, T, 2, 1>(c.s, Gq, Fields<T>{{wout[0], zc[0]}}, c.Zb(), p + 1, c.pmax, N, c.pg(), kMaxP);
    else
        launch_gdots<T, T, 4, 1>(c.s, Gq, Fields<T>{{wout[0], zc[0], wout[1], zc[1]}}, c.Zb(), p + 2, c.pmax, N,
                                 c.pg(), kMaxP);
    for (int f = 0; f < 2 * nacc; ++f)
        reduce_cols(c, c.pg() + (long long)f * kMaxP * Gq, Gq, 1, Gq, p + f / 2 + 1, HZ + f * ld);
    // H rows <z_a, w_j>, j < p + a, in one pass over W
    if (p + nacc - 1 > 0) {
        if (nacc == 1)
            launch_gdots<T, T, 1, 1>(c.s, Gq, Fields<T>{{zc[0]}}, c.Wb(), p, c.pmax, N, c.pg(), kMaxP);
        else
            launch_gdots<T, T, 2, 1>(c.s, Gq, Fields<T>{{zc[0], zc[1]}}, c.Wb(), p + 1, c.pmax, N, c.pg(), kMaxP);
        for (int a = 0; a < nacc; ++a)
            if (p + a > 0) reduce_cols(c, c.pg() + (long long)a * kMaxP * Gq, Gq, 1, Gq, p + a, RW + a * kMaxP);
    }
    for (int a = 0; a < nacc; ++a) k_border<<<1, 1, 0, c.s>>>(c.st, HZ + 2 * a * ld, RW + a * kMaxP,
                                                              HZ + (2 * a + 1) * ld, p + a);
    p += nacc;
    return nacc;
}

// Basis growth In(q, Z) after main-loop F application number it (Sec. 3:
// QR of the last two differences of q, one or two columns, H bordered by one
// JVP per column).  Returns the number of columns added, or -1 on HIP error.
template <typename T>
int grow_basis(Ctx<T>& c, int it, int nq, int& p, const rpm_options* o, int growth_index, int* want_out,
               int* jvps)
{
    const long long N = c.sh.g.N;
    double* D1 = c.template at<double>(c.L.D1);
    double* D0 = c.template at<double>(c.L.D0);
    T* tmp = c.template at<T>(c.L.tmp);
    T* tmp2 = c.template at<T>(c.L.tmp2);
    const int sa = (it - 1) & 3, sb = (it - 2) & 3, sc = (it - 3) & 3;
    const bool two = nq >= 3;
    hipEvent_t ev;
    c.mark_begin(RPM_K_GROWTH, ev);
    const int Gd = (int)((6 * N + 4 * kThreads - 1) / (4 * kThreads));
    k_growth_diff<T><<<Gd, kThreads, 0, c.s>>>(c.ring(sa), c.ring(sb), two ? c.ring(sc) : nullptr, c.Zb(), p,
                                               c.pmax,
                                               c.st->zeta_ring[sa], c.st->zeta_ring[sb], c.st->zeta_ring[sc], D1,
                                               two ? D0 : nullptr, N, c.pg());
    reduce_cols(c, c.pg(), Gd, 3, 1, 3, c.gsum());
    double gram[3];
    if (!sync_read(c, gram, c.gsum(), sizeof(gram))) return -1;
    const double T11 = std::sqrt(std::max(gram[0], 0.0));
    double T22 = 0.0;
    int want = 0;
    // modified Gram-Schmidt QR of [D1, D0]: |D0 - (g01 / g00) D1| from the Gram
    // entries (the subtraction itself is fused into the second candidate's
    // conversion below)
    const double r01 = T11 > 0.0 ? gram[1] / gram[0] : 0.0;
    if (T11 > 0.0) {
        if (two) T22 = std::sqrt(std::max(gram[2] - r01 * gram[1], 0.0));
        want = (two && T22 > o->kappa * T11) ? 2 : 1;
    }
    if (o->replay && growth_index < o->replay_len) want = o->replay[growth_index];
    *want_out = want;
    // candidates: the normalised differences, projected onto zero-mean
    // compatible fields (Lippmann-Schwinger map) and back in FP64
    const long long nel = 6 * N;
    const int gb = (int)((nel + 255) / 256);
    // (the second first: its conversion reads the first difference)
    const bool use[2] = {want >= 1 && T11 > 0.0, want >= 2 && two && T22 > 0.0};
    for (int col = 1; col >= 0; --col) {
        if (!use[col]) continue;
        double* v = col == 0 ? D1 : D0;
        if (c.sub && !c.pol) {
            // FP32 fields: projected by the FP64 pipeline, never rounded to FP32
            Ctx<double>& sd = *c.sub;
            double* a = sd.ring(3);
            if (col == 0) k_convert<double, double><<<gb, 256, 0, c.s>>>(D1, a, 1.0 / T11, nel);
            else k_convert_sub<double><<<gb, 256, 0, c.s>>>(D0, D1, r01, 1.0 / T22, a, nel);
            project_compatible<double>(sd, a, v);
            continue;
        }
        if (col == 0) k_convert<double, T><<<gb, 256, 0, c.s>>>(D1, tmp, 1.0 / T11, nel);
        else k_convert_sub<T><<<gb, 256, 0, c.s>>>(D0, D1, r01, 1.0 / T22, tmp, nel);
        if (c.pol) {
            // polarization iterates are not compatible: the differences stay as they are
            k_convert<T, double><<<gb, 256, 0, c.s>>>(tmp, v, 1.0, nel);
        } else {
            project_compatible<T>(c, tmp, tmp2);
            k_convert<T, double><<<gb, 256, 0, c.s>>>(tmp2, v, 1.0, nel);
        }
    }
    double* cand[2];
    int nc = 0;
    for (int col = 0; col < 2; ++col)
        if (use[col]) cand[nc++] = col == 0 ? D1 : D0;
    int added = 0;
    if (nc == 2 && p + 2 <= c.pmax && p <= 32) {
        const int r = add_columns<T, 2>(c, p, cand, jvps);
        if (r < 0) return -1;
        added += r;
    } else {
        for (int k = 0; k < nc && p < c.pmax; ++k) {
            const int r = add_columns<T, 1>(c, p, cand + k, jvps);
            if (r < 0) return -1;
            added += r;
        }
    }
    if (added > 0) k_factor<<<1, 64, 0, c.s>>>(c.st, p);
    c.mark_end(RPM_K_GROWTH, ev);
    c.check_launch();
    return added;
}

template <typename T>
void stats_fill(Ctx<T>& c, rpm_stats* st, const DevState& hs, int jvps, int growth, int p, double secs,
                const std::vector<int>& decisions)
{
    if (!st) return;
    st->iterations = hs.iters;
    st->jvps = jvps;
    st->basis_dim = p;
    st->growth_events = growth;
    st->residual = hs.err;
    st->seconds = secs;
    if (st->decisions && st->decisions_cap > 0) {
        for (int i = 0; i < std::min((int)decisions.size(), st->decisions_cap); ++i) st->decisions[i] = decisions[i];
    }
    for (int k = 0; k < RPM_NKERNEL; ++k) {
        st->kernel_ms[k] = c.prof.ms[k];
        st->kernel_launches[k] = c.prof.n[k];
        st->kernel_bytes[k] = c.prof.bytes[k];
    }
}

// What one run of the iteration solves: the cell problem for mean strain E
// (err_mode 0), or a correction problem d = F(d; 0) + g (err_mode 1) whose
// error is the fixed-point increment |G(d) - d| / |g|.
template <typename T>
struct Spec {
    const double* E;      // host mean strain
    const T* eps0;        // device start (nullable)
    bool zero_start;      // start from 0 (correction solves)
    const T* shift;       // device shift field g (nullable)
    int err_mode;
    double tol;
    double gnorm;
    bool reuse;
    int stall;            // stall window of the error (0 = off)
};

// Captured graphs of one iteration, one per ring slot, for the basis size p.
struct StepGraphs {
    bool on = false;
    int p = -1;
    hipGraphExec_t ex[4] = {nullptr, nullptr, nullptr, nullptr};
    void clear()
    {
        for (auto& e : ex)
            if (e) {
                hipGraphExecDestroy(e);
                e = nullptr;
            }
    }
    ~StepGraphs() { clear(); }
};

template <typename T>
struct SolveOut {
    const T* final_it = nullptr;  // the iterate whose error was evaluated last
    DevState hs;
    int jvps = 0, growth = 0, p = 0;
    std::vector<int> decisions;
};

// One run of Algorithm 1 or 2 (the iteration itself; outputs stay in the workspace).
template <typename T>
rpm_status run_solve(Ctx<T>& c, const rpm_problem* pr, const rpm_options* o, const Spec<T>& sp, SolveOut<T>& so)
{
    const Geo& g = c.sh.g;
    const long long N = g.N;
    int p = 0;
    rpm_status rs = prepare(c, pr, o, sp.reuse, &p, sp.tol, sp.gnorm, sp.stall);
    if (rs != RPM_OK) return rs;
    set_E(c, sp.E);
    const bool rpm = o->scheme == RPM_SCHEME_RPM && c.pmax > 0;
    const int* done = &c.st->done;
    double* pinc = sp.err_mode == 1 ? c.template at<double>(c.L.pinc) : nullptr;
    int jvps = 0, growth = 0;

    // initial iterate eps^0 = E (or the supplied start, or 0) and xi^0 = F(eps^0)
    if (sp.eps0) {
        hipMemcpyAsync(c.eps(), sp.eps0, sizeof(T) * 6 * N, hipMemcpyDeviceToDevice, c.s);
    } else {
        const long long nel = 6 * N;
        k_fill_uniform<T><<<(int)((nel + 255) / 256), 256, 0, c.s>>>(c.eps(), sp.zero_start ? c.st->Ezero : c.st->E,
                                                                     N);
    }
    run_F<T>(c, c.eps(), 0, nullptr, c.eps(), c.ring(1), OUT_XI, 0, DC_MEAN, c.st->E, done, sp.shift, pinc);
    if (rpm) project(c, c.ring(1), c.eps(), p, true);
    reduce_and_finalize(c, rpm ? p : 0, 1, 0, true, done, sp.err_mode);

    int it = 1, nu = 0, nq = 0;
    const int check = std::max(1, o->check_every);
    // iterations replayed from captured graphs (not with profiling events, not
    // on the legacy default stream, which cannot be captured)
    StepGraphs graphs;
    graphs.on = o->graph != 0 && !c.prof.on && c.s != nullptr;
    for (;;) {
        const bool at_growth = rpm && (nu > o->n_max) && p < c.pmax;
        if (at_growth || (it % check) == 0 || it >= o->max_iter) {
            int flags[4];
            if (!sync_read(c, flags, &c.st->done, sizeof(flags))) return RPM_E_HIP;
            if (flags[0] || flags[2] >= o->max_iter) break;
            if (at_growth) {
                int want = 0;
                const int p_before = p;
                const int added = grow_basis(c, it, nq, p, o, (int)so.decisions.size(), &want, &jvps);
                if (added < 0) return RPM_E_HIP;
                so.decisions.push_back(want);
                ++growth;
                nu = 0;
                nq = 0;
                // the current iterate: eps, or xi_prev while the basis was empty
                const T* cur = (p_before > 0 || it == 1) ? c.eps() : c.ring(it - 1);
                // projections of the current pair (eps, xi) on the grown basis, Newton step
                project(c, c.ring(it), cur, p, true);
                reduce_and_finalize(c, p, it, 1, true, done, sp.err_mode);
            }
        }
        // one RPM iteration: eps = xi + Z d, xi = F(eps), Newton step (while
        // the basis is empty eps = xi_prev, read where it lies)
        ++it;
        auto step = [&](int i) {
            const T* xprev = c.ring(i - 1);
            if (rpm && p > 0) {
                run_F<T>(c, xprev, p, c.eps(), c.eps(), c.ring(i), OUT_XI, 0, DC_MEAN, c.st->E, done, sp.shift, pinc);
                project(c, c.ring(i), c.eps(), p, false);
            } else {
                run_F<T>(c, xprev, 0, nullptr, xprev, c.ring(i), OUT_XI, 0, DC_MEAN, c.st->E, done, sp.shift, pinc);
            }
            reduce_and_finalize(c, rpm ? p : 0, i, 0, false, done, sp.err_mode);
        };
        if (graphs.on) {
            // the kernels of an iteration depend on it only through the ring slot
            // it & 3 (and on the basis size): one graph per slot, recaptured when
            // the basis grows
            if (graphs.p != p) {
                graphs.clear();
                graphs.p = p;
            }
            hipGraphExec_t& ex = graphs.ex[it & 3];
            if (!ex) {
                hipGraph_t gr = nullptr;
                if (hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal) != hipSuccess) return RPM_E_HIP;
                step(it);
                if (hipStreamEndCapture(c.s, &gr) != hipSuccess || !gr) return RPM_E_HIP;
                const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
                hipGraphDestroy(gr);
                if (ie != hipSuccess) {
                    ex = nullptr;
                    return RPM_E_HIP;
                }
            }
            if (hipGraphLaunch(ex, c.s) != hipSuccess) return RPM_E_HIP;
        } else {
            step(it);
        }
        ++nu;
        ++nq;
    }
    if (!sync_read(c, &so.hs, c.st, sizeof(DevState))) return RPM_E_HIP;
    const int itf = std::max(so.hs.iters, 1);
    // the input of the last map application: eps while a basis recombined it,
    // the previous xi otherwise (the basis only grows between executed steps)
    so.final_it = (itf == 1 || (rpm && p > 0)) ? c.eps() : c.ring(itf - 1);
    so.jvps += jvps;
    so.growth += growth;
    so.p = p;
    switch (so.hs.status) {
        case 0: return RPM_OK;
        case 2: return RPM_DIVERGED;
        case 3: return RPM_SINGULAR;
        default: return RPM_NOT_CONVERGED;
    }
}

// FP64 pipeline living in the FP32 workspace (certification and refinement).
void sub64_init(Ctx<double>& c64, Ctx<float>& c, const rpm_options* o)
{
    const int32_t n[3] = {c.sh.g.nx, c.sh.g.ny, c.sh.g.nz};
    const rpm_options b = basic_fp64_options(o);
    c64.sh = make_shapes<double>(n, spectral_comps(&b));
    c64.L = make_layout<double>(c64.sh, &b);
    c64.s = c.s;
    c64.ws = c.ws + c.L.sub64;
    c64.st = reinterpret_cast<DevState*>(c64.ws + c64.L.st);
    c64.phase = c.phase;
    c64.lam0 = c.lam0;
    c64.mu0 = c.mu0;
    c64.pmax = 0;
    c64.pol = c.pol;
    c64.alpha = c.alpha;
    c64.beta = c.beta;
    c64.prof.on = false;
}

// FP64 map application on c64.eps(): xi64 in ring(1), error and sigma_hat(0) in hs.
rpm_status eval64(Ctx<double>& c64, DevState& hs)
{
    k_reset_state<<<1, 1, 0, c64.s>>>(c64.st);
    run_F<double>(c64, c64.eps(), 0, nullptr, c64.eps(), c64.ring(1), OUT_XI, 0, DC_MEAN, c64.st->E, nullptr);
    reduce_and_finalize(c64, 0, 1, 0, true, nullptr);
    if (!sync_read(c64, &hs, c64.st, sizeof(DevState))) return RPM_E_HIP;
    return RPM_OK;
}

// Solve for E and write the caller's outputs; with FP32 fields, certify the
// result in FP64 and refine it when the FP64 error misses tol.
// After the iteration: certify an FP32 result in FP64 and refine it while the
// FP64 error misses tol (c64: the FP64 pipeline, FP32 fields only), then write
// the caller's outputs and statistics and map the stop reason to a status.
template <typename T>
rpm_status finish_solve(Ctx<T>& c, Ctx<double>& c64, const rpm_problem* pr, const rpm_options* o, SolveOut<T>& so,
                        T* eps_out, T* sig_out, double* sig_avg, rpm_stats* st,
                        std::chrono::steady_clock::time_point t0)
{
    const long long N = c.sh.g.N;
    const long long nel = 6 * N;
    const int gb = (int)((nel + 255) / 256);
    const bool refine = sizeof(T) == 4 && o->refine > 0;
    const int stall = refine ? o->stall_window : 0;
    rpm_status rs = RPM_OK;
    const DevState hs_main = so.hs;
    if (st && st->history && st->history_cap > 0) {  // before correction solves reuse the buffer
        const int n = std::min(st->history_cap, hs_main.iters);
        if (n > 0) {
            hipMemcpyAsync(st->history, c.template at<double>(c.L.hist), sizeof(double) * n, hipMemcpyDeviceToHost,
                           c.s);
            hipStreamSynchronize(c.s);
        }
    }
    double sav[6];
    for (int i = 0; i < 6; ++i) sav[i] = so.hs.sig_hat0[i] / (double)N;
    double res64 = so.hs.err;
    int nref = 0;
    const T* efin = so.final_it;
    bool rounded = false;  // outputs come from the FP64 field rounded to T
    if constexpr (sizeof(T) == 4) {
        k_convert<T, double><<<gb, 256, 0, c.s>>>(efin, c64.eps(), 1.0, nel);
        DevState h64;
        if ((rs = eval64(c64, h64)) != RPM_OK) return rs;
        res64 = h64.err;
        for (int i = 0; i < 6; ++i) sav[i] = h64.sig_hat0[i] / (double)N;
        const double zeros[6] = {0, 0, 0, 0, 0, 0};
        T* g32 = c.template at<T>(c.L.shift);
        while (rs == RPM_OK && (so.hs.status == 0 || so.hs.status == 4) && res64 > o->tol && nref < o->refine) {
            // g = F64(eps64) - eps64, |g| in FP64
            k_residual_shift<T><<<c.sh.Gp, kThreads, 0, c.s>>>(c64.ring(1), c64.eps(), g32, N, c.pg());
            reduce_cols(c, c.pg(), c.sh.Gp, 1, 1, 1, c.gsum());
            double g2;
            if (!sync_read(c, &g2, c.gsum(), sizeof(g2))) return RPM_E_HIP;
            const double gnorm = std::sqrt(std::max(g2, 0.0));
            if (!(gnorm > 0.0)) break;
            Spec<T> sc{zeros, nullptr, true, g32, 1, o->refine_tol, gnorm, true, stall};
            SolveOut<T> si;
            rpm_status ri = run_solve(c, pr, o, sc, si);
            if (ri < 0) return ri;
            so.jvps += si.jvps;
            so.growth += si.growth;
            so.p = si.p;
            so.decisions.insert(so.decisions.end(), si.decisions.begin(), si.decisions.end());
            // a diverged or singular correction solve is not applied
            if (si.hs.status == 2 || si.hs.status == 3) break;
            k_add_correction<T><<<gb, 256, 0, c.s>>>(c64.eps(), si.final_it, 1.0, nel);
            if ((rs = eval64(c64, h64)) != RPM_OK) return rs;
            ++nref;
            if (!(h64.err < res64)) {
                // the sweep did not lower the FP64 error: undo it and stop
                k_add_correction<T><<<gb, 256, 0, c.s>>>(c64.eps(), si.final_it, -1.0, nel);
                if ((rs = eval64(c64, h64)) != RPM_OK) return rs;
                res64 = h64.err;
                for (int i = 0; i < 6; ++i) sav[i] = h64.sig_hat0[i] / (double)N;
                break;
            }
            res64 = h64.err;
            for (int i = 0; i < 6; ++i) sav[i] = h64.sig_hat0[i] / (double)N;
            // a correction stopped by a stall still lowered the FP64 error
            if (si.hs.status != 0 && si.hs.status != 4) break;
        }
        if (nref > 0) {
            // the refined FP64 field, rounded, is the result
            k_convert<double, T><<<gb, 256, 0, c.s>>>(c64.eps(), c.eps(), 1.0, nel);
            efin = c.eps();
            rounded = true;
        }
    }
    if (eps_out) hipMemcpyAsync(eps_out, efin, sizeof(T) * nel, hipMemcpyDeviceToDevice, c.s);
    if (sig_out) k_stress<T><<<(int)((N + 255) / 256), 256, 0, c.s>>>(efin, c.phase, c.lame(), sig_out, N);
    if (sig_avg)
        for (int i = 0; i < 6; ++i) sig_avg[i] = sav[i];
    if (hipStreamSynchronize(c.s) != hipSuccess || c.hip_error) return RPM_E_HIP;
    if (c.prof.on) c.prof.harvest();
    (void)rounded;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats_fill(c, st, hs_main, so.jvps, so.growth, so.p, secs, so.decisions);
    if (st) {
        st->residual_fp64 = res64;
        st->refinements = nref;
    }
    (void)pr;
    switch (hs_main.status) {
        case 0:
        case 4: return (refine && res64 <= o->tol) || (!refine && hs_main.status == 0) ? RPM_OK : RPM_NOT_CONVERGED;
        case 2: return RPM_DIVERGED;
        case 3: return RPM_SINGULAR;
        default: return RPM_NOT_CONVERGED;
    }
}

template <typename T>
rpm_status solve_full(Ctx<T>& c, const rpm_problem* pr, const double E[6], const rpm_options* o, const T* eps0,
                      T* eps_out, T* sig_out, double* sig_avg, rpm_stats* st, bool reuse)
{
    auto t0 = std::chrono::steady_clock::now();
    // FP32 fields carry ~1e-7 rounding, so equilibrium errors much below 1e-6 are
    // not reliably reachable in FP32: with refinement on, the FP32 stage stops at
    // max(tol, kFp32Stage) and FP64 refinement takes the field to tol.
    const bool refine = sizeof(T) == 4 && o->refine > 0;
    const double stage_tol = refine ? std::max(o->tol, kFp32Stage) : o->tol;
    // with refinement, a stalled FP32 stage hands its field over to it
    const int stall = refine ? o->stall_window : 0;
    // FP32 fields: the FP64 pipeline (JVPs and projections of basis growth,
    // certification, refinement)
    Ctx<double> c64;
    struct SubReset {
        Ctx<T>& c;
        ~SubReset() { c.sub = nullptr; }
    } sub_reset{c};
    rpm_status rs = RPM_OK;
    if constexpr (sizeof(T) == 4) {
        sub64_init(c64, c, o);
        int p64 = 0;
        rs = prepare(c64, pr, o, false, &p64, o->tol);
        if (rs != RPM_OK) return rs;
        set_E(c64, E);
        c.sub = &c64;
    }
    Spec<T> sp{E, eps0, false, nullptr, 0, stage_tol, 1.0, reuse, stall};
    SolveOut<T> so;
    rs = run_solve(c, pr, o, sp, so);
    if (rs < 0) return rs;
    return finish_solve(c, c64, pr, o, so, eps_out, sig_out, sig_avg, st, t0);
}

bool finite(double x) { return std::isfinite(x); }

rpm_status validate(const rpm_problem* pr, const rpm_options* o)
{
    if (!pr || !o || !pr->lame) return RPM_E_INVALID;
    if (pr->n_phases < 1 || pr->n_phases > 256) return RPM_E_INVALID;
    for (int a = 0; a < 3; ++a) {
        const int n = pr->n[a];
        if (a == 2 && n == 1) continue;
        if (n < 2 || n > kMaxN || !smooth23(n)) return RPM_E_UNSUPPORTED_SIZE;
    }
    for (int i = 0; i < pr->n_phases; ++i) {
        const double l = pr->lame[2 * i], m = pr->lame[2 * i + 1];
        if (!finite(l) || !finite(m) || m < 0.0 || 3.0 * l + 2.0 * m < 0.0) return RPM_E_INVALID;
    }
    const double l0 = pr->lame0[0], m0 = pr->lame0[1];
    if (!finite(l0) || !finite(m0) || !(m0 > 0.0) || !(3.0 * l0 + 2.0 * m0 > 0.0)) return RPM_E_INVALID;
    if (!finite(o->tol) || !(o->tol > 0.0)) return RPM_E_INVALID;
    if (o->max_iter < 1 || o->n_max < 1 || o->p_max < 0 || o->p_max > kMaxP) return RPM_E_INVALID;
    if (!finite(o->kappa) || o->kappa < 0.0 || o->kappa > 1.0) return RPM_E_INVALID;
    if (o->scheme != RPM_SCHEME_BASIC && o->scheme != RPM_SCHEME_RPM) return RPM_E_INVALID;
    if (o->precision != RPM_FP64 && o->precision != RPM_FP32) return RPM_E_INVALID;
    if (o->check_every < 1) return RPM_E_INVALID;
    if (o->replay_len < 0 || (o->replay_len > 0 && !o->replay)) return RPM_E_INVALID;
    if (o->refine < 0 || !finite(o->refine_tol) || !(o->refine_tol > 0.0) || !(o->refine_tol < 1.0))
        return RPM_E_INVALID;
    if (o->map != RPM_MAP_LS && o->map != RPM_MAP_POLARIZATION) return RPM_E_INVALID;
    if (o->profile_classes < 0 || o->profile_classes >= (1 << RPM_NKERNEL)) return RPM_E_INVALID;
    if (o->stall_window < 0) return RPM_E_INVALID;
    if (o->batch_cases < 0 || o->batch_cases > 2) return RPM_E_INVALID;
    if (o->graph != 0 && o->graph != 1) return RPM_E_INVALID;
    if (o->profile_every < 0) return RPM_E_INVALID;
    if (o->tuning && (o->tuning->y_cols < 0 || o->tuning->y_blocks < 0 || o->tuning->gamma_blocks < 0 ||
                      o->tuning->y_regs < 0 || o->tuning->y_regs > 1))
        return RPM_E_INVALID;
    if (o->map == RPM_MAP_POLARIZATION &&
        (!finite(o->alpha) || !(o->alpha > 0.0) || !finite(o->beta) || !(o->beta > 0.0)))
        return RPM_E_INVALID;
    return RPM_OK;
}

template <typename T>
rpm_status ctx_init(Ctx<T>& c, const rpm_problem* pr, const rpm_options* o, void* ws, size_t ws_bytes,
                    void* stream, bool map_only = false)
{
    c.sh = make_shapes<T>(pr->n, spectral_comps(o), o->tuning);
    if (!c.sh.ok) return RPM_E_UNSUPPORTED_SIZE;
    if (!c.sh.tune_ok) return RPM_E_INVALID;
    // FP32 fields are certified by an FP64 pipeline on the same grid
    if (sizeof(T) == 4 && !map_only && !make_shapes<double>(pr->n, spectral_comps(o)).ok)
        return RPM_E_UNSUPPORTED_SIZE;
    c.L = make_layout<T>(c.sh, o, map_only);
    if (map_only && c.L.total > ws_bytes) return RPM_E_SCRATCH;
    if (!ws || ws_bytes < c.L.total) return RPM_E_WORKSPACE;
    if (!pr->phase) return RPM_E_INVALID;
    c.s = (hipStream_t)stream;
    c.ws = (char*)ws;
    c.st = reinterpret_cast<DevState*>(c.ws + c.L.st);
    c.phase = pr->phase;
    c.lam0 = pr->lame0[0];
    c.mu0 = pr->lame0[1];
    c.pmax = (o->scheme == RPM_SCHEME_RPM && !map_only) ? o->p_max : 0;
    c.pol = o->map == RPM_MAP_POLARIZATION;
    c.alpha = o->alpha;
    c.beta = o->beta;
    c.prof.on = o->profile != 0;
    c.prof.mask = o->profile_classes ? (uint32_t)o->profile_classes : ~0u;
    c.prof.every = o->profile_every > 1 ? o->profile_every : 1;
    return RPM_OK;
}

bool finite6(const double* E)
{
    for (int i = 0; i < 6; ++i)
        if (!finite(E[i])) return false;
    return true;
}

template <typename T>
rpm_status solve_typed(const rpm_problem* pr, const double E[6], const rpm_options* o, const void* eps0,
                       void* eps_out, void* sig_out, double sig_avg[6], rpm_stats* st, void* ws, size_t ws_bytes,
                       void* stream)
{
    Ctx<T> c;
    rpm_status rs = ctx_init(c, pr, o, ws, ws_bytes, stream);
    if (rs != RPM_OK) return rs;
    return solve_full<T>(c, pr, E, o, (const T*)eps0, (T*)eps_out, (T*)sig_out, sig_avg, st, o->reuse_basis != 0);
}

template <typename T>
rpm_status apply_typed(const rpm_problem* pr, const double E[6], const rpm_options* o, const void* eps, void* xi,
                       double* err, double* sig_avg, void* ws, size_t ws_bytes, void* stream, bool map_only = false)
{
    Ctx<T> c;
    rpm_status rs = ctx_init(c, pr, o, ws, ws_bytes, stream, map_only);
    if (rs != RPM_OK) return rs;
    int p = 0;
    rs = prepare(c, pr, o, false, &p, o->tol);
    if (rs != RPM_OK) return rs;
    set_E(c, E);
    run_F<T>(c, (const T*)eps, 0, nullptr, (const T*)eps, (T*)xi, OUT_XI, 0, DC_MEAN, c.st->E, nullptr);
    reduce_and_finalize(c, 0, 1, 0, true, nullptr);
    DevState hs;
    if (!sync_read(c, &hs, c.st, sizeof(hs))) return RPM_E_HIP;
    if (err) *err = hs.err;
    if (sig_avg)
        for (int i = 0; i < 6; ++i) sig_avg[i] = hs.sig_hat0[i] / (double)c.sh.g.N;
    return RPM_OK;
}

// Tile autotuner: times the map under candidate launch shapes (coordinate
// search over y_regs, y_cols, y_blocks, gamma_blocks; 0 = default first).
template <typename T>
rpm_status tune_typed(const rpm_problem* pr, const rpm_options* o, int reps, rpm_tuning* best, double* best_ms,
                      int32_t* ncand, void* ws, size_t ws_bytes, void* stream)
{
    rpm_options ob = *o;
    ob.tuning = nullptr;
    ob.profile = 0;
    Ctx<T> c;
    rpm_status rs = ctx_init(c, pr, &ob, ws, ws_bytes, stream);
    if (rs != RPM_OK) return rs;
    int p = 0;
    rs = prepare(c, pr, &ob, false, &p, ob.tol);
    if (rs != RPM_OK) return rs;
    const double E[6] = {0.01, 0.0, 0.0, 0.0, 0.0, 0.0};
    set_E(c, E);
    const Geo& g0 = c.sh.g;
    k_fill_uniform<T><<<(int)((6 * g0.N + 255) / 256), 256, 0, c.s>>>(c.eps(), c.st->E, g0.N);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return RPM_E_HIP;
    }
    const Shapes<T> base = c.sh;
    int count = 0;
    bool hip_ok = true;
    // ms per map of one shape; < 0 when the shape does not apply to the grid
    auto time_shape = [&](const rpm_tuning& tn) -> double {
        const Shapes<T> sh = make_shapes<T>(pr->n, spectral_comps(&ob), &tn);
        if (!sh.ok || !sh.tune_ok) return -1.0;
        c.sh = sh;
        run_F<T>(c, c.eps(), 0, nullptr, c.eps(), c.ring(0), OUT_XI, 0, DC_MEAN, c.st->E, nullptr);
        hipEventRecord(e0, c.s);
        for (int r = 0; r < reps; ++r)
            run_F<T>(c, c.eps(), 0, nullptr, c.eps(), c.ring(0), OUT_XI, 0, DC_MEAN, c.st->E, nullptr);
        hipEventRecord(e1, c.s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || c.hip_error)
            hip_ok = false;
        c.sh = base;
        ++count;
        return hip_ok ? (double)ms / reps : -1.0;
    };
    rpm_tuning cur{0, 0, 0, 0};
    double cur_ms = time_shape(cur);
    const Geo& g = base.g;
    // the y transforms in registers, where they apply
    {
        rpm_tuning tn = cur;
        tn.y_regs = 1;
        const Shapes<T> sh = make_shapes<T>(pr->n, spectral_comps(&ob), &tn);
        if (sh.ok && sh.tune_ok && hip_ok) {
            const double ms = time_shape(tn);
            if (ms >= 0.0 && ms < cur_ms) {
                cur = tn;
                cur_ms = ms;
            }
        }
    }
    // y_cols: admissible divisors of nz, largest first (3-D only)
    if (!g.two_d) {
        int tried = 0;
        for (int t = std::min(g.nz, 64); t >= 1 && tried < 4 && hip_ok; --t) {
            if (g.nz % t != 0 || t == g.tz) continue;
            rpm_tuning tn = cur;
            tn.y_cols = t;
            const Shapes<T> sh = make_shapes<T>(pr->n, spectral_comps(&ob), &tn);
            if (!sh.ok || !sh.tune_ok) continue;
            ++tried;
            const double ms = time_shape(tn);
            if (ms >= 0.0 && ms < cur_ms) {
                cur = tn;
                cur_ms = ms;
            }
        }
    }
    const int mult[7] = {1, 2, 3, 4, 5, 6, 8};
    // y_blocks, then gamma_blocks: 256 x mult, below the tile counts
    for (int coord = 0; coord < 2 && hip_ok; ++coord) {
        if (coord == 0 && g.two_d) continue;
        const Shapes<T> sh0 = make_shapes<T>(pr->n, spectral_comps(&ob), &cur);
        if (coord == 1 && !sh0.gpipe) continue;  // one tile per workgroup: nothing to tune
        const int tiles = coord == 0 ? sh0.Gy : sh0.Gt;
        for (int m = 0; m < 7 && hip_ok; ++m) {
            const int b = 256 * mult[m];
            if (b > tiles) break;
            rpm_tuning tn = cur;
            if (coord == 0) tn.y_blocks = b;
            else tn.gamma_blocks = b;
            const double ms = time_shape(tn);
            if (ms >= 0.0 && ms < cur_ms) {
                cur = tn;
                cur_ms = ms;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!hip_ok || cur_ms < 0.0) return RPM_E_HIP;
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    if (ncand) *ncand = count;
    return RPM_OK;
}

// Basis seed (warm start of Z): each vector goes through the steps growth
// applies to a difference of iterates (normalise, compatible projection for
// the Lippmann-Schwinger map, two Gram-Schmidt passes, JVP, H and Gram
// borders), appended to the basis the workspace holds when o->reuse_basis is
// set, else to an empty one.
template <typename T>
rpm_status seed_typed(const rpm_problem* pr, const rpm_options* o, const void* V, int p0, int32_t* p_out, void* ws,
                      size_t ws_bytes, void* stream)
{
    Ctx<T> c;
    rpm_status rs = ctx_init(c, pr, o, ws, ws_bytes, stream);
    if (rs != RPM_OK) return rs;
    if (c.pmax == 0) return RPM_E_INVALID;
    int p = 0;
    rs = prepare(c, pr, o, o->reuse_basis != 0, &p, o->tol);
    if (rs != RPM_OK) return rs;
    const long long N = c.sh.g.N;
    const long long nel = 6 * N;
    const int gb = (int)((nel + 255) / 256);
    const int rs_ = 2 * kMaxP + 3;
    double* D1 = c.template at<double>(c.L.D1);
    T* tmp = c.template at<T>(c.L.tmp);
    T* tmp2 = c.template at<T>(c.L.tmp2);
    double* nr = c.gx() + 4 * kMaxP;
    Ctx<double> c64;
    if constexpr (sizeof(T) == 4) {
        sub64_init(c64, c, o);
        int p64 = 0;
        rs = prepare(c64, pr, o, false, &p64, o->tol);
        if (rs != RPM_OK) return rs;
        c.sub = &c64;
    }
    int added = 0, jvps = 0;
    for (int k = 0; k < p0 && p < c.pmax; ++k) {
        const T* v = reinterpret_cast<const T*>(V) + (long long)k * nel;
        k_convert<T, double><<<gb, 256, 0, c.s>>>(v, D1, 1.0, nel);
        // its norm: an update pass against no columns
        launch_update<T, 1, true>(c.s, c.sh.Gq, D1, nullptr, c.Zb(), 0, c.pmax, nullptr, N, c.pg(), rs_);
        reduce_cols(c, c.pg() + kMaxP, c.sh.Gq, rs_, 1, 1, nr);
        double n2 = 0.0;
        if (!sync_read(c, &n2, nr, sizeof(n2))) return RPM_E_HIP;
        if (!(n2 > 0.0) || !finite(n2)) continue;
        if (c.sub && !c.pol) {
            // FP32 fields: normalised and projected in FP64
            Ctx<double>& sd = *c.sub;
            k_convert<double, double><<<gb, 256, 0, c.s>>>(D1, sd.ring(3), 1.0 / std::sqrt(n2), nel);
            project_compatible<double>(sd, sd.ring(3), D1);
            double* cand[1] = {D1};
            const int r = add_columns<T, 1>(c, p, cand, &jvps);
            if (r < 0) return RPM_E_HIP;
            added += r;
            continue;
        }
        k_convert<double, T><<<gb, 256, 0, c.s>>>(D1, tmp, 1.0 / std::sqrt(n2), nel);
        if (c.pol) {
            k_convert<T, double><<<gb, 256, 0, c.s>>>(tmp, D1, 1.0, nel);
        } else {
            project_compatible<T>(c, tmp, tmp2);
            k_convert<T, double><<<gb, 256, 0, c.s>>>(tmp2, D1, 1.0, nel);
        }
        double* cand[1] = {D1};
        const int r = add_columns<T, 1>(c, p, cand, &jvps);
        if (r < 0) return RPM_E_HIP;
        added += r;
    }
    if (added > 0) k_factor<<<1, 64, 0, c.s>>>(c.st, p);
    c.check_launch();
    if (hipStreamSynchronize(c.s) != hipSuccess || c.hip_error) return RPM_E_HIP;
    if (p_out) *p_out = p;
    return RPM_OK;
}

template <typename T>
rpm_status eff_typed(const rpm_problem* pr, const rpm_options* o, double* C, rpm_stats* st, void* ws,
                     size_t ws_bytes, void* stream)
{
    Ctx<T> c;
    rpm_status rs = ctx_init(c, pr, o, ws, ws_bytes, stream);
    if (rs != RPM_OK) return rs;
    const bool two_d = pr->n[2] == 1;
    const int cases3[3] = {0, 1, 5};
    const int nc = two_d ? 3 : 6;
    rpm_status worst = RPM_OK;
    for (int col = 0; col < nc; ++col) {
        const int j = two_d ? cases3[col] : col;
        double E[6] = {0, 0, 0, 0, 0, 0};
        E[j] = j < 3 ? 1.0 : 0.5;
        double sav[6];
        const bool reuse = o->reuse_basis != 0;
        c.prof.reset();
        rs = solve_full<T>(c, pr, E, o, nullptr, nullptr, nullptr, sav, st ? st + col : nullptr, reuse);
        if (rs < 0) return rs;
        if (rs != RPM_OK && worst == RPM_OK) worst = rs;
        for (int row = 0; row < nc; ++row) {
            const int i = two_d ? cases3[row] : row;
            C[row * nc + col] = sav[i];
        }
    }
    return worst;
}

// The view of load case f of a batched solve: the shared workspace (spectra,
// basis, growth temporaries, FP64 pipeline) with the case's own state,
// partial sums, fields and error history.
template <typename T>
void case_ctx(Ctx<T>& cf, const Ctx<T>& c, int f)
{
    cf.sh = c.sh;
    cf.L = c.L;
    const CaseOff& o = c.L.cs[f];
    cf.L.st = o.st;
    cf.L.pmean = o.pmean;
    cf.L.perr = o.perr;
    cf.L.pinc = o.pinc;
    cf.L.pdots = o.pdots;
    cf.L.sums = o.sums;
    cf.L.gsum = o.gsum;
    for (int i = 0; i < 4; ++i) cf.L.ring[i] = o.ring[i];
    cf.L.eps = o.eps;
    cf.L.hist = o.hist;
    cf.s = c.s;
    cf.ws = c.ws;
    cf.st = reinterpret_cast<DevState*>(c.ws + o.st);
    cf.phase = c.phase;
    cf.lam0 = c.lam0;
    cf.mu0 = c.mu0;
    cf.pmax = c.pmax;
    cf.pol = c.pol;
    cf.alpha = c.alpha;
    cf.beta = c.beta;
    cf.prof.on = false;
    cf.sub = c.sub;
}

// Stop flags of a state (the prefix of DevState up to and including err).
struct StateHead {
    int done, status, iters;
    double err;
};

template <typename T>
bool read_head(Ctx<T>& c, StateHead& h)
{
    DevState hs;
    const size_t n = offsetof(DevState, err) + sizeof(double);
    if (hipMemcpyAsync(&hs, c.st, n, hipMemcpyDeviceToHost, c.s) != hipSuccess) return false;
    if (hipStreamSynchronize(c.s) != hipSuccess) return false;
    h.done = hs.done;
    h.status = hs.status;
    h.iters = hs.iters;
    h.err = hs.err;
    return !c.hip_error;
}

template <typename T, int NB>
void launch_recombine_multi(Ctx<T>& c, const CasePtrs<T>& cp, int p)
{
    const long long nel = 6 * c.sh.g.N;
    const int VL = 16 / (int)sizeof(T);
    const int gb = (int)((nel / VL + kThreads - 1) / kThreads) + 1;
    k_recombine_multi<T, NB><<<gb, kThreads, 0, c.s>>>(cp, c.Zb(), p, c.pmax, nel);
}

// Effective tensor with the load cases solved together (Algorithm 2 for every
// unit mean strain at once): each step recombines every case from one pass
// over the basis, applies the map to each case, and projects every case on
// the basis in one more pass, so the basis streams (the bulk of an RPM step's
// bytes) are read once for all cases instead of once per case.  The cases
// share Z, W and H (F_u does not depend on E); the basis grows from the
// differences of the case with the largest error.  FP32 results are then
// certified and refined case by case.
template <typename T>
rpm_status eff_batched(const rpm_problem* pr, const rpm_options* o, double* C, rpm_stats* stv, void* ws,
                       size_t ws_bytes, void* stream)
{
    auto t0 = std::chrono::steady_clock::now();
    Ctx<T> c;
    rpm_status rs = ctx_init(c, pr, o, ws, ws_bytes, stream);
    if (rs != RPM_OK) return rs;
    const int nb = c.L.nb;
    const bool two_d = pr->n[2] == 1;
    const int cases3[3] = {0, 1, 5};
    const Geo& g = c.sh.g;
    const long long N = g.N;
    const bool refine = sizeof(T) == 4 && o->refine > 0;
    const double stage_tol = refine ? std::max(o->tol, kFp32Stage) : o->tol;
    const int stall = refine ? o->stall_window : 0;
    Ctx<double> c64;
    if constexpr (sizeof(T) == 4) {
        sub64_init(c64, c, o);
        int p64 = 0;
        rs = prepare(c64, pr, o, false, &p64, o->tol);
        if (rs != RPM_OK) return rs;
        c.sub = &c64;
    }
    Ctx<T> cx[kMaxCases];
    double Ec[kMaxCases][6];
    int p = 0;
    for (int f = 0; f < nb; ++f) {
        case_ctx(cx[f], c, f);
        const int j = two_d ? cases3[f] : f;
        for (int i = 0; i < 6; ++i) Ec[f][i] = 0.0;
        Ec[f][j] = j < 3 ? 1.0 : 0.5;
        int pf = 0;
        rs = prepare(cx[f], pr, o, f == 0 && o->reuse_basis != 0, &pf, stage_tol, 1.0, stall);
        if (rs != RPM_OK) return rs;
        if (f == 0) p = pf;
        set_E(cx[f], Ec[f]);
    }
    // a carried basis (case 0's state) serves every case
    for (int f = 1; f < nb && p > 0; ++f) k_copy_basis_state<<<1, kThreads, 0, c.s>>>(cx[f].st, cx[0].st);

    const int* done[kMaxCases];
    for (int f = 0; f < nb; ++f) done[f] = &cx[f].st->done;
    // start: eps = E_f, xi = F(eps), projections and Newton step per case
    for (int f = 0; f < nb; ++f) {
        k_fill_uniform<T><<<(int)((6 * N + 255) / 256), 256, 0, c.s>>>(cx[f].eps(), cx[f].st->E, N);
        run_F<T>(cx[f], cx[f].eps(), 0, nullptr, cx[f].eps(), cx[f].ring(1), OUT_XI, 0, DC_MEAN, cx[f].st->E,
                 done[f]);
        if (p > 0) project(cx[f], cx[f].ring(1), cx[f].eps(), p, true);
        reduce_and_finalize(cx[f], p, 1, 0, true, done[f]);
    }
    int it = 1, nu = 0, nq = 0, jvps = 0, growth = 0;
    std::vector<int> decisions;
    int p_end[kMaxCases];
    bool seen_done[kMaxCases] = {false, false, false, false, false, false};
    const int check = std::max(1, o->check_every);
    for (;;) {
        const bool at_growth = (nu > o->n_max) && p < c.pmax;
        if (at_growth || (it % check) == 0 || it >= o->max_iter) {
            bool all = true;
            int worst = -1;
            double werr = -1.0;
            double herr[kMaxCases];
            for (int f = 0; f < nb; ++f) {
                StateHead h;
                if (!read_head(cx[f], h)) return RPM_E_HIP;
                herr[f] = h.err;
                const bool d = h.done || h.iters >= o->max_iter;
                if (d && !seen_done[f]) {
                    seen_done[f] = true;
                    p_end[f] = p;
                }
                if (!d) {
                    all = false;
                    if (h.err > werr) {
                        werr = h.err;
                        worst = f;
                    }
                }
            }
            if (all) break;
            if (at_growth) {
                const int p_before = p;
                // batch_cases 1: the differences of the case with the largest
                // error; 2: of every case still iterating, largest error first
                int order[kMaxCases], no = 0;
                order[no++] = worst;
                if (o->batch_cases == 2) {
                    for (int f = 0; f < nb; ++f)
                        if (!seen_done[f] && f != worst) order[no++] = f;
                    std::sort(order + 1, order + no, [&](int a, int b) { return herr[a] > herr[b]; });
                }
                int last = worst;
                for (int k = 0; k < no && p < c.pmax; ++k) {
                    const int f = order[k];
                    if (f != last) k_copy_basis_state<<<1, kThreads, 0, c.s>>>(cx[f].st, cx[last].st);
                    int want = 0;
                    const int added = grow_basis(cx[f], it, nq, p, o, (int)decisions.size(), &want, &jvps);
                    if (added < 0) return RPM_E_HIP;
                    decisions.push_back(want);
                    last = f;
                }
                ++growth;
                nu = 0;
                nq = 0;
                for (int f = 0; f < nb; ++f) {
                    if (f != last) k_copy_basis_state<<<1, kThreads, 0, c.s>>>(cx[f].st, cx[last].st);
                    const T* cur = (p_before > 0 || it == 1) ? cx[f].eps() : cx[f].ring(it - 1);
                    project(cx[f], cx[f].ring(it), cur, p, true);
                    reduce_and_finalize(cx[f], p, it, 1, true, done[f]);
                }
            }
        }
        ++it;
        if (p > 0) {
            CasePtrs<T> cp{};
            for (int f = 0; f < nb; ++f) {
                cp.xi[f] = cx[f].ring(it - 1);
                cp.eps[f] = cx[f].eps();
                cp.d[f] = cx[f].st->d;
                cp.done[f] = done[f];
            }
            hipEvent_t ev;
            c.mark_begin(RPM_K_RECOMBINE, ev);
            if (nb == 6) launch_recombine_multi<T, 6>(c, cp, p);
            else launch_recombine_multi<T, 3>(c, cp, p);
            c.mark_end(RPM_K_RECOMBINE, ev, 6.0 * (double)N * sizeof(T) * (2 * nb + p));
        }
        for (int f = 0; f < nb; ++f) {
            const T* in = p > 0 ? cx[f].eps() : cx[f].ring(it - 1);
            run_F<T>(cx[f], in, 0, nullptr, in, cx[f].ring(it), OUT_XI, 0, DC_MEAN, cx[f].st->E, done[f]);
        }
        if (p > 0) {
            // zeta_j of every case in one pass over the basis: case f's products at
            // bpd + f kMaxP Gq (column j at + j Gq)
            Fields<T> fl{};
            for (int f = 0; f < nb; ++f) fl.f[f] = cx[f].ring(it);
            double* bpd = c.template at<double>(c.L.bpd);
            hipEvent_t ev;
            c.mark_begin(RPM_K_PROJECT, ev);
            if (nb == 6) launch_gdots<T, T, 6, 0>(c.s, c.sh.Gq, fl, c.Zb(), p, c.pmax, N, bpd, kMaxP);
            else launch_gdots<T, T, 3, 0>(c.s, c.sh.Gq, fl, c.Zb(), p, c.pmax, N, bpd, kMaxP);
            c.mark_end(RPM_K_PROJECT, ev, 6.0 * (double)N * sizeof(T) * (nb + p));
        }
        for (int f = 0; f < nb; ++f) {
            const double* bpd = c.template at<double>(c.L.bpd) + (long long)f * kMaxP * c.sh.Gq;
            k_reduce_main<<<1 + p, kThreads, 0, c.s>>>(cx[f].template at<double>(cx[f].L.perr), c.sh.G3, bpd,
                                                       c.sh.Gq, kMaxP, p, cx[f].sums(), done[f]);
            k_step_end<<<1, kThreads, 0, c.s>>>(cx[f].st, cx[f].sums(), p, it & 3, g.two_d, 0, 0, 0,
                                                cx[f].template at<double>(cx[f].L.hist), (int)c.L.hist_cap);
        }
        c.check_launch();
        ++nu;
        ++nq;
    }
    for (int f = 0; f < nb; ++f)
        if (!seen_done[f]) p_end[f] = p;
    // per case: the returned iterate, FP64 certification / refinement, outputs
    rpm_status worst = RPM_OK;
    for (int f = 0; f < nb; ++f) {
        SolveOut<T> so;
        if (!sync_read(cx[f], &so.hs, cx[f].st, sizeof(DevState))) return RPM_E_HIP;
        const int itf = std::max(so.hs.iters, 1);
        so.final_it = (itf == 1 || p_end[f] > 0) ? cx[f].eps() : cx[f].ring(itf - 1);
        so.jvps = f == 0 ? jvps : 0;
        so.growth = growth;
        so.p = p;
        so.decisions = decisions;
        if constexpr (sizeof(T) == 4) set_E(c64, Ec[f]);
        double sav[6];
        rs = finish_solve<T>(cx[f], c64, pr, o, so, nullptr, nullptr, sav, stv ? stv + f : nullptr, t0);
        if (rs < 0) return rs;
        if (rs != RPM_OK && worst == RPM_OK) worst = rs;
        for (int row = 0; row < nb; ++row) C[row * nb + f] = sav[two_d ? cases3[row] : row];
    }
    if (c.prof.on) {
        c.prof.harvest();
        if (stv)
            for (int k = 0; k < RPM_NKERNEL; ++k) {
                stv[0].kernel_ms[k] += c.prof.ms[k];
                stv[0].kernel_launches[k] += c.prof.n[k];
                stv[0].kernel_bytes[k] += c.prof.bytes[k];
            }
    }
    return worst;
}

// Prescribed mean stress (the cell problem "given the average strain or
// stress" of Sec. 2): the effective stiffness from one solve per unit mean
// strain (the basis carried from case to case), the mean strain E with
// C_eff gamma = Sigma (Voigt, engineering shear; 2-D over 11, 22, 12), then
// the strain-controlled solve for E.  st: nc + 1 entries (the load cases,
// then the final solve).
template <typename T>
rpm_status stress_typed(const rpm_problem* pr, const double S[6], const rpm_options* o, void* eps_out, void* sig_out,
                        double* sig_avg, double* E_out, rpm_stats* st, void* ws, size_t ws_bytes, void* stream)
{
    Ctx<T> c;
    rpm_status rs = ctx_init(c, pr, o, ws, ws_bytes, stream);
    if (rs != RPM_OK) return rs;
    const bool two_d = pr->n[2] == 1;
    const int cases3[3] = {0, 1, 5};
    const int nc = two_d ? 3 : 6;
    double C[36];
    rpm_status worst = RPM_OK;
    for (int col = 0; col < nc; ++col) {
        const int j = two_d ? cases3[col] : col;
        double E[6] = {0, 0, 0, 0, 0, 0};
        E[j] = j < 3 ? 1.0 : 0.5;
        double sav[6];
        c.prof.reset();
        rs = solve_full<T>(c, pr, E, o, nullptr, nullptr, nullptr, sav, st ? st + col : nullptr,
                           col > 0 || o->reuse_basis != 0);
        if (rs < 0) return rs;
        if (rs != RPM_OK && worst == RPM_OK) worst = rs;
        for (int row = 0; row < nc; ++row) C[row * nc + col] = sav[two_d ? cases3[row] : row];
    }
    // gamma = C^-1 Sigma, Gaussian elimination with partial pivoting
    double A[36], g[6];
    std::memcpy(A, C, sizeof(double) * nc * nc);
    double amax = 0.0;
    for (int i = 0; i < nc * nc; ++i) amax = std::max(amax, std::fabs(A[i]));
    for (int r = 0; r < nc; ++r) g[r] = S[two_d ? cases3[r] : r];
    for (int k = 0; k < nc; ++k) {
        int piv = k;
        for (int r = k + 1; r < nc; ++r)
            if (std::fabs(A[r * nc + k]) > std::fabs(A[piv * nc + k])) piv = r;
        if (!(std::fabs(A[piv * nc + k]) > 1e-14 * amax)) return RPM_SINGULAR;
        if (piv != k) {
            for (int j = 0; j < nc; ++j) std::swap(A[k * nc + j], A[piv * nc + j]);
            std::swap(g[k], g[piv]);
        }
        for (int r = k + 1; r < nc; ++r) {
            const double f = A[r * nc + k] / A[k * nc + k];
            for (int j = k; j < nc; ++j) A[r * nc + j] -= f * A[k * nc + j];
            g[r] -= f * g[k];
        }
    }
    for (int r = nc - 1; r >= 0; --r) {
        double v = g[r];
        for (int j = r + 1; j < nc; ++j) v -= A[r * nc + j] * g[j];
        g[r] = v / A[r * nc + r];
    }
    double E[6] = {0, 0, 0, 0, 0, 0};
    for (int r = 0; r < nc; ++r) {
        const int i = two_d ? cases3[r] : r;
        E[i] = i < 3 ? g[r] : 0.5 * g[r];  // tensor shear = engineering / 2
    }
    if (E_out) std::memcpy(E_out, E, sizeof(E));
    c.prof.reset();
    rs = solve_full<T>(c, pr, E, o, nullptr, (T*)eps_out, (T*)sig_out, sig_avg, st ? st + nc : nullptr, true);
    if (rs < 0) return rs;
    return worst != RPM_OK ? worst : rs;
}

// Scratch of rpm_fft_apply_static: one copy per GPU (each device holds its own
// instance of this array at its own address), kept until the process ends.
// Host code never uses the array's name as a device address: the address of
// the current device's copy comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[RPM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device, with it current).
rpm_status static_scratch(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RPM_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RPM_E_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RPM_OK;
}

}  // namespace

extern "C" {

void rpm_default_options(rpm_options* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-6;
    o->max_iter = 10000;
    o->n_max = 10;
    o->p_max = 32;
    o->kappa = 0.1;
    o->scheme = RPM_SCHEME_RPM;
    o->precision = RPM_FP64;
    o->reuse_basis = 0;
    o->check_every = 16;
    o->replay = nullptr;
    o->replay_len = 0;
    o->profile = 0;
    o->refine = 4;
    o->refine_tol = 1e-3;
    o->map = RPM_MAP_LS;
    o->profile_classes = 0;
    o->alpha = 2.0;
    o->beta = 2.0;
    o->stall_window = 400;
    o->batch_cases = 0;
    o->graph = 0;
    o->profile_every = 1;
    o->tuning = nullptr;
}

rpm_status rpm_lame_from_young(double E, double nu, double* lam, double* mu)
{
    if (!lam || !mu || !std::isfinite(E) || !std::isfinite(nu) || nu >= 0.5 || nu <= -1.0) return RPM_E_INVALID;
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    *mu = E / (2.0 * (1.0 + nu));
    return RPM_OK;
}

rpm_status rpm_workspace_size(const int32_t n[3], const rpm_options* o, size_t* bytes)
{
    if (!n || !o || !bytes) return RPM_E_INVALID;
    for (int a = 0; a < 3; ++a) {
        if (a == 2 && n[a] == 1) continue;
        if (n[a] < 2 || n[a] > kMaxN || !smooth23(n[a])) return RPM_E_UNSUPPORTED_SIZE;
    }
    if (o->max_iter < 1 || o->p_max < 0 || o->p_max > kMaxP) return RPM_E_INVALID;
    if (o->map != RPM_MAP_LS && o->map != RPM_MAP_POLARIZATION) return RPM_E_INVALID;
    if (o->precision == RPM_FP64) {
        Shapes<double> s = make_shapes<double>(n, spectral_comps(o));
        if (!s.ok) return RPM_E_UNSUPPORTED_SIZE;
        *bytes = make_layout<double>(s, o).total;
    } else if (o->precision == RPM_FP32) {
        Shapes<float> s = make_shapes<float>(n, spectral_comps(o));
        if (!s.ok || !make_shapes<double>(n, spectral_comps(o)).ok) return RPM_E_UNSUPPORTED_SIZE;
        *bytes = make_layout<float>(s, o).total;
    } else {
        return RPM_E_INVALID;
    }
    return RPM_OK;
}

rpm_status rpm_fft_apply(const rpm_problem* pr, const double E[6], const rpm_options* o, const void* eps, void* xi,
                         double* err, double sig_avg[6], void* workspace, size_t ws_bytes, void* hip_stream)
{
    rpm_status rs = validate(pr, o);
    if (rs != RPM_OK) return rs;
    if (!E || !finite6(E) || !eps || !xi || eps == xi) return RPM_E_INVALID;
    if (o->precision == RPM_FP64)
        return apply_typed<double>(pr, E, o, eps, xi, err, sig_avg, workspace, ws_bytes, hip_stream);
    return apply_typed<float>(pr, E, o, eps, xi, err, sig_avg, workspace, ws_bytes, hip_stream);
}

rpm_status rpm_fft_autotune(const rpm_problem* pr, const rpm_options* o, int32_t reps, rpm_tuning* best,
                            double* best_ms, int32_t* candidates, void* workspace, size_t ws_bytes, void* hip_stream)
{
    rpm_status rs = validate(pr, o);
    if (rs != RPM_OK) return rs;
    if (!best || reps < 1 || reps > 1000) return RPM_E_INVALID;
    if (o->precision == RPM_FP64)
        return tune_typed<double>(pr, o, reps, best, best_ms, candidates, workspace, ws_bytes, hip_stream);
    return tune_typed<float>(pr, o, reps, best, best_ms, candidates, workspace, ws_bytes, hip_stream);
}

rpm_status rpm_fft_apply_static(const rpm_problem* pr, const double E[6], const rpm_options* o, const void* eps,
                                void* xi, double* err, double sig_avg[6], void* hip_stream)
{
    rpm_status rs = validate(pr, o);
    if (rs != RPM_OK) return rs;
    if (!E || !finite6(E) || !eps || !xi || eps == xi) return RPM_E_INVALID;
    // the size check needs no device: reject before touching the scratch
    {
        rpm_options b = *o;
        b.scheme = RPM_SCHEME_BASIC;
        size_t need = 0;
        if (o->precision == RPM_FP64) {
            Shapes<double> s = make_shapes<double>(pr->n, spectral_comps(o));
            if (!s.ok) return RPM_E_UNSUPPORTED_SIZE;
            need = make_layout<double>(s, &b, true).total;
        } else {
            Shapes<float> s = make_shapes<float>(pr->n, spectral_comps(o));
            if (!s.ok) return RPM_E_UNSUPPORTED_SIZE;
            need = make_layout<float>(s, &b, true).total;
        }
        if (need > RPM_STATIC_SCRATCH_BYTES) return RPM_E_SCRATCH;
    }
    void* ws = nullptr;
    if ((rs = static_scratch(&ws)) != RPM_OK) return rs;
    rpm_options b = *o;
    b.profile = 0;  // no event objects either
    if (o->precision == RPM_FP64)
        return apply_typed<double>(pr, E, &b, eps, xi, err, sig_avg, ws, RPM_STATIC_SCRATCH_BYTES, hip_stream, true);
    return apply_typed<float>(pr, E, &b, eps, xi, err, sig_avg, ws, RPM_STATIC_SCRATCH_BYTES, hip_stream, true);
}

rpm_status rpm_fft_solve(const rpm_problem* pr, const double E[6], const rpm_options* o, const void* eps0,
                         void* eps_out, void* sig_out, double sig_avg[6], rpm_stats* st, void* workspace,
                         size_t ws_bytes, void* hip_stream)
{
    rpm_status rs = validate(pr, o);
    if (rs != RPM_OK) return rs;
    if (!E || !finite6(E)) return RPM_E_INVALID;
    if (o->precision == RPM_FP64)
        return solve_typed<double>(pr, E, o, eps0, eps_out, sig_out, sig_avg, st, workspace, ws_bytes, hip_stream);
    return solve_typed<float>(pr, E, o, eps0, eps_out, sig_out, sig_avg, st, workspace, ws_bytes, hip_stream);
}

rpm_status rpm_fft_effective_tensor(const rpm_problem* pr, const rpm_options* o, double* C_eff, rpm_stats* st,
                                    void* workspace, size_t ws_bytes, void* hip_stream)
{
    rpm_status rs = validate(pr, o);
    if (rs != RPM_OK) return rs;
    if (!C_eff) return RPM_E_INVALID;
    if (o->batch_cases && o->scheme == RPM_SCHEME_RPM && o->p_max > 0) {
        if (o->precision == RPM_FP64) return eff_batched<double>(pr, o, C_eff, st, workspace, ws_bytes, hip_stream);
        return eff_batched<float>(pr, o, C_eff, st, workspace, ws_bytes, hip_stream);
    }
    if (o->precision == RPM_FP64) return eff_typed<double>(pr, o, C_eff, st, workspace, ws_bytes, hip_stream);
    return eff_typed<float>(pr, o, C_eff, st, workspace, ws_bytes, hip_stream);
}

rpm_status rpm_fft_seed_basis(const rpm_problem* pr, const rpm_options* o, const void* V, int32_t p0, int32_t* p_out,
                              void* workspace, size_t ws_bytes, void* hip_stream)
{
    rpm_status rs = validate(pr, o);
    if (rs != RPM_OK) return rs;
    if (p0 < 0 || (p0 > 0 && !V) || o->scheme != RPM_SCHEME_RPM) return RPM_E_INVALID;
    if (o->precision == RPM_FP64) return seed_typed<double>(pr, o, V, p0, p_out, workspace, ws_bytes, hip_stream);
    return seed_typed<float>(pr, o, V, p0, p_out, workspace, ws_bytes, hip_stream);
}

rpm_status rpm_fft_solve_stress(const rpm_problem* pr, const double Sigma[6], const rpm_options* o, void* eps_out,
                                void* sig_out, double sig_avg[6], double E_out[6], rpm_stats* st, void* workspace,
                                size_t ws_bytes, void* hip_stream)
{
    rpm_status rs = validate(pr, o);
    if (rs != RPM_OK) return rs;
    if (!Sigma || !finite6(Sigma)) return RPM_E_INVALID;
    if (o->precision == RPM_FP64)
        return stress_typed<double>(pr, Sigma, o, eps_out, sig_out, sig_avg, E_out, st, workspace, ws_bytes,
                                    hip_stream);
    return stress_typed<float>(pr, Sigma, o, eps_out, sig_out, sig_avg, E_out, st, workspace, ws_bytes, hip_stream);
}

rpm_status rpm_workspace_basis_dim(const void* workspace, size_t ws_bytes, int32_t* p, void* hip_stream)
{
    if (!workspace || !p || ws_bytes < sizeof(DevState)) return RPM_E_INVALID;
    DevState hs;
    if (hipMemcpyAsync(&hs, workspace, sizeof(DevState), hipMemcpyDeviceToHost, (hipStream_t)hip_stream) !=
        hipSuccess)
        return RPM_E_HIP;
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return RPM_E_HIP;
    *p = hs.magic == kStateMagic ? hs.p : 0;
    return RPM_OK;
}

rpm_status rpm_workspace_h(const void* workspace, size_t ws_bytes, double* H, int32_t ld, int32_t* p,
                           void* hip_stream)
{
    if (!workspace || !H || !p || ld < 1 || ws_bytes < sizeof(DevState)) return RPM_E_INVALID;
    DevState hs;
    if (hipMemcpyAsync(&hs, workspace, sizeof(DevState), hipMemcpyDeviceToHost, (hipStream_t)hip_stream) !=
        hipSuccess)
        return RPM_E_HIP;
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) return RPM_E_HIP;
    const int pp = hs.magic == kStateMagic ? hs.p : 0;
    if (pp > ld) return RPM_E_INVALID;
    for (int i = 0; i < pp; ++i)
        for (int j = 0; j < pp; ++j) H[(long long)i * ld + j] = hs.H[i * kMaxP + j];
    *p = pp;
    return RPM_OK;
}

const char* rpm_status_string(rpm_status s)
{
    switch (s) {
        case RPM_OK: return "RPM_OK";
        case RPM_NOT_CONVERGED: return "RPM_NOT_CONVERGED";
        case RPM_DIVERGED: return "RPM_DIVERGED";
        case RPM_SINGULAR: return "RPM_SINGULAR";
        case RPM_E_INVALID: return "RPM_E_INVALID";
        case RPM_E_UNSUPPORTED_SIZE: return "RPM_E_UNSUPPORTED_SIZE";
        case RPM_E_WORKSPACE: return "RPM_E_WORKSPACE";
        case RPM_E_HIP: return "RPM_E_HIP";
        case RPM_E_SCRATCH: return "RPM_E_SCRATCH";
    }
    return "RPM_UNKNOWN";
}

}  // extern "C"
