/*
 * rpmfft.h -- C ABI of the MI355X (gfx950) RPM-FFT solver.
 *
 * The solver computes the strain and stress fields in a periodic cell of a
 * heterogeneous linear-elastic solid for a prescribed mean strain, and the
 * effective stiffness, following Peng, Nepal & Dayal, "Effective Response of
 * Heterogeneous Materials using the Recursive Projection Method", CMAME 364
 * (2020):
 *   - the cell problem and the mean/fluctuation split of Sec. 2;
 *   - the Lippmann-Schwinger fixed-point map of Algorithm 1 and the operator
 *     F of Sec. 3 (stress C(x):eps, forward FFT, reference-medium Green
 *     operator at every non-zero frequency, mean strain at k = 0, inverse
 *     FFT), with the equilibrium error of Algorithm 1;
 *   - the Recursive Projection Method of Sec. 3 / Algorithm 2 around it
 *     (projection on the basis Z, Newton on the unstable subspace with
 *     H = Z^T F_u Z, fixed point on the complement, basis growth In(q, Z)).
 *
 * Conventions
 *   - Grid n = {nx, ny, nz}; nz == 1 is 2-D plane strain.  Every extent is a
 *     product of 2s and 3s between 2 and 512 (nz may also be 1).
 *   - Fields are real arrays [6][nz][ny][nx] (x fastest) in the working
 *     precision (double for RPM_FP64, float for RPM_FP32), tensor components
 *     in the order xx, yy, zz, yz, xz, xy with tensor (not engineering)
 *     shear.  The mean strain E[6] uses the same components.
 *   - The phase map is uint8 [nz][ny][nx]; phase p has Lame constants
 *     lame[2p], lame[2p+1] (lambda, mu).  The reference medium is isotropic
 *     (lambda0, mu0).
 *   - The equilibrium error is sqrt(<|div sigma|^2>)/|<sigma>| with the
 *     divergence in voxel units (wave vectors in radians per voxel) and the
 *     Frobenius norm; in 2-D the norm of <sigma> uses the in-plane part.
 *   - Inner products between fields (projections, Gram-Schmidt) are
 *     Frobenius sums over voxels.
 *
 * Memory and ownership
 *   - Pointers documented as DEVICE point to GPU memory the caller owns
 *     (e.g. torch tensors); HOST pointers to host memory.  The library never
 *     allocates device memory: all scratch lives in the caller's workspace,
 *     sized by rpm_workspace_size.  The workspace also carries state between
 *     calls (the basis Z, W = F_u Z and H), so consecutive solves on the same
 *     workspace can reuse the basis (F_u does not depend on E).
 *   - All device work is enqueued on the caller's HIP stream (NULL = the
 *     default stream); every entry point returns after that work completed.
 *   - Calls on different workspaces are independent; calls that share a
 *     workspace must not overlap.
 *
 * Errors
 *   - Negative codes are returned before any device work and leave outputs
 *     untouched.  RPM_NOT_CONVERGED, RPM_DIVERGED and RPM_SINGULAR fill the
 *     outputs from the last iterate and the statistics.
 */
#ifndef RPMFFT_H
#define RPMFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Launch shape of the y and gamma pencil passes of one grid and precision
 * (the batched, uneven-grid workloads of the paper's benchmark families run
 * many grids; the best shape differs between them).  A field of 0 keeps the
 * library's default.  The shapes do not change a result: every element is
 * transformed with the same arithmetic; only the grouping of the per-block
 * error partial sums follows gamma_blocks.  y_regs changes the factorisation
 * of the y transforms, so their rounding.
 *   y_cols        z positions per y-pass tile: a divisor of nz, at most
 *                 128 / (2 sizeof(real)) and 8 x 256 / ny; other values make
 *                 the calls that use the tuning return RPM_E_INVALID
 *   y_blocks      workgroups of the persistent y passes (>= 1)
 *   gamma_blocks  workgroups of the persistent gamma pass (>= 1)
 *   y_regs        1: the 128-point y transforms held in registers, a row per
 *                 16 lanes, exchanged across lanes by DPP moves, without LDS
 *                 (FP32 fields, ny = 128, 3-D, nz a multiple of 16, y_cols
 *                 0 or 16, y_blocks 0; elsewhere RPM_E_INVALID); 0: the LDS
 *                 passes                                                   */
typedef struct rpm_tuning_s {
    int32_t y_cols;
    int32_t y_blocks;
    int32_t gamma_blocks;
    int32_t y_regs;
} rpm_tuning;

typedef enum {
    RPM_OK = 0,                 /* error <= tol                                  */
    RPM_NOT_CONVERGED = 1,      /* max_iter main-loop F applications reached     */
    RPM_DIVERGED = 2,           /* non-finite error or error > 1e6 x initial     */
    RPM_SINGULAR = 3,           /* I - H has a pivot below 1e-14 max|I - H|      */
    RPM_E_INVALID = -1,         /* bad argument (null pointer, range, NaN ...)   */
    RPM_E_UNSUPPORTED_SIZE = -2,/* an extent is not a 2,3-smooth size <= 512     */
    RPM_E_WORKSPACE = -3,       /* workspace missing or smaller than required    */
    RPM_E_HIP = -5,             /* a HIP runtime call failed                     */
    RPM_E_SCRATCH = -6          /* rpm_fft_apply_static: the grid needs more than
                                   the library's static device scratch          */
} rpm_status;

enum { RPM_SCHEME_BASIC = 0, /* Algorithm 1: eps <- F(eps)                       */
       RPM_SCHEME_RPM = 1 }; /* Algorithm 2                                      */

enum { RPM_MAP_LS = 0,             /* the Lippmann-Schwinger map F (Algorithm 1)  */
       RPM_MAP_POLARIZATION = 1 };  /* the polarization iteration of Algorithm 3
                                       (Sec. 5.5; Accelerated FFT for
                                       alpha = beta = 2) with the C0 term of s_b
                                       taken as -beta C0:eps                      */

enum { RPM_FP64 = 0,         /* fields, FFTs and Z in double                     */
       RPM_FP32 = 1 };       /* fields, FFTs, Z and W in float; reductions,
                                norms, Gram-Schmidt, the compatible projection
                                of new basis columns, the Jacobian-vector
                                products that form H, H and the Newton solve in
                                double                                            */

/* kernel classes of rpm_stats.kernel_* (profile = 1) */
enum { RPM_K_XFWD = 0, RPM_K_YFWD, RPM_K_GAMMA, RPM_K_YINV, RPM_K_XINV, RPM_K_REDUCE, RPM_K_FINAL,
       RPM_K_GROWTH, RPM_K_PROJECT, RPM_K_RECOMBINE, RPM_NKERNEL };

typedef struct {
    int32_t n[3];             /* nx, ny, nz                                      */
    const uint8_t *phase;     /* DEVICE [nz][ny][nx] phase labels                */
    int32_t n_phases;         /* 1..256                                          */
    const double *lame;       /* HOST [n_phases][2] (lambda, mu), mu >= 0,
                                 3 lambda + 2 mu >= 0                            */
    double lame0[2];          /* reference medium (lambda0, mu0), mu0 > 0,
                                 3 lambda0 + 2 mu0 > 0                           */
} rpm_problem;

typedef struct {
    double tol;               /* stop when the equilibrium error <= tol (> 0)   */
    int32_t max_iter;         /* cap on main-loop F applications (>= 1)         */
    int32_t n_max;            /* fixed-point count before the basis grows (>=1)*/
    int32_t p_max;            /* basis cap, 0..64 (0 with RPM = Algorithm 1)    */
    double kappa;             /* add one column when T22 <= kappa T11 (0..1)    */
    int32_t scheme;           /* RPM_SCHEME_BASIC or RPM_SCHEME_RPM              */
    int32_t precision;        /* RPM_FP64 or RPM_FP32                            */
    int32_t reuse_basis;      /* keep Z, W, H left in the workspace by the
                                 previous call on the same grid, precision,
                                 p_max and map (else start from an empty basis;
                                 max_iter may differ).  The basis holds the
                                 linear part of that call's map: a call with
                                 another reference medium, phase table,
                                 alpha/beta or phase map (a checksum of it) also
                                 starts from an empty basis                      */
    int32_t check_every;      /* host reads the convergence flag every this many
                                 iterations (>= 1); iterations queued after
                                 convergence do nothing                          */
    const int32_t *replay;    /* HOST, nullable: forced number of columns (0, 1
                                 or 2) at each growth event, in order            */
    int32_t replay_len;
    int32_t profile;          /* record per-kernel-class times with HIP events */
    int32_t refine;           /* RPM_FP32 only: at most this many FP64
                                 refinement sweeps (0 = certify only).  With
                                 refine > 0 the FP32 stage stops at
                                 max(tol, 1e-5); while the FP64 evaluation of
                                 the field misses tol, delta = F_u delta + g is
                                 solved in FP32 (g = FP64 fixed-point residual,
                                 basis reused) and added to an FP64 iterate;
                                 the status then reflects the FP64 error       */
    double refine_tol;        /* correction solves stop at |G(d) - d| <=
                                 refine_tol |g| (0 < refine_tol < 1)           */
    int32_t map;              /* RPM_MAP_LS or RPM_MAP_POLARIZATION: the fixed-
                                 point operation of both schemes (Sec. 5.5: RPM
                                 around the polarization iteration)              */
    double alpha, beta;       /* polarization parameters (> 0; default 2, 2)     */
    int32_t profile_classes;  /* with profile = 1: the kernel classes timed, bit
                                 k for class k (< 1 << RPM_NKERNEL); 0 = every
                                 class.  Fewer classes, fewer event records
                                 between the kernels of the timed solve.         */
    int32_t stall_window;     /* RPM_FP32 with refine > 0: the FP32 stage (and
                                 each correction solve) also stops when its
                                 error has not fallen below 0.9 x its lowest
                                 value for this many iterations (FP32 rounding
                                 floor); refinement then continues from that
                                 field.  0 = never (>= 0)                        */
    int32_t batch_cases;      /* rpm_fft_effective_tensor with RPM: solve the
                                 unit load cases together, one pass over the
                                 basis serving all of them per step (shared Z,
                                 W, H), growing it from the differences of the
                                 case with the largest error (1) or of every
                                 case still iterating, largest error first (2);
                                 the workspace must be sized with a non-zero
                                 value.  0 = one case after the other            */
    int32_t graph;            /* 1 = launch each main-loop iteration as a
                                 captured HIP graph (one per ring slot,
                                 recaptured when the basis grows; ignored with
                                 profile = 1 or a NULL stream, which cannot be
                                 captured); 0 = kernel by kernel                 */
    int32_t profile_every;    /* with profile = 1: events around one launch in
                                 every this many of each class (the
                                 profile_every-th, the 2 profile_every-th, ...),
                                 so a long timed solve carries few event
                                 records; 0 or 1 = every launch (>= 0)           */
    const struct rpm_tuning_s *tuning; /* HOST, nullable: launch shape of the
                                 pencil passes (rpm_fft_autotune); NULL = the
                                 library's defaults.  The workspace size does
                                 not depend on it.                               */
} rpm_options;

typedef struct {
    int32_t iterations;       /* main-loop F applications, the initial included */
    int32_t jvps;             /* F applications for H (one per basis column)     */
    int32_t basis_dim;        /* p at exit                                       */
    int32_t growth_events;
    double residual;          /* equilibrium error of the returned strain        */
    double seconds;           /* wall time of the call                           */
    double *history;          /* HOST, nullable: error after each main F call    */
    int32_t history_cap;
    int32_t *decisions;       /* HOST, nullable: columns added at each growth    */
    int32_t decisions_cap;
    double kernel_ms[RPM_NKERNEL];     /* summed HIP-event times (profile = 1)  */
    int32_t kernel_launches[RPM_NKERNEL];
    double kernel_bytes[RPM_NKERNEL];  /* summed algorithmic HBM bytes of those
                                          launches: every input read once and
                                          every output written once (profile=1) */
    double residual_fp64;     /* equilibrium error evaluated in FP64 of the FP64
                                 field behind the outputs (RPM_FP32: after
                                 refinement; RPM_FP64: equals residual)          */
    int32_t refinements;      /* refinement sweeps performed                      */
} rpm_stats;

/* Default options: tol 1e-6, max_iter 10000, n_max 10 (the near-optimal value
 * of Sec. 5.2), p_max 32, kappa 0.1, RPM, FP64, no reuse, check_every 16,
 * refine 4, refine_tol 1e-3, the Lippmann-Schwinger map, alpha = beta = 2,
 * no profiling (profile_classes 0, profile_every 1), stall_window 400,
 * batch_cases 0, graph 0. */
void rpm_default_options(rpm_options *o);

/* Lame constants (lambda, mu) of an isotropic phase from Young's modulus E and
 * Poisson's ratio nu (nu < 1/2).  Returns RPM_E_INVALID for nu >= 1/2 or
 * non-finite input. */
rpm_status rpm_lame_from_young(double E, double nu, double *lam, double *mu);

/* Bytes of device workspace needed for grid n under options o.
 * RPM_E_UNSUPPORTED_SIZE when an extent is not 2,3-smooth in [2, 512] (nz may
 * be 1), or when a pencil pass would not fit its LDS tile: with the
 * polarization map the z (2-D: y) pencils carry 12 components, which bounds
 * their length to 144 in FP64 and, since FP32 fields are certified in FP64,
 * in FP32 as well. */
rpm_status rpm_workspace_size(const int32_t n[3], const rpm_options *o, size_t *bytes);

/*
 * One application of the fixed-point map (the iteration body of Algorithm 1):
 * xi = F(eps; E) and the equilibrium error of eps, <sigma> = <C(x):eps>.
 * eps, xi: DEVICE fields in o->precision (may not alias).  err, sig_avg: HOST
 * (nullable).
 */
rpm_status rpm_fft_apply(const rpm_problem *pr, const double E[6], const rpm_options *o, const void *eps, void *xi,
                         double *err, double sig_avg[6], void *workspace, size_t ws_bytes, void *hip_stream);

/*
 * Tile autotuner of the pencil passes: times the fixed-point map of the
 * iteration body of Algorithm 1 (from the uniform strain, on the workspace's
 * own fields) under candidate launch shapes and returns the fastest.  One
 * coordinate at a time, in this order, each from the best so far: y_cols over
 * the admissible divisors of nz (largest first, at most four), then y_blocks
 * and gamma_blocks over 256 x {1, 2, 3, 4, 5, 6, 8} capped at the number of
 * tiles; 0 is tried first for each (the default).  Each candidate: one
 * untimed map, then reps maps between HIP events.
 *   reps      1 .. 1000
 *   best      HOST: the fastest shape (fields of 0 where the default won)
 *   best_ms   HOST nullable: its time per map application
 *   candidates HOST nullable: number of shapes timed
 * o->tuning is ignored.  The workspace holds rpm_workspace_size(n, o) bytes;
 * its fields are overwritten and any basis it holds is dropped, so tune before
 * the solves that would carry a basis in it (reuse_basis).
 * Errors as rpm_fft_apply; RPM_E_INVALID for reps out of range or NULL best.
 */
rpm_status rpm_fft_autotune(const rpm_problem *pr, const rpm_options *o, int32_t reps, rpm_tuning *best,
                            double *best_ms, int32_t *candidates, void *workspace, size_t ws_bytes,
                            void *hip_stream);

/*
 * Solve the cell problem for the mean strain E (Sec. 2) with Algorithm 1 or
 * Algorithm 2 until the equilibrium error of the iterate is <= tol.  With
 * RPM_FP32 the converged field is re-evaluated in FP64 (certification) and,
 * if needed, refined (rpm_options.refine); sig_avg then comes from the FP64
 * field and eps_out is that field rounded to float.
 *   eps0     DEVICE nullable: starting strain (its mean is replaced by E by
 *            the first application of F); NULL starts from the uniform E.
 *   eps_out  DEVICE nullable: the iterate whose error met tol (the input of
 *            the last F application).
 *   sig_out  DEVICE nullable: C(x):eps_out.
 *   sig_avg  HOST nullable: <sigma> of eps_out.
 *   st       HOST nullable: statistics.
 */
rpm_status rpm_fft_solve(const rpm_problem *pr, const double E[6], const rpm_options *o, const void *eps0,
                         void *eps_out, void *sig_out, double sig_avg[6], rpm_stats *st, void *workspace,
                         size_t ws_bytes, void *hip_stream);

/*
 * Effective stiffness (the effective response of the title): one solve per
 * unit mean strain, columns in Voigt order 11, 22, 33, 23, 13, 12 with
 * engineering shear (a shear load case has eps_ab = eps_ba = 1/2), so that
 * <sigma> = C_eff gamma.  3-D: C_eff is 6x6 (36 doubles, row major); 2-D
 * (nz == 1): 3x3 over 11, 22, 12 (9 doubles).  Z, W and H carry over from one
 * load case to the next when o->reuse_basis is set (F_u does not depend on E).
 *   C_eff  HOST (36 or 9 doubles);  st  HOST nullable, 6 (or 3) entries.
 */
rpm_status rpm_fft_effective_tensor(const rpm_problem *pr, const rpm_options *o, double *C_eff, rpm_stats *st,
                                    void *workspace, size_t ws_bytes, void *hip_stream);

/*
 * Seed the unstable-subspace basis of a workspace (a warm start of Z for the
 * next rpm_fft_solve / rpm_fft_effective_tensor with reuse_basis set; Sec. 3:
 * any orthonormal Z with H = Z^T F_u Z serves the Newton step).  Each vector
 * goes through the steps basis growth (Algorithm 2, In(q, Z)) applies to a
 * difference of iterates: normalised, projected onto zero-mean compatible
 * fields (Lippmann-Schwinger map), re-orthogonalised twice against the basis
 * and dropped if its norm falls to 1e-10 or below, then one Jacobian-vector
 * product for its column of W and its border of H.  Columns are appended to
 * the basis the workspace holds when o->reuse_basis is set (else to an empty
 * one), up to o->p_max; o->scheme must be RPM_SCHEME_RPM.
 *   V      DEVICE [p0][6][N] fields in o->precision (read only; may be NULL
 *          when p0 == 0).
 *   p_out  HOST nullable: the basis dimension afterwards.
 * Errors: RPM_E_INVALID for p0 < 0, a NULL V with p0 > 0 or the basic scheme,
 * before any device work.
 */
rpm_status rpm_fft_seed_basis(const rpm_problem *pr, const rpm_options *o, const void *V, int32_t p0, int32_t *p_out,
                              void *workspace, size_t ws_bytes, void *hip_stream);

/*
 * Solve the cell problem for a prescribed mean stress Sigma (Sec. 2: the
 * average strain or stress is given).  The problem is linear, so it is the
 * strain-controlled problem for the mean strain E with C_eff E = Sigma: the
 * effective stiffness comes from one solve per unit mean strain (as
 * rpm_fft_effective_tensor, the basis carried from one case to the next),
 * then E from C_eff (Voigt, engineering shear; 2-D plane strain over 11, 22,
 * 12, Sigma_33 then being the reaction), then the strain-controlled solve for E.
 *   Sigma  HOST 6 tensor components (11, 22, 33, 23, 13, 12).
 *   eps_out, sig_out  DEVICE nullable, as rpm_fft_solve.
 *   sig_avg, E_out    HOST nullable: <sigma> of eps_out and the mean strain E.
 *   st     HOST nullable: 7 entries in 3-D (4 in 2-D): the unit load cases,
 *          then the final solve.
 * Returns the first non-OK status of the solves, RPM_SINGULAR when C_eff is
 * singular (pivot below 1e-14 of its largest entry; no final solve), or a
 * negative code before any device work.
 */
rpm_status rpm_fft_solve_stress(const rpm_problem *pr, const double Sigma[6], const rpm_options *o, void *eps_out,
                                void *sig_out, double sig_avg[6], double E_out[6], rpm_stats *st, void *workspace,
                                size_t ws_bytes, void *hip_stream);

/*
 * rpm_fft_apply without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same map application, the same kernels and launch
 * shapes, with the scratch (spectra, partial sums, solver state) taken from a
 * static device array of RPM_STATIC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends.  Calls no hipMalloc/hipFree.
 *   eps, xi   DEVICE fields in o->precision on the CURRENT device, whose stream
 *             hip_stream must be (may not alias).
 *   err, sig_avg  HOST nullable, as rpm_fft_apply.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (the state it needs is re-initialised on every call): calls that
 * overlap on one GPU, on any streams, race.  Returns RPM_E_SCRATCH, before any
 * device work, when the grid needs more scratch than the array holds (128^3
 * FP32 fits; 128^3 FP64 does not); other errors as rpm_fft_apply.
 */
#define RPM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
rpm_status rpm_fft_apply_static(const rpm_problem *pr, const double E[6], const rpm_options *o, const void *eps,
                                void *xi, double *err, double sig_avg[6], void *hip_stream);

/* Current basis dimension stored in a workspace (0 if never used).  HOST p. */
rpm_status rpm_workspace_basis_dim(const void *workspace, size_t ws_bytes, int32_t *p, void *hip_stream);

/* The reduced matrix H = Z^T F_u Z of the basis a workspace holds (Sec. 3:
 * the Jacobian of the map restricted to the unstable subspace, bordered by one
 * row and column per added column): HOST H receives p x p doubles, row major
 * with leading dimension ld (>= p; at most ld x ld are written), HOST p the
 * basis dimension (0 if the workspace was never used). */
rpm_status rpm_workspace_h(const void *workspace, size_t ws_bytes, double *H, int32_t ld, int32_t *p,
                           void *hip_stream);

/* Static string naming a status code. */
const char *rpm_status_string(rpm_status s);

#ifdef __cplusplus
}
#endif

#endif /* RPMFFT_H */
