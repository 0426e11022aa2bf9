/*
 * rpmfno.h -- C ABI of the learned warm start of the MI355X RPM-FFT solver.
 *
 * A Fourier-neural-operator-style network maps the stiffness field of a cell
 * to the strain fluctuation of the six unit load cases (the localization
 * tensor).  A solve for the mean strain E then starts (rpm_fft_solve's eps0)
 * from E plus the predicted fluctuation instead of the uniform E with which
 * Algorithm 2 of Peng, Nepal & Dayal (CMAME 2020) starts; the iteration and its
 * equilibrium error still decide when the result is accepted, so a poor
 * prediction only costs iterations.  The network is not part of the paper.
 *
 * Network (x: per-voxel features, C = width, L = layers, m = modes):
 *   h_0     = W_lift x + b_lift
 *   h_{l+1} = gelu(W_l h_l + b_l + K_l h_l),  l < L
 *   y       = W_proj h_L + b_proj
 *   K_l h   = (1/N) Re sum_k exp(+2 pi i k.x/n) R_l(k) sum_x' exp(-2 pi i k.x'/n) h(x'),
 * k over the m^3 signed frequencies {-m/2 .. m/2 - 1}^3, R_l(k) complex C x C.
 * Every contraction runs on the matrix cores with bfloat16 operands (weights
 * and activations rounded to bfloat16 when loaded) and FP32 accumulation.
 *
 * Layouts: fields are [batch][channels][nz][ny][nx] FP32 (x fastest).
 * Parameters are one FP32 array (rpm_fno_param_count floats): W_lift [C][c_in],
 * b_lift [C], then per layer W_l [C][C], b_l [C], Re R_l [m^3][C][C],
 * Im R_l [m^3][C][C] (frequency index (kz, ky, kx), each kk = k + m/2, kx
 * fastest), then W_proj [c_out][C], b_proj [c_out].
 *
 * Pointers marked DEVICE are GPU memory owned by the caller; the library never
 * allocates device memory (workspace from rpm_fno_workspace_size).  Work runs
 * on hip_stream; every call returns after it completed.  Errors as rpmfft.h:
 * negative codes before any device work.
 */
#ifndef RPMFNO_H
#define RPMFNO_H

#include <stddef.h>
#include <stdint.h>

#include "rpmfft.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t c_in;    /* input channels (2 for the warm start: stiffness, Poisson)  */
    int32_t c_out;   /* output channels (36 for the warm start: six unit load
                        cases x six strain components, case-major)              */
    int32_t width;   /* hidden channels C (1..256)                                */
    int32_t layers;  /* spectral layers L (0..16)                                 */
    int32_t modes;   /* retained signed frequencies per axis m (1..32)           */
} rpm_fno_config;

/* The matrix-core product every contraction of the network uses, exposed
 * on its own: C[b] = alpha A[b] B[b] + beta C[b] for b < batch, element (i, k)
 * of A[b] at A + b sA[0] + i sA[1] + k sA[2] (B: (k, j) with sB[0..2]; C:
 * (i, j) with sC[0..2]), strides in elements (transposes and complex planes
 * are strides).  A and B are rounded to bfloat16 (nearest even) when loaded,
 * products accumulate in FP32; beta == 0 does not read C.  A, B, C: DEVICE
 * FP32.  RPM_E_INVALID for M, N, K < 1, batch outside 1..65535. */
rpm_status rpm_gemm_bf16(int32_t M, int32_t N, int32_t K, int32_t batch, const float *A, const int64_t sA[3],
                         const float *B, const int64_t sB[3], float *C, const int64_t sC[3], float alpha, float beta,
                         void *hip_stream);

/* Number of FP32 parameters.  RPM_E_INVALID for an out-of-range config. */
rpm_status rpm_fno_param_count(const rpm_fno_config *cfg, int64_t *count);

/* Workspace bytes for a grid n = {nx, ny, nz} and a batch of fields. */
rpm_status rpm_fno_workspace_size(const rpm_fno_config *cfg, const int32_t n[3], int32_t batch, size_t *bytes);

/* Initial parameters from a counter-based generator (splitmix64 of seed):
 * pointwise weights uniform in +-1/sqrt(fan_in), biases 0, spectral weights
 * uniform in [0, 1/C^2).  params: DEVICE. */
rpm_status rpm_fno_init(const rpm_fno_config *cfg, uint64_t seed, float *params, void *hip_stream);

/* y = network(x) for a batch.  x: DEVICE [batch][c_in][N]; y: DEVICE
 * [batch][c_out][N] (nullable: the output stays in the workspace).  The
 * activations stay in the workspace for rpm_fno_backward. */
rpm_status rpm_fno_forward(const rpm_fno_config *cfg, const float *params, const int32_t n[3], int32_t batch,
                           const float *x, float *y, void *workspace, size_t ws_bytes, void *hip_stream);

/* Gradient of sum(dy . y) with respect to the parameters (grad, DEVICE,
 * param_count floats, overwritten) and to the input (dx, DEVICE nullable
 * [batch][c_in][N]), for the x of the preceding rpm_fno_forward call on the
 * same workspace, grid and batch. */
rpm_status rpm_fno_backward(const rpm_fno_config *cfg, const float *params, const int32_t n[3], int32_t batch,
                            const float *x, const float *dy, float *grad, float *dx, void *workspace, size_t ws_bytes,
                            void *hip_stream);

/* One training step on a batch: forward, the mean over all outputs of
 * w (y - target)^2 with w = 10^(3 x0) from the first input feature (for the
 * warm-start features: the voxel's stiffness relative to the stiffest phase,
 * so strains inside pores, which carry no stress, hardly count; target
 * DEVICE, as y), backward, Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning
 * rate lr, step >= 1 for the bias correction) on params with the moment arrays
 * adam_m, adam_v (DEVICE, param_count floats each, zero before step 1).  grad:
 * DEVICE scratch of param_count floats.  loss: HOST nullable, the error before
 * the update. */
rpm_status rpm_fno_train_step(const rpm_fno_config *cfg, float *params, float *grad, float *adam_m, float *adam_v,
                              int32_t step, float lr, const int32_t n[3], int32_t batch, const float *x,
                              const float *target, double *loss, void *workspace, size_t ws_bytes, void *hip_stream);

/* Warm-start features of a cell (c_in = 2): x[0] = max(log10(E/E_max), -3)/3,
 * E the Young modulus of the voxel's phase and E_max that of the stiffest
 * phase of the table, x[1] = nu - 0.3.  x: DEVICE [2][N]; pr as rpmfft.h
 * (the reference medium is not used). */
rpm_status rpm_fno_features(const rpm_problem *pr, float *x, void *hip_stream);

/* Starting strain for rpm_fft_solve: eps0 = E + sum_j g_j y_j with y the
 * network output for the cell's features (c_in = 2, c_out = 36: the strain
 * fluctuation of unit load case j in channels 6j .. 6j+5, Voigt order 11, 22,
 * 33, 23, 13, 12 with engineering shear, so g_j = E_j for j < 3 and 2 E_j
 * otherwise).  eps0: DEVICE [6][N] in precision (RPM_FP64 or RPM_FP32);
 * workspace for batch 1 on the cell's grid. */
rpm_status rpm_fno_warm_start(const rpm_fno_config *cfg, const float *params, const rpm_problem *pr,
                              const double E[6], int32_t precision, void *eps0, void *workspace, size_t ws_bytes,
                              void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RPMFNO_H */
