/* Kernels of the learned warm start x0 = s * MLP(theta): a network 12 ->
 * 256 -> 256 -> n with ReLU after the hidden layers, trained with a mean
 * squared error on solutions that iccg_solve produced (scaled by 1/s) and
 * Adam.  Not part of the paper's method: a start vector for CG, whose
 * result still has to pass the solver's own residual test.
 *
 * Conventions.  All matrices are row-major, all pointers are device memory
 * unless stated, and every call is asynchronous on stream (a hipStream_t,
 * NULL = default stream).  dtype is the compute type of the products and of
 * the stored activations, weights copies and targets:
 *   MLP_BF16 -- 16-bit bfloat storage (round to nearest even), products on
 *               the matrix cores with FP32 accumulation;
 *   MLP_F32  -- FP32 storage and FP32 matrix-core products (for checking).
 * Master weights, gradients and Adam moments are FP32.  A layer maps X [M][K]
 * to X W + b with W [K][N] (in features x out features) and b [N].
 * Return: HBMC_OK, or HBMC_EINVAL (bad sizes, dtype, layout, null pointer)
 * or HBMC_EHIP; hbmc_last_error() gives the message.
 */
#ifndef HBMC_MLP_H
#define HBMC_MLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLP_BF16 0
#define MLP_F32 1

/* Layout of the operands of C = A B (logical A [M][K], B [K][N]):
 *   MLP_NN: A stored [M][K] (lda >= K), B stored [K][N] (ldb >= N);
 *   MLP_TN: A stored transposed, [K][M] (lda >= M) -- for X^T dY;
 *   MLP_NT: B stored transposed, [N][K] (ldb >= K) -- for dY W^T. */
#define MLP_NN 0
#define MLP_TN 1
#define MLP_NT 2

/* C = A B in FP32, C [M][N] with row stride ldc.  nsplit > 1 splits K into
 * nsplit ranges and writes nsplit partial products to C + z * M * ldc
 * (z = 0 .. nsplit-1; C must hold nsplit * M * ldc floats); mlp_sum_rows
 * adds them in a fixed order.  HBMC_EINVAL for an unknown layout or a
 * leading dimension below its row width (lda, ldb as listed with the
 * layouts; ldc >= N), before anything is launched. */
int mlp_gemm(int32_t dtype, int32_t layout, int32_t M, int32_t N, int32_t K, const void *A, int64_t lda,
             const void *B, int64_t ldb, float *C, int64_t ldc, int32_t nsplit, void *stream);

/* Y = act(X W + b) for X [M][K], W [K][N], bias [N] (FP32, NULL = none),
 * act = ReLU when relu != 0; Y [M][N] in dtype, and Yf [M][N] in FP32 when
 * Yf is not NULL. */
int mlp_linear_fwd(int32_t dtype, int32_t M, int32_t N, int32_t K, const void *X, const void *W,
                   const float *bias, int32_t relu, void *Y, float *Yf, void *stream);

/* Output layer with the loss: y = X W + b, d = y - T (T [M][N] in dtype);
 * dY = scale * d in dtype (scale = 2 / (M N) gives the gradient of the mean
 * of d^2); loss_part[p] = sum of d^2 over output tile p; dbias_part[r][j] =
 * sum of scale * d over the rows of row tile r.  mlp_mse_parts gives the
 * number of loss partials and of row tiles. */
int mlp_linear_fwd_mse(int32_t dtype, int32_t M, int32_t N, int32_t K, const void *X, const void *W,
                       const float *bias, const void *T, float scale, void *dY, float *loss_part,
                       float *dbias_part, void *stream);
int mlp_mse_parts(int32_t M, int32_t N, int64_t *loss_parts, int64_t *dbias_rows);

/* out[j] = sum over i < R of src[i * ld + j] (i ascending), j < N. */
int mlp_sum_rows(int64_t R, int64_t N, const float *src, int64_t ld, float *out, void *stream);

/* dz = dh * (h > 0) elementwise (dh FP32, h and dz in dtype; dzf FP32 copy
 * when not NULL). */
int mlp_relu_bwd(int32_t dtype, int64_t n, const float *dh, const void *h, void *dz, float *dzf, void *stream);

/* One Adam step (Kingma and Ba) at step number step >= 1 on FP32 master
 * weights w with moments m, v and gradient g; wc (dtype, NULL = none)
 * receives the updated weights in the compute type. */
int mlp_adam(int32_t dtype, int64_t n, float *w, float *m, float *v, const float *g, void *wc, float lr,
             float beta1, float beta2, float eps, int32_t step, void *stream);

/* dst = src in dtype (src FP32); dst = src * scale in dtype (src FP64);
 * dst = src * scale in FP64 (src FP32). */
int mlp_cast(int32_t dtype, int64_t n, const float *src, void *dst, void *stream);
int mlp_cast_f64(int32_t dtype, int64_t n, const double *src, double scale, void *dst, void *stream);
int mlp_to_f64(int64_t n, const float *src, double scale, double *dst, void *stream);

/* Training targets from single-source solutions (the solution is linear in
 * the amplitudes): T[m][i] = scale * sum over q < 4 of amp[m][q] *
 * G[idx[m][q]][i] for m < M, i < n; G [rows][n] and T [M][n] in dtype, idx
 * (int32, values < rows, not checked: the caller keeps them in range) and
 * amp (FP32) [M][4] on the device.  M <= 65535. */
int mlp_combine(int32_t dtype, int32_t M, int64_t n, const void *G, int64_t rows, const int32_t *idx,
                const float *amp, float scale, void *T, void *stream);

/* ---- the whole network ------------------------------------------------------
 * W[3]: the layers' weights in the compute type, W[k] [in_k][out_k] with
 * (in, out) = (n_in, hidden), (hidden, hidden), (hidden, n_out); b[3]: FP32
 * biases (entries may be NULL).  W and b are HOST arrays of device pointers.
 * work: device scratch of mlp_workspace_bytes(dtype, M, ...) bytes, valid
 * for batches of up to M rows of that network. */
int mlp_workspace_bytes(int32_t dtype, int32_t M, int32_t n_in, int32_t hidden, int32_t n_out, size_t *bytes);

/* Y (compute type) and/or Yf (FP32) [M][n_out] = the network at X [M][n_in]
 * (compute type); ReLU after the two hidden layers. */
int mlp_forward(int32_t dtype, int32_t M, int32_t n_in, int32_t hidden, int32_t n_out, const void *X,
                const void *const *W, const float *const *b, void *Y, float *Yf, void *work, size_t work_bytes,
                void *stream);

/* Gradients of L = mean over [M][n_out] of (MLP(X) - T)^2 into grad[6] (FP32
 * device arrays shaped like W1, b1, W2, b2, W3, b3; grad is a HOST array of
 * device pointers); *loss (device FP32, optional) = M n_out L. */
int mlp_backward(int32_t dtype, int32_t M, int32_t n_in, int32_t hidden, int32_t n_out, const void *X,
                 const void *T, const void *const *W, const float *const *b, float *const *grad, float *loss,
                 void *work, size_t work_bytes, void *stream);

/* mlp_adam on count parameter arrays (host arrays of device pointers; wc
 * may be NULL or hold NULL entries). */
int mlp_adam_step(int32_t dtype, int32_t count, const int64_t *sizes, float *const *w, float *const *m,
                  float *const *v, const float *const *g, void *const *wc, float lr, float beta1, float beta2,
                  float eps, int32_t step, void *stream);

/* One training step: mlp_backward followed by mlp_adam_step on the six
 * parameters (W1, b1, W2, b2, W3, b3), with equal results bit for bit,
 * except that the gradient of W3 is never stored (grad[4] is left as it
 * was): the product h2^T dY applies Adam to W3 as it forms each gradient
 * value, which saves writing and re-reading one FP32 value per weight of the
 * output layer.  w, m, v, grad: host arrays of six device pointers (FP32
 * master weights, Adam moments, gradients); wc: host array of six device
 * pointers to the compute-type copies, of which the weights' (wc[0], wc[2],
 * wc[4]) feed the products and are rewritten by the update (the biases'
 * may be NULL); the biases that the products add are w[1], w[3], w[5].
 * step >= 1 sets the bias corrections.  *loss as for mlp_backward, from
 * the weights before the update. */
int mlp_train_step(int32_t dtype, int32_t M, int32_t n_in, int32_t hidden, int32_t n_out, const void *X,
                   const void *T, float *const *w, float *const *m, float *const *v, float *const *grad,
                   void *const *wc, float lr, float beta1, float beta2, float eps, int32_t step, float *loss,
                   void *work, size_t work_bytes, void *stream);

/* Right-hand side of the warm-start workload: b (FP64 [N^3], index
 * x + N y + N^2 z) = sum over q < 4 of a_q exp(-|p - c_q|^2 / (2 w_q^2)) at
 * the cell centres p, c_q = o_q + s_q d_q on the four body diagonals of the
 * unit cube (o, d) = ((0,0,0), (1,1,1)), ((1,0,0), (-1,1,1)),
 * ((0,1,0), (1,-1,1)), ((0,0,1), (1,1,-1)).  theta: HOST array
 * (s_0..s_3, w_0..w_3, a_0..a_3). */
int mlp_gaussian_rhs(int32_t N, const double *theta, double *b, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HBMC_MLP_H */
