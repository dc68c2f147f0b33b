// FP32 work model: an MLP 6 -> 32 -> 32 -> 1 with ReLU hidden layers that
// predicts log2(1 + work) of a vertex from six cheap features.  Hand-written
// kernels for inference and for training (forward and deltas per sample, one
// thread per parameter for the gradient reduction, Adam).  Every reduction runs
// in a fixed order, so training is reproducible for a given seed.
//
// Parameter layout (floats): W1[32][6] b1[32] W2[32][32] b2[32] W3[32] b3[1],
// then the feature normalisation mean[6] and inv_std[6] (1325 in total).
#include "common.hpp"
#include "kernels.hpp"

#define H 32
#define F 6
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + H * F)
#define OFF_W2 (OFF_B1 + H)
#define OFF_B2 (OFF_W2 + H * H)
#define OFF_W3 (OFF_B2 + H)
#define OFF_B3 (OFF_W3 + H)
#define OFF_MEAN (OFF_B3 + 1)
#define OFF_ISTD (OFF_MEAN + F)
#define N_TRAIN (OFF_B3 + 1)   // 1313 trained parameters
#define N_ALL (OFF_ISTD + F)   // 1325

__device__ __forceinline__ void mlp_forward(const float *__restrict__ P, const float *x_raw, float *h1, float *h2,
                                            float *out) {
    float x[F];
#pragma unroll
    for (int k = 0; k < F; k++) x[k] = (x_raw[k] - P[OFF_MEAN + k]) * P[OFF_ISTD + k];
#pragma unroll
    for (int j = 0; j < H; j++) {
        float a = P[OFF_B1 + j];
#pragma unroll
        for (int k = 0; k < F; k++) a = fmaf(P[OFF_W1 + j * F + k], x[k], a);
        h1[j] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int i = 0; i < H; i++) {
        float a = P[OFF_B2 + i];
#pragma unroll
        for (int j = 0; j < H; j++) a = fmaf(P[OFF_W2 + i * H + j], h1[j], a);
        h2[i] = fmaxf(a, 0.0f);
    }
    float o = P[OFF_B3];
#pragma unroll
    for (int i = 0; i < H; i++) o = fmaf(P[OFF_W3 + i], h2[i], o);
    *out = o;
}

__global__ void __launch_bounds__(256) k_mlp_predict(i64 n, const float *__restrict__ X, const float *__restrict__ P,
                                                     float *__restrict__ pred) {
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        float x[F], h1[H], h2[H], o;
#pragma unroll
        for (int k = 0; k < F; k++) x[k] = X[r * F + k];
        mlp_forward(P, x, h1, h2, &o);
        pred[r] = o;
    }
}

// Per sample of the batch: activations, output delta (d MSE / d out) and the
// hidden-layer deltas.  Loss contributions go to lossp[b] (summed in order later).
__global__ void __launch_bounds__(256) k_mlp_fwd_bwd(i32 B, const i32 *__restrict__ idx, const float *__restrict__ X,
                                                     const float *__restrict__ y, const float *__restrict__ P,
                                                     float *__restrict__ A1, float *__restrict__ A2,
                                                     float *__restrict__ D1, float *__restrict__ D2,
                                                     float *__restrict__ G3, float *__restrict__ lossp) {
    i32 b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    i64 r = idx[b];
    float x[F], h1[H], h2[H], o;
#pragma unroll
    for (int k = 0; k < F; k++) x[k] = X[r * F + k];
    mlp_forward(P, x, h1, h2, &o);
    const float err = o - y[r];
    const float g3 = 2.0f * err / (float)B;
    lossp[b] = err * err;
    G3[b] = g3;
    float d2[H];
#pragma unroll
    for (int i = 0; i < H; i++) {
        d2[i] = h2[i] > 0.0f ? g3 * P[OFF_W3 + i] : 0.0f;
        A2[(i64)b * H + i] = h2[i];
        D2[(i64)b * H + i] = d2[i];
    }
#pragma unroll
    for (int j = 0; j < H; j++) {
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i < H; i++) a = fmaf(d2[i], P[OFF_W2 + i * H + j], a);
        A1[(i64)b * H + j] = h1[j];
        D1[(i64)b * H + j] = h1[j] > 0.0f ? a : 0.0f;
    }
}

// One thread per trained parameter: its gradient summed over the batch in order.
__global__ void __launch_bounds__(256) k_mlp_grad(i32 B, const i32 *__restrict__ idx, const float *__restrict__ X,
                                                  const float *__restrict__ P, const float *__restrict__ A1,
                                                  const float *__restrict__ A2, const float *__restrict__ D1,
                                                  const float *__restrict__ D2, const float *__restrict__ G3,
                                                  float *__restrict__ grad) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N_TRAIN) return;
    float g = 0.0f;
    if (p < OFF_B1) {  // W1[j][k]
        int j = p / F, k = p % F;
        float m = P[OFF_MEAN + k], s = P[OFF_ISTD + k];
        for (i32 b = 0; b < B; b++) g = fmaf(D1[(i64)b * H + j], (X[(i64)idx[b] * F + k] - m) * s, g);
    } else if (p < OFF_W2) {  // b1[j]
        int j = p - OFF_B1;
        for (i32 b = 0; b < B; b++) g += D1[(i64)b * H + j];
    } else if (p < OFF_B2) {  // W2[i][j]
        int q = p - OFF_W2, i = q / H, j = q % H;
        for (i32 b = 0; b < B; b++) g = fmaf(D2[(i64)b * H + i], A1[(i64)b * H + j], g);
    } else if (p < OFF_W3) {  // b2[i]
        int i = p - OFF_B2;
        for (i32 b = 0; b < B; b++) g += D2[(i64)b * H + i];
    } else if (p < OFF_B3) {  // W3[i]
        int i = p - OFF_W3;
        for (i32 b = 0; b < B; b++) g = fmaf(G3[b], A2[(i64)b * H + i], g);
    } else {  // b3
        for (i32 b = 0; b < B; b++) g += G3[b];
    }
    grad[p] = g;
}

__global__ void k_mlp_adam(float *__restrict__ P, const float *__restrict__ grad, float *__restrict__ m1,
                           float *__restrict__ m2, float lr, float b1, float b2, float eps, int step) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N_TRAIN) return;
    float g = grad[p];
    float a = b1 * m1[p] + (1.0f - b1) * g;
    float v = b2 * m2[p] + (1.0f - b2) * g * g;
    m1[p] = a;
    m2[p] = v;
    float ah = a / (1.0f - powf(b1, (float)step));
    float vh = v / (1.0f - powf(b2, (float)step));
    P[p] -= lr * ah / (sqrtf(vh) + eps);
}

// Column sums of X (and of X^2) in double, per block then in block order.
__global__ void __launch_bounds__(256) k_feat_partial(i64 n, const float *__restrict__ X, double *__restrict__ part) {
    __shared__ double s1[256][F];
    __shared__ double s2[256][F];
    double a1[F] = {0}, a2[F] = {0};
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x)
        for (int k = 0; k < F; k++) {
            double v = X[r * F + k];
            a1[k] += v;
            a2[k] += v * v;
        }
    for (int k = 0; k < F; k++) {
        s1[threadIdx.x][k] = a1[k];
        s2[threadIdx.x][k] = a2[k];
    }
    __syncthreads();
    if (threadIdx.x < 2 * F) {
        int k = threadIdx.x % F;
        bool sq = threadIdx.x >= F;
        double t = 0;
        for (int i = 0; i < 256; i++) t += sq ? s2[i][k] : s1[i][k];
        part[(i64)blockIdx.x * 2 * F + threadIdx.x] = t;
    }
}

__global__ void k_feat_finish(i64 n, int nblocks, const double *__restrict__ part, float *__restrict__ P) {
    if (threadIdx.x >= F) return;
    int k = threadIdx.x;
    double s = 0, q = 0;
    for (int b = 0; b < nblocks; b++) {
        s += part[(i64)b * 2 * F + k];
        q += part[(i64)b * 2 * F + F + k];
    }
    double mean = n > 0 ? s / (double)n : 0.0;
    double var = n > 0 ? q / (double)n - mean * mean : 0.0;
    P[OFF_MEAN + k] = (float)mean;
    P[OFF_ISTD + k] = (float)(1.0 / sqrt(var > 1e-8 ? var : 1e-8));
}

// Squared error of the model over all samples: per block, then in block order.
__global__ void __launch_bounds__(256) k_mlp_sse(i64 n, const float *__restrict__ pred, const float *__restrict__ y,
                                                 double *__restrict__ part) {
    __shared__ double s[256];
    double a = 0;
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        double e = (double)pred[r] - (double)y[r];
        a += e * e;
    }
    s[threadIdx.x] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int i = 0; i < 256; i++) t += s[i];
        part[blockIdx.x] = t;
    }
}

// Mean and standard deviation of the targets (per block in double, then in order),
// and the standardised copy the training runs on.
__global__ void __launch_bounds__(256) k_target_partial(i64 n, const float *__restrict__ y, double *__restrict__ part) {
    __shared__ double s1[256], s2[256];
    double a = 0, q = 0;
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        double v = y[r];
        a += v;
        q += v * v;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t1 = 0, t2 = 0;
        for (int i = 0; i < 256; i++) {
            t1 += s1[i];
            t2 += s2[i];
        }
        part[2 * blockIdx.x] = t1;
        part[2 * blockIdx.x + 1] = t2;
    }
}

__global__ void k_target_finish(i64 n, int nblocks, const double *__restrict__ part, float *__restrict__ ms) {
    if (threadIdx.x != 0) return;
    double s = 0, q = 0;
    for (int b = 0; b < nblocks; b++) {
        s += part[2 * b];
        q += part[2 * b + 1];
    }
    double mean = s / (double)n, var = q / (double)n - mean * mean;
    ms[0] = (float)mean;
    ms[1] = (float)sqrt(var > 1e-12 ? var : 1e-12);
}

__global__ void k_target_standardise(i64 n, const float *__restrict__ y, const float *__restrict__ ms,
                                     float *__restrict__ ys) {
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x)
        ys[r] = (y[r] - ms[0]) / ms[1];
}

// Output layer rescaled so that the model predicts the original targets.
__global__ void k_fold_output(float *__restrict__ P, const float *__restrict__ ms) {
    int i = threadIdx.x;
    if (i < H) P[OFF_W3 + i] *= ms[1];
    if (i == 0) P[OFF_B3] = P[OFF_B3] * ms[1] + ms[0];
}

hipError_t mlp_standardise_targets(i64 n, const float *y, double *part, int nblocks, float *ms, float *ys,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_target_partial, dim3(nblocks), dim3(256), 0, s, n, y, part);
    hipLaunchKernelGGL(k_target_finish, dim3(1), dim3(64), 0, s, n, nblocks, part, ms);
    hipLaunchKernelGGL(k_target_standardise, dim3(nblocks), dim3(256), 0, s, n, y, ms, ys);
    return hipGetLastError();
}

hipError_t mlp_fold_output(float *P, const float *ms, hipStream_t s) {
    hipLaunchKernelGGL(k_fold_output, dim3(1), dim3(64), 0, s, P, ms);
    return hipGetLastError();
}

int mlp_num_trained() { return N_TRAIN; }
int mlp_num_all() { return N_ALL; }

hipError_t mlp_predict(i64 n, const float *X, const float *P, float *pred, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    i64 blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_mlp_predict, dim3((u32)blocks), dim3(256), 0, s, n, X, P, pred);
    return hipGetLastError();
}

hipError_t mlp_feature_stats(i64 n, const float *X, double *part, int nblocks, float *P, hipStream_t s) {
    hipLaunchKernelGGL(k_feat_partial, dim3(nblocks), dim3(256), 0, s, n, X, part);
    hipLaunchKernelGGL(k_feat_finish, dim3(1), dim3(64), 0, s, n, nblocks, part, P);
    return hipGetLastError();
}

hipError_t mlp_train_step(i32 B, const i32 *idx, const float *X, const float *y, float *P, float *A1, float *A2,
                          float *D1, float *D2, float *G3, float *lossp, float *grad, float *m1, float *m2, float lr,
                          int step, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((B + 255) / 256), dim3(256), 0, s, B, idx, X, y, P, A1, A2, D1, D2, G3,
                       lossp);
    hipLaunchKernelGGL(k_mlp_grad, dim3((N_TRAIN + 255) / 256), dim3(256), 0, s, B, idx, X, P, A1, A2, D1, D2, G3,
                       grad);
    hipLaunchKernelGGL(k_mlp_adam, dim3((N_TRAIN + 255) / 256), dim3(256), 0, s, P, grad, m1, m2, lr, 0.9f, 0.999f,
                       1e-8f, step);
    return hipGetLastError();
}

hipError_t mlp_sse(i64 n, const float *pred, const float *y, double *part, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_sse, dim3(nblocks), dim3(256), 0, s, n, pred, y, part);
    return hipGetLastError();
}
