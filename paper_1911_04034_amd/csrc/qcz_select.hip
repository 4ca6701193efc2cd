// HIP kernels (gfx950) of the per-block level selector.
//
// The variable error bound of Sec. 3.7 picks one level for the whole state;
// the selector picks one level per block from 16 statistics of the block's
// stored values with a small network (16 -> 64 -> 64 -> 6, ReLU, softmax over
// the six levels), trained on the device with cross-entropy and Adam.
//
//   block_features_kernel  per-chunk statistics -> 16 float features per block
//   mlp_forward_kernel     one thread per sample, parameters in LDS
//   mlp_sample_kernel      forward + backward of one sample per thread; the
//                          activations and the back-propagated errors go to a
//                          feature-major workspace
//   mlp_grad_kernel        one workgroup per slice of samples: tiles of 32
//                          samples staged in LDS, every parameter's gradient
//                          is a dot product of two staged rows
//   mlp_adam_kernel        slice partials summed in a fixed order, Adam step
//
// Sums are taken in a fixed order, so results do not vary from run to run.
#include "qcz_internal.h"

#include <math.h>

#include <map>
#include <mutex>

namespace qcz {

// ---------------------------------------------------------------------------
// block features
// ---------------------------------------------------------------------------
constexpr int kFeatSums = 11;   // accumulated per block: the kChunkStats fields 0..10

// one workgroup per block of this launch (cs, blevel, X and n2out start at its first block)
__global__ __launch_bounds__(kWG) void block_features_kernel(const double *cs, const uint8_t *blevel, FeatCtx ctx,
                                                             float *X, double *n2out)
{
    __shared__ double red[kWG / 64][kFeatSums];
    const uint64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    double a[kFeatSums];
    for (int j = 0; j < kFeatSums; ++j) a[j] = 0.0;
    a[CS_EMAX] = -1.0;
    a[CS_EMIN] = 4096.0;
    for (int k = tid; k < ctx.cpb; k += kWG) {
        const double *r = cs + (b * (uint64_t)ctx.cpb + (uint64_t)k) * kChunkStats;
        for (int j = 0; j < kFeatSums; ++j) {
            if (j == CS_EMAX) a[j] = fmax(a[j], r[j]);
            else if (j == CS_EMIN) a[j] = fmin(a[j], r[j]);
            else a[j] += r[j];
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        for (int j = 0; j < kFeatSums; ++j) {
            const double o = __shfl_down(a[j], d, 64);
            if (j == CS_EMAX) a[j] = fmax(a[j], o);
            else if (j == CS_EMIN) a[j] = fmin(a[j], o);
            else a[j] += o;
        }
    }
    if ((tid & 63) == 0)
        for (int j = 0; j < kFeatSums; ++j) red[tid >> 6][j] = a[j];
    __syncthreads();
    if (tid != 0) return;
    for (int w = 1; w < kWG / 64; ++w)
        for (int j = 0; j < kFeatSums; ++j) {
            if (j == CS_EMAX) red[0][j] = fmax(red[0][j], red[w][j]);
            else if (j == CS_EMIN) red[0][j] = fmin(red[0][j], red[w][j]);
            else red[0][j] += red[w][j];
        }
    const double *t = red[0];
    const double M = ldexp(1.0, ctx.block_log2 + 1);   // stored doubles per block
    const double nz = t[CS_NZ];
    double f[kNIn];
    f[0] = log2(fmax(t[CS_N2] * (double)ctx.nblocks, ldexp(1.0, -60))) / 64.0;
    f[1] = 1.0 - nz / M;
    f[2] = nz > 0.0 ? (t[CS_ESUM] / nz - 1023.0) / 64.0 : 0.0;
    f[3] = nz > 0.0 ? (t[CS_EMAX] - t[CS_EMIN]) / 64.0 : 0.0;
    f[4] = t[CS_EQ8] / M;
    f[5] = t[CS_EQ16] / M;
    f[6] = t[CS_EQ24] / M;
    f[7] = t[CS_SGN] / M;
    f[8] = t[CS_CONST2] / (double)ctx.cpb;
    f[9] = t[CS_BYTES] / (16.0 * ldexp(1.0, ctx.block_log2));
    f[10] = (double)blevel[b] / 5.0;
    f[11] = nz > 0.0 ? (t[CS_EMAX] - 1023.0) / 64.0 : -17.0;
    f[12] = ctx.f12;
    f[13] = ctx.f13;
    f[14] = ctx.f14;
    f[15] = ctx.f15;
    for (int j = 0; j < kNIn; ++j) X[b * kNIn + j] = (float)f[j];
    if (n2out) n2out[b] = t[CS_N2];
}

// ---------------------------------------------------------------------------
// network
// ---------------------------------------------------------------------------
constexpr int kMlpWG = 256;

__device__ __forceinline__ void load_params(float *Ps, const float *params)
{
    for (int i = threadIdx.x; i < kNParams; i += blockDim.x) Ps[i] = params[i];
    __syncthreads();
}

// h1 = relu(W1 x + b1)
__device__ __forceinline__ void layer1(const float *Ps, const float (&x)[kNIn], float (&h1)[kNH])
{
#pragma unroll
    for (int j = 0; j < kNH; ++j) {
        float a = Ps[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kNIn; ++i) a = fmaf(Ps[kOffW1 + j * kNIn + i], x[i], a);
        h1[j] = a > 0.f ? a : 0.f;
    }
}

// h2 = relu(W2 h1 + b2), z = W3 h2 + b3.  The loop over hidden units k stays
// rolled (register arrays are only indexed by unrolled loop counters); with
// h2_row != nullptr unit k's activation is stored at h2_row[k * N].
__device__ __forceinline__ void layer23(const float *Ps, const float (&h1)[kNH], float (&z)[kNOut], float *h2_row,
                                        uint64_t N)
{
#pragma unroll
    for (int c = 0; c < kNOut; ++c) z[c] = Ps[kOffB3 + c];
#pragma unroll 1
    for (int k = 0; k < kNH; ++k) {
        float a = Ps[kOffB2 + k];
#pragma unroll
        for (int j = 0; j < kNH; ++j) a = fmaf(Ps[kOffW2 + k * kNH + j], h1[j], a);
        a = a > 0.f ? a : 0.f;
        if (h2_row) h2_row[(uint64_t)k * N] = a;
#pragma unroll
        for (int c = 0; c < kNOut; ++c) z[c] = fmaf(Ps[kOffW3 + c * kNH + k], a, z[c]);
    }
}

__global__ __launch_bounds__(kMlpWG) void mlp_forward_kernel(const float *params, const float *X, uint64_t N,
                                                             float *probs, uint8_t *argmax)
{
    __shared__ float Ps[kNParams];
    load_params(Ps, params);
    const uint64_t n = (uint64_t)blockIdx.x * kMlpWG + threadIdx.x;
    if (n >= N) return;
    float x[kNIn], h1[kNH], z[kNOut];
#pragma unroll
    for (int i = 0; i < kNIn; ++i) x[i] = X[n * kNIn + i];
    layer1(Ps, x, h1);
    layer23(Ps, h1, z, nullptr, 0);
    float m = z[0];
    int best = 0;
#pragma unroll
    for (int c = 1; c < kNOut; ++c)
        if (z[c] > m) { m = z[c]; best = c; }
    if (probs) {
        float e[kNOut], s = 0.f;
#pragma unroll
        for (int c = 0; c < kNOut; ++c) { e[c] = expf(z[c] - m); s += e[c]; }
#pragma unroll
        for (int c = 0; c < kNOut; ++c) probs[n * kNOut + c] = e[c] / s;
    }
    if (argmax) argmax[n] = (uint8_t)best;
}

// Workspace rows (feature-major, N floats each): h1 (64), h2 (64), da1 (64),
// da2 (64), dz (6).  The gradient kernel also stages x (16) and a row of ones.
constexpr int kRowH1 = 0, kRowH2 = 64, kRowD1 = 128, kRowD2 = 192, kRowDZ = 256, kWsRows = 262;

__global__ __launch_bounds__(kMlpWG) void mlp_sample_kernel(const float *params, const float *X,
                                                            const uint8_t *labels, uint64_t N, float *ws,
                                                            float *loss_part)
{
    __shared__ float Ps[kNParams];
    __shared__ float red[kMlpWG / 64];
    load_params(Ps, params);
    const uint64_t n = (uint64_t)blockIdx.x * kMlpWG + threadIdx.x;
    float ln = 0.f;
    if (n < N) {
        float x[kNIn], h1[kNH], z[kNOut];
#pragma unroll
        for (int i = 0; i < kNIn; ++i) x[i] = X[n * kNIn + i];
        layer1(Ps, x, h1);
#pragma unroll
        for (int j = 0; j < kNH; ++j) ws[(uint64_t)(kRowH1 + j) * N + n] = h1[j];
        layer23(Ps, h1, z, ws + (uint64_t)kRowH2 * N + n, N);
        float m = z[0];
#pragma unroll
        for (int c = 1; c < kNOut; ++c) m = fmaxf(m, z[c]);
        float e[kNOut], s = 0.f;
#pragma unroll
        for (int c = 0; c < kNOut; ++c) { e[c] = expf(z[c] - m); s += e[c]; }
        const int y = labels[n];
        float zy = z[0];
#pragma unroll
        for (int c = 1; c < kNOut; ++c) zy = (c == y) ? z[c] : zy;
        ln = -(zy - m - logf(s));
        const float invN = 1.0f / (float)N;
        float dz[kNOut];
#pragma unroll
        for (int c = 0; c < kNOut; ++c) {
            dz[c] = (e[c] / s - (c == y ? 1.f : 0.f)) * invN;
            ws[(uint64_t)(kRowDZ + c) * N + n] = dz[c];
        }
        // da2_k = (W3^T dz)_k relu'(a2_k); da1 = (W2^T da2) relu'(a1), accumulated over k
        float g1[kNH];
#pragma unroll
        for (int j = 0; j < kNH; ++j) g1[j] = 0.f;
#pragma unroll 1
        for (int k = 0; k < kNH; ++k) {
            float a = 0.f;
#pragma unroll
            for (int c = 0; c < kNOut; ++c) a = fmaf(Ps[kOffW3 + c * kNH + k], dz[c], a);
            const float h2k = ws[(uint64_t)(kRowH2 + k) * N + n];
            a = h2k > 0.f ? a : 0.f;
            ws[(uint64_t)(kRowD2 + k) * N + n] = a;
#pragma unroll
            for (int j = 0; j < kNH; ++j) g1[j] = fmaf(Ps[kOffW2 + k * kNH + j], a, g1[j]);
        }
#pragma unroll
        for (int j = 0; j < kNH; ++j) ws[(uint64_t)(kRowD1 + j) * N + n] = h1[j] > 0.f ? g1[j] : 0.f;
    }
    for (int d = 32; d >= 1; d >>= 1) ln += __shfl_down(ln, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ln;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < kMlpWG / 64; ++w) t += red[w];
        loss_part[blockIdx.x] = t;
    }
}

// Staged rows of a 32-sample tile: x (16), h1, h2, da1, da2 (64 each), dz (6), ones.
constexpr int kTile = 32, kTileStride = kTile + 1;   // +1: rows start in different LDS banks
constexpr int kStX = 0, kStH1 = 16, kStH2 = 80, kStD1 = 144, kStD2 = 208, kStDZ = 272, kStOne = 278, kStRows = 279;
constexpr int kSlice = 512;                          // samples per gradient workgroup
constexpr int kPPT = (kNParams + kMlpWG - 1) / kMlpWG;   // parameters per thread (23)

// (row, col) of the staged tile whose dot product is parameter p's gradient
__device__ __forceinline__ void param_rows(int p, int &r, int &c)
{
    if (p < kOffB1) { r = kStD1 + p / kNIn; c = kStX + p % kNIn; }
    else if (p < kOffW2) { r = kStD1 + (p - kOffB1); c = kStOne; }
    else if (p < kOffB2) { const int q = p - kOffW2; r = kStD2 + q / kNH; c = kStH1 + q % kNH; }
    else if (p < kOffW3) { r = kStD2 + (p - kOffB2); c = kStOne; }
    else if (p < kOffB3) { const int q = p - kOffW3; r = kStDZ + q / kNH; c = kStH2 + q % kNH; }
    else { r = kStDZ + (p - kOffB3); c = kStOne; }
}

__global__ __launch_bounds__(kMlpWG) void mlp_grad_kernel(const float *X, const float *ws, uint64_t N,
                                                          float *partial)
{
    __shared__ float T[kStRows * kTileStride];
    const int tid = threadIdx.x;
    int rr[kPPT], cc[kPPT];
    float acc[kPPT];
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        const int p = tid + k * kMlpWG;
        param_rows(p < kNParams ? p : kNParams - 1, rr[k], cc[k]);
        acc[k] = 0.f;
    }
    const uint64_t n0 = (uint64_t)blockIdx.x * kSlice;
    const uint64_t n1 = n0 + kSlice < N ? n0 + kSlice : N;
    for (uint64_t t0 = n0; t0 < n1; t0 += kTile) {
        const int cnt = (int)(n1 - t0 < (uint64_t)kTile ? n1 - t0 : (uint64_t)kTile);
        // stage: rows of the workspace are contiguous in n (coalesced)
        for (int e = tid; e < kStRows * kTile; e += kMlpWG) {
            const int row = e / kTile, j = e % kTile;
            float v = 0.f;
            if (j < cnt) {
                const uint64_t n = t0 + (uint64_t)j;
                if (row < kStH1) v = X[n * kNIn + row];
                else if (row < kStOne) v = ws[(uint64_t)(row - kStH1) * N + n];
                else v = 1.f;
            }
            T[row * kTileStride + j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            const float *a = T + rr[k] * kTileStride, *b = T + cc[k] * kTileStride;
            float s = acc[k];
            for (int j = 0; j < kTile; ++j) s = fmaf(a[j], b[j], s);
            acc[k] = s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        const int p = tid + k * kMlpWG;
        if (p < kNParams) partial[(uint64_t)blockIdx.x * kNParams + p] = acc[k];
    }
}

__global__ __launch_bounds__(kMlpWG) void mlp_adam_kernel(float *params, float *m, float *v, const float *partial,
                                                          int nslices, const float *loss_part, int nloss, uint64_t N,
                                                          float lr, uint32_t step, float *grad_out, float *loss_out)
{
    const int p = blockIdx.x * kMlpWG + threadIdx.x;
    if (p == 0 && loss_out) {
        double t = 0.0;
        for (int i = 0; i < nloss; ++i) t += (double)loss_part[i];
        loss_out[0] = (float)(t / (double)N);
    }
    if (p >= kNParams) return;
    double g = 0.0;
    for (int s = 0; s < nslices; ++s) g += (double)partial[(uint64_t)s * kNParams + p];
    if (grad_out) grad_out[p] = (float)g;
    if (step == 0) return;   // gradient only
    // Adam (Kingma and Ba, 2015): beta1 = 0.9, beta2 = 0.999, eps = 1e-8
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double mm = b1 * (double)m[p] + (1.0 - b1) * g;
    const double vv = b2 * (double)v[p] + (1.0 - b2) * g * g;
    const double mhat = mm / (1.0 - pow(b1, (double)step));
    const double vhat = vv / (1.0 - pow(b2, (double)step));
    m[p] = (float)mm;
    v[p] = (float)vv;
    params[p] = (float)((double)params[p] - (double)lr * mhat / (sqrt(vhat) + eps));
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_block_features(const double *cstats, const uint8_t *block_level, const FeatCtx &ctx, uint64_t nb,
                                 float *X, double *n2, hipStream_t st)
{
    if (nb == 0 || nb > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(block_features_kernel, dim3((unsigned)nb), dim3(kWG), 0, st, cstats, block_level, ctx, X, n2);
    return hipGetLastError();
}

static unsigned sample_blocks(uint64_t N) { return (unsigned)((N + kMlpWG - 1) / kMlpWG); }
static unsigned slices(uint64_t N) { return (unsigned)((N + kSlice - 1) / kSlice); }

hipError_t launch_mlp_forward(const float *params, const float *X, uint64_t N, float *probs, uint8_t *argmax,
                              hipStream_t st)
{
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(sample_blocks(N)), dim3(kMlpWG), 0, st, params, X, N, probs, argmax);
    return hipGetLastError();
}

static constexpr size_t ws_bytes(uint64_t N)
{
    return (((size_t)kWsRows * N * sizeof(float) + 255) & ~(size_t)255) +
           (((size_t)((N + kSlice - 1) / kSlice) * kNParams * sizeof(float) + 255) & ~(size_t)255) +
           (((size_t)((N + kMlpWG - 1) / kMlpWG) * sizeof(float) + 255) & ~(size_t)255);
}

size_t mlp_workspace_bytes(uint64_t N) { return ws_bytes(N); }

// Workspace of the training step for callers that cannot allocate: a static
// device array holding the workspace of kMlpStaticSamples samples (about
// 8.5 MiB; every GPU the library runs on holds its own copy until the process
// ends).  Every step reads only what it wrote itself, so no clearing is needed.
static __device__ __align__(256) uint8_t scratch[ws_bytes(kMlpStaticSamples)];

// The device address of this GPU's copy of `scratch`, looked up once per
// device (with that device current) on the first call from it.  In host code
// the array's name is not a device address; only the looked-up pointer may be
// handed to kernels.
hipError_t mlp_static_workspace(void **out, size_t *bytes)
{
    static std::mutex mu;
    static std::map<int, void *> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = addr.emplace(dev, p).first;
    }
    *out = it->second;
    *bytes = sizeof(scratch);
    return hipSuccess;
}

hipError_t launch_mlp_train(float *params, float *m, float *v, const float *X, const uint8_t *labels, uint64_t N,
                            float lr, uint32_t step, float *grad_out, float *loss_out, void *work, hipStream_t st)
{
    if (N == 0) return hipErrorInvalidValue;
    uint8_t *w = (uint8_t *)work;
    float *ws = (float *)w;
    w += ((size_t)kWsRows * N * sizeof(float) + 255) & ~(size_t)255;
    float *partial = (float *)w;
    w += ((size_t)slices(N) * kNParams * sizeof(float) + 255) & ~(size_t)255;
    float *loss_part = (float *)w;
    hipLaunchKernelGGL(mlp_sample_kernel, dim3(sample_blocks(N)), dim3(kMlpWG), 0, st, params, X, labels, N, ws,
                       loss_part);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(slices(N)), dim3(kMlpWG), 0, st, X, ws, N, partial);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNParams + kMlpWG - 1) / kMlpWG), dim3(kMlpWG), 0, st, params, m, v,
                       partial, (int)slices(N), loss_part, (int)sample_blocks(N), N, lr, step, grad_out, loss_out);
    return hipGetLastError();
}

}  // namespace qcz
