// Learned warm start of the dual PCGP: training and inference kernels of a
// 3-layer perceptron with bfloat16 weights and activations and FP32
// accumulation (forward, masked-MSE backward, Adam).
//
// One tiled GEMM kernel (64 x 64 outputs per workgroup, 4 x 4 per thread,
// K staged through LDS in steps of 16) serves every product; each output is
// accumulated by one thread in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "kernels.h"

namespace tfeti {

namespace {

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}

template <typename T>
__device__ __forceinline__ float ld(const T* p, int64_t i);
template <>
__device__ __forceinline__ float ld<float>(const float* p, int64_t i) {
  return p[i];
}
template <>
__device__ __forceinline__ float ld<uint16_t>(const uint16_t* p, int64_t i) {
  return bf2f(p[i]);
}

constexpr int BM = 64, BN = 64, BK = 16;

}  // namespace

// C(m, n) = sum_k A(m, k) B(k, n) with A(m, k) = A[m*lda + k] (or A[k*lda + m]
// if TRA) and B(k, n) = B[k*ldb + n] (or B[n*ldb + k] if TRB).  Epilogue:
// EPI_F32: C32 = acc;  EPI_BIAS_RELU_BF16: Cb = bf16(relu(acc + bias[n]));
// EPI_BIAS_F32: C32 = acc + bias[n];  EPI_MASK_F32: C32 = acc * (Mb(m,n) > 0).
enum { EPI_F32 = 0, EPI_BIAS_RELU_BF16 = 1, EPI_BIAS_F32 = 2, EPI_MASK_F32 = 3 };

template <typename TA, typename TB, bool TRA, bool TRB, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const TA* __restrict__ A, int lda,
                                                   const TB* __restrict__ B, int ldb, float* __restrict__ C32,
                                                   uint16_t* __restrict__ Cb, int ldc,
                                                   const float* __restrict__ bias,
                                                   const uint16_t* __restrict__ Mb) {
  __shared__ float As[BK][BM + 1];
  __shared__ float Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  // split K: slice z covers [z * kc, min(K, (z + 1) * kc)) and writes its
  // partial product to C32 + z * M * ldc (EPI_F32 only)
  const int kc = (K + gridDim.z - 1) / gridDim.z;
  const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
  if (gridDim.z > 1) C32 += (int64_t)blockIdx.z * M * ldc;
  const int ty = tid / 16, tx = tid % 16;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    for (int q = tid; q < BK * BM; q += 256) {
      int kk, mm;
      if (TRA) {
        mm = q % BM;
        kk = q / BM;
      } else {
        kk = q % BK;
        mm = q / BK;
      }
      int gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < M && gk < kend) v = TRA ? ld(A, (int64_t)gk * lda + gm) : ld(A, (int64_t)gm * lda + gk);
      As[kk][mm] = v;
    }
    for (int q = tid; q < BK * BN; q += 256) {
      int kk, nn;
      if (TRB) {
        kk = q % BK;
        nn = q / BK;
      } else {
        nn = q % BN;
        kk = q / BN;
      }
      int gn = n0 + nn, gk = k0 + kk;
      float v = 0.f;
      if (gn < N && gk < kend) v = TRB ? ld(B, (int64_t)gn * ldb + gk) : ld(B, (int64_t)gk * ldb + gn);
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
      if (gm >= M || gn >= N) continue;
      int64_t o = (int64_t)gm * ldc + gn;
      float v = acc[i][j];
      if (EPI == EPI_F32) {
        C32[o] = v;
      } else if (EPI == EPI_BIAS_RELU_BF16) {
        v += bias[gn];
        Cb[o] = f2bf(v > 0.f ? v : 0.f);
      } else if (EPI == EPI_BIAS_F32) {
        C32[o] = v + bias[gn];
      } else {
        C32[o] = (bf2f(Mb[o]) > 0.f) ? v : 0.f;
      }
    }
}

template <typename TA, typename TB, bool TRA, bool TRB, int EPI>
static void gemm(int M, int N, int K, const TA* A, int lda, const TB* B, int ldb, float* C32, uint16_t* Cb, int ldc,
                 const float* bias, const uint16_t* Mb, hipStream_t st, int splits = 1) {
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, splits);
  gemm_kernel<TA, TB, TRA, TRB, EPI><<<grid, dim3(256), 0, st>>>(M, N, K, A, lda, B, ldb, C32, Cb, ldc, bias, Mb);
}

// out[i] = sum over z < S of part[z * n + i], in order of z
__global__ void reduce_slices_kernel(int64_t n, int S, const float* __restrict__ part, float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int z = 0; z < S; ++z) acc += part[(int64_t)z * n + i];
  out[i] = acc;
}

constexpr int MAX_SPLITS = 64;
constexpr int SPLIT_ROWS = 256;  // rows of the batch per K slice of a weight gradient

static int splits_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(MAX_SPLITS, (n + SPLIT_ROWS - 1) / SPLIT_ROWS));
}

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// dY = M (Y - T) / n and per-block partial sums of 1/2 M (Y - T)^2 / n
__global__ void loss_grad_kernel(int64_t total, int64_t n, const float* __restrict__ Y, const float* __restrict__ T,
                                 const float* __restrict__ Mk, float* __restrict__ dY, float* __restrict__ part) {
  __shared__ float sh[256];
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    float d = Y[i] - T[i];
    float m = Mk[i];
    dY[i] = m * d / (float)n;
    acc += 0.5f * m * d * d / (float)n;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void sum_f32_kernel(const float* __restrict__ part, int n, float* __restrict__ out) {
  __shared__ float sh[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// column sums of an (n x c) matrix over row slice z = blockIdx.y of S:
// part[z * c + j], one thread per column, rows in order
__global__ void colsum_kernel(int64_t n, int c, const float* __restrict__ X, float* __restrict__ part) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= c) return;
  const int64_t rc = (n + gridDim.y - 1) / gridDim.y;
  const int64_t r0 = (int64_t)blockIdx.y * rc, r1 = r0 + rc < n ? r0 + rc : n;
  float acc = 0.f;
  for (int64_t i = r0; i < r1; ++i) acc += X[i * c + j];
  part[(int64_t)blockIdx.y * c + j] = acc;
}

// Adam (Kingma and Ba, 2015) on FP32 master weights, refreshing the bf16 shadow
__global__ void adam_kernel(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, uint16_t* __restrict__ wb, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float mh = mi / c1, vh = vi / c2;
  float wi = w[i] - lr * mh / (sqrtf(vh) + eps);
  w[i] = wi;
  if (wb) wb[i] = f2bf(wi);
}

// ------------------------------------------------------------------ drivers
int mlp_check(const tfeti_mlp* net) {
  if (!net || net->d_in <= 0 || net->d_h <= 0 || net->d_out <= 0) return TFETI_E_INVALID;
  for (int l = 0; l < 3; ++l)
    if (!net->W[l] || !net->b[l] || !net->Wb[l]) return TFETI_E_INVALID;
  return TFETI_OK;
}

// work (floats): Xb, h1, h2 (bf16), dY, dA, dB (FP32), partial sums
int64_t mlp_work_floats(const tfeti_mlp* net, int64_t n) {
  int64_t din = net->d_in, dh = net->d_h, dout = net->d_out;
  const int64_t dm = std::max<int64_t>(dh, std::max<int64_t>(din, dout));
  return (n * din + 1) / 2 + 2 * ((n * dh + 1) / 2) + n * dout + 2 * n * dh + 1024 + 64 +
         (int64_t)MAX_SPLITS * dm * dm + (int64_t)MAX_SPLITS * dm;
}

struct MlpWork {
  uint16_t *Xb, *h1, *h2;
  float *dY, *dA, *dB, *part, *slices, *bslices;
};

// the buffers of the forward pass (bf16 inputs, both hidden layers) at the
// start of the workspace; returns the first float past them
static float* carve_forward(const tfeti_mlp* net, int64_t n, float* work, MlpWork& w) {
  const int64_t din = net->d_in, dh = net->d_h;
  float* p = work;
  w.Xb = reinterpret_cast<uint16_t*>(p);
  p += (n * din + 1) / 2;
  w.h1 = reinterpret_cast<uint16_t*>(p);
  p += (n * dh + 1) / 2;
  w.h2 = reinterpret_cast<uint16_t*>(p);
  p += (n * dh + 1) / 2;
  return p;
}

static MlpWork carve(const tfeti_mlp* net, int64_t n, float* work) {
  MlpWork w;
  int64_t din = net->d_in, dh = net->d_h, dout = net->d_out;
  float* p = carve_forward(net, n, work, w);
  w.dY = p;
  p += n * dout;
  w.dA = p;
  p += n * dh;
  w.dB = p;
  p += n * dh;
  w.part = p;
  p += 1024 + 64;
  const int64_t dm = std::max<int64_t>(dh, std::max<int64_t>(din, dout));
  w.slices = p;
  p += (int64_t)MAX_SPLITS * dm * dm;
  w.bslices = p;
  return w;
}

static void forward(const tfeti_mlp* net, int64_t n, const float* X, float* Y, const MlpWork& w, hipStream_t st) {
  const int din = net->d_in, dh = net->d_h, dout = net->d_out;
  int64_t nx = n * din;
  if (nx > 0) to_bf16_kernel<<<dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st>>>(nx, X, w.Xb);
  // h = bf16(relu(x W^T + b)); W row-major (out x in): B(k, j) = W[j*in + k]
  gemm<uint16_t, uint16_t, false, true, EPI_BIAS_RELU_BF16>((int)n, dh, din, w.Xb, din, net->Wb[0], din, nullptr,
                                                            w.h1, dh, net->b[0], nullptr, st);
  gemm<uint16_t, uint16_t, false, true, EPI_BIAS_RELU_BF16>((int)n, dh, dh, w.h1, dh, net->Wb[1], dh, nullptr, w.h2,
                                                            dh, net->b[1], nullptr, st);
  gemm<uint16_t, uint16_t, false, true, EPI_BIAS_F32>((int)n, dout, dh, w.h2, dh, net->Wb[2], dh, Y, nullptr, dout,
                                                      net->b[2], nullptr, st);
}

// ------------------------------------------------------------------ allocation-free forward pass
// Device scratch of tfeti_mlp_forward_noalloc: the bf16 inputs and both
// hidden layers (the three buffers the forward pass carves from the caller's
// workspace).  One copy per GPU for the life of the process.
constexpr int64_t kNoallocBytes = 8 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
thread_local std::string g_noalloc_err;
}  // namespace

// Bytes of scratch the forward pass of n rows needs (carve_forward()).
static int64_t mlp_forward_scratch_bytes(const tfeti_mlp* net, int64_t n) {
  return 4 * ((n * net->d_in + 1) / 2 + 2 * ((n * net->d_h + 1) / 2));
}

// Device address of this GPU's scratch array, looked up once per device
// with that device current; nullptr on failure.
static void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

const char* call_error() { return g_noalloc_err.empty() ? nullptr : g_noalloc_err.c_str(); }

void set_call_error(const std::string& msg) { g_noalloc_err = msg; }

}  // namespace tfeti

using namespace tfeti;

extern "C" {

int tfeti_mlp_forward_noalloc(const tfeti_mlp* net, int64_t n, const float* X, float* Y, void* stream) {
  g_noalloc_err.clear();
  if (mlp_check(net) || n < 0 || (n > 0 && (!X || !Y))) {
    g_noalloc_err = "tfeti_mlp_forward_noalloc: invalid network or buffers";
    return TFETI_E_INVALID;
  }
  if (n == 0) return TFETI_OK;
  const int64_t need = mlp_forward_scratch_bytes(net, n);
  if (need > kNoallocBytes) {
    g_noalloc_err = "tfeti_mlp_forward_noalloc: " + std::to_string(n) + " rows need " + std::to_string(need) +
                    " bytes of scratch; the maximum is " + std::to_string(kNoallocBytes) +
                    " bytes (split the rows into smaller calls)";
    return TFETI_E_INVALID;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    g_noalloc_err = "tfeti_mlp_forward_noalloc: no usable current device";
    return TFETI_E_HIP;
  }
  void* ptr = scratch_ptr(dev);
  if (!ptr) {
    g_noalloc_err = "tfeti_mlp_forward_noalloc: hipGetSymbolAddress of the scratch array failed";
    return TFETI_E_HIP;
  }
  MlpWork w{};
  (void)carve_forward(net, n, static_cast<float*>(ptr), w);
  forward(net, n, X, Y, w, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? TFETI_OK : TFETI_E_HIP;
}

int tfeti_mlp_work_size(const tfeti_mlp* net, int64_t n, int64_t* floats) {
  if (mlp_check(net) || n < 0 || !floats) return TFETI_E_INVALID;
  *floats = mlp_work_floats(net, n);
  return TFETI_OK;
}

int tfeti_mlp_sync_bf16(const tfeti_mlp* net, void* stream) {
  if (mlp_check(net)) return TFETI_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  const int64_t sz[3] = {(int64_t)net->d_h * net->d_in, (int64_t)net->d_h * net->d_h, (int64_t)net->d_out * net->d_h};
  for (int l = 0; l < 3; ++l)
    to_bf16_kernel<<<dim3((unsigned)((sz[l] + 255) / 256)), dim3(256), 0, st>>>(sz[l], net->W[l], net->Wb[l]);
  return hipGetLastError() == hipSuccess ? TFETI_OK : TFETI_E_HIP;
}

int tfeti_mlp_forward(const tfeti_mlp* net, int64_t n, const float* X, float* Y, float* work, void* stream) {
  if (mlp_check(net) || n < 0 || (n > 0 && (!X || !Y || !work)) || n > (1 << 28)) return TFETI_E_INVALID;
  if (n == 0) return TFETI_OK;
  forward(net, n, X, Y, carve(net, n, work), (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? TFETI_OK : TFETI_E_HIP;
}

int tfeti_mlp_loss_grad(const tfeti_mlp* net, int64_t n, const float* X, const float* T, const float* Mk, float* Y,
                        float* loss, float* work, void* stream) {
  if (mlp_check(net) || n <= 0 || !X || !T || !Mk || !Y || !loss || !work || n > (1 << 28)) return TFETI_E_INVALID;
  for (int l = 0; l < 3; ++l)
    if (!net->gW[l] || !net->gb[l]) return TFETI_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  const int din = net->d_in, dh = net->d_h, dout = net->d_out;
  MlpWork w = carve(net, n, work);
  forward(net, n, X, Y, w, st);
  const int64_t tot = n * dout;
  const int nb = (int)std::min<int64_t>(1024, (tot + 255) / 256);
  loss_grad_kernel<<<dim3(nb), dim3(256), 0, st>>>(tot, n, Y, T, Mk, w.dY, w.part);
  sum_f32_kernel<<<dim3(1), dim3(256), 0, st>>>(w.part, nb, loss);
  // weight gradients: split-K over the batch rows into slices, summed in order
  const int S = splits_for(n);
  auto wgrad = [&](int M, int N, const float* G, const uint16_t* H, float* gW, float* gb) {
    gemm<float, uint16_t, true, false, EPI_F32>(M, N, (int)n, G, M, H, N, S > 1 ? w.slices : gW, nullptr, N, nullptr,
                                                nullptr, st, S);
    if (S > 1)
      reduce_slices_kernel<<<dim3((unsigned)(((int64_t)M * N + 255) / 256)), dim3(256), 0, st>>>((int64_t)M * N, S,
                                                                                               w.slices, gW);
    colsum_kernel<<<dim3((M + 63) / 64, S), dim3(64), 0, st>>>(n, M, G, w.bslices);
    reduce_slices_kernel<<<dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st>>>(M, S, w.bslices, gb);
  };
  // layer 3: gW3 = dY^T h2, gb3 = colsum(dY), dA = (dY W3) * [h2 > 0]
  wgrad(dout, dh, w.dY, w.h2, net->gW[2], net->gb[2]);
  gemm<float, uint16_t, false, false, EPI_MASK_F32>((int)n, dh, dout, w.dY, dout, net->Wb[2], dh, w.dA, nullptr, dh,
                                                    nullptr, w.h2, st);
  // layer 2: gW2 = dA^T h1, gb2 = colsum(dA), dB = (dA W2) * [h1 > 0]
  wgrad(dh, dh, w.dA, w.h1, net->gW[1], net->gb[1]);
  gemm<float, uint16_t, false, false, EPI_MASK_F32>((int)n, dh, dh, w.dA, dh, net->Wb[1], dh, w.dB, nullptr, dh,
                                                    nullptr, w.h1, st);
  // layer 1: gW1 = dB^T Xb, gb1 = colsum(dB)
  wgrad(dh, din, w.dB, w.Xb, net->gW[0], net->gb[0]);
  return hipGetLastError() == hipSuccess ? TFETI_OK : TFETI_E_HIP;
}

int tfeti_mlp_adam(const tfeti_mlp* net, int32_t step, float lr, float b1, float b2, float eps, void* stream) {
  if (mlp_check(net) || step <= 0) return TFETI_E_INVALID;
  for (int l = 0; l < 3; ++l)
    if (!net->gW[l] || !net->gb[l] || !net->mW[l] || !net->vW[l] || !net->mb[l] || !net->vb[l]) return TFETI_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  const int64_t szW[3] = {(int64_t)net->d_h * net->d_in, (int64_t)net->d_h * net->d_h,
                          (int64_t)net->d_out * net->d_h};
  const int64_t szb[3] = {net->d_h, net->d_h, net->d_out};
  for (int l = 0; l < 3; ++l) {
    adam_kernel<<<dim3((unsigned)((szW[l] + 255) / 256)), dim3(256), 0, st>>>(
        szW[l], net->W[l], net->gW[l], net->mW[l], net->vW[l], net->Wb[l], lr, b1, b2, eps, c1, c2);
    adam_kernel<<<dim3((unsigned)((szb[l] + 255) / 256)), dim3(256), 0, st>>>(
        szb[l], net->b[l], net->gb[l], net->mb[l], net->vb[l], nullptr, lr, b1, b2, eps, c1, c2);
  }
  return hipGetLastError() == hipSuccess ? TFETI_OK : TFETI_E_HIP;
}

}  // extern "C"
