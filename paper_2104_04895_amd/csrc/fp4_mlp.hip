// fp4_mlp.hip -- small multilayer perceptron for the learned rate surrogate: FP32 training
// (forward, backward, Adam) and BF16 inference on the matrix cores, all in hand-written
// kernels.
//
// Network: nin -> width (SiLU) -> ... -> width (SiLU) -> 2, with `depth` linear layers in
// total.  Output 0 is the predicted log rate mu, output 1 the predicted log standard
// deviation s of that prediction; the training loss is the Gaussian negative
// log-likelihood  0.5 (y - mu)^2 exp(-2 s) + s  averaged over the mini-batch.
// Parameters are one flat FP32 array: for each layer l, W_l [out_l][in_l] then b_l [out_l].
#include "fp4_mlp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

namespace {

constexpr int TM = 64, TN = 64, TK = 16;

// C[i][j] = sum_k A(i,k) B(k,j) (+ bias[j]) for i < M, j < N, with A(i,k) = A[i*sai + k*sak]
// and B(k,j) = B[k*sbk + j*sbj]; optionally Z = C and C = silu(C).  64x64 tiles staged in
// LDS, 256 threads, 4x4 outputs per thread.
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *A, long sai,
                                              long sak, const float *B, long sbk, long sbj,
                                              const float *bias, float *Z, float *C, long ldc,
                                              int act, int accumulate) {
  __shared__ float As[TK][TM + 1];
  __shared__ float Bs[TK][TN + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += TK) {
    for (int e = threadIdx.x; e < TK * TM; e += 256) {
      const int kk = e / TM, ii = e % TM;
      const int i = i0 + ii, k = k0 + kk;
      As[kk][ii] = (i < M && k < K) ? A[(long)i * sai + (long)k * sak] : 0.f;
    }
    for (int e = threadIdx.x; e < TK * TN; e += 256) {
      const int kk = e / TN, jj = e % TN;
      const int j = j0 + jj, k = k0 + kk;
      Bs[kk][jj] = (j < N && k < K) ? B[(long)k * sbk + (long)j * sbj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[kk][tx * 4 + q];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = fmaf(a[r], b[q], acc[r][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + ty * 4 + r, j = j0 + tx * 4 + q;
      if (i >= M || j >= N) continue;
      float v = acc[r][q] + (bias ? bias[j] : 0.f);
      const long o = (long)i * ldc + j;
      if (accumulate) v += C[o];
      if (Z) Z[o] = v;
      if (act) v = v / (1.f + expf(-v));
      C[o] = v;
    }
}

// dZ = dH * silu'(Z) element-wise (in place on dH)
__global__ void k_silu_back(float *dH, const float *Z, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float z = Z[i];
  const float s = 1.f / (1.f + expf(-z));
  dH[i] *= s + z * s * (1.f - s);
}

// Gaussian NLL per sample and its gradient with respect to the two outputs (scaled by 1/M)
__global__ void k_loss(const float *out, const float *y, int M, float *dout, float *loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const float mu = out[2 * i], s = out[2 * i + 1];
  const float r = y[i] - mu;
  const float ie = expf(-2.f * s);
  loss[i] = 0.5f * r * r * ie + s;
  dout[2 * i] = -r * ie / (float)M;
  dout[2 * i + 1] = (1.f - r * r * ie) / (float)M;
}

// db[j] = sum_i dZ[i][j]
__global__ void k_colsum(const float *dZ, int M, int N, float *db) {
  const int j = blockIdx.x;
  float acc = 0.f;
  for (int i = threadIdx.x; i < M; i += blockDim.x) acc += dZ[(long)i * N + j];
  __shared__ float red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[j] = red[0];
}

// Adam step (bias-corrected), element-wise
__global__ void k_adam(float *p, const float *g, float *m, float *v, long n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_gather(const float *X, const float *Y, const int *idx, int M, int nin, float *Xb,
                         float *Yb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int r = idx[i];
  for (int k = 0; k < nin; ++k) Xb[(long)i * nin + k] = X[(long)r * nin + k];
  Yb[i] = Y[r];
}

// ---------------------------------------------------------------- BF16 inference on MFMA
//
// Inputs and weights are stored as BF16 (round to nearest even), products accumulate in
// FP32 on the matrix cores (v_mfma_f32_16x16x16_bf16), bias and SiLU are applied in FP32 and
// hidden activations are rounded to BF16 for the next layer.  Operand layouts of the 16x16x16
// instruction (lane l, element e of the 4-wide register): A[i][k] with i = l % 16,
// k = 4 (l / 16) + e; B[k][j] with j = l % 16, k = 4 (l / 16) + e; D[i][j] with j = l % 16,
// i = 4 (l / 16) + e.
typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// dst[r][c] (rows_pad x cols_pad) = bf16(src[r * lds + c]) inside rows x cols, 0 outside
__global__ void k_pack_bf16(const float *src, int rows, int cols, long lds, unsigned short *dst,
                            int rows_pad, int cols_pad) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)rows_pad * cols_pad) return;
  const int r = (int)(e / cols_pad), c = (int)(e % cols_pad);
  dst[e] = (r < rows && c < cols) ? bf16bits(src[(long)r * lds + c]) : (unsigned short)0;
}

// One layer: X [Mp][Kp] BF16 (Mp a multiple of 64, Kp of 16, zero padded), W [Np][Kp] BF16
// (Np a multiple of 16, zero padded), bias [N].  Work-group: 4 wavefronts x 16 rows, the
// 128-column group blockIdx.y.  Hidden layers write Hb [Mp][Np] BF16 (the next layer's
// input), the last layer Hf [M][N] FP32.
__global__ __launch_bounds__(256) void k_fwd_mfma(int M, int Kp, int N, int Np,
                                                  const unsigned short *__restrict__ X,
                                                  const unsigned short *__restrict__ W,
                                                  const float *__restrict__ bias,
                                                  unsigned short *Hb, float *Hf, int act) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.x * 64 + wave * 16;
  const int nt0 = blockIdx.y * 8;
  const int ntiles = min(8, Np / 16 - nt0);
  const int i = lane & 15, kq = lane >> 4;
  v4f32 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = v4f32{0.f, 0.f, 0.f, 0.f};
  const unsigned short *xa = X + (long)(m0 + i) * Kp + 4 * kq;
  for (int k0 = 0; k0 < Kp; k0 += 16) {
    const v4i16 a = *reinterpret_cast<const v4i16 *>(xa + k0);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t < ntiles) {
        const v4i16 b = *reinterpret_cast<const v4i16 *>(W + (long)((nt0 + t) * 16 + i) * Kp + 4 * kq + k0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (t >= ntiles) continue;
    const int col = (nt0 + t) * 16 + i;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = m0 + 4 * kq + e;
      if (col >= N) continue;
      float v = acc[t][e] + bias[col];
      if (act) {
        v = v / (1.f + expf(-v));
        Hb[(long)row * Np + col] = bf16bits(v);
      } else if (row < M) {
        Hf[(long)row * N + col] = v;
      }
    }
  }
}

}  // namespace

struct fp4_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  int nin = 0, width = 0, depth = 0;
  std::vector<int> in_dim, out_dim;
  std::vector<size_t> w_off, b_off;
  size_t nparam = 0;
  float *d_p = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr;
  long adam_t = 0;
  std::string err;
  int fail(int code, const std::string &m) {
    err = m;
    return code;
  }
};

namespace {

#define MLP_HIP(m, expr)                                                               \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return (m)->fail(FP4_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

hipError_t gemm(hipStream_t s, int M, int N, int K, const float *A, long sai, long sak,
                const float *B, long sbk, long sbj, const float *bias, float *Z, float *C, long ldc,
                int act, int accumulate) {
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, M, N, K, A, sai, sak, B, sbk, sbj, bias, Z, C,
                     ldc, act, accumulate);
  return hipGetLastError();
}

struct Work {
  std::vector<float *> H, Z;  // activations per layer output (H[0] = input)
  float *dA = nullptr, *dB = nullptr, *loss = nullptr, *y = nullptr;
  size_t M = 0;
};

void free_work(Work &w) {
  for (float *p : w.H) (void)hipFree(p);
  for (float *p : w.Z) (void)hipFree(p);
  (void)hipFree(w.dA);
  (void)hipFree(w.dB);
  (void)hipFree(w.loss);
  (void)hipFree(w.y);
  w = Work{};
}

int alloc_work(fp4_mlp *m, Work &w, size_t M) {
  w.M = M;
  w.H.assign(m->depth + 1, nullptr);
  w.Z.assign(m->depth, nullptr);
  MLP_HIP(m, hipMalloc(&w.H[0], sizeof(float) * M * m->nin));
  for (int l = 0; l < m->depth; ++l) {
    MLP_HIP(m, hipMalloc(&w.H[l + 1], sizeof(float) * M * m->out_dim[l]));
    MLP_HIP(m, hipMalloc(&w.Z[l], sizeof(float) * M * m->out_dim[l]));
  }
  const size_t mx = (size_t)std::max(m->width, m->nin);
  MLP_HIP(m, hipMalloc(&w.dA, sizeof(float) * M * mx));
  MLP_HIP(m, hipMalloc(&w.dB, sizeof(float) * M * mx));
  MLP_HIP(m, hipMalloc(&w.loss, sizeof(float) * M));
  MLP_HIP(m, hipMalloc(&w.y, sizeof(float) * M));
  return FP4_OK;
}

// BF16 forward pass on MFMA from w.H[0] (M rows, FP32) into w.H[depth] (FP32 [M][2]).
int forward_bf16_mfma(fp4_mlp *m, Work &w, int M) {
  const int Mp = (M + 63) / 64 * 64;
  auto pad16 = [](int v) { return (v + 15) / 16 * 16; };
  int maxk = pad16(m->nin);
  for (int l = 0; l < m->depth; ++l) maxk = std::max(maxk, pad16(m->out_dim[l]));
  unsigned short *act[2] = {nullptr, nullptr}, *wb = nullptr;
  size_t wtot = 0;
  for (int l = 0; l < m->depth; ++l) wtot += (size_t)pad16(m->out_dim[l]) * pad16(m->in_dim[l]);
  hipError_t e = hipMalloc(&act[0], sizeof(unsigned short) * (size_t)Mp * maxk);
  if (e == hipSuccess) e = hipMalloc(&act[1], sizeof(unsigned short) * (size_t)Mp * maxk);
  if (e == hipSuccess) e = hipMalloc(&wb, sizeof(unsigned short) * wtot);
  int rc = FP4_OK;
  if (e != hipSuccess) rc = m->fail(FP4_E_NOMEM, std::string("BF16 work buffers: ") + hipGetErrorString(e));
  if (!rc) {
    // zero-padded BF16 copies of the input rows and of every weight matrix
    const int k0 = pad16(m->nin);
    hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)(((long)Mp * k0 + 255) / 256)), dim3(256), 0,
                       m->stream, w.H[0], M, m->nin, (long)m->nin, act[0], Mp, k0);
    size_t off = 0;
    std::vector<size_t> woff(m->depth);
    for (int l = 0; l < m->depth && !rc; ++l) {
      const int np = pad16(m->out_dim[l]), kp = pad16(m->in_dim[l]);
      woff[l] = off;
      hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)(((long)np * kp + 255) / 256)), dim3(256), 0,
                         m->stream, m->d_p + m->w_off[l], m->out_dim[l], m->in_dim[l],
                         (long)m->in_dim[l], wb + off, np, kp);
      off += (size_t)np * kp;
    }
    for (int l = 0; l < m->depth && !rc; ++l) {
      const int np = pad16(m->out_dim[l]), kp = pad16(m->in_dim[l]);
      const int last = l + 1 == m->depth;
      dim3 grid((unsigned)(Mp / 64), (unsigned)((np / 16 + 7) / 8));
      hipLaunchKernelGGL(k_fwd_mfma, grid, dim3(256), 0, m->stream, M, kp, m->out_dim[l], np,
                         act[l & 1], wb + woff[l], m->d_p + m->b_off[l], act[(l + 1) & 1],
                         w.H[m->depth], last ? 0 : 1);
    }
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) rc = m->fail(FP4_E_DEVICE, hipGetErrorString(le));
    // the buffers are freed after the stream has finished with them
    const hipError_t se = hipStreamSynchronize(m->stream);
    if (!rc && se != hipSuccess) rc = m->fail(FP4_E_DEVICE, hipGetErrorString(se));
  }
  (void)hipFree(act[0]);
  (void)hipFree(act[1]);
  (void)hipFree(wb);
  return rc;
}

// forward pass from w.H[0] (M rows); FP32 parameters p
int forward(fp4_mlp *m, Work &w, int M, const float *p) {
  for (int l = 0; l < m->depth; ++l) {
    const int act = l + 1 < m->depth;
    MLP_HIP(m, gemm(m->stream, M, m->out_dim[l], m->in_dim[l], w.H[l], m->in_dim[l], 1,
                    p + m->w_off[l], 1, m->in_dim[l], p + m->b_off[l], w.Z[l], w.H[l + 1],
                    m->out_dim[l], act, 0));
  }
  return FP4_OK;
}

// loss and gradient (into m->d_g) for the M rows in w.H[0] / w.y
int forward_backward(fp4_mlp *m, Work &w, int M) {
  int rc = forward(m, w, M, m->d_p);
  if (rc) return rc;
  const int L = m->depth;
  hipLaunchKernelGGL(k_loss, dim3((M + 255) / 256), dim3(256), 0, m->stream, w.H[L], w.y, M,
                     w.dA, w.loss);
  MLP_HIP(m, hipGetLastError());
  float *dcur = w.dA, *dnext = w.dB;
  for (int l = L - 1; l >= 0; --l) {
    const int out = m->out_dim[l], in = m->in_dim[l];
    if (l + 1 < L) {
      hipLaunchKernelGGL(k_silu_back, dim3((unsigned)(((long)M * out + 255) / 256)), dim3(256), 0,
                         m->stream, dcur, w.Z[l], (long)M * out);
      MLP_HIP(m, hipGetLastError());
    }
    // dW[o][k] = sum_i dZ[i][o] H[i][k]
    MLP_HIP(m, gemm(m->stream, out, in, M, dcur, 1, out, w.H[l], in, 1, nullptr, nullptr,
                    m->d_g + m->w_off[l], in, 0, 0));
    hipLaunchKernelGGL(k_colsum, dim3(out), dim3(256), 0, m->stream, dcur, M, out,
                       m->d_g + m->b_off[l]);
    MLP_HIP(m, hipGetLastError());
    if (l > 0) {
      // dH_prev[i][k] = sum_o dZ[i][o] W[o][k]
      MLP_HIP(m, gemm(m->stream, M, in, out, dcur, out, 1, m->d_p + m->w_off[l], in, 1, nullptr,
                      nullptr, dnext, in, 0, 0));
      std::swap(dcur, dnext);
    }
  }
  return FP4_OK;
}

}  // namespace

extern "C" {

int fp4_mlp_create(fp4_mlp **out, int device_id, int32_t nin, int32_t width, int32_t depth,
                   uint64_t seed) {
  if (!out) return FP4_E_INVAL;
  *out = nullptr;
  if (nin < 1 || nin > 256 || width < 1 || width > 1024 || depth < 2 || depth > 16) return FP4_E_INVAL;
  fp4_mlp *m = new (std::nothrow) fp4_mlp();
  if (!m) return FP4_E_NOMEM;
  if (hipSetDevice(device_id) != hipSuccess || hipStreamCreate(&m->stream) != hipSuccess) {
    (void)hipGetLastError();
    delete m;
    return FP4_E_DEVICE;
  }
  m->device = device_id;
  m->nin = nin;
  m->width = width;
  m->depth = depth;
  size_t off = 0;
  for (int l = 0; l < depth; ++l) {
    const int in = l == 0 ? nin : width;
    const int o = l + 1 == depth ? 2 : width;
    m->in_dim.push_back(in);
    m->out_dim.push_back(o);
    m->w_off.push_back(off);
    off += (size_t)in * o;
    m->b_off.push_back(off);
    off += o;
  }
  m->nparam = off;
  // He-style initialisation from a seeded generator (host), biases zero
  std::vector<float> p(off, 0.f);
  std::mt19937_64 rng(seed);
  for (int l = 0; l < depth; ++l) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (float)m->in_dim[l]) * (l + 1 == depth ? 0.1f : 1.f));
    for (size_t i = 0; i < (size_t)m->in_dim[l] * m->out_dim[l]; ++i) p[m->w_off[l] + i] = nd(rng);
  }
  hipError_t e = hipMalloc(&m->d_p, off * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->d_g, off * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->d_m, off * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->d_v, off * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(m->d_p, p.data(), off * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->d_m, 0, off * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->d_v, 0, off * sizeof(float));
  if (e != hipSuccess) {
    fp4_mlp_destroy(m);
    return FP4_E_NOMEM;
  }
  *out = m;
  return FP4_OK;
}

void fp4_mlp_destroy(fp4_mlp *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipFree(m->d_p);
  (void)hipFree(m->d_g);
  (void)hipFree(m->d_m);
  (void)hipFree(m->d_v);
  if (m->stream) (void)hipStreamDestroy(m->stream);
  delete m;
}

const char *fp4_mlp_last_error(const fp4_mlp *m) { return m ? m->err.c_str() : "null network"; }

int64_t fp4_mlp_num_params(const fp4_mlp *m) { return m ? (int64_t)m->nparam : -1; }

int fp4_mlp_get_params(fp4_mlp *m, float *p) {
  if (!m || !p) return FP4_E_INVAL;
  (void)hipSetDevice(m->device);
  MLP_HIP(m, hipMemcpy(p, m->d_p, m->nparam * sizeof(float), hipMemcpyDeviceToHost));
  return FP4_OK;
}

int fp4_mlp_set_params(fp4_mlp *m, const float *p) {
  if (!m || !p) return FP4_E_INVAL;
  for (size_t i = 0; i < m->nparam; ++i)
    if (!std::isfinite(p[i])) return m->fail(FP4_E_INVAL, "parameters contain NaN or Inf");
  (void)hipSetDevice(m->device);
  MLP_HIP(m, hipMemcpy(m->d_p, p, m->nparam * sizeof(float), hipMemcpyHostToDevice));
  return FP4_OK;
}

int fp4_mlp_loss_grad(fp4_mlp *m, const float *X, const float *y, int32_t n, double *loss,
                      float *grad) {
  if (!m || !X || !y || n < 1 || n > (1 << 24)) return FP4_E_INVAL;
  (void)hipSetDevice(m->device);
  Work w;
  int rc = alloc_work(m, w, n);
  if (!rc) {
    hipError_t e = hipMemcpy(w.H[0], X, sizeof(float) * (size_t)n * m->nin, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.y, y, sizeof(float) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = m->fail(FP4_E_DEVICE, hipGetErrorString(e));
  }
  if (!rc) rc = forward_backward(m, w, n);
  if (!rc) {
    std::vector<float> l(n);
    hipError_t e = hipMemcpyAsync(l.data(), w.loss, sizeof(float) * n, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess && grad)
      e = hipMemcpyAsync(grad, m->d_g, sizeof(float) * m->nparam, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) rc = m->fail(FP4_E_DEVICE, hipGetErrorString(e));
    double s = 0.0;
    for (float v : l) s += v;
    if (loss) *loss = s / n;
  }
  free_work(w);
  return rc;
}

int fp4_mlp_train(fp4_mlp *m, const float *X, const float *y, int32_t n, int32_t epochs,
                  int32_t batch, float lr, uint64_t seed, double *loss_per_epoch) {
  if (!m || !X || !y || n < 1 || epochs < 1 || batch < 1 || !(lr > 0.f)) return FP4_E_INVAL;
  (void)hipSetDevice(m->device);
  batch = std::min(batch, n);
  float *dX = nullptr, *dY = nullptr;
  int *didx = nullptr;
  Work w;
  int rc = alloc_work(m, w, batch);
  hipError_t e = hipSuccess;
  if (!rc) e = hipMalloc(&dX, sizeof(float) * (size_t)n * m->nin);
  if (!rc && e == hipSuccess) e = hipMalloc(&dY, sizeof(float) * n);
  if (!rc && e == hipSuccess) e = hipMalloc(&didx, sizeof(int) * n);
  if (!rc && e == hipSuccess) e = hipMemcpy(dX, X, sizeof(float) * (size_t)n * m->nin, hipMemcpyHostToDevice);
  if (!rc && e == hipSuccess) e = hipMemcpy(dY, y, sizeof(float) * n, hipMemcpyHostToDevice);
  if (!rc && e != hipSuccess) rc = m->fail(FP4_E_DEVICE, hipGetErrorString(e));
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::mt19937_64 rng(seed);
  std::vector<float> lbuf(batch);
  for (int ep = 0; ep < epochs && !rc; ++ep) {
    std::shuffle(idx.begin(), idx.end(), rng);
    e = hipMemcpyAsync(didx, idx.data(), sizeof(int) * n, hipMemcpyHostToDevice, m->stream);
    if (e != hipSuccess) { rc = m->fail(FP4_E_DEVICE, hipGetErrorString(e)); break; }
    double eloss = 0.0;
    long nseen = 0;
    for (int b0 = 0; b0 + batch <= n && !rc; b0 += batch) {
      hipLaunchKernelGGL(k_gather, dim3((batch + 255) / 256), dim3(256), 0, m->stream, dX, dY,
                         didx + b0, batch, m->nin, w.H[0], w.y);
      rc = forward_backward(m, w, batch);
      if (rc) break;
      m->adam_t++;
      const float b1 = 0.9f, b2 = 0.999f;
      const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
      hipLaunchKernelGGL(k_adam, dim3((unsigned)((m->nparam + 255) / 256)), dim3(256), 0, m->stream,
                         m->d_p, m->d_g, m->d_m, m->d_v, (long)m->nparam, lr, b1, b2, 1e-8f, c1, c2);
      if (loss_per_epoch) {
        e = hipMemcpyAsync(lbuf.data(), w.loss, sizeof(float) * batch, hipMemcpyDeviceToHost, m->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
        if (e != hipSuccess) { rc = m->fail(FP4_E_DEVICE, hipGetErrorString(e)); break; }
        for (float v : lbuf) eloss += v;
        nseen += batch;
      }
    }
    if (loss_per_epoch) loss_per_epoch[ep] = nseen ? eloss / nseen : 0.0;
  }
  if (!rc) {
    e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) rc = m->fail(FP4_E_DEVICE, hipGetErrorString(e));
  }
  (void)hipFree(dX);
  (void)hipFree(dY);
  (void)hipFree(didx);
  free_work(w);
  return rc;
}

int fp4_mlp_predict(fp4_mlp *m, const float *X, int32_t n, int32_t bf16, float *out,
                    double *ms) {
  if (!m || !X || !out || n < 1 || n > (1 << 24)) return FP4_E_INVAL;
  (void)hipSetDevice(m->device);
  Work w;
  int rc = alloc_work(m, w, n);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc) {
    hipError_t e = hipMemcpy(w.H[0], X, sizeof(float) * (size_t)n * m->nin, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, m->stream);
    if (e != hipSuccess) rc = m->fail(FP4_E_DEVICE, hipGetErrorString(e));
  }
  if (!rc) {
    if (bf16) {
      rc = forward_bf16_mfma(m, w, n);
    } else {
      rc = forward(m, w, n, m->d_p);
    }
  }
  if (!rc) {
    hipError_t e = hipEventRecord(e1, m->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, w.H[m->depth], sizeof(float) * 2 * (size_t)n, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) rc = m->fail(FP4_E_DEVICE, hipGetErrorString(e));
    if (ms) *ms = t;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  free_work(w);
  return rc;
}

}  // extern "C"
