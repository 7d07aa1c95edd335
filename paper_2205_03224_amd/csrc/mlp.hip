// Learned warm start: a 3-layer perceptron that maps per-node features of
// the interface unknowns to a starting basis for the low-rank setup (the
// block iteration of gs_lowrank), trained on bases the library's own Arnoldi
// produces.  Forward, subspace loss, backward and Adam are kernels of this
// file; all in float32, reductions over rows in a fixed order.
//
//   a1 = tanh(X W1 + b1),  a2 = tanh(a1 W2 + b2),  Y = a2 W3 + b3
//   loss = ||Y^T Y||_F^2 - 2 ||W^T Y||_F^2 + k_w    (= ||Y Y^T - W W^T||_F^2
//                                                   for orthonormal W)
//   dloss/dY = 4 Y (Y^T Y) - 4 W (W^T Y)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "device.h"
#include "engine.h"

namespace gs {

namespace {

constexpr int kMaxDim = 64;       // widest layer supported (LDS tiles below)
constexpr int kRowsPerBlock = 64; // rows of one dense-layer tile
constexpr int kAtbRows = 64;      // rows per partial of A^T B

// Z = act(A W + b): A rows x in (row-major), W in x out, Z rows x out.
// One workgroup per 64-row tile; W and the A tile staged in LDS.
template <int ACT>
__global__ __launch_bounds__(256) void k_dense(const float* A, int64_t rows, int in,
                                               const float* W, const float* b, int out,
                                               float* Z) {
  extern __shared__ __align__(16) float sm[];
  float* Ws = sm;                         // in x out
  float* As = sm + in * out;              // 64 x in
  const int tid = threadIdx.x;
  for (int i = tid; i < in * out; i += blockDim.x) Ws[i] = W[i];
  const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
  for (int i = tid; i < kRowsPerBlock * in; i += blockDim.x) {
    const int64_t r = r0 + i / in;
    As[i] = r < rows ? A[r * in + i % in] : 0.0f;
  }
  __syncthreads();
  const int lr = tid % kRowsPerBlock;
  const int64_t r = r0 + lr;
  if (r >= rows) return;
  for (int o = tid / kRowsPerBlock; o < out; o += blockDim.x / kRowsPerBlock) {
    float acc = b ? b[o] : 0.0f;
    for (int i = 0; i < in; ++i) acc = fmaf(As[lr * in + i], Ws[i * out + o], acc);
    Z[r * out + o] = ACT ? tanhf(acc) : acc;
  }
}

// dA = (dZ W^T) * (1 - act^2): dZ rows x out, W in x out, act rows x in.
__global__ __launch_bounds__(256) void k_dense_bwd(const float* dZ, int64_t rows, int out,
                                                   const float* W, int in, const float* act,
                                                   float* dA) {
  extern __shared__ __align__(16) float sm[];
  float* Ws = sm;                         // in x out
  float* Ds = sm + in * out;              // 64 x out
  const int tid = threadIdx.x;
  for (int i = tid; i < in * out; i += blockDim.x) Ws[i] = W[i];
  const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
  for (int i = tid; i < kRowsPerBlock * out; i += blockDim.x) {
    const int64_t r = r0 + i / out;
    Ds[i] = r < rows ? dZ[r * out + i % out] : 0.0f;
  }
  __syncthreads();
  const int lr = tid % kRowsPerBlock;
  const int64_t r = r0 + lr;
  if (r >= rows) return;
  for (int i = tid / kRowsPerBlock; i < in; i += blockDim.x / kRowsPerBlock) {
    float acc = 0.0f;
    for (int o = 0; o < out; ++o) acc = fmaf(Ds[lr * out + o], Ws[i * out + o], acc);
    const float a = act[r * in + i];
    dA[r * in + i] = acc * (1.0f - a * a);
  }
}

// partial[blk][i*n + j] = sum over the block's rows of A[r,i] B[r,j]
// (A rows x m, B rows x n); with B == null, column sums of A (n = 1).
__global__ __launch_bounds__(256) void k_atb(const float* A, int m, const float* B, int n,
                                             int64_t rows, float* partial) {
  extern __shared__ __align__(16) float sm[];
  float* As = sm;                          // kAtbRows x m
  float* Bs = sm + kAtbRows * m;           // kAtbRows x n
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kAtbRows;
  for (int i = tid; i < kAtbRows * m; i += blockDim.x) {
    const int64_t r = r0 + i / m;
    As[i] = r < rows ? A[r * m + i % m] : 0.0f;
  }
  for (int i = tid; i < kAtbRows * n; i += blockDim.x) {
    const int64_t r = r0 + i / n;
    Bs[i] = (r < rows) ? (B ? B[r * n + i % n] : 1.0f) : 0.0f;
  }
  __syncthreads();
  float* out = partial + (int64_t)blockIdx.x * m * n;
  for (int e = tid; e < m * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    float acc = 0.0f;
    for (int rr = 0; rr < kAtbRows; ++rr) acc = fmaf(As[rr * m + i], Bs[rr * n + j], acc);
    out[e] = acc;
  }
}

// out[e] (+)= sum_b partial[b][e], fixed order over b
__global__ void k_sum_blocks(const float* partial, int nblk, int len, float* out, int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  float acc = 0.0f;
  for (int b = 0; b < nblk; ++b) acc += partial[(int64_t)b * len + e];
  out[e] = accumulate ? out[e] + acc : acc;
}

// dY = 4 (Y G1 - W G2): Y rows x ky, W rows x kw, G1 ky x ky, G2 kw x ky
__global__ __launch_bounds__(256) void k_lossgrad(const float* Y, int ky, const float* Wt, int kw,
                                                  const float* G1, const float* G2,
                                                  int64_t rows, float* dY) {
  extern __shared__ __align__(16) float sm[];
  float* g1 = sm;
  float* g2 = sm + ky * ky;
  for (int i = threadIdx.x; i < ky * ky; i += blockDim.x) g1[i] = G1[i];
  for (int i = threadIdx.x; i < kw * ky; i += blockDim.x) g2[i] = G2[i];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * ky) return;
  const int64_t r = e / ky;
  const int c = (int)(e % ky);
  float acc = 0.0f;
  for (int i = 0; i < ky; ++i) acc = fmaf(Y[r * ky + i], g1[i * ky + c], acc);
  for (int i = 0; i < kw; ++i) acc = fmaf(-Wt[r * kw + i], g2[i * ky + c], acc);
  dY[e] = 4.0f * acc;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

struct Mlp {
  int in = 0, hid = 0, out = 0;
  hipStream_t st = nullptr;
  DevMem mem;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  int nparams = 0, step = 0;
  std::unique_ptr<DevMem> work;
  int64_t cap_rows = 0;
  float *a1 = nullptr, *a2 = nullptr, *y = nullptr, *dy = nullptr, *d2 = nullptr, *d1 = nullptr;
  float *partial = nullptr, *g1 = nullptr, *g2 = nullptr;
  std::string err;

  float* W1() { return params; }
  float* b1() { return W1() + in * hid; }
  float* W2() { return b1() + hid; }
  float* b2() { return W2() + hid * hid; }
  float* W3() { return b2() + hid; }
  float* b3() { return W3() + hid * out; }

  void ensure(int64_t rows) {
    if (rows <= cap_rows) return;
    // the old buffers may still be read by queued kernels
    hipcheck(hipStreamSynchronize(st), "mlp grow");
    work = std::make_unique<DevMem>();
    cap_rows = rows;
    a1 = work->alloc<float>(rows * hid);
    a2 = work->alloc<float>(rows * hid);
    y = work->alloc<float>(rows * kMaxDim);
    dy = work->alloc<float>(rows * kMaxDim);
    d2 = work->alloc<float>(rows * hid);
    d1 = work->alloc<float>(rows * hid);
    const int64_t nblk = (rows + kAtbRows - 1) / kAtbRows;
    partial = work->alloc<float>(nblk * kMaxDim * kMaxDim);
    g1 = work->alloc<float>(kMaxDim * kMaxDim);
    g2 = work->alloc<float>(kMaxDim * kMaxDim);
  }

  void dense(const float* A, int64_t rows, int i_, const float* W, const float* b, int o_,
             float* Z, bool act) {
    const int nb = (int)((rows + kRowsPerBlock - 1) / kRowsPerBlock);
    const size_t lds = (size_t)(i_ * o_ + kRowsPerBlock * i_) * sizeof(float);
    if (act) hipLaunchKernelGGL(k_dense<1>, dim3(nb), dim3(256), lds, st, A, rows, i_, W, b, o_, Z);
    else hipLaunchKernelGGL(k_dense<0>, dim3(nb), dim3(256), lds, st, A, rows, i_, W, b, o_, Z);
  }
  void dense_bwd(const float* dZ, int64_t rows, int o_, const float* W, int i_, const float* act,
                 float* dA) {
    const int nb = (int)((rows + kRowsPerBlock - 1) / kRowsPerBlock);
    const size_t lds = (size_t)(i_ * o_ + kRowsPerBlock * o_) * sizeof(float);
    hipLaunchKernelGGL(k_dense_bwd, dim3(nb), dim3(256), lds, st, dZ, rows, o_, W, i_, act, dA);
  }
  // out (+)= A^T B over all rows (B null: column sums of A)
  void atb(const float* A, int m_, const float* B, int n_, int64_t rows, float* outp, bool acc) {
    const int nb = (int)((rows + kAtbRows - 1) / kAtbRows);
    const int nn = B ? n_ : 1;
    const size_t lds = (size_t)kAtbRows * (m_ + nn) * sizeof(float);
    hipLaunchKernelGGL(k_atb, dim3(nb), dim3(256), lds, st, A, m_, B, nn, rows, partial);
    const int len = m_ * nn;
    hipLaunchKernelGGL(k_sum_blocks, dim3((len + 255) / 256), dim3(256), 0, st, partial, nb, len,
                       outp, acc ? 1 : 0);
  }
  // Y must be valid for `rows` rows: callers that use the internal y buffer
  // call ensure(rows) first and pass it afterwards
  void forward(const float* X, int64_t rows, float* Y) {
    ensure(rows);
    if (!Y) throw Error(GS_EINVAL, "null network output");
    dense(X, rows, in, W1(), b1(), hid, a1, true);
    dense(a1, rows, hid, W2(), b2(), hid, a2, true);
    dense(a2, rows, hid, W3(), b3(), out, Y, false);
  }
};

}  // namespace gs

using gs::Error;
using gs::Mlp;

struct gs_mlp {
  Mlp m;
};

#define MLP_GUARD(h, ...)                       \
  try {                                         \
    __VA_ARGS__;                                \
  } catch (const Error& e) {                    \
    if (h) (h)->m.err = e.what();               \
    return e.code;                              \
  } catch (const std::exception& e) {           \
    if (h) (h)->m.err = e.what();               \
    return GS_EINVAL;                           \
  }

extern "C" {

int gs_mlp_create(gs_mlp** out, int in_dim, int hidden, int out_dim, uint64_t seed, int device,
                  void* stream) {
  if (!out) return GS_EINVAL;
  *out = nullptr;
  if (in_dim < 1 || hidden < 1 || out_dim < 1 || in_dim > gs::kMaxDim || hidden > gs::kMaxDim ||
      out_dim > gs::kMaxDim)
    return GS_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return GS_EDEVICE;
  auto h = std::make_unique<gs_mlp>();
  MLP_GUARD(h.get(), {
    Mlp& m = h->m;
    m.in = in_dim;
    m.hid = hidden;
    m.out = out_dim;
    m.st = (hipStream_t)stream;
    m.nparams = in_dim * hidden + hidden + hidden * hidden + hidden + hidden * out_dim + out_dim;
    m.params = m.mem.alloc<float>(m.nparams);
    m.grads = m.mem.alloc<float>(m.nparams);
    m.m = m.mem.alloc<float>(m.nparams);
    m.v = m.mem.alloc<float>(m.nparams);
    // Glorot-uniform weights, zero biases: packed parameter j (weights only)
    // is sqrt(6 / (fan_in + fan_out)) of its layer times v_j, v the
    // SplitMix64 start vector of `seed` over all nparams positions
    {
      std::vector<double> v((size_t)m.nparams);
      gs::start_vector(seed, m.nparams, v.data());
      std::vector<float> p((size_t)m.nparams, 0.0f);
      const int dims[4] = {in_dim, hidden, hidden, out_dim};
      size_t o = 0;
      for (int layer = 0; layer < 3; ++layer) {
        const int a = dims[layer], b = dims[layer + 1];
        const double lim = std::sqrt(6.0 / (double)(a + b));
        for (int e = 0; e < a * b; ++e, ++o) p[o] = (float)(lim * v[o]);
        o += (size_t)b;  // biases stay zero
      }
      gs::hipcheck(hipMemcpyAsync(m.params, p.data(), p.size() * sizeof(float),
                                  hipMemcpyHostToDevice, m.st),
                   "mlp init");
      gs::hipcheck(hipStreamSynchronize(m.st), "mlp init");
    }
    gs::launch_fill<float>(m.grads, 0.0f, m.nparams, m.st);
    gs::launch_fill<float>(m.m, 0.0f, m.nparams, m.st);
    gs::launch_fill<float>(m.v, 0.0f, m.nparams, m.st);
    gs::hipcheck(hipStreamSynchronize(m.st), "mlp create");
    *out = h.release();
    return GS_OK;
  });
}

void gs_mlp_destroy(gs_mlp* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->m.st);
  delete h;
}

int gs_mlp_nparams(const gs_mlp* h) { return h ? h->m.nparams : 0; }

const char* gs_mlp_last_error(const gs_mlp* h) { return h ? h->m.err.c_str() : ""; }

int gs_mlp_set_params(gs_mlp* h, const float* params) {
  if (!h || !params) return GS_EINVAL;
  MLP_GUARD(h, {
    gs::hipcheck(hipMemcpyAsync(h->m.params, params, h->m.nparams * sizeof(float),
                                hipMemcpyHostToDevice, h->m.st), "set params");
    gs::launch_fill<float>(h->m.m, 0.0f, h->m.nparams, h->m.st);
    gs::launch_fill<float>(h->m.v, 0.0f, h->m.nparams, h->m.st);
    h->m.step = 0;
    gs::hipcheck(hipStreamSynchronize(h->m.st), "set params");
    return GS_OK;
  });
}

static int copy_out(gs_mlp* h, const float* src, float* dst) {
  MLP_GUARD(h, {
    gs::hipcheck(hipMemcpyAsync(dst, src, h->m.nparams * sizeof(float), hipMemcpyDeviceToHost,
                                h->m.st), "copy out");
    gs::hipcheck(hipStreamSynchronize(h->m.st), "copy out");
    return GS_OK;
  });
}

int gs_mlp_get_params(const gs_mlp* h, float* params) {
  if (!h || !params) return GS_EINVAL;
  return copy_out(const_cast<gs_mlp*>(h), h->m.params, params);
}

int gs_mlp_get_grads(const gs_mlp* h, float* grads) {
  if (!h || !grads) return GS_EINVAL;
  return copy_out(const_cast<gs_mlp*>(h), h->m.grads, grads);
}

int gs_mlp_zero_grad(gs_mlp* h) {
  if (!h) return GS_EINVAL;
  gs::launch_fill<float>(h->m.grads, 0.0f, h->m.nparams, h->m.st);
  return GS_OK;
}

int gs_mlp_forward(gs_mlp* h, const float* X, int64_t rows, float* Y) {
  if (!h || !X || !Y || rows < 0) return GS_EINVAL;
  MLP_GUARD(h, {
    if (rows == 0) return GS_OK;
    h->m.forward(X, rows, Y);
    gs::hipcheck(hipGetLastError(), "mlp forward");
    return GS_OK;
  });
}

int gs_mlp_loss_backward(gs_mlp* h, const float* X, const float* Wt, int64_t rows, int kw,
                         double* loss) {
  if (!h || !X || !Wt || !loss || rows <= 0 || kw < 1 || kw > gs::kMaxDim) return GS_EINVAL;
  MLP_GUARD(h, {
    Mlp& m = h->m;
    m.ensure(rows);  // before taking m.y: growing reallocates it
    m.forward(X, rows, m.y);
    const int ky = m.out;
    // Gram matrices G1 = Y^T Y (ky x ky), G2 = W^T Y (kw x ky)
    m.atb(m.y, ky, m.y, ky, rows, m.g1, false);
    m.atb(Wt, kw, m.y, ky, rows, m.g2, false);
    std::vector<float> g1((size_t)ky * ky), g2((size_t)kw * ky);
    gs::hipcheck(hipMemcpyAsync(g1.data(), m.g1, g1.size() * 4, hipMemcpyDeviceToHost, m.st), "loss");
    gs::hipcheck(hipMemcpyAsync(g2.data(), m.g2, g2.size() * 4, hipMemcpyDeviceToHost, m.st), "loss");
    gs::hipcheck(hipStreamSynchronize(m.st), "loss");
    double l = kw;
    for (float x : g1) l += (double)x * x;
    for (float x : g2) l -= 2.0 * (double)x * x;
    *loss = l;
    // dY, then back through the layers (gradients accumulate)
    const int64_t ne = rows * ky;
    hipLaunchKernelGGL(gs::k_lossgrad, dim3((unsigned)((ne + 255) / 256)), dim3(256),
                       (size_t)(ky * ky + kw * ky) * sizeof(float), m.st, m.y, ky, Wt, kw, m.g1,
                       m.g2, rows, m.dy);
    float* gW1 = m.grads;
    float* gb1 = gW1 + m.in * m.hid;
    float* gW2 = gb1 + m.hid;
    float* gb2 = gW2 + m.hid * m.hid;
    float* gW3 = gb2 + m.hid;
    float* gb3 = gW3 + m.hid * m.out;
    m.atb(m.a2, m.hid, m.dy, ky, rows, gW3, true);
    m.atb(m.dy, ky, nullptr, 1, rows, gb3, true);
    m.dense_bwd(m.dy, rows, ky, m.W3(), m.hid, m.a2, m.d2);
    m.atb(m.a1, m.hid, m.d2, m.hid, rows, gW2, true);
    m.atb(m.d2, m.hid, nullptr, 1, rows, gb2, true);
    m.dense_bwd(m.d2, rows, m.hid, m.W2(), m.hid, m.a1, m.d1);
    m.atb(X, m.in, m.d1, m.hid, rows, gW1, true);
    m.atb(m.d1, m.hid, nullptr, 1, rows, gb1, true);
    gs::hipcheck(hipGetLastError(), "mlp backward");
    return GS_OK;
  });
}

int gs_mlp_adam_step(gs_mlp* h, float lr, float beta1, float beta2, float eps) {
  if (!h) return GS_EINVAL;
  MLP_GUARD(h, {
    Mlp& m = h->m;
    m.step += 1;
    const float c1 = 1.0f - std::pow(beta1, (float)m.step);
    const float c2 = 1.0f - std::pow(beta2, (float)m.step);
    hipLaunchKernelGGL(gs::k_adam, dim3((m.nparams + 255) / 256), dim3(256), 0, m.st, m.params,
                       m.grads, m.m, m.v, m.nparams, lr, beta1, beta2, eps, c1, c2);
    gs::hipcheck(hipGetLastError(), "adam");
    return GS_OK;
  });
}

}  // extern "C"
