// Host side of the loop surrogate network: parameters, Adam state,
// workspaces, forward pass, loss gradient, Adam step and a training loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "kernels.h"
#include "tufrg.h"

using namespace tufrg;

struct tufrg_mlp {
  hipStream_t st = nullptr;
  std::vector<int> sizes;  // n_in, hidden..., n_out
  std::vector<long long> woff, boff;
  long long n_params = 0;
  int maxw = 0;
  float *d_p = nullptr, *d_m = nullptr, *d_v = nullptr, *d_g = nullptr;
  int t = 0;  // Adam steps taken
  // workspaces for a chunk of rows
  int cap = 0;
  std::vector<float *> act, pre;  // per hidden layer [cap][width]
  float *d_y = nullptr, *d_dy = nullptr, *d_da = nullptr, *d_part = nullptr;
  double *d_loss = nullptr, *h_loss = nullptr;
  int *d_idx = nullptr, *h_idx = nullptr;
  long long idx_cap = 0;
  float *d_xb = nullptr, *d_tb = nullptr;
  int xb_cap = 0;
  std::vector<void *> allocs;
  std::string err;
};

namespace {

constexpr int FWD_CHUNK = 16384;

thread_local std::string g_mlp_err;

tufrg_status mfail(tufrg_mlp *m, tufrg_status s, const std::string &msg) {
  if (m)
    m->err = msg;
  else
    g_mlp_err = msg;
  return s;
}

template <typename T>
tufrg_status malloc_d(tufrg_mlp *m, T **p, size_t n) {
  void *v = nullptr;
  if (hipMalloc(&v, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return mfail(m, TUFRG_E_NOMEM, "hipMalloc failed");
  }
  m->allocs.push_back(v);
  *p = (T *)v;
  return TUFRG_OK;
}

void free_one(tufrg_mlp *m, void *p) {
  if (!p) return;
  auto it = std::find(m->allocs.begin(), m->allocs.end(), p);
  if (it != m->allocs.end()) m->allocs.erase(it);
  (void)hipFree(p);
}

bool on_device(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

#define MTRY(x)                       \
  do {                                \
    tufrg_status s_ = (x);            \
    if (s_ != TUFRG_OK) return s_;    \
  } while (0)
#define MHIP(m, x)                                                                 \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      (void)hipGetLastError();                                                     \
      return mfail(m, TUFRG_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    }                                                                              \
  } while (0)

// workspaces for chunks of up to rows rows
tufrg_status reserve(tufrg_mlp *m, int rows) {
  if (rows <= m->cap) return TUFRG_OK;
  MHIP(m, hipStreamSynchronize(m->st));
  for (float *p : m->act) free_one(m, p);
  for (float *p : m->pre) free_one(m, p);
  free_one(m, m->d_y);
  free_one(m, m->d_dy);
  free_one(m, m->d_da);
  free_one(m, m->d_part);
  m->act.clear();
  m->pre.clear();
  const int L = (int)m->sizes.size() - 1;
  for (int l = 1; l < L; ++l) {
    float *a = nullptr, *z = nullptr;
    MTRY(malloc_d(m, &a, (size_t)rows * m->sizes[l]));
    MTRY(malloc_d(m, &z, (size_t)rows * m->sizes[l]));
    m->act.push_back(a);
    m->pre.push_back(z);
  }
  MTRY(malloc_d(m, &m->d_y, (size_t)rows * m->sizes[L]));
  MTRY(malloc_d(m, &m->d_dy, (size_t)rows * m->maxw));
  MTRY(malloc_d(m, &m->d_da, (size_t)rows * m->maxw));
  MTRY(malloc_d(m, &m->d_part, (size_t)((rows + 63) / 64) * m->maxw));
  m->cap = rows;
  return TUFRG_OK;
}

// forward of rows [0, n) of X (n <= cap); hidden activations stay in the
// workspace, the output goes to Y (leading dimension n_out)
tufrg_status forward_chunk(tufrg_mlp *m, int n, const float *X, float *Y) {
  const int L = (int)m->sizes.size() - 1;
  const float *a = X;
  for (int l = 0; l < L; ++l) {
    const int ni = m->sizes[l], no = m->sizes[l + 1];
    const float *W = m->d_p + m->woff[l], *b = m->d_p + m->boff[l];
    const bool last = l + 1 == L;
    float *out = last ? Y : m->act[l];
    MHIP(m, launch_gemm_f32(n, no, ni, a, ni, 0, W, ni, 1, b, last ? 1 : 2, out, no, last ? nullptr : m->pre[l],
                            m->st));
    a = out;
  }
  return TUFRG_OK;
}

tufrg_status loss_grad_internal(tufrg_mlp *m, int n, const float *X, const float *T, float *grad) {
  const int L = (int)m->sizes.size() - 1;
  MTRY(reserve(m, n));
  MTRY(forward_chunk(m, n, X, m->d_y));
  const int nout = m->sizes[L];
  MHIP(m, launch_mse_grad((long long)n * nout, m->d_y, T, m->d_dy, m->d_loss, m->st));
  // d_dy holds dZ of the last layer; walk back
  float *dz = m->d_dy, *spare = m->d_da;
  for (int l = L - 1; l >= 0; --l) {
    const int ni = m->sizes[l], no = m->sizes[l + 1];
    const float *ain = l == 0 ? X : m->act[l - 1];
    // dW[o][i] = sum_r dz[r][o] a[r][i]
    MHIP(m, launch_gemm_f32(no, ni, n, dz, no, 1, ain, ni, 0, nullptr, 0, grad + m->woff[l], ni, nullptr, m->st));
    MHIP(m, launch_colsum(n, no, dz, m->d_part, grad + m->boff[l], m->st));
    if (l > 0) {
      // dA[r][i] = sum_o dz[r][o] W[o][i], then times GELU'(z) of layer l - 1
      MHIP(m, launch_gemm_f32(n, ni, no, dz, no, 0, m->d_p + m->woff[l], ni, 0, nullptr, 0, spare, ni, nullptr,
                              m->st));
      MHIP(m, launch_gelu_bwd((long long)n * ni, m->pre[l - 1], spare, m->st));
      std::swap(dz, spare);
    }
  }
  return TUFRG_OK;
}

}  // namespace

namespace tufrg {
// used by the context to run the surrogate over its loop blocks
tufrg_status mlp_forward_internal(tufrg_mlp *m, long long n, const float *X, float *Y) {
  const int nin = m->sizes.front(), nout = m->sizes.back();
  MTRY(reserve(m, (int)std::min<long long>(n, FWD_CHUNK)));
  for (long long r = 0; r < n; r += m->cap) {
    const int rows = (int)std::min<long long>(m->cap, n - r);
    MTRY(forward_chunk(m, rows, X + r * nin, Y + r * nout));
  }
  return TUFRG_OK;
}
int mlp_n_in(const tufrg_mlp *m) { return m->sizes.front(); }
hipStream_t mlp_stream(const tufrg_mlp *m) { return m->st; }
int mlp_n_out(const tufrg_mlp *m) { return m->sizes.back(); }
}  // namespace tufrg

extern "C" const char *tufrg_mlp_last_error(const tufrg_mlp *m) { return m ? m->err.c_str() : g_mlp_err.c_str(); }

extern "C" tufrg_status tufrg_mlp_create(int32_t n_sizes, const int32_t *sizes, const float *params, void *stream,
                                         tufrg_mlp **out) {
  if (!out) return mfail(nullptr, TUFRG_E_INVAL, "null output pointer");
  *out = nullptr;
  if (n_sizes < 2 || !sizes) return mfail(nullptr, TUFRG_E_INVAL, "need at least an input and an output size");
  for (int i = 0; i < n_sizes; ++i)
    if (sizes[i] <= 0 || sizes[i] > 65536) return mfail(nullptr, TUFRG_E_INVAL, "layer sizes must be in [1, 65536]");
  tufrg_mlp *m = new tufrg_mlp();
  m->st = (hipStream_t)stream;
  m->sizes.assign(sizes, sizes + n_sizes);
  long long o = 0;
  for (int l = 0; l + 1 < n_sizes; ++l) {
    m->woff.push_back(o);
    o += (long long)sizes[l] * sizes[l + 1];
    m->boff.push_back(o);
    o += sizes[l + 1];
  }
  m->n_params = o;
  m->maxw = *std::max_element(m->sizes.begin() + 1, m->sizes.end());
  auto bail = [&](tufrg_status s) {
    g_mlp_err = m->err;
    for (void *p : m->allocs) (void)hipFree(p);
    if (m->h_loss) (void)hipHostFree(m->h_loss);
    delete m;
    return s;
  };
  tufrg_status s;
  if ((s = malloc_d(m, &m->d_p, o)) || (s = malloc_d(m, &m->d_m, o)) || (s = malloc_d(m, &m->d_v, o)) ||
      (s = malloc_d(m, &m->d_g, o)) || (s = malloc_d(m, &m->d_loss, 1)))
    return bail(s);
  if (hipHostMalloc((void **)&m->h_loss, sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    m->err = "hipHostMalloc failed";
    return bail(TUFRG_E_NOMEM);
  }
  hipError_t e = hipSuccess;
  if (params)
    e = hipMemcpyAsync(m->d_p, params, o * sizeof(float), hipMemcpyHostToDevice, m->st);
  else
    e = hipMemsetAsync(m->d_p, 0, o * sizeof(float), m->st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_m, 0, o * sizeof(float), m->st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_v, 0, o * sizeof(float), m->st);
  if (e == hipSuccess) e = hipStreamSynchronize(m->st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    m->err = std::string("upload failed: ") + hipGetErrorString(e);
    return bail(TUFRG_E_HIP);
  }
  *out = m;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_mlp_destroy(tufrg_mlp *m) {
  if (!m) return TUFRG_OK;
  (void)hipStreamSynchronize(m->st);
  for (void *p : m->allocs) (void)hipFree(p);
  if (m->h_loss) (void)hipHostFree(m->h_loss);
  if (m->h_idx) (void)hipHostFree(m->h_idx);
  delete m;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_mlp_n_params(const tufrg_mlp *m, int64_t *n) {
  if (!m || !n) return mfail(nullptr, TUFRG_E_INVAL, "null argument");
  *n = m->n_params;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_mlp_params(tufrg_mlp *m, float *dst) {
  if (!m) return mfail(nullptr, TUFRG_E_INVAL, "null network");
  if (!on_device(dst)) return mfail(m, TUFRG_E_INVAL, "params must be a device pointer");
  MHIP(m, hipMemcpyAsync(dst, m->d_p, m->n_params * sizeof(float), hipMemcpyDeviceToDevice, m->st));
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_mlp_set_params(tufrg_mlp *m, const float *src) {
  if (!m) return mfail(nullptr, TUFRG_E_INVAL, "null network");
  if (!on_device(src)) return mfail(m, TUFRG_E_INVAL, "params must be a device pointer");
  MHIP(m, hipMemcpyAsync(m->d_p, src, m->n_params * sizeof(float), hipMemcpyDeviceToDevice, m->st));
  MHIP(m, hipMemsetAsync(m->d_m, 0, m->n_params * sizeof(float), m->st));
  MHIP(m, hipMemsetAsync(m->d_v, 0, m->n_params * sizeof(float), m->st));
  m->t = 0;
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_mlp_forward(tufrg_mlp *m, int64_t n, const float *X, float *Y) {
  if (!m) return mfail(nullptr, TUFRG_E_INVAL, "null network");
  if (n < 0) return mfail(m, TUFRG_E_INVAL, "negative row count");
  if (n == 0) return TUFRG_OK;
  if (!on_device(X) || !on_device(Y)) return mfail(m, TUFRG_E_INVAL, "X, Y must be device pointers");
  return mlp_forward_internal(m, n, X, Y);
}

extern "C" tufrg_status tufrg_mlp_loss_grad(tufrg_mlp *m, int32_t n, const float *X, const float *T, float *grad,
                                            double *loss) {
  if (!m) return mfail(nullptr, TUFRG_E_INVAL, "null network");
  if (n <= 0 || n > 65536) return mfail(m, TUFRG_E_INVAL, "batch must be in [1, 65536]");
  if (!on_device(X) || !on_device(T) || (grad && !on_device(grad)))
    return mfail(m, TUFRG_E_INVAL, "X, T, grad must be device pointers");
  MHIP(m, hipMemsetAsync(m->d_loss, 0, sizeof(double), m->st));
  MTRY(loss_grad_internal(m, n, X, T, grad ? grad : m->d_g));
  if (loss) {
    MHIP(m, hipMemcpyAsync(m->h_loss, m->d_loss, sizeof(double), hipMemcpyDeviceToHost, m->st));
    MHIP(m, hipStreamSynchronize(m->st));
    *loss = *m->h_loss;
  }
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_mlp_adam_step(tufrg_mlp *m, const float *grad, float lr) {
  if (!m) return mfail(nullptr, TUFRG_E_INVAL, "null network");
  if (grad && !on_device(grad)) return mfail(m, TUFRG_E_INVAL, "grad must be a device pointer");
  m->t++;
  MHIP(m, launch_adam(m->n_params, m->d_p, grad ? grad : m->d_g, m->d_m, m->d_v, lr, 0.9f, 0.999f, 1e-8f, m->t,
                      m->st));
  return TUFRG_OK;
}

extern "C" tufrg_status tufrg_mlp_train(tufrg_mlp *m, int64_t n, const float *X, const float *T, int32_t batch,
                                        int32_t epochs, float lr, uint64_t seed, double *last_epoch_loss) {
  if (!m) return mfail(nullptr, TUFRG_E_INVAL, "null network");
  if (n <= 0 || batch <= 0 || batch > 65536 || epochs < 0) return mfail(m, TUFRG_E_INVAL, "bad sizes");
  if (!on_device(X) || !on_device(T)) return mfail(m, TUFRG_E_INVAL, "X, T must be device pointers");
  const int nin = m->sizes.front(), nout = m->sizes.back();
  const int b = (int)std::min<long long>(batch, n);
  if (n > m->idx_cap) {
    MHIP(m, hipStreamSynchronize(m->st));
    free_one(m, m->d_idx);
    if (m->h_idx) (void)hipHostFree(m->h_idx);
    m->h_idx = nullptr;
    MTRY(malloc_d(m, &m->d_idx, n));
    if (hipHostMalloc((void **)&m->h_idx, n * sizeof(int), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return mfail(m, TUFRG_E_NOMEM, "hipHostMalloc failed");
    }
    m->idx_cap = n;
  }
  if (b > m->xb_cap) {
    MHIP(m, hipStreamSynchronize(m->st));
    free_one(m, m->d_xb);
    free_one(m, m->d_tb);
    m->d_xb = m->d_tb = nullptr;
    m->xb_cap = 0;
    MTRY(malloc_d(m, &m->d_xb, (size_t)b * nin));
    MTRY(malloc_d(m, &m->d_tb, (size_t)b * nout));
    m->xb_cap = b;
  }
  MTRY(reserve(m, b));
  std::mt19937_64 rng(seed);
  std::vector<int> perm(n);
  const int nb = (int)((n + b - 1) / b);
  double last = 0.0;
  for (int ep = 0; ep < epochs; ++ep) {
    for (long long i = 0; i < n; ++i) perm[i] = (int)i;
    std::shuffle(perm.begin(), perm.end(), rng);
    // the previous epoch's index upload has completed (synchronised below)
    std::memcpy(m->h_idx, perm.data(), n * sizeof(int));
    MHIP(m, hipMemcpyAsync(m->d_idx, m->h_idx, n * sizeof(int), hipMemcpyHostToDevice, m->st));
    MHIP(m, hipMemsetAsync(m->d_loss, 0, sizeof(double), m->st));
    for (int k = 0; k < nb; ++k) {
      const int r0 = k * b, rows = (int)std::min<long long>(b, n - r0);
      MHIP(m, launch_gather_rows(rows, nin, m->d_idx + r0, X, m->d_xb, m->st));
      MHIP(m, launch_gather_rows(rows, nout, m->d_idx + r0, T, m->d_tb, m->st));
      MTRY(loss_grad_internal(m, rows, m->d_xb, m->d_tb, m->d_g));
      m->t++;
      MHIP(m, launch_adam(m->n_params, m->d_p, m->d_g, m->d_m, m->d_v, lr, 0.9f, 0.999f, 1e-8f, m->t, m->st));
    }
    MHIP(m, hipMemcpyAsync(m->h_loss, m->d_loss, sizeof(double), hipMemcpyDeviceToHost, m->st));
    MHIP(m, hipStreamSynchronize(m->st));
    last = *m->h_loss / nb;
  }
  if (last_epoch_loss) *last_epoch_loss = last;
  return TUFRG_OK;
}
