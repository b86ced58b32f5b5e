// C ABI of the spin surrogate network (see include/spintrack.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mlp_kernels.h"
#include "spintrack.h"

struct st_mlp {
  int device = 0;
  int n_in = 0;
  std::string err;
  st::MlpOffsets off{};
  int64_t n_params = 0;
  int64_t step = 0;                 // Adam steps taken
  float frame_ref[4] = {0.0f, 0.0f, 0.0f, 0.0f};    // output frame (st_mlp_set_frame)
  float frame_scale[4] = {1.0f, 1.0f, 1.0f, 1.0f};
  float frame_lin[4][st::kMlpMaxIn] = {};            // linear part (st_mlp_set_linear_frame)
  float* params = nullptr;          // fp32 master weights
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  float* grad = nullptr;
  __bf16* wb = nullptr;             // W2, W3, W2ᵀ, W3ᵀ in bf16 (4 × 256²), then W4 split (16 × 256)
  // training scratch, sized for the largest batch seen
  int64_t cap_ld = 0;
  std::vector<void*> scratch;
  __bf16 *hT[2] = {nullptr, nullptr};
  __bf16 *dzT[2] = {nullptr, nullptr};
  __bf16* dsT2 = nullptr;
  float *loss_part = nullptr, *red_tmp = nullptr;
  float *gW1 = nullptr, *gb1 = nullptr, *gb2 = nullptr, *gb3 = nullptr, *gW4 = nullptr, *gb4 = nullptr;
  float *gW2 = nullptr, *gW3 = nullptr;
};

namespace {

constexpr int kSplits = 64;

struct DeviceGuard {
  int old = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    if (old != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
  }
};

st_status fail(st_mlp* m, st_status s, const std::string& msg) {
  if (m) m->err = msg;
  return s;
}

st_status hip_fail(st_mlp* m, hipError_t e, const char* what) {
  return fail(m, ST_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// splitmix64 (Steele, Lea & Flood 2014): a counter-based 64-bit generator.
uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

void free_scratch(st_mlp* m) {
  for (void* p : m->scratch) (void)hipFree(p);
  m->scratch.clear();
  m->cap_ld = 0;
}

template <class T>
hipError_t alloc(st_mlp* m, T** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) m->scratch.push_back(*p);
  return e;
}

st_status ensure_scratch(st_mlp* m, int64_t ld) {
  if (ld <= m->cap_ld) return ST_OK;
  free_scratch(m);
  const int64_t W = st::kMlpWidth;
  const int64_t nb = ld / st::mlp_tile();
  hipError_t e = hipSuccess;
  for (int l = 0; l < 2 && e == hipSuccess; ++l) e = alloc(m, &m->hT[l], (size_t)(W * ld));
  for (int l = 0; l < 2 && e == hipSuccess; ++l) e = alloc(m, &m->dzT[l], (size_t)(W * ld));
  if (e == hipSuccess) e = alloc(m, &m->dsT2, (size_t)(W * ld));
  if (e == hipSuccess) e = alloc(m, &m->loss_part, (size_t)nb);
  // multi-pass reduction buffers of the per-workgroup partials, one double
  // buffer per tensor (all reduced together)
  if (e == hipSuccess) {
    const int P = (int)nb;
    const size_t need = st::sum_partials_tmp(W * m->n_in, P) + 3 * st::sum_partials_tmp(W, P) +
                        st::sum_partials_tmp(4 * W, P) + st::sum_partials_tmp(4, P) +
                        st::sum_partials_tmp(1, P) + 2 * st::sum_partials_tmp(W * W, kSplits);
    e = alloc(m, &m->red_tmp, std::max<size_t>(need, 1));
  }
  if (e == hipSuccess) e = alloc(m, &m->gW1, (size_t)(nb * W * m->n_in));
  if (e == hipSuccess) e = alloc(m, &m->gb1, (size_t)(nb * W));
  if (e == hipSuccess) e = alloc(m, &m->gb2, (size_t)(nb * W));
  if (e == hipSuccess) e = alloc(m, &m->gb3, (size_t)(nb * W));
  if (e == hipSuccess) e = alloc(m, &m->gW4, (size_t)(nb * 4 * W));
  if (e == hipSuccess) e = alloc(m, &m->gb4, (size_t)(nb * 4));
  if (e == hipSuccess) e = alloc(m, &m->gW2, (size_t)(kSplits * W * W));
  if (e == hipSuccess) e = alloc(m, &m->gW3, (size_t)(kSplits * W * W));
  if (e != hipSuccess) {
    free_scratch(m);
    return fail(m, ST_ENOMEM, std::string("training scratch: ") + hipGetErrorString(e));
  }
  m->cap_ld = ld;
  return ST_OK;
}

st::MlpArgs base_args(st_mlp* m) {
  st::MlpArgs a;
  std::memset(&a, 0, sizeof(a));
  const int64_t W2 = (int64_t)st::kMlpWidth * st::kMlpWidth;
  a.n_in = m->n_in;
  a.off = m->off;
  a.n_params = m->n_params;
  a.params = m->params;
  a.params_rw = m->params;
  a.W2b = m->wb;
  a.W3b = m->wb + W2;
  a.W2Tb = m->wb + 2 * W2;
  a.W3Tb = m->wb + 3 * W2;
  a.W2b_rw = m->wb;
  a.W3b_rw = m->wb + W2;
  a.W2Tb_rw = m->wb + 2 * W2;
  a.W3Tb_rw = m->wb + 3 * W2;
  a.W4s = m->wb + 4 * W2;
  a.W4s_rw = m->wb + 4 * W2;
  a.grad = m->grad;
  a.adam_m = m->adam_m;
  a.adam_v = m->adam_v;
  for (int j = 0; j < 4; ++j) {
    a.out_ref[j] = m->frame_ref[j];
    a.out_scale[j] = m->frame_scale[j];
    for (int k = 0; k < st::kMlpMaxIn; ++k) a.out_lin[j][k] = m->frame_lin[j][k];
  }
  return a;
}

// Forward, backward and the gradient reduction for one batch into m->grad.
// With pend set, the reduction stops after its first pass and pend receives
// what is left for the Adam kernel to add (the per-tile partials of a large
// batch; the split-K weight partials are complete after one pass).
st_status compute_gradient(st_mlp* m, const float* x, const float* t, int64_t batch, float* d_loss,
                           hipStream_t s, st::AdamPending* pend = nullptr) {
  const int64_t tile = st::mlp_tile();
  const int64_t ld = (batch + tile - 1) / tile * tile;
  st_status st = ensure_scratch(m, ld);
  if (st != ST_OK) return st;
  st::MlpArgs a = base_args(m);
  a.batch = batch;
  a.ld = ld;
  a.x = x;
  a.target = t;
  a.inv_loss_norm = 1.0f / (float)batch;
  a.loss_part = m->loss_part;
  a.dsT2 = m->dsT2;
  a.hT1 = m->hT[0]; a.hT2 = m->hT[1];
  a.dzT2 = m->dzT[0]; a.dzT3 = m->dzT[1];
  a.gpart_W1 = m->gW1; a.gpart_b1 = m->gb1; a.gpart_b2 = m->gb2; a.gpart_b3 = m->gb3;
  a.gpart_W4 = m->gW4; a.gpart_b4 = m->gb4; a.gpart_W2 = m->gW2; a.gpart_W3 = m->gW3;
  a.n_splits = kSplits;
  a.split_chunk = ((ld + kSplits - 1) / kSplits + 31) / 32 * 32;
  const int nb = (int)(ld / tile);
  const int64_t W = st::kMlpWidth;
  hipError_t e;
  if ((e = st::launch_mlp_forward(a, true, s)) != hipSuccess) return hip_fail(m, e, "forward and backward");
  if ((e = st::launch_mlp_weight_grad(a, s)) != hipSuccess) return hip_fail(m, e, "weight gradients");
  const st::MlpOffsets& o = m->off;
  // every tensor's partials (and the loss) reduced together, one launch per pass
  st::SumSegment red[] = {
      {m->gW1, W * m->n_in, nb, m->grad + o.W1}, {m->gb1, W, nb, m->grad + o.b1},
      {m->gW2, W * W, kSplits, m->grad + o.W2},  {m->gb2, W, nb, m->grad + o.b2},
      {m->gW3, W * W, kSplits, m->grad + o.W3},  {m->gb3, W, nb, m->grad + o.b3},
      {m->gW4, 4 * W, nb, m->grad + o.W4},       {m->gb4, 4, nb, m->grad + o.b4},
      {m->loss_part, 1, nb, d_loss}};
  const int nseg = d_loss ? 9 : 8;
  st::SumLeft left[9];
  if ((e = st::launch_sum_partials_multi(red, nseg, m->red_tmp, s, pend ? 1 : (1 << 30), left)) !=
      hipSuccess)
    return hip_fail(m, e, "gradient reduction");
  if (pend) {
    *pend = st::AdamPending{};
    for (int k = 0; k < 8; ++k)
      if (left[k].rows > 0)
        pend->seg[pend->n++] = {left[k].src, red[k].out - m->grad, left[k].len, left[k].rows};
    if (d_loss && left[8].rows > 0) {
      pend->loss_src = left[8].src;
      pend->loss_rows = left[8].rows;
      pend->loss_out = d_loss;
    }
  }
  return ST_OK;
}

st_status check_batch(st_mlp* m, const void* x, const void* t, int64_t batch) {
  if (!m) return ST_EINVAL;
  if (batch <= 0 || batch > (int64_t)1 << 26) return fail(m, ST_EINVAL, "batch must be in 1..2^26");
  if (!x || !t) return fail(m, ST_EINVAL, "inputs or targets are NULL");
  return ST_OK;
}

}  // namespace

extern "C" {

st_status st_mlp_create(st_mlp** out, int device, int32_t n_in, int32_t width, uint64_t seed) {
  if (!out) return ST_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return ST_EINVAL;
  if (n_in < 1 || n_in > st::kMlpMaxIn || width != st::kMlpWidth) return ST_EINVAL;
  st_mlp* m = new (std::nothrow) st_mlp();
  if (!m) return ST_ENOMEM;
  m->device = device;
  m->n_in = n_in;
  m->off = st::mlp_offsets(n_in);
  m->n_params = m->off.total;
  std::vector<float> p((size_t)m->n_params, 0.0f);
  uint64_t ctr = seed * 0x100000001B3ull;
  auto fill = [&](int64_t off, int64_t count, int fan_in) {
    const double lim = 1.0 / std::sqrt((double)fan_in);
    for (int64_t i = 0; i < count; ++i) {
      const double u = (double)(splitmix64(ctr++) >> 11) * 0x1.0p-53;   // [0, 1)
      p[(size_t)(off + i)] = (float)((2.0 * u - 1.0) * lim);
    }
  };
  const int64_t W = st::kMlpWidth;
  fill(m->off.W1, W * n_in, n_in);
  fill(m->off.W2, W * W, (int)W);
  fill(m->off.W3, W * W, (int)W);
  fill(m->off.W4, 4 * W, (int)W);
  DeviceGuard g(device);
  hipError_t e = hipSuccess;
  const size_t nbytes = (size_t)m->n_params * sizeof(float);
  if (e == hipSuccess) e = hipMalloc(&m->params, nbytes);
  if (e == hipSuccess) e = hipMalloc(&m->adam_m, nbytes);
  if (e == hipSuccess) e = hipMalloc(&m->adam_v, nbytes);
  if (e == hipSuccess) e = hipMalloc(&m->grad, nbytes);
  if (e == hipSuccess) e = hipMalloc(&m->wb, ((size_t)4 * W * W + 16 * W) * sizeof(__bf16));
  if (e == hipSuccess) e = hipMemcpy(m->params, p.data(), nbytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->adam_m, 0, nbytes);
  if (e == hipSuccess) e = hipMemset(m->adam_v, 0, nbytes);
  if (e == hipSuccess) e = st::launch_refresh_bf16(base_args(m), nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    st_mlp_destroy(m);
    return ST_ENOMEM;
  }
  *out = m;
  return ST_OK;
}

st_status st_mlp_destroy(st_mlp* m) {
  if (!m) return ST_OK;
  {
    DeviceGuard g(m->device);
    free_scratch(m);
    for (void* p : {(void*)m->params, (void*)m->adam_m, (void*)m->adam_v, (void*)m->grad, (void*)m->wb})
      if (p) (void)hipFree(p);
  }
  delete m;
  return ST_OK;
}

const char* st_mlp_last_error(const st_mlp* m) { return m ? m->err.c_str() : "null network"; }

}  // extern "C"

int st_mlp_device_of(const st_mlp* m) { return m->device; }
int st_mlp_inputs_of(const st_mlp* m) { return m->n_in; }

extern "C" {

st_status st_mlp_params(st_mlp* m, float* h_get, const float* h_set, int64_t* n_params) {
  if (!m) return ST_EINVAL;
  if (n_params) *n_params = m->n_params;
  DeviceGuard g(m->device);
  const size_t nbytes = (size_t)m->n_params * sizeof(float);
  hipError_t e;
  if (h_get && (e = hipMemcpy(h_get, m->params, nbytes, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(m, e, "read parameters");
  if (h_set) {
    if ((e = hipMemcpy(m->params, h_set, nbytes, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(m, e, "write parameters");
    if ((e = st::launch_refresh_bf16(base_args(m), nullptr)) != hipSuccess)
      return hip_fail(m, e, "refresh bf16 weights");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(m, e, "synchronise");
  }
  return ST_OK;
}

st_status st_mlp_set_frame(st_mlp* m, const double* ref, const double* scale) {
  if (!m) return ST_EINVAL;
  if (!ref || !scale) return fail(m, ST_EINVAL, "frame is NULL");
  for (int j = 0; j < 4; ++j)
    if (!std::isfinite(ref[j]) || !std::isfinite(scale[j]) || !(scale[j] > 0.0))
      return fail(m, ST_EINVAL, "frame values must be finite with scale > 0");
  for (int j = 0; j < 4; ++j) { m->frame_ref[j] = (float)ref[j]; m->frame_scale[j] = (float)scale[j]; }
  return ST_OK;
}

st_status st_mlp_set_linear_frame(st_mlp* m, const double* lin) {
  if (!m) return ST_EINVAL;
  if (lin)
    for (int i = 0; i < 4 * m->n_in; ++i)
      if (!std::isfinite(lin[i])) return fail(m, ST_EINVAL, "linear frame values must be finite");
  for (int j = 0; j < 4; ++j)
    for (int k = 0; k < st::kMlpMaxIn; ++k)
      m->frame_lin[j][k] = (lin && k < m->n_in) ? (float)lin[j * m->n_in + k] : 0.0f;
  return ST_OK;
}

st_status st_mlp_fit_frame(st_mlp* m, const float* d_x, const float* d_t, int64_t n, double floor,
                           st_frame_fit* out, void* stream) {
  if (!m) return ST_EINVAL;
  const int D = m->n_in + 1, V = D * D + 4 * D;
  if (!d_x || !d_t) return fail(m, ST_EINVAL, "inputs or targets are NULL");
  if (n < D || n > ((int64_t)1 << 40)) return fail(m, ST_EINVAL, "need at least n_in + 1 samples");
  if (!(floor > 0.0) || !std::isfinite(floor)) return fail(m, ST_EINVAL, "floor must be > 0");
  DeviceGuard g(m->device);
  hipStream_t s = (hipStream_t)stream;
  double* part = nullptr;
  const int B = st::kFitBlocks;
  hipError_t e = hipMalloc((void**)&part, (size_t)B * V * sizeof(double));
  if (e != hipSuccess) return fail(m, ST_ENOMEM, std::string("fit scratch: ") + hipGetErrorString(e));
  std::vector<double> h((size_t)B * V);
  auto done = [&](st_status st) { (void)hipFree(part); return st; };
  if ((e = st::launch_fit_normal(d_x, d_t, n, m->n_in, part, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess ||
      (e = hipMemcpy(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
    return done(hip_fail(m, e, "frame fit, normal equations"));
  // block partials summed in block order
  std::vector<double> sum((size_t)V, 0.0);
  for (int b = 0; b < B; ++b)
    for (int v = 0; v < V; ++v) sum[(size_t)v] += h[(size_t)b * V + v];
  double G[st::kMlpMaxIn + 1][st::kMlpMaxIn + 1], R[st::kMlpMaxIn + 1][4];
  double trace = 0.0;
  for (int p = 0; p < D; ++p) {
    for (int q = 0; q < D; ++q) G[p][q] = sum[(size_t)(p * D + q)];
    for (int c = 0; c < 4; ++c) R[p][c] = sum[(size_t)(D * D + p * 4 + c)];
    trace += G[p][p];
  }
  // a ridge of 1e-12 of the mean diagonal on the input columns keeps a
  // constant-zero input (a band of one energy) solvable, with coefficient 0
  for (int p = 1; p < D; ++p) G[p][p] += 1e-12 * trace / D;
  // Cholesky G = L Lᵀ, then L Lᵀ c = R for the four components
  double L[st::kMlpMaxIn + 1][st::kMlpMaxIn + 1] = {};
  for (int p = 0; p < D; ++p) {
    for (int q = 0; q <= p; ++q) {
      double v = G[p][q];
      for (int k = 0; k < q; ++k) v -= L[p][k] * L[q][k];
      if (p == q) {
        if (!(v > 0.0)) return done(fail(m, ST_EINVAL, "frame fit: inputs are degenerate"));
        L[p][p] = std::sqrt(v);
      } else {
        L[p][q] = v / L[q][q];
      }
    }
  }
  st::FitCoef cf{};
  for (int c = 0; c < 4; ++c) {
    double y[st::kMlpMaxIn + 1];
    for (int p = 0; p < D; ++p) {
      double v = R[p][c];
      for (int k = 0; k < p; ++k) v -= L[p][k] * y[k];
      y[p] = v / L[p][p];
    }
    for (int p = D - 1; p >= 0; --p) {
      double v = y[p];
      for (int k = p + 1; k < D; ++k) v -= L[k][p] * cf.c[c][k];
      cf.c[c][p] = v / L[p][p];
    }
  }
  if ((e = st::launch_fit_residual(d_x, d_t, n, m->n_in, cf, part, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess ||
      (e = hipMemcpy(h.data(), part, (size_t)B * 8 * sizeof(double), hipMemcpyDeviceToHost)) !=
          hipSuccess)
    return done(hip_fail(m, e, "frame fit, residuals"));
  double ss[4] = {0.0, 0.0, 0.0, 0.0}, mx[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < B; ++b)
    for (int c = 0; c < 4; ++c) {
      ss[c] += h[(size_t)b * 8 + c];
      mx[c] = std::max(mx[c], h[(size_t)b * 8 + 4 + c]);
    }
  st_frame_fit f;
  std::memset(&f, 0, sizeof(f));
  for (int c = 0; c < 4; ++c) {
    f.ref[c] = cf.c[c][0];
    for (int k = 0; k < m->n_in; ++k) f.lin[c][k] = cf.c[c][1 + k];
    f.resid_rms[c] = std::sqrt(ss[c] / (double)n);
    f.resid_max[c] = mx[c];
    f.scale[c] = std::max(f.resid_rms[c], floor);
  }
  for (int c = 0; c < 4; ++c) {
    m->frame_ref[c] = (float)f.ref[c];
    m->frame_scale[c] = (float)f.scale[c];
    for (int k = 0; k < st::kMlpMaxIn; ++k) m->frame_lin[c][k] = (float)f.lin[c][k];
  }
  if (out) *out = f;
  return done(ST_OK);
}

st_status st_mlp_gradient(st_mlp* m, const float* d_x, const float* d_t, int64_t batch,
                          float* d_grad, float* d_loss, void* stream) {
  st_status st = check_batch(m, d_x, d_t, batch);
  if (st != ST_OK) return st;
  if (!d_grad) return fail(m, ST_EINVAL, "gradient output is NULL");
  DeviceGuard g(m->device);
  hipStream_t s = (hipStream_t)stream;
  if ((st = compute_gradient(m, d_x, d_t, batch, d_loss, s)) != ST_OK) return st;
  hipError_t e = hipMemcpyAsync(d_grad, m->grad, (size_t)m->n_params * sizeof(float),
                                hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(m, e, "copy gradient");
  return ST_OK;
}

st_status st_mlp_train_step(st_mlp* m, const float* d_x, const float* d_t, int64_t batch, float lr,
                            float* d_loss, void* stream) {
  st_status st = check_batch(m, d_x, d_t, batch);
  if (st != ST_OK) return st;
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(m, ST_EINVAL, "learning rate must be > 0");
  DeviceGuard g(m->device);
  hipStream_t s = (hipStream_t)stream;
  // the reduction's last pass (the per-tile partials of a large batch) runs
  // inside the Adam kernel
  st::AdamPending pend;
  if ((st = compute_gradient(m, d_x, d_t, batch, d_loss, s, &pend)) != ST_OK) return st;
  m->step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)st::kAdamBeta1, (double)m->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)st::kAdamBeta2, (double)m->step)));
  hipError_t e = st::launch_adam(base_args(m), lr, c1, c2, s, &pend);
  if (e != hipSuccess) return hip_fail(m, e, "adam");
  return ST_OK;
}

st_status st_mlp_infer(st_mlp* m, const float* d_x, float* d_q, int64_t n, void* stream) {
  if (!m) return ST_EINVAL;
  if (n < 0) return fail(m, ST_EINVAL, "negative count");
  if (n == 0) return ST_OK;
  if (!d_x || !d_q) return fail(m, ST_EINVAL, "inputs or outputs are NULL");
  DeviceGuard g(m->device);
  st::MlpArgs a = base_args(m);
  a.batch = n;
  a.x = d_x;
  a.q_out = d_q;
  hipError_t e = st::launch_mlp_forward(a, false, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(m, e, "inference");
  return ST_OK;
}

st_status st_mlp_features(st_mlp* m, const double* d_z, int64_t n, const double* center,
                          const double* inv_scale, double extra, float* d_x, void* stream) {
  if (!m) return ST_EINVAL;
  if (n < 0 || (n > 0 && (!d_z || !d_x)) || !center || !inv_scale)
    return fail(m, ST_EINVAL, "bad feature arguments");
  st::FeatureMap f;
  for (int i = 0; i < 6; ++i) { f.center[i] = center[i]; f.inv_scale[i] = inv_scale[i]; }
  f.extra = extra;
  DeviceGuard g(m->device);
  hipError_t e = st::launch_features(d_z, n, f, m->n_in, d_x, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(m, e, "features");
  return ST_OK;
}

st_status st_mlp_targets(st_mlp* m, const double* d_q, int64_t n, const double* ref, float* d_t,
                         void* stream) {
  if (!m) return ST_EINVAL;
  if (n < 0 || (n > 0 && (!d_q || !d_t)) || !ref) return fail(m, ST_EINVAL, "bad target arguments");
  DeviceGuard g(m->device);
  hipError_t e = st::launch_targets(d_q, n, ref, d_t, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(m, e, "targets");
  return ST_OK;
}

}  // extern "C"
