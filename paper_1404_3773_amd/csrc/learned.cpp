// Learned start density of the C interface (declared in include/ces.h): per-
// atom descriptors (host), the atom-centred correction functions and their
// quadrature Gram matrix against a target density, the correction applied to
// a start density, a dense per-atom network (FP32, SiLU) with forward,
// backward and Adam on the device, and the per-cluster quadratic loss.
// Not part of the paper's method: it only chooses the SCF's start density.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ces_internal.h"

struct ces_mlp_s {
  int device = -1;
  std::vector<int> sizes;              // n_in, width x depth, n_out
  std::vector<int64_t> w_off, b_off;   // offsets into the parameter vector
  int64_t n_params = 0;
  float* params = nullptr;
  float* grads = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* mean = nullptr;
  float* sd = nullptr;
  void* block = nullptr;
};

namespace ces {
namespace {

constexpr int kFeat = CES_MLP_FEATURES;
constexpr int kChan = CES_MLP_CHANNELS;

// descriptor parameters
constexpr double kRc = 10.0, kEta2 = 2.0, kEta4 = 0.02, kEnvSigma = 3.0;

double fcut(double r) { return r < kRc ? 0.5 * (std::cos(M_PI * r / kRc) + 1.0) : 0.0; }

// splitmix64 (Steele, Lea, Flood 2014) and Box-Muller normals for the
// initial weights.
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return (static_cast<double>(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  }
};

size_t fit_bytes(const Basis& b, int n_atoms) {
  const int nc = kChan * n_atoms + 1;
  return align256(size_t(b.n_grid) * nc * 8) + align256(size_t(gram_chunks(b.n_grid, nc)) * nc * nc * 8) +
         align256(size_t(6) * std::max(n_atoms, 1) * 8);
}

int64_t mlp_work_floats(const ces_mlp_s& m, int rows) {
  int64_t f = int64_t(rows) * m.sizes[0];
  int wmax = 0;
  for (size_t l = 1; l < m.sizes.size(); ++l) {
    f += 2 * int64_t(rows) * m.sizes[l];
    wmax = std::max(wmax, m.sizes[l]);
  }
  return f + 2 * int64_t(rows) * wmax;
}

// Workspace pointers: H0, then (Z_l, H_{l+1}) per layer, then two gradient buffers.
struct MlpWork {
  std::vector<float*> H, Z;
  float* G[2];
};
MlpWork mlp_work(const ces_mlp_s& m, int rows, void* work) {
  MlpWork w;
  float* p = static_cast<float*>(work);
  const int L = static_cast<int>(m.sizes.size()) - 1;
  w.H.push_back(p);
  p += int64_t(rows) * m.sizes[0];
  int wmax = 0;
  for (int l = 0; l < L; ++l) {
    w.Z.push_back(p);
    p += int64_t(rows) * m.sizes[l + 1];
    w.H.push_back(p);
    p += int64_t(rows) * m.sizes[l + 1];
    wmax = std::max(wmax, m.sizes[l + 1]);
  }
  w.G[0] = p;
  w.G[1] = p + int64_t(rows) * wmax;
  return w;
}

ces_status check_mlp(ces_mlp m) {
  if (!m) return fail(CES_ERR_INVALID_ARG, "null network");
  int dev = 0;
  CES_HIP(hipGetDevice(&dev));
  if (dev != m->device) return fail(CES_ERR_INVALID_ARG, "network lives on another device");
  return CES_OK;
}

}  // namespace
}  // namespace ces

using namespace ces;

extern "C" {

ces_status ces_atom_descriptors(int n_atoms, const double* h_atoms, float* h_desc,
                                double* h_dirs) {
  if (n_atoms < 0 || (n_atoms > 0 && (!h_atoms || !h_desc || !h_dirs)))
    return fail(CES_ERR_INVALID_ARG, "bad descriptor arguments");
  const int n = n_atoms;
  auto at = [&](int i, int c) { return h_atoms[3 * i + c]; };
  auto dist = [&](int i, int j) {
    const double dx = at(i, 0) - at(j, 0), dy = at(i, 1) - at(j, 1), dz = at(i, 2) - at(j, 2);
    return std::sqrt(dx * dx + dy * dy + dz * dz);
  };
  for (int j = 0; j < n; ++j) {
    double f[kFeat] = {};
    double u[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
      if (i == j) continue;
      const double r = dist(i, j);
      const double fc = fcut(r);
      for (int s = 0; s < 16; ++s) {
        const double mu = 2.0 + 0.5 * s;
        f[s] += std::exp(-kEta2 * (r - mu) * (r - mu)) * fc;
      }
      const double g = std::exp(-r * r / (2 * kEnvSigma * kEnvSigma));
      f[22] += g / 10.0;
      for (int c = 0; c < 3; ++c) u[c] += g * (at(i, c) - at(j, c)) / r;
    }
    for (int i = 0; i < n; ++i) {
      if (i == j) continue;
      const double ri = dist(i, j);
      for (int k = i + 1; k < n; ++k) {
        if (k == j) continue;
        const double rk = dist(k, j);
        double dot = 0;
        for (int c = 0; c < 3; ++c) dot += (at(i, c) - at(j, c)) * (at(k, c) - at(j, c));
        const double cosv = dot / (ri * rk);
        const double g = std::exp(-kEta4 * (ri * ri + rk * rk)) * fcut(ri) * fcut(rk);
        f[16] += (1 + cosv) * g;
        f[17] += (1 - cosv) * g;
        f[18] += 0.125 * std::pow(1 + cosv, 4) * g;
        f[19] += 0.125 * std::pow(1 - cosv, 4) * g;
      }
    }
    f[20] = std::sqrt(at(j, 0) * at(j, 0) + at(j, 1) * at(j, 1) + at(j, 2) * at(j, 2)) / 8.0;
    f[21] = n / 40.0;
    const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    f[23] = un;
    for (int c = 0; c < kFeat; ++c) h_desc[size_t(j) * kFeat + c] = static_cast<float>(f[c]);
    for (int c = 0; c < 3; ++c) h_dirs[3 * j + c] = un > 1e-6 ? u[c] / un : 0.0;
  }
  return CES_OK;
}

ces_status ces_density_fit_workspace_size(ces_ham hh, int n_atoms, size_t* bytes) {
  if (!hh || !bytes || n_atoms < 1) return fail(CES_ERR_INVALID_ARG, "bad arguments");
  *bytes = fit_bytes(*hh->h.basis, n_atoms);
  return CES_OK;
}

ces_status ces_density_fit_gram(ces_ham hh, int n_atoms, const double* h_atoms,
                                const double* h_dirs, const double* d_target, double* d_gram,
                                void* d_work, size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  const Basis& b = *hh->h.basis;
  if (n_atoms < 1 || !h_atoms || !h_dirs || !d_gram)
    return fail(CES_ERR_INVALID_ARG, "bad density-fit arguments");
  const size_t need = fit_bytes(b, n_atoms);
  if (!d_work || work_bytes < need)
    return fail(CES_ERR_WORKSPACE, "density-fit workspace too small: need " + std::to_string(need));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nc = kChan * n_atoms + 1;
  char* w = static_cast<char*>(d_work);
  double* F = reinterpret_cast<double*>(w);
  double* part = reinterpret_cast<double*>(w + align256(size_t(b.n_grid) * nc * 8));
  double* geo = reinterpret_cast<double*>(
      w + align256(size_t(b.n_grid) * nc * 8) + align256(size_t(gram_chunks(b.n_grid, nc)) * nc * nc * 8));
  std::vector<double> buf(6 * size_t(n_atoms));
  std::copy(h_atoms, h_atoms + 3 * n_atoms, buf.begin());
  std::copy(h_dirs, h_dirs + 3 * n_atoms, buf.begin() + 3 * n_atoms);
  CES_HIP(hipMemcpyAsync(geo, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, s));
  launch_fit_columns(b, geo, geo + 3 * n_atoms, n_atoms, d_target, F, s);
  launch_gram(F, b.n_grid, F, b.n_grid, d_gram, part, b.n_grid, nc, s);
  CES_HIP(hipGetLastError());
  CES_HIP(hipStreamSynchronize(s));
  return CES_OK;
}

ces_status ces_density_correction(ces_ham hh, int n_atoms, const double* h_atoms,
                                  const double* h_dirs, const float* d_coef, double* d_rho,
                                  void* d_work, size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  const Basis& b = *hh->h.basis;
  if (n_atoms < 1 || !h_atoms || !h_dirs || !d_coef || !d_rho)
    return fail(CES_ERR_INVALID_ARG, "bad density-correction arguments");
  if (!d_work || work_bytes < size_t(48) * n_atoms)
    return fail(CES_ERR_WORKSPACE, "density-correction workspace needs 48 bytes per atom");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<double> buf(6 * size_t(n_atoms));
  std::copy(h_atoms, h_atoms + 3 * n_atoms, buf.begin());
  std::copy(h_dirs, h_dirs + 3 * n_atoms, buf.begin() + 3 * n_atoms);
  double* geo = static_cast<double*>(d_work);
  CES_HIP(hipMemcpyAsync(geo, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, s));
  launch_density_correction(b, geo, geo + 3 * n_atoms, n_atoms, d_coef, d_rho, s);
  CES_HIP(hipGetLastError());
  CES_HIP(hipStreamSynchronize(s));
  return CES_OK;
}

// ------------------------------------------------------------------- MLP

ces_status ces_mlp_create(int n_in, int width, int depth, int n_out, uint64_t seed, ces_mlp* out) {
  if (!out) return fail(CES_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (n_in < 1 || width < 1 || depth < 0 || n_out < 1 || n_in > 4096 || width > 4096 ||
      n_out > 4096 || depth > 64)
    return fail(CES_ERR_INVALID_ARG, "bad network shape");
  ces_mlp_s* m = new (std::nothrow) ces_mlp_s();
  if (!m) return fail(CES_ERR_ALLOC, "out of host memory");
  m->sizes.push_back(n_in);
  for (int i = 0; i < depth; ++i) m->sizes.push_back(width);
  m->sizes.push_back(n_out);
  int64_t off = 0;
  for (size_t l = 0; l + 1 < m->sizes.size(); ++l) {
    m->w_off.push_back(off);
    off += int64_t(m->sizes[l]) * m->sizes[l + 1];
    m->b_off.push_back(off);
    off += m->sizes[l + 1];
  }
  m->n_params = off;
  // weights N(0, 1 / fan_in), zero biases; scaling mean 0, std 1
  std::vector<float> host(off, 0.0f);
  SplitMix rng{seed};
  for (size_t l = 0; l + 1 < m->sizes.size(); ++l) {
    const double sc = 1.0 / std::sqrt(static_cast<double>(m->sizes[l]));
    for (int64_t e = 0; e < int64_t(m->sizes[l]) * m->sizes[l + 1]; ++e)
      host[m->w_off[l] + e] = static_cast<float>(sc * rng.normal());
  }
  const size_t pb = align256(size_t(off) * 4), sb = align256(size_t(n_in) * 4);
  auto cleanup = [&](ces_status st) {
    if (m->block) (void)hipFree(m->block);
    delete m;
    return st;
  };
  if (hipGetDevice(&m->device) != hipSuccess) return cleanup(fail(CES_ERR_DEVICE, "no device"));
  if (hipMalloc(&m->block, 4 * pb + 2 * sb) != hipSuccess)
    return cleanup(fail(CES_ERR_ALLOC, "hipMalloc of network storage failed"));
  char* p = static_cast<char*>(m->block);
  m->params = reinterpret_cast<float*>(p);
  m->grads = reinterpret_cast<float*>(p + pb);
  m->m = reinterpret_cast<float*>(p + 2 * pb);
  m->v = reinterpret_cast<float*>(p + 3 * pb);
  m->mean = reinterpret_cast<float*>(p + 4 * pb);
  m->sd = reinterpret_cast<float*>(p + 4 * pb + sb);
  std::vector<float> ones(n_in, 1.0f);
  if (hipMemcpy(m->params, host.data(), size_t(off) * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->grads, 0, 3 * pb) != hipSuccess ||
      hipMemset(m->mean, 0, size_t(n_in) * 4) != hipSuccess ||
      hipMemcpy(m->sd, ones.data(), size_t(n_in) * 4, hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(CES_ERR_DEVICE, "network upload failed"));
  *out = m;
  return CES_OK;
}

ces_status ces_mlp_destroy(ces_mlp m) {
  if (!m) return CES_OK;
  if (m->block) (void)hipFree(m->block);
  delete m;
  return CES_OK;
}

ces_status ces_mlp_num_params(ces_mlp m, int64_t* n) {
  if (!m || !n) return fail(CES_ERR_INVALID_ARG, "null argument");
  *n = m->n_params;
  return CES_OK;
}

ces_status ces_mlp_get_params(ces_mlp m, float* h_params, float* h_mean, float* h_std) {
  CES_TRY(check_mlp(m));
  if (h_params) CES_HIP(hipMemcpy(h_params, m->params, size_t(m->n_params) * 4, hipMemcpyDeviceToHost));
  if (h_mean) CES_HIP(hipMemcpy(h_mean, m->mean, size_t(m->sizes[0]) * 4, hipMemcpyDeviceToHost));
  if (h_std) CES_HIP(hipMemcpy(h_std, m->sd, size_t(m->sizes[0]) * 4, hipMemcpyDeviceToHost));
  return CES_OK;
}

ces_status ces_mlp_set_params(ces_mlp m, const float* h_params, const float* h_mean,
                              const float* h_std) {
  CES_TRY(check_mlp(m));
  if (h_std)
    for (int c = 0; c < m->sizes[0]; ++c)
      if (!(h_std[c] > 0.0f)) return fail(CES_ERR_INVALID_ARG, "input scales must be positive");
  if (h_params) CES_HIP(hipMemcpy(m->params, h_params, size_t(m->n_params) * 4, hipMemcpyHostToDevice));
  if (h_mean) CES_HIP(hipMemcpy(m->mean, h_mean, size_t(m->sizes[0]) * 4, hipMemcpyHostToDevice));
  if (h_std) CES_HIP(hipMemcpy(m->sd, h_std, size_t(m->sizes[0]) * 4, hipMemcpyHostToDevice));
  return CES_OK;
}

ces_status ces_mlp_workspace_size(ces_mlp m, int rows, size_t* bytes) {
  if (!m || !bytes || rows < 1) return fail(CES_ERR_INVALID_ARG, "bad arguments");
  *bytes = align256(size_t(mlp_work_floats(*m, rows)) * 4);
  return CES_OK;
}

ces_status ces_mlp_forward(ces_mlp m, int rows, const float* d_in, float* d_out, void* d_work,
                           size_t work_bytes, void* stream) {
  CES_TRY(check_mlp(m));
  if (rows < 1 || !d_in || !d_out) return fail(CES_ERR_INVALID_ARG, "bad forward arguments");
  if (!d_work || work_bytes < size_t(mlp_work_floats(*m, rows)) * 4)
    return fail(CES_ERR_WORKSPACE, "network workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MlpWork w = mlp_work(*m, rows, d_work);
  const int L = static_cast<int>(m->sizes.size()) - 1;
  launch_standardize(d_in, m->mean, m->sd, w.H[0], rows, m->sizes[0], s);
  for (int l = 0; l < L; ++l) {
    const int ni = m->sizes[l], no = m->sizes[l + 1];
    launch_gemm_f32(false, false, w.H[l], ni, m->params + m->w_off[l], no, w.Z[l], no, rows, no, ni,
                    1.0f, 0.0f, s);
    launch_bias_act(w.Z[l], m->params + m->b_off[l], w.H[l + 1], rows, no, l + 1 < L, s);
  }
  CES_HIP(hipMemcpyAsync(d_out, w.H[L], size_t(rows) * m->sizes[L] * 4, hipMemcpyDeviceToDevice, s));
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_mlp_backward(ces_mlp m, int rows, const float* d_gout, void* d_work,
                            size_t work_bytes, void* stream) {
  CES_TRY(check_mlp(m));
  if (rows < 1 || !d_gout) return fail(CES_ERR_INVALID_ARG, "bad backward arguments");
  if (!d_work || work_bytes < size_t(mlp_work_floats(*m, rows)) * 4)
    return fail(CES_ERR_WORKSPACE, "network workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MlpWork w = mlp_work(*m, rows, d_work);
  const int L = static_cast<int>(m->sizes.size()) - 1;
  float* G = w.G[0];
  float* Gn = w.G[1];
  CES_HIP(hipMemcpyAsync(G, d_gout, size_t(rows) * m->sizes[L] * 4, hipMemcpyDeviceToDevice, s));
  for (int l = L - 1; l >= 0; --l) {
    const int ni = m->sizes[l], no = m->sizes[l + 1];
    if (l + 1 < L) launch_act_grad(G, w.Z[l], int64_t(rows) * no, s);
    // dW = H_l^T G  (ni x no), db = column sums of G
    launch_gemm_f32(true, false, w.H[l], ni, G, no, m->grads + m->w_off[l], no, ni, no, rows, 1.0f,
                    0.0f, s);
    launch_colsum(G, m->grads + m->b_off[l], rows, no, s);
    if (l > 0) {
      // dH_l = G W^T  (rows x ni)
      launch_gemm_f32(false, true, G, no, m->params + m->w_off[l], no, Gn, ni, rows, ni, no, 1.0f,
                      0.0f, s);
      std::swap(G, Gn);
    }
  }
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_mlp_get_grads(ces_mlp m, float* h_grads) {
  CES_TRY(check_mlp(m));
  if (!h_grads) return fail(CES_ERR_INVALID_ARG, "null output");
  CES_HIP(hipMemcpy(h_grads, m->grads, size_t(m->n_params) * 4, hipMemcpyDeviceToHost));
  return CES_OK;
}

ces_status ces_mlp_adam_step(ces_mlp m, float lr, float beta1, float beta2, float eps, int step,
                             void* stream) {
  CES_TRY(check_mlp(m));
  if (step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0))
    return fail(CES_ERR_INVALID_ARG, "bad Adam parameters");
  const float c1 = 1.0f - std::pow(beta1, static_cast<float>(step));
  const float c2 = 1.0f - std::pow(beta2, static_cast<float>(step));
  launch_adam(m->params, m->grads, m->m, m->v, m->n_params, lr, beta1, beta2, eps, c1, c2,
              static_cast<hipStream_t>(stream));
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_cluster_quad_loss(int n_clusters, int max_atoms, const int64_t* d_row_off,
                                 const int64_t* d_m_off, const float* d_M, const float* d_p,
                                 const float* d_t, const float* d_out, float* d_gout,
                                 float* d_loss, float scale, void* stream) {
  if (n_clusters < 1 || max_atoms < 1 || max_atoms > 2048 || !d_row_off || !d_m_off || !d_M ||
      !d_p || !d_t || !d_out || !d_gout || !d_loss)
    return fail(CES_ERR_INVALID_ARG, "bad loss arguments");
  launch_cluster_quad_loss(n_clusters, d_row_off, d_m_off, d_M, d_p, d_t, d_out, d_gout, d_loss,
                           scale, kChan * max_atoms, static_cast<hipStream_t>(stream));
  CES_HIP(hipGetLastError());
  return CES_OK;
}

}  // extern "C"
