// C ABI entry points of libmds: argument validation, model lifetime, and
// dispatch to the HIP kernels.  Semantics are documented in include/mds.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "mds_internal.h"

struct mds_model {
  mds::Model m;
};

namespace mds {

namespace {
thread_local std::string g_err;
thread_local int32_t g_hip_err = 0;
}  // namespace

mds_status set_error(mds_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

mds_status hip_fail(hipError_t e, const char* what) {
  g_hip_err = (int32_t)e;
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? MDS_ERR_OOM : MDS_ERR_HIP;
}

// Freed model blocks are kept for reuse by later fits of the same size, so
// a steady stream of fit/free pairs does not pay hipMalloc / hipFree (which
// synchronises the device) every time.  Bounded by count and bytes.
namespace {
constexpr size_t kCacheBlocks = 8;
constexpr size_t kCacheBytes = (size_t)1 << 30;
std::mutex g_cache_mu;
std::vector<std::tuple<int, size_t, void*>> g_cache;  // (device, bytes, pointer)
size_t g_cache_total = 0;
}  // namespace

void* model_alloc(int dev, size_t bytes) {
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (size_t i = 0; i < g_cache.size(); ++i) {
      if (std::get<0>(g_cache[i]) == dev && std::get<1>(g_cache[i]) == bytes) {
        void* p = std::get<2>(g_cache[i]);
        g_cache_total -= bytes;
        g_cache.erase(g_cache.begin() + (ptrdiff_t)i);
        return p;
      }
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void model_release(int dev, size_t bytes, void* p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_cache.size() < kCacheBlocks && g_cache_total + bytes <= kCacheBytes) {
      g_cache.emplace_back(dev, bytes, p);
      g_cache_total += bytes;
      return;
    }
  }
  (void)hipFree(p);
}

namespace {

void free_model(Model& m) {
  if (m.base) model_release(m.dev, (size_t)m.bytes, m.base);
  delete[] m.idx_host;
  delete[] m.lam_host;
  m = Model();
}

}  // namespace
}  // namespace mds

using namespace mds;

extern "C" {

const char* mds_last_error(void) { return g_err.c_str(); }
int32_t mds_last_hip_error(void) { return g_hip_err; }

mds_status mds_sample_landmarks(int64_t n, int64_t l, uint64_t seed, int64_t* idx_out) {
  if (!idx_out) return set_error(MDS_ERR_INVALID_ARG, "idx_out is NULL");
  if (l < 1 || l > n) return set_error(MDS_ERR_INVALID_ARG, "need 1 <= l <= n");
  try {
    sample_landmarks_host(n, l, seed, idx_out);
  } catch (const std::bad_alloc&) {
    return set_error(MDS_ERR_OOM, "host allocation failed in sampler");
  }
  return MDS_OK;
}

mds_status mds_fit_landmarks(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx, int64_t l,
                             int32_t r, uint64_t seed, const int64_t* idx_or_null, void* stream,
                             mds_model** out) {
  if (!out) return set_error(MDS_ERR_INVALID_ARG, "out is NULL");
  if (!X) return set_error(MDS_ERR_INVALID_ARG, "X is NULL");
  if (dt != MDS_F32 && dt != MDS_F64) return set_error(MDS_ERR_INVALID_ARG, "dt must be MDS_F32 or MDS_F64");
  if (p < 1) return set_error(MDS_ERR_INVALID_ARG, "p must be >= 1");
  if (ldx < p) return set_error(MDS_ERR_INVALID_ARG, "ldx < p");
  if (l < 2 || l > n) return set_error(MDS_ERR_INVALID_ARG, "need 2 <= l <= n");
  if (r < 1 || r > l - 1 || r > MDS_MAX_R)
    return set_error(MDS_ERR_INVALID_ARG, "need 1 <= r <= min(l - 1, MDS_MAX_R)");
  if (p > (int64_t)1 << 24) return set_error(MDS_ERR_INVALID_ARG, "p too large");
  if (l > (int64_t)1 << 16) return set_error(MDS_ERR_INVALID_ARG, "l too large (max 65536)");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  mds_model* h = nullptr;
  try {
    h = new mds_model();
    Model& m = h->m;
    m.n_fit = n;
    m.p = p;
    m.l = l;
    m.l_pad = round_up(l, BN);
    m.r = r;
    m.rb = (int32_t)((r + 15) / 16);
    if (m.rb == 3) m.rb = 4;
    (void)hipGetDevice(&m.dev);
    m.idx_host = new int64_t[(size_t)l];
    if (idx_or_null) {
      std::vector<int64_t> v(idx_or_null, idx_or_null + l);
      std::sort(v.begin(), v.end());
      for (int64_t i = 0; i < l; ++i) {
        if (v[i] < 0 || v[i] >= n) {
          free_model(m);
          delete h;
          return set_error(MDS_ERR_INVALID_ARG, "landmark index out of range");
        }
        if (i > 0 && v[i] == v[i - 1]) {
          free_model(m);
          delete h;
          return set_error(MDS_ERR_INVALID_ARG, "duplicate landmark index");
        }
      }
      std::memcpy(m.idx_host, v.data(), sizeof(int64_t) * l);
    } else {
      sample_landmarks_host(n, l, seed, m.idx_host);
    }
  } catch (const std::bad_alloc&) {
    if (h) {
      free_model(h->m);
      delete h;
    }
    return set_error(MDS_ERR_OOM, "host allocation failed");
  }
  Model& m = h->m;
  int64_t* idx_dev = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&idx_dev), sizeof(int64_t) * l, st);
  if (e != hipSuccess) {
    free_model(m);
    delete h;
    return hip_fail(e, "hipMallocAsync(idx)");
  }
  e = hipMemcpyAsync(idx_dev, m.idx_host, sizeof(int64_t) * l, hipMemcpyHostToDevice, st);
  mds_status s = (e == hipSuccess) ? fit_on_device(m, X, dt, ldx, idx_dev, nullptr, 0, st)
                                   : hip_fail(e, "hipMemcpyAsync(idx)");
  (void)hipFreeAsync(idx_dev, st);
  if (s == MDS_OK) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = hip_fail(e, "fit synchronize");
  } else {
    (void)hipStreamSynchronize(st);
  }
  if (s != MDS_OK) {
    free_model(m);
    delete h;
    return s;
  }
  *out = h;
  return MDS_OK;
}

mds_status mds_embed(const mds_model* h, const void* X, int32_t dt, int64_t n_new, int64_t ldx,
                     int32_t prec, void* Y, int64_t ldy, void* stream) {
  if (!h) return set_error(MDS_ERR_INVALID_ARG, "model is NULL");
  const Model& m = h->m;
  if (n_new < 0) return set_error(MDS_ERR_INVALID_ARG, "n_new < 0");
  if (prec < MDS_PREC_FP64 || prec > MDS_PREC_SPLIT_FP16)
    return set_error(MDS_ERR_INVALID_ARG, "unknown precision");
  if (dt != MDS_F32 && dt != MDS_F64) return set_error(MDS_ERR_INVALID_ARG, "dt must be MDS_F32 or MDS_F64");
  if (prec != MDS_PREC_FP64 && dt != MDS_F32)
    return set_error(MDS_ERR_INVALID_ARG, "FP32 and split precisions take MDS_F32 input");
  if (!m.vectors)
    return set_error(MDS_ERR_INVALID_ARG,
                     "model was fitted on dissimilarities: use mds_embed_from_sqdist");
  if (n_new == 0) return MDS_OK;
  if (!X || !Y) return set_error(MDS_ERR_INVALID_ARG, "X or Y is NULL");
  if (ldx < m.p) return set_error(MDS_ERR_INVALID_ARG, "ldx < p");
  if (ldy < m.r) return set_error(MDS_ERR_INVALID_ARG, "ldy < r");
  int mode = MODE_F32;
  switch (prec) {
    case MDS_PREC_FP64: mode = MODE_F64; break;
    case MDS_PREC_FP32: mode = MODE_F32; break;
    case MDS_PREC_SPLIT_BF16: mode = MODE_BF16; break;
    default: mode = MODE_F16; break;
  }
  return launch_embed(m, mode, X, dt, n_new, ldx, Y, ldy, reinterpret_cast<hipStream_t>(stream));
}

mds_status mds_fit_from_sqdist(const double* D1, int64_t l, int64_t ldd, int32_t r, void* stream,
                               mds_model** out) {
  if (!out) return set_error(MDS_ERR_INVALID_ARG, "out is NULL");
  if (!D1) return set_error(MDS_ERR_INVALID_ARG, "D1 is NULL");
  if (l < 2) return set_error(MDS_ERR_INVALID_ARG, "need l >= 2");
  if (ldd < l) return set_error(MDS_ERR_INVALID_ARG, "ldd < l");
  if (r < 1 || r > l - 1 || r > MDS_MAX_R)
    return set_error(MDS_ERR_INVALID_ARG, "need 1 <= r <= min(l - 1, MDS_MAX_R)");
  if (l > (int64_t)1 << 16) return set_error(MDS_ERR_INVALID_ARG, "l too large (max 65536)");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  mds_model* h = nullptr;
  try {
    h = new mds_model();
    Model& m = h->m;
    m.n_fit = l;
    m.p = 0;
    m.l = l;
    m.l_pad = round_up(l, BN);
    m.r = r;
    m.rb = (int32_t)((r + 15) / 16);
    if (m.rb == 3) m.rb = 4;
    m.vectors = false;
    (void)hipGetDevice(&m.dev);
    m.idx_host = new int64_t[(size_t)l];
    for (int64_t i = 0; i < l; ++i) m.idx_host[i] = i;
  } catch (const std::bad_alloc&) {
    if (h) {
      free_model(h->m);
      delete h;
    }
    return set_error(MDS_ERR_OOM, "host allocation failed");
  }
  Model& m = h->m;
  mds_status s = fit_on_device(m, nullptr, MDS_F64, 0, nullptr, D1, ldd, st);
  if (s == MDS_OK) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = hip_fail(e, "fit synchronize");
  } else {
    (void)hipStreamSynchronize(st);
  }
  if (s != MDS_OK) {
    free_model(m);
    delete h;
    return s;
  }
  *out = h;
  return MDS_OK;
}

mds_status mds_maxmin_landmarks(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx, int64_t l,
                                int64_t first, int64_t* idx_out, void* stream) {
  if (!X || !idx_out) return set_error(MDS_ERR_INVALID_ARG, "X or idx_out is NULL");
  if (dt != MDS_F32 && dt != MDS_F64) return set_error(MDS_ERR_INVALID_ARG, "dt must be MDS_F32 or MDS_F64");
  if (p < 1 || ldx < p) return set_error(MDS_ERR_INVALID_ARG, "need p >= 1 and ldx >= p");
  if (l < 1 || l > n) return set_error(MDS_ERR_INVALID_ARG, "need 1 <= l <= n");
  if (first < 0 || first >= n) return set_error(MDS_ERR_INVALID_ARG, "first out of range");
  if (n > ((int64_t)1 << 36)) return set_error(MDS_ERR_INVALID_ARG, "n too large");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  mds_status s = maxmin_on_device(X, dt, n, p, ldx, l, first, idx_out, st);
  if (s != MDS_OK) (void)hipStreamSynchronize(st);
  return s;
}

mds_status mds_maxmin_landmarks_noalloc(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx,
                                        int64_t l, int64_t first, int64_t* idx_out, void* stream) {
  if (!X || !idx_out) return set_error(MDS_ERR_INVALID_ARG, "X or idx_out is NULL");
  if (dt != MDS_F32 && dt != MDS_F64) return set_error(MDS_ERR_INVALID_ARG, "dt must be MDS_F32 or MDS_F64");
  if (p < 1 || ldx < p) return set_error(MDS_ERR_INVALID_ARG, "need p >= 1 and ldx >= p");
  if (l < 1 || l > n) return set_error(MDS_ERR_INVALID_ARG, "need 1 <= l <= n");
  if (first < 0 || first >= n) return set_error(MDS_ERR_INVALID_ARG, "first out of range");
  if (n > MDS_NOALLOC_MAX_N)
    return set_error(MDS_ERR_INVALID_ARG, "n exceeds MDS_NOALLOC_MAX_N (1048576) for the no-allocation MaxMin");
  if (l > MDS_NOALLOC_MAX_L)
    return set_error(MDS_ERR_INVALID_ARG, "l exceeds MDS_NOALLOC_MAX_L (16384) for the no-allocation MaxMin");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  mds_status s = maxmin_on_device_noalloc(X, dt, n, p, ldx, l, first, idx_out, st);
  if (s != MDS_OK) (void)hipStreamSynchronize(st);
  return s;
}

mds_status mds_pivot_mds(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx, int64_t l, int32_t r,
                         uint64_t seed, const int64_t* idx_or_null, double* Y, int64_t ldy, double* lam,
                         int32_t* r_eff, void* stream) {
  if (!X || !Y) return set_error(MDS_ERR_INVALID_ARG, "X or Y is NULL");
  if (dt != MDS_F32 && dt != MDS_F64) return set_error(MDS_ERR_INVALID_ARG, "dt must be MDS_F32 or MDS_F64");
  if (p < 1 || ldx < p) return set_error(MDS_ERR_INVALID_ARG, "need p >= 1 and ldx >= p");
  if (p > 4096) return set_error(MDS_ERR_INVALID_ARG, "p too large (max 4096)");
  if (l < 2 || l > n) return set_error(MDS_ERR_INVALID_ARG, "need 2 <= l <= n");
  if (l > MDS_DC_MAX_L) return set_error(MDS_ERR_INVALID_ARG, "l too large (max 2048)");
  if (r < 1 || r > l - 1 || r > MDS_MAX_R)
    return set_error(MDS_ERR_INVALID_ARG, "need 1 <= r <= min(l - 1, MDS_MAX_R)");
  if (ldy < r) return set_error(MDS_ERR_INVALID_ARG, "ldy < r");
  if (n > ((int64_t)1 << 36)) return set_error(MDS_ERR_INVALID_ARG, "n too large");
  std::vector<int64_t> idx((size_t)l);
  try {
    if (idx_or_null) {
      std::vector<int64_t> v(idx_or_null, idx_or_null + l);
      std::sort(v.begin(), v.end());
      for (int64_t i = 0; i < l; ++i) {
        if (v[i] < 0 || v[i] >= n) return set_error(MDS_ERR_INVALID_ARG, "pivot index out of range");
        if (i > 0 && v[i] == v[i - 1]) return set_error(MDS_ERR_INVALID_ARG, "duplicate pivot index");
      }
      std::memcpy(idx.data(), idx_or_null, sizeof(int64_t) * l);  // the caller's order
    } else {
      sample_landmarks_host(n, l, seed, idx.data());
    }
  } catch (const std::bad_alloc&) {
    return set_error(MDS_ERR_OOM, "host allocation failed");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  mds_status s = pivot_on_device(X, dt, n, p, ldx, l, r, idx.data(), Y, ldy, lam, r_eff, st);
  if (s != MDS_OK) (void)hipStreamSynchronize(st);
  return s;
}

mds_status mds_embed_affine(const mds_model* h, const void* X, int32_t dt, int64_t n_new, int64_t ldx,
                            int32_t prec, void* Y, int64_t ldy, void* stream) {
  if (!h) return set_error(MDS_ERR_INVALID_ARG, "model is NULL");
  const Model& m = h->m;
  if (!m.vectors)
    return set_error(MDS_ERR_INVALID_ARG,
                     "model was fitted on dissimilarities: the affine form needs landmark vectors");
  if (n_new < 0) return set_error(MDS_ERR_INVALID_ARG, "n_new < 0");
  if (prec != MDS_PREC_FP64 && prec != MDS_PREC_FP32)
    return set_error(MDS_ERR_INVALID_ARG, "the affine form takes FP64 or FP32");
  if (dt != MDS_F32 && dt != MDS_F64) return set_error(MDS_ERR_INVALID_ARG, "dt must be MDS_F32 or MDS_F64");
  if (prec == MDS_PREC_FP32 && dt != MDS_F32)
    return set_error(MDS_ERR_INVALID_ARG, "FP32 precision takes MDS_F32 input");
  if (n_new == 0) return MDS_OK;
  if (!X || !Y) return set_error(MDS_ERR_INVALID_ARG, "X or Y is NULL");
  if (ldx < m.p) return set_error(MDS_ERR_INVALID_ARG, "ldx < p");
  if (ldy < m.r) return set_error(MDS_ERR_INVALID_ARG, "ldy < r");
  if (n_new > ((int64_t)1 << 36)) return set_error(MDS_ERR_INVALID_ARG, "n_new too large");
  return launch_embed_affine(m, prec == MDS_PREC_FP64 ? 1 : 0, X, dt, n_new, ldx, Y, ldy,
                             reinterpret_cast<hipStream_t>(stream));
}

mds_status mds_divide_conquer(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx, int64_t l,
                              int64_t c, int32_t r, uint64_t seed, double* Y, int64_t ldy,
                              double* lam_bar, int32_t* r_eff, int64_t* order_out, void* stream) {
  if (!X || !Y) return set_error(MDS_ERR_INVALID_ARG, "X or Y is NULL");
  if (dt != MDS_F32 && dt != MDS_F64) return set_error(MDS_ERR_INVALID_ARG, "dt must be MDS_F32 or MDS_F64");
  if (p < 1) return set_error(MDS_ERR_INVALID_ARG, "p must be >= 1");
  if (p > (int64_t)1 << 24) return set_error(MDS_ERR_INVALID_ARG, "p too large");
  if (ldx < p) return set_error(MDS_ERR_INVALID_ARG, "ldx < p");
  if (r < 1 || r > MDS_MAX_R) return set_error(MDS_ERR_INVALID_ARG, "need 1 <= r <= MDS_MAX_R");
  if (ldy < r) return set_error(MDS_ERR_INVALID_ARG, "ldy < r");
  if (c < (int64_t)r + 1) return set_error(MDS_ERR_INVALID_ARG, "need c >= r + 1");
  if (l <= c) return set_error(MDS_ERR_INVALID_ARG, "need l > c");
  if (l > MDS_DC_MAX_L) return set_error(MDS_ERR_INVALID_ARG, "l too large (max 2048)");
  if (n <= c) return set_error(MDS_ERR_INVALID_ARG, "need n > c");
  if (n > ((int64_t)1 << 40)) return set_error(MDS_ERR_INVALID_ARG, "n too large");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  mds_status s = dc_on_device(X, dt, n, p, ldx, l, c, r, seed, Y, ldy, lam_bar, r_eff, order_out, st);
  if (s != MDS_OK) (void)hipStreamSynchronize(st);
  return s;
}

mds_status mds_embed_from_sqdist(const mds_model* h, const void* A2, int32_t dt, int64_t n_new,
                                 int64_t lda, int32_t prec, void* Y, int64_t ldy, void* stream) {
  if (!h) return set_error(MDS_ERR_INVALID_ARG, "model is NULL");
  const Model& m = h->m;
  if (n_new < 0) return set_error(MDS_ERR_INVALID_ARG, "n_new < 0");
  if (prec != MDS_PREC_FP64 && prec != MDS_PREC_FP32)
    return set_error(MDS_ERR_INVALID_ARG, "embedding from dissimilarities takes FP64 or FP32");
  if (dt != MDS_F32 && dt != MDS_F64) return set_error(MDS_ERR_INVALID_ARG, "dt must be MDS_F32 or MDS_F64");
  if (prec == MDS_PREC_FP32 && dt != MDS_F32)
    return set_error(MDS_ERR_INVALID_ARG, "FP32 precision takes MDS_F32 input");
  if (n_new == 0) return MDS_OK;
  if (!A2 || !Y) return set_error(MDS_ERR_INVALID_ARG, "A2 or Y is NULL");
  if (lda < m.l) return set_error(MDS_ERR_INVALID_ARG, "lda < l");
  if (ldy < m.r) return set_error(MDS_ERR_INVALID_ARG, "ldy < r");
  return launch_embed_sqdist(m, prec == MDS_PREC_FP64 ? 1 : 0, A2, dt, n_new, lda, Y, ldy,
                             reinterpret_cast<hipStream_t>(stream));
}

void mds_free(mds_model* h) {
  if (!h) return;
  free_model(h->m);
  delete h;
}

mds_status mds_model_info(const mds_model* h, int64_t* n_fit, int64_t* p, int64_t* l, int32_t* r,
                          int32_t* r_eff) {
  if (!h) return set_error(MDS_ERR_INVALID_ARG, "model is NULL");
  if (n_fit) *n_fit = h->m.n_fit;
  if (p) *p = h->m.p;
  if (l) *l = h->m.l;
  if (r) *r = h->m.r;
  if (r_eff) *r_eff = h->m.r_eff;
  return MDS_OK;
}

mds_status mds_get_landmarks(const mds_model* h, int64_t* idx) {
  if (!h || !idx) return set_error(MDS_ERR_INVALID_ARG, "NULL argument");
  std::memcpy(idx, h->m.idx_host, sizeof(int64_t) * h->m.l);
  return MDS_OK;
}

mds_status mds_get_eigenvalues(const mds_model* h, double* lam) {
  if (!h || !lam) return set_error(MDS_ERR_INVALID_ARG, "NULL argument");
  std::memcpy(lam, h->m.lam_host, sizeof(double) * h->m.r);
  return MDS_OK;
}

// X1 and q stay in the model's device memory; these getters copy them out
// on request (the model is immutable, so no stream ordering is needed)
mds_status mds_get_landmark_coords(const mds_model* h, double* X1) {
  if (!h || !X1) return set_error(MDS_ERR_INVALID_ARG, "NULL argument");
  const hipError_t e = hipMemcpy(X1, h->m.x1_64, sizeof(double) * h->m.l * h->m.r, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "copy of the landmark coordinates");
  return MDS_OK;
}

mds_status mds_get_q(const mds_model* h, double* q) {
  if (!h || !q) return set_error(MDS_ERR_INVALID_ARG, "NULL argument");
  const hipError_t e = hipMemcpy(q, h->m.q64, sizeof(double) * h->m.l, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "copy of q");
  return MDS_OK;
}

int64_t mds_model_bytes(const mds_model* h) { return h ? h->m.bytes : 0; }

mds_status mds_fit_stats(const mds_model* h, int32_t* steps, int32_t* restarts) {
  if (!h) return set_error(MDS_ERR_INVALID_ARG, "model is NULL");
  if (steps) *steps = h->m.lanczos_steps;
  if (restarts) *restarts = h->m.restarts;
  return MDS_OK;
}

}  // extern "C"

// Internal accessor used by the serving layer.
namespace mds {
const Model* model_of(const mds_model* h) { return h ? &h->m : nullptr; }
}  // namespace mds
