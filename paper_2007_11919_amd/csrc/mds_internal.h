// Internal declarations shared by the host sources and the HIP kernels of
// libmds.  Nothing here is part of the C ABI (see include/mds.h).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <mutex>
#include <set>
#include <string>
#include <utility>

#include "../../include/mds.h"

namespace mds {

// ---- tiling constants of the fused embed kernel ------------------------
// A block owns BM data rows and walks the landmarks BN at a time; the
// contraction over p is staged through LDS in chunks of CHUNK_BYTES per
// row (32 FP32, 16 FP64, or 32 hi + 32 lo 16-bit values).
constexpr int BM = 128;
constexpr int BN = 128;
constexpr int CHUNK_BYTES = 128;
constexpr int THREADS = 256;

enum Mode { MODE_F64 = 0, MODE_F32 = 1, MODE_BF16 = 2, MODE_F16 = 3 };

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// elements of the contraction per chunk in each mode
inline int chunk_elems(int mode) { return mode == MODE_F64 ? 16 : 32; }

// Models with one 16-column output block run the variant of the embed kernel
// that walks the landmarks 512 at a time when it pays: when at least 512
// landmark rows are padded and fewer than a quarter of the last 512-landmark
// pass would be idle, and in the split precisions also whenever p >=
// kWideMinP (a 128-row tile of X no longer stays in L2 across landmark
// tiles).  The choice depends on the model only (plain and serving launches
// alike), so a row's result does not depend on the launch it arrives in.
constexpr int kWideMinP = 256;
constexpr int kSplitPackRows = 512;  // landmark packs hold round_up(l_pad, this) rows
constexpr int kEmbedClasses = 5;
constexpr int kWideClass = 3;    // wide variant (FP32, or split with landmark lo parts)
constexpr int kWideHiClass = 4;  // wide split variant, landmark lo parts all zero
inline bool embed_wide(int mode, int64_t p, int rb, int64_t l_pad) {
  if (rb != 1 || mode == MODE_F64) return false;
  const int64_t span = round_up(l_pad, kSplitPackRows);
  const bool fills = l_pad >= kSplitPackRows && 4 * (span - l_pad) < span;
  if (mode == MODE_F32) return fills;
  return fills || p >= kWideMinP;
}

// Device-side view of one model for one precision, passed by value.
struct EmbedModelView {
  const void* mpack;   // l_pad rows x nchunks x CHUNK_BYTES landmark operands
  const void* w;       // projection weights: FP64 l_pad x (16*rb) row-major;
                       // FP32 (16*rb) x l_pad (column-major, leading dim ldwt)
  const void* c;       // l_pad: q - |m|^2 (float or double)
  int p;               // data dimension
  int nchunks;         // ceil(p / chunk_elems)
  int ntl;             // l_pad / BN landmark tiles
  int r;               // output columns written
  int rb;              // 16-wide blocks of output columns (1..4)
  int m_lo_zero;       // split modes: every landmark lo part is zero
  float prescale;      // split FP16: data scaled by 2^s before splitting
  float postscale;     // split FP16: 2^-2s applied to the dot products
  int64_t ldwt;        // leading dimension of the FP32 weights
  const void* spack;   // split modes: chunk-major hi and lo planes (Model::sbf / sh)
  int64_t lsplit;      // landmark rows of each chunk in spack
};

// One row tile of one request, for the persistent serving kernel.
struct TileWork {
  const void* x;
  void* y;
  int64_t ldx;
  int64_t ldy;
  int64_t row0;
  int32_t nrows;       // rows of this tile (<= BM)
  int32_t model;       // index into the model-view table
};

struct Model {
  int64_t n_fit = 0, p = 0, l = 0, l_pad = 0;
  int32_t r = 0, r_eff = 0, rb = 1;
  int dev = 0;
  int32_t lanczos_steps = 0, restarts = 0;
  // host copies
  int64_t* idx_host = nullptr;
  double* lam_host = nullptr;   // r
  // device buffers: one allocation (base), the rest point into it
  void* base = nullptr;
  void* m64 = nullptr;    // l_pad x nchunks64 x 16 doubles (FP64 operand and fit input)
  void* m32 = nullptr;    // round_up(l_pad, kSplitPackRows) x nchunks32 x 32 floats
  void* mbf = nullptr;    // round_up(l_pad, kSplitPackRows) x nchunks32 x (32 hi + 32 lo) bf16
  void* mh = nullptr;     // same for FP16 (scaled)
  void* sbf = nullptr;    // chunk-major BF16 parts: hi plane, lo plane (fit.hip k_pack32)
  void* sh = nullptr;     // same for FP16 (scaled)
  int64_t l_split = 0;    // round_up(l_pad, kSplitPackRows)
  void* w32 = nullptr;    // 16rb x l_pad float (column-major: output column, landmark)
  void* w64 = nullptr;    // l_pad x 16rb double
  void* c32 = nullptr;    // l_pad float
  void* c64 = nullptr;    // l_pad double
  void* q32 = nullptr;    // l_pad float: diag(Q1), for embedding from dissimilarities
  void* q64 = nullptr;    // l_pad double
  void* x1_64 = nullptr;  // l x r double: landmark coordinates X1 (read by the getter)
  void* aff64 = nullptr;  // r x p double: A = 2 W' M of the affine form y = A x + b
  void* aff32 = nullptr;  // r x p float
  void* affb64 = nullptr; // r double: b = W' c
  void* affb32 = nullptr; // r float
  bool vectors = true;    // fitted on data rows (false: on a dissimilarity matrix)
  int bf_lo_zero = 0, h_lo_zero = 0;
  float h_prescale = 1.f, h_postscale = 1.f;
  int64_t bytes = 0;

  EmbedModelView view(int mode) const;
};

// ---- error plumbing -----------------------------------------------------
mds_status set_error(mds_status st, const std::string& msg);
mds_status hip_fail(hipError_t e, const char* what);
#define MDS_HIP(call)                                                  \
  do {                                                                 \
    hipError_t _e = (call);                                            \
    if (_e != hipSuccess) return ::mds::hip_fail(_e, #call);           \
  } while (0)

// ---- model memory (api.cpp): a small cache of freed model blocks --------
void* model_alloc(int dev, size_t bytes);
void model_release(int dev, size_t bytes, void* p);

// ---- host sampler (sampler.cpp) -----------------------------------------
void sample_landmarks_host(int64_t n, int64_t l, uint64_t seed, int64_t* out);

// ---- fit kernels (fit.hip) ------------------------------------------------
struct FitScratch;
// D1 == nullptr: fit on the landmark rows of X; otherwise on the caller's
// l x l squared-dissimilarity matrix D1 (device, leading dimension ldd).
mds_status fit_on_device(Model& m, const void* X, int dt, int64_t ldx, const int64_t* idx_dev,
                         const double* D1, int64_t ldd, hipStream_t st);

// ---- embed kernels (embed.hip) -----------------------------------------
mds_status launch_embed(const Model& m, int mode, const void* X, int dt, int64_t n, int64_t ldx,
                        void* Y, int64_t ldy, hipStream_t st);
// Divide-and-conquer MDS (dc.hip); arguments as mds_divide_conquer, already
// validated.  Synchronous.
mds_status dc_on_device(const void* X, int dt, int64_t n, int64_t p, int64_t ldx, int64_t l, int64_t c,
                        int r, uint64_t seed, double* Y, int64_t ldy, double* lam_bar, int32_t* r_eff,
                        int64_t* order_out, hipStream_t st);
// y = A x + b for rows of X (embed_affine.hip); prec64: FP64 arithmetic and
// double Y, else FP32 arithmetic and float Y (X float).
mds_status launch_embed_affine(const Model& m, int prec64, const void* X, int dt, int64_t n,
                               int64_t ldx, void* Y, int64_t ldy, hipStream_t st);
// the same for an affine map given by device pointers (A: r x p, b: r)
mds_status launch_affine_raw(const void* A, const void* b, int prec64, int64_t p, int r, const void* X,
                             int dt, int64_t n, int64_t ldx, void* Y, int64_t ldy, hipStream_t st);
// top-r eigenpairs of the symmetric d x d FP64 matrix G (device, destroyed):
// lam (device, r, descending; zero beyond d), U (device, d x r row-major),
// status[0] = 1 when lambda_1 <= 0 (dc.hip)
mds_status dense_top_eigen(double* G, int d, int r, double* lam, double* U, int* status,
                           hipStream_t st);
// MaxMin landmarks and pivot MDS (pivot.hip); arguments validated by the API
mds_status maxmin_on_device(const void* X, int dt, int64_t n, int64_t p, int64_t ldx, int64_t l,
                            int64_t first, int64_t* idx_host, hipStream_t st);
// the same on the library's static scratch array (no allocation); sizes
// checked by the API against MDS_NOALLOC_MAX_N / _L
mds_status maxmin_on_device_noalloc(const void* X, int dt, int64_t n, int64_t p, int64_t ldx, int64_t l,
                                    int64_t first, int64_t* idx_host, hipStream_t st);
mds_status pivot_on_device(const void* X, int dt, int64_t n, int64_t p, int64_t ldx, int64_t l, int r,
                           const int64_t* idx_host, double* Y, int64_t ldy, double* lam_host,
                           int32_t* r_eff, hipStream_t st);
mds_status launch_embed_sqdist(const Model& m, int prec64, const void* A2, int dt, int64_t n,
                               int64_t lda, void* Y, int64_t ldy, hipStream_t st);
// persistent serving launch over a device table of tiles
// rbc = embed_class(...): 0 for rb 1, 1 for rb 2, 2 for rb 3..4, and
// kWideClass / kWideHiClass for the 512-landmark variants
mds_status launch_embed_worklist(int mode, int rbc, const EmbedModelView* views_dev,
                                 const TileWork* work_dev, const int32_t* nwork_dev,
                                 int grid, hipStream_t st);
int embed_max_rb();
// Raises kernel fn's dynamic LDS limit to bytes on the current device,
// once per (kernel, device): the limit is a per-device setting, so a
// process that uses several devices sets it on each.  Host only; safe from
// several threads.
inline hipError_t lds_limit_once(const void* fn, int bytes) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({fn, dev})) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) done.insert({fn, dev});
  return e;
}
// compute units of the current device (cached)
int num_cu();
int rb_class(int rb);
int embed_class(int mode, int64_t p, int rb, int64_t l_pad, int m_lo_zero);
int embed_blocks_per_cu(int mode, int rbc);
mds_status prepare_embed_worklist(int mode, int rbc);

}  // namespace mds
