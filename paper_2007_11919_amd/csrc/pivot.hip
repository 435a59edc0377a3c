// MaxMin landmark selection and pivot MDS (Section 3.1), FP64.
//
// MaxMin (the landmark choice of LMDS): from a given first point, add the
// point whose smallest squared distance to the chosen points is largest.
// Each step is one pass over X: a block stages 256 rows x 32 columns
// through LDS with coalesced loads; thread t sums (x - m)^2 over its row's
// columns in order, with a separately rounded product and sum per column
// (so the values do not depend on how rows are grouped), keeps the running
// minimum, and the block reports its largest minimum (smallest row on
// ties).  A one-block kernel merges the block results in order and appends
// the next landmark; the steps run back to back on the stream.
//
// Pivot MDS: C is the double-centred n x l block of squared distances
// between all points and the pivots, and its singular value decomposition
// C = U Sigma W' stands in for the eigendecomposition of Q; Q's eigenvalues
// are estimated as lambda = sigma sqrt(n / l) and the configuration is
// U_r Lambda_r^{1/2}; direction k is live when sigma_k^2 > TAU sigma_1^2.
// For squared Euclidean distances the double-centred
// block is C = Xc Mc' (Xc: rows minus their mean, Mc: pivots minus their
// mean), so C'C = Mc S Mc' with S = Xc'Xc (p x p), and
//     U_r Lambda_r^{1/2} = Xc Mc' W_r diag(lambda^{1/2} / sigma),
// an affine map of the rows.  The work is one pass for the means, one for
// S, an l x l symmetric eigenproblem, and one streaming pass for Y.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "mds_internal.h"

namespace mds {
namespace {

struct Buf {
  void* p = nullptr;
  hipStream_t st = nullptr;
  ~Buf() {
    if (p) (void)hipFreeAsync(p, st);
  }
  template <typename T>
  T* get() const {
    return static_cast<T*>(p);
  }
};

#define PV_HIP(call)                                     \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) return hip_fail(_e, #call);    \
  } while (0)

#define PV_LAUNCH(what)                                  \
  do {                                                   \
    hipError_t _e = hipGetLastError();                   \
    if (_e != hipSuccess) return hip_fail(_e, what);     \
  } while (0)

constexpr int MM_ROWS = 256;
constexpr int MM_COLS = 32;

// ---------------------------------------------------------------- MaxMin
// Step s: distances to landmark idx[s]; dmin <- min(dmin, d) (set on the
// first step); per block the largest dmin and its smallest row.
template <typename TX>
__global__ __launch_bounds__(256) void k_mm_step(const TX* __restrict__ X, int64_t ldx, int64_t n,
                                                 int64_t p, const int64_t* __restrict__ idx, int s,
                                                 double* __restrict__ dmin, double* __restrict__ bval,
                                                 int64_t* __restrict__ bidx) {
  __shared__ TX xs[MM_ROWS][MM_COLS + 1];
  __shared__ double ms[MM_COLS];
  __shared__ double wv[4];
  __shared__ int64_t wi[4];
  const int t = threadIdx.x;
  // odd steps walk the row blocks backwards, so each step starts on the rows
  // the previous one read last (still in the memory-side cache when X is
  // larger than it); a row's result does not depend on the order
  const int64_t blk = (s & 1) ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x;
  const int64_t row0 = blk * MM_ROWS;
  const int nrows = (int)((n - row0) < MM_ROWS ? (n - row0) : MM_ROWS);
  const TX* mrow = X + idx[s] * ldx;
  // thread t stages column t % 32, rows t / 32 + 8 u, of each 256 x 32
  // chunk; the next chunk is loaded into registers while the current one is
  // summed
  constexpr int PER = MM_ROWS * MM_COLS / 256;
  constexpr int RSTEP = 256 / MM_COLS;
  const int cc0 = t % MM_COLS, rb = t / MM_COLS;
  const TX* xbase = X + (row0 + rb) * ldx + cc0;
  const int64_t rstride = (int64_t)RSTEP * ldx;
  // FP32 rows 16-byte aligned with p a multiple of 4: thread t loads the
  // 16-byte segment t % 8 of rows t / 8 + 32 v instead (a quarter of the
  // load instructions, whole 16-byte accesses)
  constexpr int VE = 16 / (int)sizeof(TX);  // values per 16 bytes
  constexpr int VSEG = MM_COLS / VE;        // segments per row chunk
  constexpr int VRSTEP = 256 / VSEG;
  const bool vec = sizeof(TX) == 4 && (p % VE == 0) && ((((uintptr_t)X) & 15) == 0) &&
                   ((ldx * (int64_t)sizeof(TX)) % 16 == 0);
  const int vs = t % VSEG, vr = t / VSEG;
  const TX* vbase = X + (row0 + vr) * ldx + vs * VE;
  const int64_t vrstride = (int64_t)VRSTEP * ldx;
  TX reg[PER];
  auto load = [&](int64_t c0) {
    if (vec) {
      const bool cin = c0 + vs * VE < p;
#pragma unroll
      for (int u = 0; u < PER / VE; ++u) {
        typedef TX tv __attribute__((ext_vector_type(VE)));
        tv v = {};
        if (cin && vr + VRSTEP * u < nrows) v = *reinterpret_cast<const tv*>(vbase + c0 + u * vrstride);
#pragma unroll
        for (int e = 0; e < VE; ++e) reg[u * VE + e] = v[e];
      }
      return;
    }
    const bool cin = c0 + cc0 < p;
    const TX* src = xbase + c0;
#pragma unroll
    for (int u = 0; u < PER; ++u) reg[u] = (cin && rb + RSTEP * u < nrows) ? src[u * rstride] : (TX)0;
  };
  double acc = 0.0;
  load(0);
  for (int64_t c0 = 0; c0 < p; c0 += MM_COLS) {
    const int nc = (int)((p - c0) < MM_COLS ? (p - c0) : MM_COLS);
    if (vec) {
#pragma unroll
      for (int u = 0; u < PER / VE; ++u)
#pragma unroll
        for (int e = 0; e < VE; ++e) xs[vr + VRSTEP * u][vs * VE + e] = reg[u * VE + e];
    } else {
#pragma unroll
      for (int u = 0; u < PER; ++u) xs[rb + RSTEP * u][cc0] = reg[u];
    }
    if (t < MM_COLS) ms[t] = (t < nc) ? (double)mrow[c0 + t] : 0.0;
    __syncthreads();
    if (c0 + MM_COLS < p) load(c0 + MM_COLS);
    for (int cc = 0; cc < nc; ++cc) {
      const double d = (double)xs[t][cc] - ms[cc];
      acc = __dadd_rn(acc, __dmul_rn(d, d));
    }
    __syncthreads();
  }
  double best = -1.0;
  int64_t at = INT64_MAX;
  if (t < nrows) {
    const int64_t i = row0 + t;
    const double v = (s == 0) ? acc : fmin(dmin[i], acc);
    dmin[i] = v;
    best = v;
    at = i;
  }
  // largest value, smallest row on ties: a total order, so any merge order
  // gives the same result
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(best, off, 64);
    const int64_t oi = __shfl_xor(at, off, 64);
    if (ov > best || (ov == best && oi < at)) {
      best = ov;
      at = oi;
    }
  }
  if ((t & 63) == 0) {
    wv[t >> 6] = best;
    wi[t >> 6] = at;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < 4; ++w)
      if (wv[w] > best || (wv[w] == best && wi[w] < at)) {
        best = wv[w];
        at = wi[w];
      }
    bval[blk] = best;
    bidx[blk] = at;
  }
}

// The same step on a column-major copy Xt of X (p rows of ldt values; ldt
// a whole number of blocks): thread t of a block owns rows VE t .. VE t +
// VE - 1 (one 16-byte load per column), so a step reads each column as one
// contiguous run instead of 128-byte pieces of rows.  Per row the sum runs
// over the columns in the same order with the same rounding as k_mm_step,
// so the distances, and the landmarks, are the same.
constexpr int MM_MAXP = 4096;
template <typename TX>
__global__ __launch_bounds__(256) void k_mm_transpose(const TX* __restrict__ X, int64_t ldx, int64_t n,
                                                      int64_t p, TX* __restrict__ Xt, int64_t ldt) {
  __shared__ TX tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    tile[k][tx] = (r < n && c < p) ? X[r * ldx + c] : (TX)0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (c < p) Xt[c * ldt + r] = tile[tx][k];
  }
}

template <typename TX>
__global__ __launch_bounds__(256) void k_mm_step_t(const TX* __restrict__ Xt, int64_t ldt, int64_t n,
                                                   int64_t p, const TX* __restrict__ X, int64_t ldx,
                                                   const int64_t* __restrict__ idx, int s,
                                                   double* __restrict__ dmin, double* __restrict__ bval,
                                                   int64_t* __restrict__ bidx) {
  constexpr int VE = 16 / (int)sizeof(TX);  // rows per thread
  constexpr int ROWS = 256 * VE;            // rows per block
  typedef TX tv __attribute__((ext_vector_type(VE)));
  __shared__ double ms[MM_MAXP];
  __shared__ double wv[4];
  __shared__ int64_t wi[4];
  const int t = threadIdx.x;
  // odd steps walk the row blocks backwards, as in k_mm_step
  const int64_t blk = (s & 1) ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x;
  const int64_t i0 = blk * ROWS + (int64_t)t * VE;
  const TX* mrow = X + idx[s] * ldx;
  for (int k = t; k < p; k += 256) ms[k] = (double)mrow[k];
  __syncthreads();
  double acc[VE];
#pragma unroll
  for (int e = 0; e < VE; ++e) acc[e] = 0.0;
  const TX* col = Xt + i0;
#pragma unroll 8
  for (int64_t k = 0; k < p; ++k) {
    const tv v = *reinterpret_cast<const tv*>(col + k * ldt);
    const double m = ms[k];
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const double d = (double)v[e] - m;
      acc[e] = __dadd_rn(acc[e], __dmul_rn(d, d));
    }
  }
  double best = -1.0;
  int64_t at = INT64_MAX;
#pragma unroll
  for (int e = 0; e < VE; ++e) {
    const int64_t i = i0 + e;
    if (i < n) {
      const double v = (s == 0) ? acc[e] : fmin(dmin[i], acc[e]);
      dmin[i] = v;
      if (v > best) {  // rows ascending: ties keep the smaller row
        best = v;
        at = i;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(best, off, 64);
    const int64_t oi = __shfl_xor(at, off, 64);
    if (ov > best || (ov == best && oi < at)) {
      best = ov;
      at = oi;
    }
  }
  if ((t & 63) == 0) {
    wv[t >> 6] = best;
    wi[t >> 6] = at;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < 4; ++w)
      if (wv[w] > best || (wv[w] == best && wi[w] < at)) {
        best = wv[w];
        at = wi[w];
      }
    bval[blk] = best;
    bidx[blk] = at;
  }
}

// merge the block results of step s - 1 into landmark s; flag[0] = 1 when
// the largest smallest distance is zero (fewer than l distinct points)
__global__ __launch_bounds__(256) void k_mm_pick(const double* __restrict__ bval,
                                                 const int64_t* __restrict__ bidx, int nb,
                                                 int64_t* __restrict__ idx, int s,
                                                 int* __restrict__ flag) {
  __shared__ double wv[4];
  __shared__ int64_t wi[4];
  const int t = threadIdx.x;
  double best = -1.0;
  int64_t at = INT64_MAX;
  // eight block results in flight per thread (the order of the merge does
  // not matter: largest value, smallest row on ties is a total order)
  for (int b0 = t; b0 < nb; b0 += 256 * 8) {
    double v[8];
    int64_t ix[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + 256 * u;
      v[u] = (b < nb) ? bval[b] : -1.0;
      ix[u] = (b < nb) ? bidx[b] : INT64_MAX;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (v[u] > best || (v[u] == best && ix[u] < at)) {
        best = v[u];
        at = ix[u];
      }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(best, off, 64);
    const int64_t oi = __shfl_xor(at, off, 64);
    if (ov > best || (ov == best && oi < at)) {
      best = ov;
      at = oi;
    }
  }
  if ((t & 63) == 0) {
    wv[t >> 6] = best;
    wi[t >> 6] = at;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < 4; ++w)
      if (wv[w] > best || (wv[w] == best && wi[w] < at)) {
        best = wv[w];
        at = wi[w];
      }
    if (!(best > 0.0)) {
      flag[0] = 1;
      at = idx[s - 1];  // keep a valid row; the host reports the error
    }
    idx[s] = at;
  }
}

// ---------------------------------------------------------- pivot MDS
// Column sums of rows [c * rows_per, (c + 1) * rows_per): a block covers 64
// columns of one chunk, its four waves take the rows i = w (mod 4), and the
// four partials are added in order.
template <typename TX>
__global__ __launch_bounds__(256) void k_colsum_part(const TX* __restrict__ X, int64_t ldx, int64_t n,
                                                     int64_t p, int64_t rows_per,
                                                     double* __restrict__ part, int* __restrict__ bad) {
  __shared__ double ws[4][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * 64 + lane;
  const int64_t c = blockIdx.y;
  const int64_t i0 = c * rows_per, i1 = std::min(n, i0 + rows_per);
  double acc = 0.0;
  bool fin = true;
  if (k < p)
    for (int64_t i = i0 + g; i < i1; i += 4) {
      const double v = (double)X[i * ldx + k];
      fin = fin && isfinite(v);
      acc += v;
    }
  ws[g][lane] = acc;
  if (!fin) bad[0] = 1;
  __syncthreads();
  if (g == 0 && k < p) part[c * p + k] = ((ws[0][lane] + ws[1][lane]) + ws[2][lane]) + ws[3][lane];
}

// out[k] = scale * sum over c of part[c][k]: the chunks are split into
// PSEG segments summed in parallel, then the segments in order.
constexpr int PSEG = 16;
__global__ void k_sum_seg(const double* __restrict__ part, int64_t nparts, int64_t len,
                          double* __restrict__ seg) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int sg = blockIdx.y;
  if (k >= len) return;
  const int64_t per = (nparts + PSEG - 1) / PSEG;
  const int64_t c0 = sg * per, c1 = std::min(nparts, c0 + per);
  double acc = 0.0;
  for (int64_t c = c0; c < c1; ++c) acc += part[c * len + k];
  seg[sg * len + k] = acc;
}

__global__ void k_sum_parts(const double* __restrict__ seg, int64_t len, double scale,
                            double* __restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= len) return;
  double acc = 0.0;
  for (int sg = 0; sg < PSEG; ++sg) acc += seg[sg * len + k];
  out[k] = acc * scale;
}

// Partial S over rows [c * rows_per, (c + 1) * rows_per): 64x64 tile per
// block, 4x4 per thread, rows staged 16 at a time, centred on the mean.
// S[a][b] and S[b][a] are the same sums of the same products.
template <typename TX>
__global__ __launch_bounds__(256) void k_cov_part(const TX* __restrict__ X, int64_t ldx, int64_t n,
                                                  int64_t p, const double* __restrict__ mean,
                                                  int64_t rows_per, double* __restrict__ part) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int64_t a0 = (int64_t)blockIdx.y * 64, b0 = (int64_t)blockIdx.x * 64;
  const int64_t c = blockIdx.z;
  const int64_t i0 = c * rows_per, i1 = std::min(n, i0 + rows_per);
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int64_t s0 = i0; s0 < i1; s0 += 16) {
    for (int e = t; e < 16 * 64; e += 256) {
      const int ii = e >> 6, cc = e & 63;
      const int64_t i = s0 + ii;
      double va = 0.0, vb = 0.0;
      if (i < i1) {
        const TX* row = X + i * ldx;
        if (a0 + cc < p) va = (double)row[a0 + cc] - mean[a0 + cc];
        if (b0 + cc < p) vb = (double)row[b0 + cc] - mean[b0 + cc];
      }
      As[ii][cc] = va;
      Bs[ii][cc] = vb;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = As[kk][ty + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) bv[v] = Bs[kk][tx + 16 * v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
    }
    __syncthreads();
  }
  double* Sp = part + c * p * p;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t a = a0 + ty + 16 * u, b = b0 + tx + 16 * v;
      if (a < p && b < p) Sp[a * p + b] = acc[u][v];
    }
}

// The same partial S for p <= 128 on the FP64 matrix cores.  The chunk is
// walked 32 rows at a time: thread t owns column t % 128 of rows t / 128,
// t / 128 + 2, ..., loads the next step's values into registers while the
// matrix cores work on the current step, and writes them centred into LDS.
// The 16 x 16 output tiles on and above the diagonal (T (T + 1) / 2 of them,
// T = ceil(p / 16)) are shared out over the four waves, each accumulating
// S[a][b] = sum_i x_ia x_ib with v_mfma_f64_16x16x4f64 (lane (i, q) holds
// x[k + q][16 t + i] of both operands).  Every output is written to both
// symmetric positions.
constexpr int PV_COV_MAXP = 128;
constexpr int PV_COV_ROWS = 32;
constexpr int PV_COV_TILES = (PV_COV_MAXP / 16) * (PV_COV_MAXP / 16 + 1) / 2;  // 36
constexpr int PV_COV_PER_WAVE = (PV_COV_TILES + 3) / 4;                       // 9
template <typename TX>
__global__ __launch_bounds__(256) void k_cov_mfma(const TX* __restrict__ X, int64_t ldx, int64_t n,
                                                  int64_t p, const double* __restrict__ mean,
                                                  int64_t rows_per, double* __restrict__ part) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NV = PV_COV_ROWS / 2;  // values a thread carries per step
  __shared__ double xs[PV_COV_ROWS][PV_COV_MAXP + 1];
  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // the same in every lane of a wave
  const int li = lane & 15, lq = lane >> 4;
  const int T = (int)((p + 15) / 16);
  const int npairs = T * (T + 1) / 2;
  const int64_t c = blockIdx.x;
  const int64_t i0 = c * rows_per, i1 = std::min(n, i0 + rows_per);
  // the wave's tile pairs q = wv + 4 m, unranked row by row (ta <= tb)
  int ta[PV_COV_PER_WAVE], tb[PV_COV_PER_WAVE];
#pragma unroll
  for (int m = 0; m < PV_COV_PER_WAVE; ++m) {
    int q = wv + 4 * m, a = 0;
    ta[m] = -1;
    tb[m] = -1;
    if (q < npairs) {
      while (q >= T - a) {
        q -= T - a;
        ++a;
      }
      ta[m] = a;
      tb[m] = a + q;
    }
  }
  d4 acc[PV_COV_PER_WAVE];
#pragma unroll
  for (int m = 0; m < PV_COV_PER_WAVE; ++m) acc[m] = d4{0, 0, 0, 0};
  const int cc = t & (PV_COV_MAXP - 1), r0 = t / PV_COV_MAXP;
  const bool colok = cc < p;
  const double mu = colok ? mean[cc] : 0.0;
  TX v[NV];
  auto fetch = [&](int64_t s0) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int64_t i = s0 + r0 + 2 * u;
      v[u] = (colok && i < i1) ? X[i * ldx + cc] : TX(0);
    }
  };
  fetch(i0);
  for (int64_t s0 = i0; s0 < i1; s0 += PV_COV_ROWS) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int64_t i = s0 + r0 + 2 * u;
      xs[r0 + 2 * u][cc] = (colok && i < i1) ? (double)v[u] - mu : 0.0;
    }
    __syncthreads();
    if (s0 + PV_COV_ROWS < i1) fetch(s0 + PV_COV_ROWS);
#pragma unroll
    for (int k = 0; k < PV_COV_ROWS; k += 4) {
#pragma unroll
      for (int m = 0; m < PV_COV_PER_WAVE; ++m) {
        if (ta[m] >= 0) {
          const double av = xs[k + lq][16 * ta[m] + li];
          const double bv = xs[k + lq][16 * tb[m] + li];
          acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[m], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // FP64 result layout: element v of lane (j, g) is row g + 4 v, column j
  double* Sp = part + c * p * p;
#pragma unroll
  for (int m = 0; m < PV_COV_PER_WAVE; ++m) {
    if (ta[m] < 0) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t ra = 16 * ta[m] + lq + 4 * e, cb = 16 * tb[m] + li;
      if (ra < p && cb < p) {
        Sp[ra * p + cb] = acc[m][e];
        Sp[cb * p + ra] = acc[m][e];
      }
    }
  }
}

// Mc[j][k] = X[idx[j]][k] - mbar[k]; mbar = mean of the pivot rows: a block
// takes 64 columns, wave g the pivots j = g (mod 4) in order, and the four
// partial sums are added in a fixed order.
template <typename TX>
__global__ __launch_bounds__(256) void k_pivots_centred(const TX* __restrict__ X, int64_t ldx, int64_t p,
                                                        const int64_t* __restrict__ idx, int64_t l,
                                                        double* __restrict__ Mc) {
  __shared__ double ws[4][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (k < p) {
#pragma unroll 4
    for (int64_t j = g; j < l; j += 4) acc += (double)X[idx[j] * ldx + k];
  }
  ws[g][lane] = acc;
  __syncthreads();
  const double mb = (((ws[0][lane] + ws[1][lane]) + ws[2][lane]) + ws[3][lane]) / (double)l;
  if (k < p) {
#pragma unroll 4
    for (int64_t j = g; j < l; j += 4) Mc[j * p + k] = (double)X[idx[j] * ldx + k] - mb;
  }
}

// T = Mc S (l x p), one output per thread
__global__ void k_mc_s(const double* __restrict__ Mc, const double* __restrict__ S, int64_t l,
                       int64_t p, double* __restrict__ T) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= l * p) return;
  const int64_t j = e / p, k = e % p;
  double acc = 0.0;
  for (int64_t q = 0; q < p; ++q) acc = fma(Mc[j * p + q], S[q * p + k], acc);
  T[e] = acc;
}

// K = T Mc' (l x l), then symmetrised: K[i][j] = (K[i][j] + K[j][i]) / 2,
// computed identically for both entries
__global__ void k_t_mct(const double* __restrict__ T, const double* __restrict__ Mc, int64_t l,
                        int64_t p, double* __restrict__ K) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= l * l) return;
  const int64_t i = e / l, j = e % l;
  double a = 0.0, b = 0.0;
  for (int64_t q = 0; q < p; ++q) {
    a = fma(T[i * p + q], Mc[j * p + q], a);
    b = fma(T[j * p + q], Mc[i * p + q], b);
  }
  K[e] = (i <= j) ? 0.5 * (a + b) : 0.5 * (b + a);
}

// ---- the p x p route (p < l): C'C = Mc S Mc' = B B' with B = Mc L and
// S = L L' (Cholesky), so its nonzero eigenpairs are those of G = B'B
// (p x p): eigenvalue lambda with vector w = B u / sqrt(lambda) for the unit
// eigenvector u of G.  The dense solver then works on a p x p matrix (in
// LDS for p <= 100 or so) instead of l x l.
constexpr int PV_CHOL_MAXP = 128;
// S = L L' in one block (right-looking, S in LDS); L lower triangular with
// zeros above the diagonal.  flag[0] = 1 on a pivot that is not positive
// and finite (S singular to working precision): L is then zero and the
// caller takes the l x l route.
__global__ __launch_bounds__(1024) void k_chol(const double* __restrict__ S, int p, double* __restrict__ L,
                                               int* __restrict__ flag) {
  extern __shared__ double a[];  // p x (p + 1)
  const int t = threadIdx.x;
  const int ld = p + 1;
  for (int e = t; e < p * p; e += 1024) a[(e / p) * ld + e % p] = S[e];
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < p; ++k) {
    const double d = a[k * ld + k];
    if (!(d > 0.0) || !isfinite(d)) {
      bad = true;
      break;  // uniform: every thread reads the same pivot
    }
    const double piv = sqrt(d);
    __syncthreads();  // every thread has read a[k][k]
    for (int i = k + t; i < p; i += 1024) a[i * ld + k] = (i == k) ? piv : a[i * ld + k] / piv;
    __syncthreads();
    // trailing lower part: thread (ti, tj) of a 32 x 32 grid takes rows
    // k + 1 + ti + 32 u and columns k + 1 + tj + 32 v up to the diagonal
    const int ti = t >> 5, tj = t & 31;
    for (int i = k + 1 + ti; i < p; i += 32) {
      const double lik = a[i * ld + k];
      for (int j = k + 1 + tj; j <= i; j += 32) a[i * ld + j] -= lik * a[j * ld + k];
    }
    __syncthreads();
  }
  if (t == 0) flag[0] = bad ? 1 : 0;
  // on failure L is all zeros, so the p x p chain launched behind this
  // kernel (before the host reads the flag) works on defined values
  for (int e = t; e < p * p; e += 1024) {
    const int i = e / p, j = e % p;
    L[e] = (!bad && j <= i) ? a[i * ld + j] : 0.0;
  }
}

// B = Mc L (l x p), L lower triangular
__global__ void k_mc_l(const double* __restrict__ Mc, const double* __restrict__ L, int64_t l, int64_t p,
                       double* __restrict__ B) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= l * p) return;
  const int64_t i = e / p, j = e % p;
  double acc = 0.0;
  for (int64_t q = j; q < p; ++q) acc = fma(Mc[i * p + q], L[q * p + j], acc);
  B[e] = acc;
}

// G = B'B (p x p), computed identically for both entries of each pair
__global__ void k_btb(const double* __restrict__ B, int64_t l, int64_t p, double* __restrict__ G) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= p * p) return;
  const int64_t a = e / p, b = e % p;
  const int64_t lo = a < b ? a : b, hi = a < b ? b : a;
  double acc = 0.0;
  for (int64_t i = 0; i < l; ++i) acc = fma(B[i * p + lo], B[i * p + hi], acc);
  G[e] = acc;
}

// W[i][t] = sum_a B[i][a] U[a][t] / sqrt(lambda_t) (l x r; zero when
// lambda_t <= 0: such a direction is dead)
__global__ void k_w_from_u(const double* __restrict__ B, const double* __restrict__ U,
                           const double* __restrict__ lam, int64_t l, int64_t p, int r,
                           double* __restrict__ W) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= l * r) return;
  const int64_t i = e / r;
  const int t = (int)(e % r);
  const double lt = lam[t];
  if (!(lt > 0.0)) {
    W[e] = 0.0;
    return;
  }
  double acc = 0.0;
  for (int64_t a2 = 0; a2 < p; ++a2) acc = fma(B[i * p + a2], U[a2 * r + t], acc);
  W[e] = acc / sqrt(lt);
}

// A[t][k] = fac[t] * sum_j Mc[j][k] W[j][t] (r x p); b[t] = -sum_k A[t][k] xbar[k]
__global__ void k_pivot_affine(const double* __restrict__ Mc, const double* __restrict__ W, int64_t l,
                               int64_t p, int r, const double* __restrict__ fac,
                               double* __restrict__ A) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * p) return;
  const int64_t t = e / p, k = e % p;
  double acc = 0.0;
  for (int64_t j = 0; j < l; ++j) acc = fma(Mc[j * p + k], W[j * r + t], acc);
  A[e] = fac[t] * acc;
}

__global__ void k_affine_shift(const double* __restrict__ A, const double* __restrict__ xbar, int64_t p,
                               int r, double* __restrict__ b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r) return;
  double acc = 0.0;
  for (int64_t k = 0; k < p; ++k) acc = fma(A[(int64_t)t * p + k], xbar[k], acc);
  b[t] = -acc;
}

// idx[0] = first and flag = 0 (a fill kernel rather than a memset and a
// host copy, so the steps need no host data once launched)
__global__ void k_mm_init(int64_t* __restrict__ idx, int64_t first, int* __restrict__ flag) {
  if (threadIdx.x == 0) {
    idx[0] = first;
    flag[0] = 0;
  }
}

// The steps of MaxMin on buffers the caller provides: dmin (n), bval and
// bidx (one per row block), idx (l), flag (1); Xt (p x ldt) when the
// column-major copy is used, else NULL.  Copies idx to the host and waits.
template <typename TX>
mds_status maxmin_steps(const TX* X, int64_t ldx, int64_t n, int64_t p, int64_t l, int64_t first,
                        int64_t* idx_host, hipStream_t st, double* dmin, double* bval, int64_t* bidx,
                        int64_t* idx, int* flag, TX* Xt, int64_t ldt) {
  const int nb = (int)((n + MM_ROWS - 1) / MM_ROWS);
  k_mm_init<<<1, 64, 0, st>>>(idx, first, flag);
  PV_LAUNCH("maxmin init");
  if (Xt) {
    k_mm_transpose<TX><<<dim3((unsigned)(ldt / 32), (unsigned)((p + 31) / 32)), 256, 0, st>>>(X, ldx, n, p,
                                                                                               Xt, ldt);
    PV_LAUNCH("maxmin column-major copy");
  }
  constexpr int64_t ROWS_T = 256 * (16 / (int64_t)sizeof(TX));
  const int nbs = Xt ? (int)(ldt / ROWS_T) : nb;
  for (int s = 0; s + 1 < l; ++s) {
    if (Xt)
      k_mm_step_t<TX><<<nbs, 256, 0, st>>>(Xt, ldt, n, p, X, ldx, idx, s, dmin, bval, bidx);
    else
      k_mm_step<TX><<<nbs, 256, 0, st>>>(X, ldx, n, p, idx, s, dmin, bval, bidx);
    k_mm_pick<<<1, 256, 0, st>>>(bval, bidx, nbs, idx, s + 1, flag);
  }
  PV_LAUNCH("maxmin steps");
  int hflag = 0;
  PV_HIP(hipMemcpyAsync(idx_host, idx, sizeof(int64_t) * l, hipMemcpyDeviceToHost, st));
  PV_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  PV_HIP(hipStreamSynchronize(st));
  if (hflag) return set_error(MDS_ERR_DEGENERATE, "fewer than l distinct points");
  return MDS_OK;
}

template <typename TX>
mds_status maxmin_run(const TX* X, int64_t ldx, int64_t n, int64_t p, int64_t l, int64_t first,
                      int64_t* idx_host, hipStream_t st) {
  const int nb = (int)((n + MM_ROWS - 1) / MM_ROWS);
  Buf dmin, bval, bidx, idx, flag;
  auto alloc = [&](Buf& b, size_t bytes) -> hipError_t {
    b.st = st;
    return hipMallocAsync(&b.p, std::max<size_t>(bytes, 256), st);
  };
  PV_HIP(alloc(dmin, sizeof(double) * n));
  PV_HIP(alloc(bval, sizeof(double) * nb));
  PV_HIP(alloc(bidx, sizeof(int64_t) * nb));
  PV_HIP(alloc(idx, sizeof(int64_t) * l));
  PV_HIP(alloc(flag, sizeof(int)));
  // column-major copy when there is room for it (else the row-major steps)
  constexpr int64_t ROWS_T = 256 * (16 / (int64_t)sizeof(TX));
  const int64_t ldt = (n + ROWS_T - 1) / ROWS_T * ROWS_T;
  Buf Xt;
  bool col_major = l > 1 && p <= MM_MAXP && alloc(Xt, sizeof(TX) * p * ldt) == hipSuccess;
  if (!col_major) (void)hipGetLastError();
  return maxmin_steps<TX>(X, ldx, n, p, l, first, idx_host, st, dmin.get<double>(), bval.get<double>(),
                          bidx.get<int64_t>(), idx.get<int64_t>(), flag.get<int>(),
                          col_major ? Xt.get<TX>() : nullptr, ldt);
}

// ---- MaxMin without allocation ----
// One static device array per GPU holds the step buffers, laid out for the
// largest accepted call (MDS_NOALLOC_MAX_N rows, MDS_NOALLOC_MAX_L
// landmarks); every call on a GPU reuses that GPU's copy, so calls that
// overlap on one GPU race.  Only the row-major steps run (the column-major
// copy of X would not fit a bounded array).
constexpr int64_t NA_NB = (MDS_NOALLOC_MAX_N + MM_ROWS - 1) / MM_ROWS;
constexpr size_t na_round(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t NA_OFF_BVAL = na_round(sizeof(double) * MDS_NOALLOC_MAX_N);
constexpr size_t NA_OFF_BIDX = NA_OFF_BVAL + na_round(sizeof(double) * NA_NB);
constexpr size_t NA_OFF_IDX = NA_OFF_BIDX + na_round(sizeof(int64_t) * NA_NB);
constexpr size_t NA_OFF_FLAG = NA_OFF_IDX + na_round(sizeof(int64_t) * MDS_NOALLOC_MAX_L);
constexpr size_t NA_BYTES = NA_OFF_FLAG + 256;
static_assert(NA_BYTES == MDS_NOALLOC_SCRATCH_BYTES, "scratch size stated in the header");

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

// device address of this GPU's scratch array, looked up once per device
// (the name `scratch` is a host-side stand-in and must not reach a kernel)
constexpr int NA_MAX_DEV = 64;
std::mutex na_mu;
void* na_ptr[NA_MAX_DEV] = {};

mds_status scratch_for_current_device(unsigned char** out) {
  int dev = 0;
  PV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NA_MAX_DEV) return set_error(MDS_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> g(na_mu);
  if (!na_ptr[dev]) {
    void* ptr = nullptr;
    PV_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return set_error(MDS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    na_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(na_ptr[dev]);
  return MDS_OK;
}

template <typename TX>
mds_status maxmin_run_noalloc(const TX* X, int64_t ldx, int64_t n, int64_t p, int64_t l, int64_t first,
                              int64_t* idx_host, hipStream_t st) {
  unsigned char* base = nullptr;
  mds_status s = scratch_for_current_device(&base);
  if (s != MDS_OK) return s;
  return maxmin_steps<TX>(X, ldx, n, p, l, first, idx_host, st, reinterpret_cast<double*>(base),
                          reinterpret_cast<double*>(base + NA_OFF_BVAL),
                          reinterpret_cast<int64_t*>(base + NA_OFF_BIDX),
                          reinterpret_cast<int64_t*>(base + NA_OFF_IDX), reinterpret_cast<int*>(base + NA_OFF_FLAG),
                          nullptr, 0);
}

template <typename TX>
mds_status pivot_run(const TX* X, int dt, int64_t ldx, int64_t n, int64_t p, int64_t l, int r,
                     const int64_t* idx_host, double* Y, int64_t ldy, double* lam_host, int32_t* r_eff,
                     hipStream_t st) {
  // row chunks of at least 1024 rows, partial S within ~512 MB; at most 768
  // chunks, so the matrix-core covariance (three blocks per compute unit)
  // covers all of them in one pass over 256 compute units
  const int64_t by_mem = std::max<int64_t>(1, ((int64_t)512 << 20) / (int64_t)(sizeof(double) * p * p));
  const int64_t nchunks = std::max<int64_t>(1, std::min<int64_t>({(n + 1023) / 1024, 768, by_mem}));
  const int64_t rows_per = (n + nchunks - 1) / nchunks;
  Buf idx, part, xbar, Spart, S, Mc, T, K, lam, W, stat, fac, A, b, bad, seg;
  auto alloc = [&](Buf& bb, size_t bytes) -> hipError_t {
    bb.st = st;
    return hipMallocAsync(&bb.p, std::max<size_t>(bytes, 256), st);
  };
  PV_HIP(alloc(idx, sizeof(int64_t) * l));
  PV_HIP(alloc(part, sizeof(double) * nchunks * p));
  PV_HIP(alloc(xbar, sizeof(double) * p));
  PV_HIP(alloc(Spart, sizeof(double) * nchunks * p * p));
  PV_HIP(alloc(S, sizeof(double) * p * p));
  PV_HIP(alloc(seg, sizeof(double) * PSEG * p * p));
  PV_HIP(alloc(Mc, sizeof(double) * l * p));
  PV_HIP(alloc(T, sizeof(double) * l * p));
  PV_HIP(alloc(K, sizeof(double) * l * l));
  PV_HIP(alloc(lam, sizeof(double) * r));
  PV_HIP(alloc(W, sizeof(double) * l * r));
  PV_HIP(alloc(stat, sizeof(int)));
  PV_HIP(alloc(fac, sizeof(double) * r));
  PV_HIP(alloc(A, sizeof(double) * r * p));
  PV_HIP(alloc(b, sizeof(double) * r));
  PV_HIP(alloc(bad, sizeof(int)));
  PV_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
  PV_HIP(hipMemcpyAsync(idx.p, idx_host, sizeof(int64_t) * l, hipMemcpyHostToDevice, st));
  {
    dim3 g((unsigned)((p + 63) / 64), (unsigned)nchunks);
    k_colsum_part<TX><<<g, 256, 0, st>>>(X, ldx, n, p, rows_per, part.get<double>(), bad.get<int>());
    dim3 gs((unsigned)((p + 255) / 256), PSEG);
    k_sum_seg<<<gs, 256, 0, st>>>(part.get<double>(), nchunks, p, seg.get<double>());
    k_sum_parts<<<(unsigned)((p + 255) / 256), 256, 0, st>>>(seg.get<double>(), p, 1.0 / (double)n,
                                                            xbar.get<double>());
    const unsigned tiles = (unsigned)((p + 63) / 64);
    dim3 gc(tiles, tiles, (unsigned)nchunks);
    if (p <= PV_COV_MAXP)
      k_cov_mfma<TX><<<(unsigned)nchunks, 256, 0, st>>>(X, ldx, n, p, xbar.get<double>(), rows_per,
                                                        Spart.get<double>());
    else
      k_cov_part<TX><<<gc, 256, 0, st>>>(X, ldx, n, p, xbar.get<double>(), rows_per, Spart.get<double>());
    dim3 gs2((unsigned)((p * p + 255) / 256), PSEG);
    k_sum_seg<<<gs2, 256, 0, st>>>(Spart.get<double>(), nchunks, p * p, seg.get<double>());
    k_sum_parts<<<(unsigned)((p * p + 255) / 256), 256, 0, st>>>(seg.get<double>(), p * p, 1.0,
                                                                S.get<double>());
    k_pivots_centred<TX><<<(unsigned)((p + 63) / 64), 256, 0, st>>>(X, ldx, p, idx.get<int64_t>(), l,
                                                                    Mc.get<double>());
    PV_LAUNCH("pivot Gram matrices");
  }
  // l x l route: K = Mc S Mc' and its top eigenpairs
  auto l_route = [&]() -> mds_status {
    k_mc_s<<<(unsigned)((l * p + 255) / 256), 256, 0, st>>>(Mc.get<double>(), S.get<double>(), l, p,
                                                           T.get<double>());
    k_t_mct<<<(unsigned)((l * l + 255) / 256), 256, 0, st>>>(T.get<double>(), Mc.get<double>(), l, p,
                                                            K.get<double>());
    PV_LAUNCH("pivot C'C");
    return dense_top_eigen(K.get<double>(), (int)l, r, lam.get<double>(), W.get<double>(),
                           stat.get<int>(), st);
  };
  // p x p route when p < l (see k_chol); cflag says whether it held
  const bool p_route = p < l && p <= PV_CHOL_MAXP;
  Buf Lc, Bm, G, U, cflag;
  mds_status s = MDS_OK;
  if (p_route) {
    PV_HIP(alloc(Lc, sizeof(double) * p * p));
    PV_HIP(alloc(Bm, sizeof(double) * l * p));
    PV_HIP(alloc(G, sizeof(double) * p * p));
    PV_HIP(alloc(U, sizeof(double) * p * r));
    PV_HIP(alloc(cflag, sizeof(int)));
    PV_HIP(lds_limit_once(reinterpret_cast<const void*>(&k_chol),
                          (int)(sizeof(double) * PV_CHOL_MAXP * (PV_CHOL_MAXP + 1))));
    k_chol<<<1, 1024, sizeof(double) * (size_t)p * (p + 1), st>>>(S.get<double>(), (int)p, Lc.get<double>(),
                                                                   cflag.get<int>());
    k_mc_l<<<(unsigned)((l * p + 255) / 256), 256, 0, st>>>(Mc.get<double>(), Lc.get<double>(), l, p,
                                                           Bm.get<double>());
    k_btb<<<(unsigned)((p * p + 255) / 256), 256, 0, st>>>(Bm.get<double>(), l, p, G.get<double>());
    PV_LAUNCH("pivot p x p Gram");
    s = dense_top_eigen(G.get<double>(), (int)p, r, lam.get<double>(), U.get<double>(), stat.get<int>(), st);
    if (s != MDS_OK) return s;
    k_w_from_u<<<(unsigned)((l * r + 255) / 256), 256, 0, st>>>(Bm.get<double>(), U.get<double>(),
                                                               lam.get<double>(), l, p, r, W.get<double>());
    PV_LAUNCH("pivot vectors");
  } else {
    s = l_route();
    if (s != MDS_OK) return s;
  }
  std::vector<double> th(r), hw((size_t)l * r);
  int hstat = 0, hbad = 0, hchol = 0;
  PV_HIP(hipMemcpyAsync(th.data(), lam.p, sizeof(double) * r, hipMemcpyDeviceToHost, st));
  PV_HIP(hipMemcpyAsync(hw.data(), W.p, sizeof(double) * l * r, hipMemcpyDeviceToHost, st));
  PV_HIP(hipMemcpyAsync(&hstat, stat.p, sizeof(int), hipMemcpyDeviceToHost, st));
  PV_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  if (p_route) PV_HIP(hipMemcpyAsync(&hchol, cflag.p, sizeof(int), hipMemcpyDeviceToHost, st));
  PV_HIP(hipStreamSynchronize(st));
  if (hbad) return set_error(MDS_ERR_INVALID_ARG, "non-finite value in X");
  if (p_route && hchol) {  // S singular to working precision: the l x l route
    s = l_route();
    if (s != MDS_OK) return s;
    PV_HIP(hipMemcpyAsync(th.data(), lam.p, sizeof(double) * r, hipMemcpyDeviceToHost, st));
    PV_HIP(hipMemcpyAsync(hw.data(), W.p, sizeof(double) * l * r, hipMemcpyDeviceToHost, st));
    PV_HIP(hipMemcpyAsync(&hstat, stat.p, sizeof(int), hipMemcpyDeviceToHost, st));
    PV_HIP(hipStreamSynchronize(st));
  }
  if (hstat) return set_error(MDS_ERR_DEGENERATE, "largest eigenvalue is not positive");
  // sigma^2 = eigenvalues of C'C; lambda = sigma sqrt(n / l); column signs
  // from W (largest-|.| entry positive, first on ties)
  // a direction is live when sigma^2 > TAU sigma_1^2: Section 2's test on
  // the eigenvalues of the matrix pivot MDS decomposes, C'C; dead directions
  // report lambda = 0
  std::vector<double> hfac(r, 0.0);
  int live = 0;
  for (int t = 0; t < r; ++t) {
    const double sigma = std::sqrt(std::max(th[t], 0.0));
    const double lamt = sigma * std::sqrt((double)n / (double)l);
    const bool is_live = th[t] > MDS_TAU * th[0];
    if (lam_host) lam_host[t] = is_live ? lamt : 0.0;
    if (!is_live) continue;
    ++live;
    double best = -1.0, val = 0.0;
    for (int64_t j = 0; j < l; ++j) {
      const double v = hw[(size_t)j * r + t];
      if (std::fabs(v) > best) {
        best = std::fabs(v);
        val = v;
      }
    }
    hfac[t] = (val < 0.0 ? -1.0 : 1.0) * std::sqrt(lamt) / sigma;
  }
  if (r_eff) *r_eff = live;
  PV_HIP(hipMemcpyAsync(fac.p, hfac.data(), sizeof(double) * r, hipMemcpyHostToDevice, st));
  k_pivot_affine<<<(unsigned)((r * p + 255) / 256), 256, 0, st>>>(Mc.get<double>(), W.get<double>(), l, p,
                                                                 r, fac.get<double>(), A.get<double>());
  k_affine_shift<<<1, 64, 0, st>>>(A.get<double>(), xbar.get<double>(), p, r, b.get<double>());
  PV_LAUNCH("pivot affine map");
  s = launch_affine_raw(A.p, b.p, 1, p, r, X, dt, n, ldx, Y, ldy, st);
  if (s != MDS_OK) return s;
  PV_HIP(hipStreamSynchronize(st));
  return MDS_OK;
}

}  // namespace

mds_status maxmin_on_device(const void* X, int dt, int64_t n, int64_t p, int64_t ldx, int64_t l,
                            int64_t first, int64_t* idx_host, hipStream_t st) {
  if (l == 1) {
    idx_host[0] = first;
    return MDS_OK;
  }
  if (dt == MDS_F32)
    return maxmin_run<float>(static_cast<const float*>(X), ldx, n, p, l, first, idx_host, st);
  return maxmin_run<double>(static_cast<const double*>(X), ldx, n, p, l, first, idx_host, st);
}

mds_status maxmin_on_device_noalloc(const void* X, int dt, int64_t n, int64_t p, int64_t ldx, int64_t l,
                                    int64_t first, int64_t* idx_host, hipStream_t st) {
  if (l == 1) {
    idx_host[0] = first;
    return MDS_OK;
  }
  if (dt == MDS_F32)
    return maxmin_run_noalloc<float>(static_cast<const float*>(X), ldx, n, p, l, first, idx_host, st);
  return maxmin_run_noalloc<double>(static_cast<const double*>(X), ldx, n, p, l, first, idx_host, st);
}

mds_status pivot_on_device(const void* X, int dt, int64_t n, int64_t p, int64_t ldx, int64_t l, int r,
                           const int64_t* idx_host, double* Y, int64_t ldy, double* lam_host,
                           int32_t* r_eff, hipStream_t st) {
  if (dt == MDS_F32)
    return pivot_run<float>(static_cast<const float*>(X), dt, ldx, n, p, l, r, idx_host, Y, ldy, lam_host,
                            r_eff, st);
  return pivot_run<double>(static_cast<const double*>(X), dt, ldx, n, p, l, r, idx_host, Y, ldy, lam_host,
                           r_eff, st);
}

}  // namespace mds
