// Fit: classical MDS on the landmarks, all in FP64 on the GPU.
//
//   gather      M = X[idx]                                  (Section 3.1)
//   sqdist      Delta1_ij = sum_k (M_ik - M_jk)^2            (Section 2)
//   centring    Q1 = -1/2 (Delta1 - d1 1' - 1 d1' + dbar 11'),  q1 = diag(Q1)
//               (the element-wise form of -1/2 P Delta1 P, Section 2)
//   eigen       the r largest eigenpairs of Q1 by Lanczos with full
//               reorthogonalisation; the paper also uses a Lanczos solver
//               (Section 2).  Ritz pairs come from a bisection / inverse
//               iteration solve of the small tridiagonal matrix.
//   finalise    sign convention, X1 = V Lambda^{1/2}, W = 1/2 V Lambda^{-1/2}
//               (eq. (2) after (1/l) X1 S1^{-1} = V Lambda^{-1/2}, Section 3.1),
//               c = q1 - |m|^2, and the operand packs of the embed kernels.
//
// Every reduction has a fixed order, so a fit is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "mds_internal.h"
#include "tridiag_dev.h"

namespace mds {

namespace {

constexpr int RED_THREADS = 256;

__device__ inline double block_sum(double v, double* sh) {
  // fixed-order tree reduction over a 256-thread block
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- gather
template <typename TX>
__global__ void k_gather(const TX* __restrict__ X, int64_t ldx, const int64_t* __restrict__ idx,
                         int64_t l, int64_t p, int64_t ldm, double* __restrict__ M,
                         int* __restrict__ bad) {
  const int64_t total = l * p;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / p, k = e - (e / p) * p;
    const double v = (double)X[idx[i] * ldx + k];
    if (!isfinite(v)) bad[0] = 1;
    M[i * ldm + k] = v;
  }
}

// ------------------------------------------------ landmark squared distances
// 64x64 output tile per block, 4x4 per thread, contraction staged by 16.
// Blocks take the tiles on and above the diagonal (linear index t -> tile
// row bi <= tile column bj) and also write the mirrored tile: each entry is
// a sum of (a_k - b_k)^2 over k in order, which is the same number with a
// and b exchanged, so Delta1 comes out exactly symmetric.
__global__ __launch_bounds__(256) void k_sqdist(const double* __restrict__ M, int64_t ldm,
                                                int64_t l, int64_t p, double* __restrict__ D) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  __shared__ double Tt[64][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int tl = (int)blockIdx.x;
  int bj = (int)((sqrt(8.0 * tl + 1.0) - 1.0) * 0.5);
  while ((bj + 1) * (bj + 2) / 2 <= tl) ++bj;
  while (bj * (bj + 1) / 2 > tl) --bj;
  const int bi = tl - bj * (bj + 1) / 2;
  const int64_t i0 = (int64_t)bi * 64, j0 = (int64_t)bj * 64;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int64_t k0 = 0; k0 < p; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int row = e >> 4, kk = e & 15;
      const int64_t gk = k0 + kk;
      const int64_t gi = i0 + row, gj = j0 + row;
      As[kk][row] = (gi < l && gk < p) ? M[gi * ldm + gk] : 0.0;
      Bs[kk][row] = (gj < l && gk < p) ? M[gj * ldm + gk] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        a[x] = As[kk][ty * 4 + x];
        b[x] = Bs[kk][tx * 4 + x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const double d = a[x] - b[y];
          acc[x][y] = fma(d, d, acc[x][y]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int64_t i = i0 + ty * 4 + x, j = j0 + tx * 4 + y;
      if (i < l && j < l) D[i * l + j] = acc[x][y];
    }
  if (bi == bj) return;
  // the mirrored tile, transposed through LDS so that the writes are rows
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) Tt[tx * 4 + y][ty * 4 + x] = acc[x][y];
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int jl = e >> 6, il = e & 63;
    const int64_t j = j0 + jl, i = i0 + il;
    if (i < l && j < l) D[j * l + i] = Tt[jl][il];
  }
}

// Copy a caller's squared-dissimilarity matrix into Delta1, flagging
// non-finite entries (flag[0]) and asymmetry (flag[1]); the copy is made
// exactly symmetric as (d_ij + d_ji) / 2.
__global__ __launch_bounds__(256) void k_load_sqdist(const double* __restrict__ D1, int64_t ldd,
                                                     int64_t l, double* __restrict__ D,
                                                     int* __restrict__ flags) {
  const int64_t total = l * l;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / l, j = e - (e / l) * l;
    const double a = D1[i * ldd + j], b = D1[j * ldd + i];
    if (!isfinite(a)) flags[0] = 1;
    if (fabs(a - b) > 1e-12 * (fabs(a) + fabs(b))) flags[1] = 1;
    D[e] = 0.5 * (a + b);
  }
}

// ------------------------------------------------------------- centring
__global__ __launch_bounds__(256) void k_rowmean(const double* __restrict__ D, int64_t l,
                                                 double* __restrict__ d1) {
  __shared__ double sh[RED_THREADS];
  const int64_t i = blockIdx.x;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < l; j += RED_THREADS) s += D[i * l + j];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) d1[i] = s / (double)l;
}

__global__ __launch_bounds__(256) void k_mean(const double* __restrict__ v, int64_t l,
                                              double* __restrict__ out) {
  __shared__ double sh[RED_THREADS];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < l; j += RED_THREADS) s += v[j];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = s / (double)l;
}

// Q1_ij = -1/2 (Delta_ij - (d1_i + d1_j) + dbar), in place; exactly symmetric.
__global__ __launch_bounds__(256) void k_centre(double* __restrict__ DQ, int64_t l,
                                                const double* __restrict__ d1,
                                                const double* __restrict__ dbar,
                                                double* __restrict__ q, double* __restrict__ rowsq) {
  __shared__ double sh[RED_THREADS];
  const int64_t i = blockIdx.x;
  const double di = d1[i], db = dbar[0];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < l; j += RED_THREADS) {
    const double v = -0.5 * ((DQ[i * l + j] - (di + d1[j])) + db);
    DQ[i * l + j] = v;
    if (j == i) q[i] = v;
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) rowsq[i] = s;
}

__global__ __launch_bounds__(256) void k_sqrt_sum(const double* __restrict__ v, int64_t l,
                                                  double* __restrict__ out) {
  __shared__ double sh[RED_THREADS];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < l; j += RED_THREADS) s += v[j];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

// -------------------------------------------------------------- Lanczos
// ctrl[0] = stop flag (an invariant subspace was reached), ctrl[1] = the
// step at which it happened.  Kernels of later steps in the same batch
// return at once when the flag is set.

__global__ void k_fill_random(double* __restrict__ w, int64_t l, uint64_t salt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < l) w[i] = hash_unit((uint64_t)i, salt);
}

// w = Q v, one block per row
__global__ __launch_bounds__(256) void k_symv(const double* __restrict__ Q, int64_t l,
                                              const double* __restrict__ v,
                                              double* __restrict__ w, const int* __restrict__ ctrl) {
  if (ctrl[0]) return;
  __shared__ double sh4[4];
  const int64_t row = blockIdx.x;
  const double* qr = Q + row * l;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < l; c += 256) s = fma(qr[c], v[c], s);
  s = block_sum4(s, sh4);
  if (threadIdx.x == 0) w[row] = s;
}

// w = Q v for l <= kSymvRowsMaxL: v staged in LDS once per block, one row
// per wave (four rows per block), four independent sums per lane combined
// in a fixed order, then a fixed butterfly over the wave.  Against one
// block per row, each block reads v from L2 once for four rows.  For
// larger l one block per row (k_symv) keeps more of Q in flight.
constexpr int64_t kSymvRowsMaxL = 1024;
__global__ __launch_bounds__(256) void k_symv_rows(const double* __restrict__ Q, int64_t l,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ w, const int* __restrict__ ctrl) {
  if (ctrl[0]) return;
  extern __shared__ double vs[];
  for (int64_t i = threadIdx.x; i < l; i += 256) vs[i] = v[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= l) return;
  const double* qr = Q + row * l;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t c = lane;
  for (; c + 192 < l; c += 256) {
    s0 = fma(qr[c], vs[c], s0);
    s1 = fma(qr[c + 64], vs[c + 64], s1);
    s2 = fma(qr[c + 128], vs[c + 128], s2);
    s3 = fma(qr[c + 192], vs[c + 192], s3);
  }
  for (; c < l; c += 64) s0 = fma(qr[c], vs[c], s0);
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) w[row] = s;
}

// h_c = V_c' w for c < ncols (one block per column)
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ V, int64_t l,
                                              const double* __restrict__ w, double* __restrict__ h,
                                              const int* __restrict__ ctrl) {
  if (ctrl[0]) return;
  __shared__ double sh4[4];
  const int64_t c = blockIdx.x;
  const double* vc = V + c * l;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < l; i += 256) s = fma(vc[i], w[i], s);
  s = block_sum4(s, sh4);
  if (threadIdx.x == 0) h[c] = s;
}

// w -= V[:, :ncols] h; a block owns 64 rows, four column groups combined in order
__global__ __launch_bounds__(256) void k_update(const double* __restrict__ V, int64_t l, int ncols,
                                                const double* __restrict__ h,
                                                double* __restrict__ w, const int* __restrict__ ctrl) {
  if (ctrl[0]) return;
  extern __shared__ double hs[];
  __shared__ double part[4][64];
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) hs[c] = h[c];
  __syncthreads();
  const int rl = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + rl;
  double s = 0.0;
  if (i < l)
    for (int c = g; c < ncols; c += 4) s = fma(V[(int64_t)c * l + i], hs[c], s);
  part[g][rl] = s;
  __syncthreads();
  if (g == 0 && i < l) w[i] -= ((part[0][rl] + part[1][rl]) + part[2][rl]) + part[3][rl];
}

// alpha_j, beta_j = |w|, v_{j+1} = w / beta_j, or flag an invariant subspace.
__global__ __launch_bounds__(1024) void k_finish(double* __restrict__ V, int64_t l, int j,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ h1,
                                                 const double* __restrict__ h2,
                                                 double* __restrict__ alpha, double* __restrict__ beta,
                                                 const double* __restrict__ qnorm, int* __restrict__ ctrl,
                                                 int write_next) {
  if (ctrl[0]) return;
  __shared__ double sh[1024];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < l; i += 1024) s = fma(w[i], w[i], s);
  sh[t] = s;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if (t < st) sh[t] += sh[t + st];
    __syncthreads();
  }
  const double nrm = sqrt(sh[0]);
  const bool breakdown = !(nrm > 1e-12 * qnorm[0]);
  if (t == 0) {
    alpha[j] = h1[j] + h2[j];
    beta[j] = breakdown ? 0.0 : nrm;
  }
  if (breakdown) {
    if (t == 0) {
      ctrl[0] = 1;
      ctrl[1] = j;
    }
    return;
  }
  if (write_next) {
    const double inv = 1.0 / nrm;
    double* vn = V + (int64_t)(j + 1) * l;
    for (int64_t i = t; i < l; i += 1024) vn[i] = w[i] * inv;
  }
}

// The same two Gram-Schmidt passes and the normalisation (k_dots, k_update
// twice, then k_finish) in one block of 1024 threads, for a small basis:
// w stays in LDS, wave g forms the dots of columns g, g + 16, ... (lanes
// down the rows, fixed butterfly), and thread t updates rows t, t + 1024, ...
// over the columns in order.  One launch per step instead of five.
// The first pass's dots also copy the first ncache columns of V into LDS
// (as many as fit beside w), so the update and the second pass read those
// from LDS: each such column leaves memory once per step instead of four
// times.  The copies are exact, so the sums are unchanged.
constexpr int kOrthThreads = 1024;
constexpr int kOrthMaxL = 4096;           // w and the dots in the default 64 KB of LDS
constexpr int64_t kOrthMaxBasis = 40000;  // (j + 1) l values of V read per pass
constexpr int kOrthLdsMax = 159 * 1024;   // dynamic LDS of one k_orth block (160 KB with red[])
// columns of V that k_orth keeps in LDS for a step with nc columns
__host__ __device__ inline int orth_cache_cols(int64_t l, int nc) {
  const int64_t fixed = (int64_t)sizeof(double) * (l + 2 * (int64_t)nc);
  const int64_t room = (kOrthLdsMax - fixed) / ((int64_t)sizeof(double) * l);
  return (int)(room < 0 ? 0 : (room < nc ? room : nc));
}
inline size_t orth_lds_bytes(int64_t l, int nc) {
  return sizeof(double) * (size_t)(l + 2 * (int64_t)nc + (int64_t)orth_cache_cols(l, nc) * l);
}
__global__ __launch_bounds__(kOrthThreads) void k_orth(double* __restrict__ V, int64_t l, int j,
                                                       const double* __restrict__ w_in,
                                                       double* __restrict__ h1, double* __restrict__ h2,
                                                       double* __restrict__ alpha,
                                                       double* __restrict__ beta,
                                                       const double* __restrict__ qnorm,
                                                       int* __restrict__ ctrl, int write_next) {
  if (ctrl[0]) return;
  // LDS: l values of w, the j + 1 dots of each pass, then columns
  // 0 .. ncache - 1 of V
  extern __shared__ double ws[];
  __shared__ double red[kOrthThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  constexpr int NW = kOrthThreads / 64;
  const int nc = j + 1;
  const int ncache = orth_cache_cols(l, nc);
  double* hs = ws + l;
  double* vs = hs + 2 * nc;
  for (int64_t i = t; i < l; i += kOrthThreads) ws[i] = w_in[i];
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    double* h = pass == 0 ? h1 : h2;
    double* hp = hs + pass * nc;
    for (int c = wv; c < nc; c += NW) {
      // the first pass reads the column from memory (and keeps a copy when
      // it fits); the second reads the copy
      const bool cached = c < ncache;
      const double* vc = (pass == 1 && cached) ? vs + (int64_t)c * l : V + (int64_t)c * l;
      double* keep = (pass == 0 && cached) ? vs + (int64_t)c * l : nullptr;
      // four independent sums (rows i, i + 64, i + 128, i + 192 mod 256),
      // combined in a fixed order
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int64_t i = lane;
      for (; i + 192 < l; i += 256) {
        const double a0 = vc[i], a1 = vc[i + 64], a2 = vc[i + 128], a3 = vc[i + 192];
        if (keep) {
          keep[i] = a0;
          keep[i + 64] = a1;
          keep[i + 128] = a2;
          keep[i + 192] = a3;
        }
        s0 = fma(a0, ws[i], s0);
        s1 = fma(a1, ws[i + 64], s1);
        s2 = fma(a2, ws[i + 128], s2);
        s3 = fma(a3, ws[i + 192], s3);
      }
      for (; i < l; i += 64) {
        const double a0 = vc[i];
        if (keep) keep[i] = a0;
        s0 = fma(a0, ws[i], s0);
      }
      double s = (s0 + s1) + (s2 + s3);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) {
        hp[c] = s;
        h[c] = s;
      }
    }
    __syncthreads();
    for (int64_t i = t; i < l; i += kOrthThreads) {
      // four independent sums over the columns (c mod 4), combined in order;
      // whole groups of four held in LDS are read there, the rest from
      // memory (the same values)
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int c = 0;
      for (; c + 3 < nc && c + 3 < ncache; c += 4) {
        s0 = fma(vs[(int64_t)c * l + i], hp[c], s0);
        s1 = fma(vs[(int64_t)(c + 1) * l + i], hp[c + 1], s1);
        s2 = fma(vs[(int64_t)(c + 2) * l + i], hp[c + 2], s2);
        s3 = fma(vs[(int64_t)(c + 3) * l + i], hp[c + 3], s3);
      }
      for (; c + 3 < nc; c += 4) {
        s0 = fma(V[(int64_t)c * l + i], hp[c], s0);
        s1 = fma(V[(int64_t)(c + 1) * l + i], hp[c + 1], s1);
        s2 = fma(V[(int64_t)(c + 2) * l + i], hp[c + 2], s2);
        s3 = fma(V[(int64_t)(c + 3) * l + i], hp[c + 3], s3);
      }
      for (; c < nc; ++c) s0 = fma(c < ncache ? vs[(int64_t)c * l + i] : V[(int64_t)c * l + i], hp[c], s0);
      ws[i] -= (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
  }
  double s = 0.0;
  for (int64_t i = t; i < l; i += kOrthThreads) s = fma(ws[i], ws[i], s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) red[wv] = s;
  __syncthreads();
  double tot = 0.0;
#pragma unroll
  for (int g = 0; g < NW; ++g) tot += red[g];
  const double nrm = sqrt(tot);
  const bool breakdown = !(nrm > 1e-12 * qnorm[0]);
  if (t == 0) {
    alpha[j] = hs[j] + hs[nc + j];  // first- and second-pass dots with v_j
    beta[j] = breakdown ? 0.0 : nrm;
  }
  if (breakdown) {
    if (t == 0) {
      ctrl[0] = 1;
      ctrl[1] = j;
    }
    return;
  }
  if (write_next) {
    const double inv = 1.0 / nrm;
    double* vn = V + (int64_t)(j + 1) * l;
    for (int64_t i = t; i < l; i += kOrthThreads) vn[i] = ws[i] * inv;
  }
}

// normalise w into column col (start vector or restart); ok[0] = success
__global__ __launch_bounds__(1024) void k_set_column(double* __restrict__ V, int64_t l, int col,
                                                     const double* __restrict__ w, double min_norm,
                                                     int* __restrict__ ok) {
  __shared__ double sh[1024];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < l; i += 1024) s = fma(w[i], w[i], s);
  sh[t] = s;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if (t < st) sh[t] += sh[t + st];
    __syncthreads();
  }
  const double nrm = sqrt(sh[0]);
  const bool good = nrm > min_norm;
  if (t == 0) ok[0] = good ? 1 : 0;
  if (!good) return;
  const double inv = 1.0 / nrm;
  for (int64_t i = t; i < l; i += 1024) V[(int64_t)col * l + i] = w[i] * inv;
}

// ------------------------------------------------ tridiagonal Ritz solver
// T (k x k) has diagonal alpha[0..k) and off-diagonal beta[0..k-1).
// Computes its r largest eigenvalues by bisection on Sturm counts
// (multisection over the 256 threads) and their eigenvectors by inverse
// iteration with partial pivoting, orthogonalising within clusters.
// Output: theta[t], bound[t] = |beta[k-1] * s_{k-1,t}| (Lanczos residual
// norm of Ritz pair t), S[t*ldS + i], and kout[0] = k.  With report given,
// it also receives the 16 control words (word 6 = k) and, as double 8, qn[0],
// so that one copy brings the host everything a convergence check needs.
// A second block (grid of 2) solves the leading (k - d_probe) x (k - d_probe)
// matrix, i.e. the Ritz pairs d_probe steps earlier, into theta2/bound2
// (S2, gwork2 its own work space): with both the host can estimate how fast
// the residual bounds fall.

constexpr int kTriThreads = 256;  // multisection points of the bisection
__global__ __launch_bounds__(kTriThreads) void k_tridiag(const double* __restrict__ alpha,
                                                 const double* __restrict__ beta,
                                                 const int* __restrict__ ctrl, int k_host, int r,
                                                 double* __restrict__ theta_out,
                                                 double* __restrict__ bound_out,
                                                 double* __restrict__ S, int ldS,
                                                 double* __restrict__ gwork, int* __restrict__ kout,
                                                 int work_in_lds, double* __restrict__ report,
                                                 const double* __restrict__ qn, int d_probe,
                                                 double* __restrict__ theta2,
                                                 double* __restrict__ bound2,
                                                 double* __restrict__ S2,
                                                 double* __restrict__ gwork2) {
  extern __shared__ double sm[];
  __shared__ double theta[MDS_MAX_R];
  const int t = threadIdx.x;
  const bool probe = blockIdx.x == 1;
  const int kfull = ctrl[0] ? ctrl[1] + 1 : k_host;
  const int k = probe ? kfull - d_probe : kfull;
  if (k < 1) return;  // (probe only: the host ignores its output then)
  if (probe) {
    theta_out = theta2;
    bound_out = bound2;
    S = S2;
    gwork = gwork2;
  }
  const int nr = min(r, k);
  double* al = sm;
  double* be = sm + k;
  for (int i = t; i < k; i += kTriThreads) {
    al[i] = alpha[i];
    be[i] = beta[i];
  }
  __syncthreads();
  double* be2 = sm + 2 * k;
  // with work_in_lds, the work arrays ([4][k][nr]) and the vectors (nr x k)
  // live in LDS, and the vectors are copied out at the end
  double* wk = work_in_lds ? (sm + 3 * k) : gwork;
  double* Z = work_in_lds ? (wk + (int64_t)4 * k * nr) : S;
  const int ldz = work_in_lds ? k : ldS;
  tridiag_top<kTriThreads>(al, be, k, nr, theta, Z, ldz, wk, be2);
  if (t < nr) {
    const double coupling = fabs(be[k - 1 < 0 ? 0 : k - 1]);
    theta_out[t] = theta[t];
    bound_out[t] = coupling * fabs(Z[(int64_t)t * ldz + (k - 1)]);
  }
  if (work_in_lds)
    for (int e = t; e < k * nr; e += kTriThreads) {
      const int tt = e / k, i = e - tt * k;
      S[(int64_t)tt * ldS + i] = Z[e];
    }
  if (probe) return;
  if (t == 0) kout[0] = k;
  if (report) {
    if (t < 16) reinterpret_cast<int*>(report)[t] = (t == 6) ? k : ctrl[t];
    if (t == 16) report[8] = qn[0];
  }
}

// Ritz vectors V_r[i][t] = sum_c Vk[c][i] S[t][c]   (output row-major l x r)
__global__ __launch_bounds__(256) void k_ritz(const double* __restrict__ Vk, int64_t l, int k,
                                              const double* __restrict__ S, int ldS, int r,
                                              double* __restrict__ Vr) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int tt = blockIdx.y;
  if (i >= l) return;
  const double* s = S + (int64_t)tt * ldS;
  double acc = 0.0;
  for (int c = 0; c < k; ++c) acc = fma(Vk[(int64_t)c * l + i], s[c], acc);
  Vr[i * r + tt] = acc;
}

// Sign convention (largest-|.| entry positive, smallest index on ties),
// then X1 = V Lambda^{1/2} and W = 1/2 V Lambda^{-1/2} for live columns.
__global__ __launch_bounds__(256) void k_finalize_cols(double* __restrict__ Vr, int64_t l, int r,
                                                       const double* __restrict__ lam,
                                                       double* __restrict__ X1,
                                                       double* __restrict__ W64, int ldw,
                                                       float* __restrict__ W32t, int64_t l_pad) {
  __shared__ double shv[256];
  __shared__ int64_t shi[256];
  const int tt = blockIdx.x;
  const int t = threadIdx.x;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = t; i < l; i += 256) {
    const double a = fabs(Vr[i * r + tt]);
    if (a > best || (a == best && i < bi)) {
      best = a;
      bi = i;
    }
  }
  shv[t] = best;
  shi[t] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      const double a = shv[t + s];
      const int64_t ai = shi[t + s];
      if (a > shv[t] || (a == shv[t] && ai < shi[t])) {
        shv[t] = a;
        shi[t] = ai;
      }
    }
    __syncthreads();
  }
  const double sgn = (Vr[shi[0] * r + tt] < 0.0) ? -1.0 : 1.0;
  // live direction: the same FP64 comparison the host makes for r_eff
  const bool on = lam[tt] > MDS_TAU * lam[0];
  const double lt = lam[tt];
  const double sx = on ? sqrt(lt) : 0.0;
  const double sw = on ? 0.5 / sqrt(lt) : 0.0;
  for (int64_t i = t; i < l; i += 256) {
    const double v = sgn * Vr[i * r + tt];
    Vr[i * r + tt] = v;
    X1[i * r + tt] = on ? v * sx : 0.0;
    const double wv = on ? v * sw : 0.0;
    W64[i * ldw + tt] = wv;
    W32t[(int64_t)tt * l_pad + i] = (float)wv;
  }
}

// c = q - |m|^2 per landmark (zero for padding rows), FP64 and FP32; also
// the largest |m| of each landmark row.  One wave per row, fixed order.
__global__ __launch_bounds__(256) void k_bias(const double* __restrict__ M, int64_t ldm, int64_t l,
                                              int64_t l_pad, int64_t p,
                                              const double* __restrict__ q,
                                              double* __restrict__ c64, float* __restrict__ c32,
                                              double* __restrict__ rowmax) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= l_pad) return;
  double nn = 0.0, mx = 0.0;
  if (i < l)
    for (int64_t k = lane; k < p; k += 64) {
      const double x = M[i * ldm + k];
      nn = fma(x, x, nn);
      mx = fmax(mx, fabs(x));
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    nn += __shfl_xor(nn, off, 64);
    mx = fmax(mx, __shfl_xor(mx, off, 64));
  }
  if (lane == 0) {
    const double v = (i < l) ? q[i] - nn : 0.0;
    if (i < l) rowmax[i] = mx;
    c64[i] = v;
    c32[i] = (float)v;
  }
}

// q as FP64 and FP32 (zero for padding landmarks), for embedding from
// dissimilarities
// Affine form of eq. (2) for Euclidean input: y = A x + b with
// A[k][i] = 2 sum_j W[j][k] M[j][i] and b[k] = sum_j W[j][k] c[j] (the
// |x|^2 term drops out because the columns of V sum to zero).  Column i == p
// of the grid computes b.  Block (column block, landmark chunk z): its four
// waves take the landmarks j = w (mod 4) of chunk z, each lane one column i
// and 16 outputs k at a time; the wave partials are added in order and the
// chunk partials are summed in order by k_affine_sum.
__global__ __launch_bounds__(256) void k_affine_map(const double* __restrict__ M, int64_t ldm,
                                                    int64_t l, int64_t p,
                                                    const double* __restrict__ W, int ldw,
                                                    const double* __restrict__ c, int r,
                                                    double* __restrict__ part) {
  __shared__ double ws[4][16][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int64_t nz = gridDim.y;
  const int64_t per = (l + nz - 1) / nz;
  const int64_t j0 = blockIdx.y * per, j1 = (j0 + per < l) ? j0 + per : l;
  for (int k0 = 0; k0 < r; k0 += 16) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    if (i <= p) {
      for (int64_t j = j0 + g; j < j1; j += 4) {
        const double mv = (i < p) ? M[j * ldm + i] : c[j];
        const double* wr = W + j * ldw + k0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (k0 + u < r) acc[u] = fma(wr[u], mv, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) ws[g][u][lane] = acc[u];
    __syncthreads();
    if (g == 0 && i <= p) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (k0 + u >= r) break;
        const double s = ((ws[0][u][lane] + ws[1][u][lane]) + ws[2][u][lane]) + ws[3][u][lane];
        part[((int64_t)blockIdx.y * r + k0 + u) * (p + 1) + i] = s;
      }
    }
    __syncthreads();
  }
}

// A = 2 x (sum of the chunk partials of columns i < p), b = sum for i == p
__global__ void k_affine_sum(const double* __restrict__ part, int nz, int64_t p, int r,
                             double* __restrict__ A64, float* __restrict__ A32,
                             double* __restrict__ b64, float* __restrict__ b32) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * (p + 1)) return;
  const int64_t k = e / (p + 1), i = e % (p + 1);
  const int64_t zs = (int64_t)r * (p + 1);
  const double* pp = part + k * (p + 1) + i;
  double s = 0.0;
  int z = 0;
  for (; z + 8 <= nz; z += 8) {  // eight loads in flight, added in order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = pp[(z + u) * zs];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; z < nz; ++z) s += pp[z * zs];
  if (i < p) {
    A64[k * p + i] = 2.0 * s;
    A32[k * p + i] = (float)(2.0 * s);
  } else {
    b64[k] = s;
    b32[k] = (float)s;
  }
}

__global__ void k_copy_q(const double* __restrict__ q, int64_t l, int64_t l_pad,
                         double* __restrict__ q64, float* __restrict__ q32) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= l_pad) return;
  const double v = (i < l) ? q[i] : 0.0;
  q64[i] = v;
  q32[i] = (float)v;
}

// The host needs four small words after the fit: the two lo-part flags of
// the split packs and the FP16 split scales.  They are gathered next to the
// control words, so the fit ends with one small copy to the host.
__global__ void k_stage_words(const int* __restrict__ lo_flags, const float* __restrict__ scales,
                              int* __restrict__ stage) {
  if (threadIdx.x == 0) {
    stage[0] = lo_flags[0];
    stage[1] = lo_flags[1];
    stage[2] = __float_as_int(scales[0]);
    stage[3] = __float_as_int(scales[1]);
  }
}

// FP16 split scale: 2^s with the largest landmark magnitude at 2^12, so data
// up to 16x larger than every landmark stays below the FP16 maximum.
__global__ __launch_bounds__(256) void k_scale(const double* __restrict__ rowmax, int64_t l,
                                               float* __restrict__ scales) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < l; i += 256) m = fmax(m, rowmax[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s2]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int e2 = 0;
    if (sh[0] > 0.0) (void)frexp(sh[0], &e2);
    const int sexp = 12 - e2;
    scales[0] = ldexpf(1.0f, sexp);
    scales[1] = ldexpf(1.0f, -2 * sexp);
  }
}

// Operand packs of the embed kernels (see embed.hip for the layout):
// FP32: row i, chunk ch -> 32 floats; split modes: 32 hi then 32 lo.
// Chunk-major split packs (sbf, sh): plane P (hi, lo), chunk ch, landmark i
// -> 64 bytes at ((P nch + ch) l_split + i) * 64, whose 16-byte segment g
// (values 8 g .. 8 g + 7 of the chunk) sits at position g ^ ((i >> 2) & 3),
// the order in which the kernels keep a landmark row in LDS.
__global__ void k_pack32(const double* __restrict__ M, int64_t ldm, int64_t l_pad, int64_t p,
                         int nch, float* __restrict__ m32, uint16_t* __restrict__ mbf,
                         uint16_t* __restrict__ mh, uint16_t* __restrict__ sbf,
                         uint16_t* __restrict__ sh, int64_t l_split, const float* __restrict__ scales,
                         int* __restrict__ lo_flags) {
  const float prescale = scales[0];
  const int64_t total = l_pad * (int64_t)nch * 32;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / ((int64_t)nch * 32);
    const int64_t rem = e - row * ((int64_t)nch * 32);
    const int ch = (int)(rem >> 5), kk = (int)(rem & 31);
    const int64_t k = (int64_t)ch * 32 + kk;
    const float x = (k < p) ? (float)M[row * ldm + k] : 0.0f;
    // FP32 pack: the 16-value k-block holding value p - 1 (p not a multiple
    // of 16) is transposed, value 4 a + b at position 4 b + a, so that each
    // group of four MFMA inputs holds consecutive values and the embed can
    // skip those past p
    const int kb0 = ch * 32 + (kk & 16);
    const int kin = kk & 15;
    const int kdst = (p - kb0 < 16) ? ((kin & 3) * 4 + (kin >> 2)) : kin;
    m32[e - kin + kdst] = x;
    const __bf16 bh = (__bf16)x;
    const __bf16 bl = (__bf16)(x - (float)bh);
    const int64_t base = (row * nch + ch) * 64;
    mbf[base + kk] = __builtin_bit_cast(uint16_t, bh);
    mbf[base + 32 + kk] = __builtin_bit_cast(uint16_t, bl);
    const float xs = x * prescale;
    const _Float16 hh = (_Float16)xs;
    const _Float16 hl = (_Float16)(xs - (float)hh);
    mh[base + kk] = __builtin_bit_cast(uint16_t, hh);
    mh[base + 32 + kk] = __builtin_bit_cast(uint16_t, hl);
    const int64_t plane = (int64_t)nch * l_split * 32;
    const int64_t soff = ((int64_t)ch * l_split + row) * 32 + (((kk >> 3) ^ ((row >> 2) & 3)) << 3) + (kk & 7);
    sbf[soff] = __builtin_bit_cast(uint16_t, bh);
    sbf[plane + soff] = __builtin_bit_cast(uint16_t, bl);
    sh[soff] = __builtin_bit_cast(uint16_t, hh);
    sh[plane + soff] = __builtin_bit_cast(uint16_t, hl);
    if ((float)bl != 0.0f) lo_flags[0] = 1;
    if ((float)hl != 0.0f) lo_flags[1] = 1;
  }
}

// The fit's scratch: one block from the library's device-block cache (so
// repeated fits of one shape reuse it without an allocation), handed back
// when the fit returns, once the stream has drained.
struct Scratch {
  int dev = 0;
  size_t bytes = 0;
  void* p = nullptr;
  hipStream_t st = nullptr;
  ~Scratch() {
    if (!p) return;
    (void)hipStreamSynchronize(st);
    model_release(dev, bytes, p);
  }
};

}  // namespace

#define LAUNCH_CHECK(what)                                    \
  do {                                                        \
    hipError_t _e = hipGetLastError();                        \
    if (_e != hipSuccess) return hip_fail(_e, what);          \
  } while (0)

namespace {

constexpr size_t kTriLdsMax = 144 * 1024;  // beside about 13 KB of static LDS

// Ritz solve of the k x k tridiagonal matrix; its work arrays live in LDS
// when they fit.
hipError_t launch_tridiag(const double* alpha, const double* beta, const int* ctrl, int k_host,
                          int r, double* theta, double* bound, double* S, int ldS, double* gwork,
                          int* kout, hipStream_t st, double* report = nullptr,
                          const double* qn = nullptr, int d_probe = 0, double* theta2 = nullptr,
                          double* bound2 = nullptr, double* S2 = nullptr, double* gwork2 = nullptr) {
  {
    hipError_t e = lds_limit_once(reinterpret_cast<const void*>(&k_tridiag), (int)kTriLdsMax);
    if (e != hipSuccess) return e;
  }
  const int nr = std::min(r, k_host);
  const size_t base = sizeof(double) * 3 * (size_t)k_host;
  const size_t work = sizeof(double) * 5 * (size_t)k_host * nr;  // work arrays and vectors
  const int in_lds = (base + work <= kTriLdsMax) ? 1 : 0;
  const unsigned grid = (d_probe > 0) ? 2u : 1u;
  k_tridiag<<<grid, kTriThreads, base + (in_lds ? work : 0), st>>>(alpha, beta, ctrl, k_host, r, theta, bound, S,
                                                          ldS, gwork, kout, in_lds, report, qn, d_probe,
                                                          theta2, bound2, S2, gwork2);
  return hipGetLastError();
}

struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  }
};

}  // namespace

mds_status fit_on_device(Model& m, const void* X, int dt, int64_t ldx, const int64_t* idx_dev,
                         const double* D1, int64_t ldd, hipStream_t st) {
  const bool vectors = (D1 == nullptr);
  const int64_t l = m.l, p = m.p, l_pad = m.l_pad;
  const int r = m.r;
  const int nch64 = (int)((p + 15) / 16);
  const int nch32 = (int)((p + 31) / 32);
  const int64_t ldm = (int64_t)nch64 * 16;
  const int ldw = 16 * m.rb;
  const int kcap = (int)l;  // Krylov space can grow to the full dimension

  // ---- model buffers: one allocation ----
  Layout lay;
  const size_t o64 = lay.take(sizeof(double) * l_pad * ldm);
  // FP32 and split packs: rows up to a multiple of kSplitPackRows (zero past
  // l_pad) for the variant of the embed that walks 512 landmarks at a time
  const int64_t l_split = round_up(l_pad, kSplitPackRows);
  const size_t o32 = lay.take(sizeof(float) * l_split * nch32 * 32);
  const size_t obf = lay.take(sizeof(uint16_t) * l_split * nch32 * 64);
  const size_t oh = lay.take(sizeof(uint16_t) * l_split * nch32 * 64);
  // the same parts chunk-major for the 32 x 32 split kernels: a hi plane
  // then a lo plane, each nch32 x l_split x 32 values
  const size_t osbf = lay.take(sizeof(uint16_t) * l_split * nch32 * 64);
  const size_t osh = lay.take(sizeof(uint16_t) * l_split * nch32 * 64);
  const size_t ow32 = lay.take(sizeof(float) * l_pad * ldw);
  const size_t ow64 = lay.take(sizeof(double) * l_pad * ldw);
  const size_t oc32 = lay.take(sizeof(float) * l_pad);
  const size_t oc64 = lay.take(sizeof(double) * l_pad);
  const size_t oq32 = lay.take(sizeof(float) * l_pad);
  const size_t oq64 = lay.take(sizeof(double) * l_pad);
  const size_t ox1 = lay.take(sizeof(double) * (size_t)l * r);
  const size_t oa64 = lay.take(sizeof(double) * (size_t)r * p);
  const size_t oa32 = lay.take(sizeof(float) * (size_t)r * p);
  const size_t ob64 = lay.take(sizeof(double) * (size_t)r);
  const size_t ob32 = lay.take(sizeof(float) * (size_t)r);
  m.base = model_alloc(m.dev, lay.off);
  if (!m.base) return set_error(MDS_ERR_OOM, "device allocation of the model failed");
  char* b = static_cast<char*>(m.base);
  m.m64 = b + o64;
  m.m32 = b + o32;
  m.mbf = b + obf;
  m.mh = b + oh;
  m.sbf = b + osbf;
  m.sh = b + osh;
  m.l_split = l_split;
  m.w32 = b + ow32;
  m.w64 = b + ow64;
  m.c32 = b + oc32;
  m.c64 = b + oc64;
  m.q32 = b + oq32;
  m.q64 = b + oq64;
  m.x1_64 = b + ox1;
  m.aff64 = b + oa64;
  m.aff32 = b + oa32;
  m.affb64 = b + ob64;
  m.affb32 = b + ob32;
  m.bytes = (int64_t)lay.off;
  MDS_HIP(hipMemsetAsync(m.base, 0, lay.off, st));

  // ---- scratch (stream-ordered, freed when the fit returns) ----
  // affine-map partials: landmark chunks (each wave walks a few landmarks,
  // so the loop is not a chain of memory latencies), up to 64, within 64 MB
  const int64_t aff_cols = (int64_t)r * (p + 1);
  const int aff_nz = (int)std::max<int64_t>(1, std::min<int64_t>({64, (l + 15) / 16,
                                                                   (int64_t)(8 << 20) / aff_cols}));
  Layout sl;
  const size_t sDQ = sl.take(sizeof(double) * l * l);
  const size_t sV = sl.take(sizeof(double) * l * (kcap + 1));
  const size_t ssmall = sl.take(sizeof(double) * ((size_t)l * 7 + 64));
  const size_t sS = sl.take(sizeof(double) * (size_t)(kcap + 1) * (2 * r + 1));
  const size_t swork = sl.take(sizeof(double) * (size_t)(kcap + 1) * 4 * (2 * r + 1));
  const size_t sVr = sl.take(sizeof(double) * l * r);
  const size_t sab = sl.take(sizeof(double) * ((size_t)2 * (kcap + 1) + 6 * MDS_MAX_R + 32));
  const size_t saff = sl.take(vectors ? sizeof(double) * (size_t)aff_nz * aff_cols : 0);
  Scratch scr;
  scr.dev = m.dev;
  scr.bytes = sl.off;
  scr.st = st;
  scr.p = model_alloc(m.dev, sl.off);
  if (!scr.p) return set_error(MDS_ERR_OOM, "device allocation of the fit scratch failed");
  char* sb = static_cast<char*>(scr.p);
  struct {
    void* p;
  } bDQ{sb + sDQ}, bV{sb + sV}, bsmall{sb + ssmall}, bS{sb + sS}, bwork{sb + swork}, bVr{sb + sVr},
      bab{sb + sab}, baff{sb + saff};
  double* DQ = (double*)bDQ.p;
  double* Vk = (double*)bV.p;
  double* d1 = (double*)bsmall.p;
  double* q = d1 + l;
  double* rowsq = q + l;
  double* w = rowsq + l;
  double* h1 = w + l;
  double* h2 = h1 + l;
  double* rowmax = h2 + l;
  double* scal = rowmax + l;  // [0] dbar, [1] |Q|_F, [2..3] FP16 scales (as floats)
  float* scales = reinterpret_cast<float*>(scal + 2);
  // ctrl: [0] stop, [1] stop step, [2] ok, [3] bad input, [4] asymmetric
  // input, [6] k of the last tridiagonal solve, [7] always 0 (no-stop view),
  // [8] k of the newest-run solve, [10..11] lo flags of the split packs,
  // [16..19] the words read back at the end (lo flags, FP16 scales)
  int* ctrl = reinterpret_cast<int*>(scal + 8);
  double* alpha = (double*)bab.p;
  double* beta = alpha + (kcap + 1);
  // check report: 16 control words (8 doubles), qn, then theta and bound,
  // read back with one copy
  double* report = beta + (kcap + 1);
  double* theta = report + 16;
  double* bound = theta + 2 * MDS_MAX_R;
  double* theta2 = bound + 2 * MDS_MAX_R;  // the probe's pairs (d_probe steps earlier)
  double* bound2 = theta2 + MDS_MAX_R;
  const size_t report_doubles = 16 + 6 * MDS_MAX_R;
  MDS_HIP(hipMemsetAsync(ctrl, 0, sizeof(int) * 16, st));
  MDS_HIP(hipMemsetAsync(beta, 0, sizeof(double) * (kcap + 1), st));

  // ---- gather, distances (or the caller's matrix), centring ----
  if (!vectors) {
    const int grid = (int)std::min<int64_t>((l * l + 255) / 256, 8192);
    k_load_sqdist<<<grid, 256, 0, st>>>(D1, ldd, l, DQ, ctrl + 3);
    LAUNCH_CHECK("load dissimilarities");
  } else {
    const int64_t total = l * p;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    if (dt == MDS_F32)
      k_gather<float><<<grid, 256, 0, st>>>((const float*)X, ldx, idx_dev, l, p, ldm, (double*)m.m64,
                                            ctrl + 3);
    else
      k_gather<double><<<grid, 256, 0, st>>>((const double*)X, ldx, idx_dev, l, p, ldm,
                                             (double*)m.m64, ctrl + 3);
    LAUNCH_CHECK("gather");
    const int64_t sq_tiles = (l + 63) / 64;
    k_sqdist<<<(unsigned)(sq_tiles * (sq_tiles + 1) / 2), 256, 0, st>>>((const double*)m.m64, ldm, l, p, DQ);
    LAUNCH_CHECK("sqdist");
  }
  k_rowmean<<<(unsigned)l, 256, 0, st>>>(DQ, l, d1);
  k_mean<<<1, 256, 0, st>>>(d1, l, scal);
  k_centre<<<(unsigned)l, 256, 0, st>>>(DQ, l, d1, scal, q, rowsq);
  k_sqrt_sum<<<1, 256, 0, st>>>(rowsq, l, scal + 1);
  LAUNCH_CHECK("centring");
  // The input flags and |Q1|_F are read with the first convergence check
  // (no host round trip here); on bad input the first batch of Lanczos
  // steps runs on meaningless values and is discarded.
  int hctrl[16];
  std::vector<double> hrep(report_doubles);

  // ---- Lanczos with full reorthogonalisation ----
  const int upd_blocks = (int)((l + 63) / 64);
  const int fill_blocks = (int)((l + 255) / 256);
  MDS_HIP(lds_limit_once(reinterpret_cast<const void*>(&k_orth), kOrthLdsMax));  // up to all of a CU's LDS
  k_fill_random<<<fill_blocks, 256, 0, st>>>(w, l, 0x5EEDull);
  k_set_column<<<1, 1024, 0, st>>>(Vk, l, 0, w, 0.0, ctrl + 2);
  LAUNCH_CHECK("lanczos start");
  const double conv_tol = 1e-13;
  int j = 0;            // next step to run; column j holds v_j
  int block_start = 0;  // first column of the current Lanczos run
  int restarts = 0;
  std::vector<double> htheta(r), hbound(r);
  int k_final = 0;
  // Steps until the next convergence check: grown from the observed decay
  // rate of the slowest residual bound (a check costs a host round trip).
  int batch = std::max(8, 2 * r + 4);
  int prev_j = -1;
  double prev_worst = 0.0;
  for (;;) {
    const int jend = std::min(kcap, j + batch);
    for (; j < jend; ++j) {
      const size_t shm = sizeof(double) * (size_t)(j + 1);
      if (l <= kSymvRowsMaxL)
        k_symv_rows<<<(unsigned)((l + 3) / 4), 256, sizeof(double) * (size_t)l, st>>>(DQ, l, Vk + (int64_t)j * l,
                                                                                    w, ctrl);
      else
        k_symv<<<(unsigned)l, 256, 0, st>>>(DQ, l, Vk + (int64_t)j * l, w, ctrl);
      if (l <= kOrthMaxL && (int64_t)(j + 1) * l <= kOrthMaxBasis) {
        k_orth<<<1, kOrthThreads, orth_lds_bytes(l, j + 1), st>>>(
            Vk, l, j, w, h1, h2, alpha, beta, scal + 1, ctrl, (j + 1 < kcap) ? 1 : 0);
        continue;
      }
      k_dots<<<j + 1, 256, 0, st>>>(Vk, l, w, h1, ctrl);
      k_update<<<upd_blocks, 256, shm, st>>>(Vk, l, j + 1, h1, w, ctrl);
      k_dots<<<j + 1, 256, 0, st>>>(Vk, l, w, h2, ctrl);
      k_update<<<upd_blocks, 256, shm, st>>>(Vk, l, j + 1, h2, w, ctrl);
      k_finish<<<1, 1024, 0, st>>>(Vk, l, j, w, h1, h2, alpha, beta, scal + 1, ctrl,
                                   (j + 1 < kcap) ? 1 : 0);
    }
    LAUNCH_CHECK("lanczos steps");
    // the probe solves the Krylov matrix d_probe steps back (same run only)
    const int d_probe = (j - block_start >= r + 4) ? std::max(4, (j - block_start) / 4) : 0;
    MDS_HIP(launch_tridiag(alpha, beta, ctrl, j, r, theta, bound, (double*)bS.p, kcap + 1,
                           (double*)bwork.p, ctrl + 6, st, report, scal + 1, d_probe, theta2, bound2,
                           (double*)bS.p + (size_t)(kcap + 1) * (r + 1),
                           (double*)bwork.p + (size_t)(kcap + 1) * 4 * (r + 1)));
    MDS_HIP(hipMemcpyAsync(hrep.data(), report, sizeof(double) * report_doubles,
                           hipMemcpyDeviceToHost, st));
    MDS_HIP(hipStreamSynchronize(st));
    std::memcpy(hctrl, hrep.data(), sizeof(hctrl));
    if (hctrl[3])
      return set_error(MDS_ERR_INVALID_ARG, vectors ? "non-finite value in a landmark row"
                                                    : "non-finite squared dissimilarity");
    if (!vectors && hctrl[4]) return set_error(MDS_ERR_INVALID_ARG, "dissimilarity matrix is not symmetric");
    if (!(hrep[8] > 0.0)) return set_error(MDS_ERR_DEGENERATE, "all landmarks coincide (Q1 = 0)");
    for (int t = 0; t < r; ++t) {
      htheta[t] = hrep[16 + t];
      hbound[t] = hrep[16 + 2 * MDS_MAX_R + t];
    }
    // the probe's worst bound, when it saw the same run without a stop
    double probe_worst = -1.0;
    if (d_probe > 0 && hctrl[0] == 0 && j - d_probe >= r) {
      probe_worst = 0.0;
      for (int t = 0; t < r; ++t)
        probe_worst = std::max(probe_worst, hrep[16 + 5 * MDS_MAX_R + t] / fabs(hrep[16 + 4 * MDS_MAX_R]));
    }
    const int k = hctrl[6];
    const bool stopped = hctrl[0] != 0;
    bool conv = k >= r;
    for (int t = 0; conv && t < r; ++t)
      if (!(hbound[t] <= conv_tol * fabs(htheta[0]))) conv = false;
    if (conv && block_start == 0 && stopped) {
      // A run that ends in an invariant subspace shows one copy of each
      // distinct eigenvalue it touched: look at the complement before
      // trusting the top r.
      conv = false;
    } else if (conv && block_start > 0) {
      // The newest run started in the complement of everything found
      // before it; once its largest Ritz value mu has converged, mu is the
      // largest eigenvalue left there.  Stop only if mu does not exceed
      // theta_r; otherwise further copies may hide in the complement.
      MDS_HIP(launch_tridiag(alpha + block_start, beta + block_start, ctrl + 7, k - block_start, 1,
                             theta + r, bound + r, (double*)bS.p + (size_t)(kcap + 1) * r, kcap + 1,
                             (double*)bwork.p + (size_t)(kcap + 1) * 4 * r, ctrl + 8, st));
      double hmu[2];
      MDS_HIP(hipMemcpyAsync(&hmu[0], theta + r, sizeof(double), hipMemcpyDeviceToHost, st));
      MDS_HIP(hipMemcpyAsync(&hmu[1], bound + r, sizeof(double), hipMemcpyDeviceToHost, st));
      MDS_HIP(hipStreamSynchronize(st));
      const double slack = 1e-12 * fabs(htheta[0]);
      conv = hmu[1] <= conv_tol * fabs(htheta[0]) && hmu[0] <= htheta[r - 1] + slack;
    }
    if (conv || k >= kcap) {
      k_final = k;
      break;
    }
    {
      double worst = 0.0;
      for (int t = 0; t < std::min(r, k); ++t) worst = std::max(worst, hbound[t] / fabs(htheta[0]));
      if (probe_worst > 0.0) {  // the rate from the probe d_probe steps back
        prev_j = j - d_probe;
        prev_worst = probe_worst;
      }
      int next = 8;
      if (prev_j >= 0 && worst > 0.0 && prev_worst > worst && j > prev_j) {
        const double rate = (log(prev_worst) - log(worst)) / (double)(j - prev_j);  // per step
        const double need = (log(worst) - log(conv_tol)) / rate;
        // the bounds fall faster as the Ritz values settle, so a long
        // extrapolation overshoots: aim short of it and check again
        next = (int)std::ceil(need > 10.0 ? 0.85 * need : need) + 1;
      } else if (prev_j >= 0) {
        next = std::max(8, j / 4);
      }
      batch = std::min(std::max(next, 4), std::max(8, j));
      prev_j = j;
      prev_worst = worst;
    }
    if (stopped) {
      // Invariant subspace: continue with a fresh vector orthogonal to it.
      bool ok = false;
      for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
        MDS_HIP(hipMemsetAsync(ctrl, 0, sizeof(int) * 2, st));
        k_fill_random<<<fill_blocks, 256, 0, st>>>(w, l, 0xABCDull + 131ull * (uint64_t)(k + attempt));
        const size_t shm = sizeof(double) * (size_t)k;
        for (int pass = 0; pass < 2; ++pass) {
          k_dots<<<k, 256, 0, st>>>(Vk, l, w, h1, ctrl);
          k_update<<<upd_blocks, 256, shm, st>>>(Vk, l, k, h1, w, ctrl);
        }
        k_set_column<<<1, 1024, 0, st>>>(Vk, l, k, w, 1e-6, ctrl + 2);
        LAUNCH_CHECK("lanczos restart");
        int okflag = 0;
        MDS_HIP(hipMemcpyAsync(&okflag, ctrl + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        MDS_HIP(hipStreamSynchronize(st));
        ok = okflag != 0;
      }
      ++restarts;
      if (!ok) {  // the whole space is spanned: T is exact
        k_final = k;
        break;
      }
      j = k;
      block_start = k;
      prev_j = -1;  // a new run: its residuals start over
      batch = 8;
    } else if (j >= kcap) {
      k_final = k;
      break;
    }
  }
  if (k_final < r) return set_error(MDS_ERR_NOT_CONVERGED, "Krylov space smaller than r");
  m.lanczos_steps = k_final;
  m.restarts = restarts;

  // ---- Ritz vectors, rank decision, finalisation ----
  {
    dim3 grid((unsigned)((l + 255) / 256), (unsigned)r);
    k_ritz<<<grid, 256, 0, st>>>(Vk, l, k_final, (const double*)bS.p, kcap + 1, r, (double*)bVr.p);
    LAUNCH_CHECK("ritz vectors");
  }
  if (!(htheta[0] > 0.0)) return set_error(MDS_ERR_DEGENERATE, "largest eigenvalue is not positive");
  int r_eff = 0;
  for (int t = 0; t < r; ++t) r_eff += htheta[t] > MDS_TAU * htheta[0] ? 1 : 0;
  m.r_eff = r_eff;
  k_finalize_cols<<<r, 256, 0, st>>>((double*)bVr.p, l, r, theta, (double*)m.x1_64, (double*)m.w64,
                                     ldw, (float*)m.w32, l_pad);
  k_copy_q<<<(unsigned)((l_pad + 255) / 256), 256, 0, st>>>(q, l, l_pad, (double*)m.q64,
                                                            (float*)m.q32);
  if (vectors) {
    k_bias<<<(unsigned)((l_pad + 3) / 4), 256, 0, st>>>((const double*)m.m64, ldm, l, l_pad, p, q,
                                                        (double*)m.c64, (float*)m.c32, rowmax);
    k_scale<<<1, 256, 0, st>>>(rowmax, l, scales);
    const int64_t total = l_pad * (int64_t)nch32 * 32;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
    k_pack32<<<grid, 256, 0, st>>>((const double*)m.m64, ldm, l_pad, p, nch32, (float*)m.m32,
                                   (uint16_t*)m.mbf, (uint16_t*)m.mh, (uint16_t*)m.sbf, (uint16_t*)m.sh,
                                   m.l_split, scales, ctrl + 10);
    dim3 agrid((unsigned)((p + 1 + 63) / 64), (unsigned)aff_nz);
    k_affine_map<<<agrid, 256, 0, st>>>((const double*)m.m64, ldm, l, p, (const double*)m.w64, ldw,
                                        (const double*)m.c64, r, (double*)baff.p);
    k_affine_sum<<<(unsigned)((aff_cols + 255) / 256), 256, 0, st>>>(
        (const double*)baff.p, aff_nz, p, r, (double*)m.aff64, (float*)m.aff32, (double*)m.affb64,
        (float*)m.affb32);
  } else {
    k_scale<<<1, 256, 0, st>>>(rowmax, 0, scales);  // unused without vectors
  }
  int* words_dev = ctrl + 16;
  k_stage_words<<<1, 64, 0, st>>>(ctrl + 10, scales, words_dev);
  LAUNCH_CHECK("finalise");
  // ---- host copies ----
  m.lam_host = new double[r];
  for (int t = 0; t < r; ++t) m.lam_host[t] = htheta[t];
  int words[4];
  MDS_HIP(hipMemcpyAsync(words, words_dev, sizeof(words), hipMemcpyDeviceToHost, st));
  MDS_HIP(hipStreamSynchronize(st));
  m.bf_lo_zero = words[0] ? 0 : 1;
  m.h_lo_zero = words[1] ? 0 : 1;
  std::memcpy(&m.h_prescale, &words[2], sizeof(float));
  std::memcpy(&m.h_postscale, &words[3], sizeof(float));
  return MDS_OK;
}

}  // namespace mds
