// Divide-and-conquer MDS (Section 3.2) on the GPU, all in FP64.
//
//   partition   row i gets the key SplitMix64(seed) output i+1; a radix sort
//               orders rows by (key, index).  The first c rows of that order
//               are the connecting points; the rest are cut into consecutive
//               pieces of l - c.  Part j holds the connecting rows followed
//               by its own piece, so all parts have l rows except perhaps
//               the last, and there are ceil(1 + (n - l) / (l - c)) parts.
//   per part    classical MDS (Section 2): the top r eigenpairs of
//               Q_j = -1/2 P Delta_j P and X_j = V Lambda^{1/2}.
//   alignment   every X_j (j >= 1) is mapped onto X_0 by the Procrustes
//               rotation T_j and shift t_j fitted on the connecting rows;
//               its own rows become X_j T_j + t_j and are written to their
//               input positions.
//
// For squared Euclidean distances Q_j = B B' with B the centred rows of the
// part (m x p); B'B (p x p) has the same non-zero eigenvalues, and its unit
// eigenvectors u give the coordinates X_j = B u.  Each part is solved
// through whichever Gram matrix is smaller, by a dense symmetric solver in
// one workgroup: Householder reduction to tridiagonal form (in LDS when the
// matrix fits), the largest eigenpairs of the tridiagonal matrix by
// bisection and inverse iteration, and the back-transformation of those
// vectors.  Every reduction has a fixed order, so a run is reproducible.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mds_internal.h"
#include "tridiag_dev.h"

namespace mds {
namespace {

struct DcShape {
  int64_t n, p, l, c;
  int64_t nparts;
  int64_t m_max;  // rows of a full part
  int r;
};

__host__ __device__ inline int64_t dc_part_size(int64_t j, const DcShape& s) {
  if (s.nparts == 1) return s.n;
  const int64_t lo = s.c + j * (s.l - s.c);
  const int64_t hi = std::min(s.c + (j + 1) * (s.l - s.c), s.n);
  return s.c + (hi - lo);
}

// position in the sorted order of row i of part j
__device__ inline int64_t dc_pos(int64_t j, int64_t i, const DcShape& s) {
  return i < s.c ? i : s.c + j * (s.l - s.c) + (i - s.c);
}

// ------------------------------------------------------------- partition
__global__ void k_dc_keys(int64_t n, uint64_t seed, uint64_t* __restrict__ keys,
                          int64_t* __restrict__ vals) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // SplitMix64: the state after i+1 steps is seed + (i+1) * gamma
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    keys[i] = z ^ (z >> 31);
    vals[i] = i;
  }
}

// ----------------------------------------------------------- part means
// mean[j][k] over the rows of part j: a block takes 64 columns, wave g the
// rows i = g (mod 4) in order, and the four partial sums are added in a
// fixed order; flags non-finite input.
template <typename TX>
__global__ __launch_bounds__(256) void k_dc_mean(const TX* __restrict__ X, int64_t ldx,
                                                 const int64_t* __restrict__ order, DcShape s,
                                                 double* __restrict__ mean, int* __restrict__ bad) {
  __shared__ double part[4][64];
  const int t = threadIdx.x, kk = t & 63, g = t >> 6;
  const int64_t j = blockIdx.x;
  const int64_t k = (int64_t)blockIdx.y * 64 + kk;
  const int64_t m = dc_part_size(j, s);
  double acc = 0.0;
  bool fin = true;
  if (k < s.p) {
#pragma unroll 4
    for (int64_t i = g; i < m; i += 4) {
      const double v = (double)X[order[dc_pos(j, i, s)] * ldx + k];
      fin = fin && isfinite(v);
      acc += v;
    }
  }
  part[g][kk] = acc;
  if (!fin) bad[0] = 1;
  __syncthreads();
  if (g == 0 && k < s.p)
    mean[j * s.p + k] = (((part[0][kk] + part[1][kk]) + part[2][kk]) + part[3][kk]) / (double)m;
}

// -------------------------------------------------------- Gram matrices
// B'B of a part (p x p): G[a][b] = sum_i (x_ia - mu_a)(x_ib - mu_b) over the
// part's rows in order.  64x64 tile per block, 4x4 per thread, rows staged
// 16 at a time.  G[a][b] and G[b][a] are the same sums of the same products,
// so the result is exactly symmetric.
template <typename TX>
__global__ __launch_bounds__(256) void k_dc_gram_feat(const TX* __restrict__ X, int64_t ldx,
                                                      const int64_t* __restrict__ order, DcShape s,
                                                      const double* __restrict__ mean, int64_t j0,
                                                      double* __restrict__ G) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int64_t j = j0 + blockIdx.z;
  const int64_t a0 = (int64_t)blockIdx.y * 64, b0 = (int64_t)blockIdx.x * 64;
  const int64_t m = dc_part_size(j, s);
  const double* mu = mean + j * s.p;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int64_t i0 = 0; i0 < m; i0 += 16) {
    for (int e = t; e < 16 * 64; e += 256) {
      const int ii = e >> 6, cc = e & 63;
      const int64_t i = i0 + ii;
      double va = 0.0, vb = 0.0;
      if (i < m) {
        const TX* row = X + order[dc_pos(j, i, s)] * ldx;
        if (a0 + cc < s.p) va = (double)row[a0 + cc] - mu[a0 + cc];
        if (b0 + cc < s.p) vb = (double)row[b0 + cc] - mu[b0 + cc];
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
  double* Gp = G + (int64_t)blockIdx.z * s.p * s.p;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t a = a0 + ty + 16 * u, b = b0 + tx + 16 * v;
      if (a < s.p && b < s.p) Gp[a * s.p + b] = acc[u][v];
    }
}

// The same B'B for p <= 128 on the FP64 matrix cores, one block per part.
// The part's rows are walked 32 at a time through the partition order:
// thread t owns column t % 128 of rows t / 128, t / 128 + 2, ..., loads the
// next step's values into registers while the matrix cores work on the
// current step, and writes them centred into LDS.  The 16 x 16 output tiles
// on and above the diagonal are shared out over the four waves, each
// accumulating G[a][b] = sum_i x_ia x_ib with v_mfma_f64_16x16x4f64 (lane
// (i, q) holds x[k + q][16 t + i] of both operands); every output is
// written to both symmetric positions, so G is exactly symmetric.
constexpr int DCG_MAXP = 128;
constexpr int DCG_ROWS = 32;
constexpr int DCG_PER_WAVE = ((DCG_MAXP / 16) * (DCG_MAXP / 16 + 1) / 2 + 3) / 4;  // 9
template <typename TX>
__global__ __launch_bounds__(256) void k_dc_gram_mfma(const TX* __restrict__ X, int64_t ldx,
                                                      const int64_t* __restrict__ order, DcShape s,
                                                      const double* __restrict__ mean, int64_t j0,
                                                      double* __restrict__ G) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int NV = DCG_ROWS / 2;  // values a thread carries per step
  __shared__ double xs[DCG_ROWS][DCG_MAXP + 1];
  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);  // the same in every lane of a wave
  const int li = lane & 15, lq = lane >> 4;
  const int64_t p = s.p;
  const int T = (int)((p + 15) / 16);
  const int npairs = T * (T + 1) / 2;
  const int64_t jc = blockIdx.x, j = j0 + jc;
  const int64_t m = dc_part_size(j, s);
  // the wave's tile pairs q = wv + 4 u, unranked row by row (ta <= tb)
  int ta[DCG_PER_WAVE], tb[DCG_PER_WAVE];
#pragma unroll
  for (int u = 0; u < DCG_PER_WAVE; ++u) {
    int q = wv + 4 * u, a = 0;
    ta[u] = -1;
    tb[u] = -1;
    if (q < npairs) {
      while (q >= T - a) {
        q -= T - a;
        ++a;
      }
      ta[u] = a;
      tb[u] = a + q;
    }
  }
  d4 acc[DCG_PER_WAVE];
#pragma unroll
  for (int u = 0; u < DCG_PER_WAVE; ++u) acc[u] = d4{0, 0, 0, 0};
  const int cc = t & (DCG_MAXP - 1), r0 = t / DCG_MAXP;
  const bool colok = cc < p;
  const double mu = colok ? mean[j * p + cc] : 0.0;
  TX v[NV];
  auto fetch = [&](int64_t s0) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int64_t i = s0 + r0 + 2 * u;
      v[u] = (colok && i < m) ? X[order[dc_pos(j, i, s)] * ldx + cc] : TX(0);
    }
  };
  fetch(0);
  for (int64_t s0 = 0; s0 < m; s0 += DCG_ROWS) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int64_t i = s0 + r0 + 2 * u;
      xs[r0 + 2 * u][cc] = (colok && i < m) ? (double)v[u] - mu : 0.0;
    }
    __syncthreads();
    if (s0 + DCG_ROWS < m) fetch(s0 + DCG_ROWS);
#pragma unroll
    for (int k = 0; k < DCG_ROWS; k += 4) {
#pragma unroll
      for (int u = 0; u < DCG_PER_WAVE; ++u) {
        if (ta[u] >= 0) {
          const double av = xs[k + lq][16 * ta[u] + li];
          const double bv = xs[k + lq][16 * tb[u] + li];
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // FP64 result layout: element e of lane (j, g) is row g + 4 e, column j
  double* Gp = G + jc * p * p;
#pragma unroll
  for (int u = 0; u < DCG_PER_WAVE; ++u) {
    if (ta[u] < 0) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t ra = 16 * ta[u] + lq + 4 * e, cb = 16 * tb[u] + li;
      if (ra < p && cb < p) {
        Gp[ra * p + cb] = acc[u][e];
        Gp[cb * p + ra] = acc[u][e];
      }
    }
  }
}

// B B' of a part (m x m, leading dimension m_max): G[i][i'] =
// sum_k (x_ik - mu_k)(x_i'k - mu_k), features staged 16 at a time.
template <typename TX>
__global__ __launch_bounds__(256) void k_dc_gram_rows(const TX* __restrict__ X, int64_t ldx,
                                                      const int64_t* __restrict__ order, DcShape s,
                                                      const double* __restrict__ mean, int64_t j0,
                                                      double* __restrict__ G) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int64_t j = j0 + blockIdx.z;
  const int64_t i0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64;
  const int64_t m = dc_part_size(j, s);
  const int64_t ld = s.m_max;
  if (i0 >= m || k0 >= m) return;
  const double* mu = mean + j * s.p;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int64_t f0 = 0; f0 < s.p; f0 += 16) {
    for (int e = t; e < 16 * 64; e += 256) {
      const int rr = e >> 4, ff = e & 15;
      const int64_t f = f0 + ff;
      double va = 0.0, vb = 0.0;
      if (f < s.p) {
        if (i0 + rr < m) va = (double)X[order[dc_pos(j, i0 + rr, s)] * ldx + f] - mu[f];
        if (k0 + rr < m) vb = (double)X[order[dc_pos(j, k0 + rr, s)] * ldx + f] - mu[f];
      }
      As[ff][rr] = va;
      Bs[ff][rr] = vb;
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
  double* Gp = G + (int64_t)blockIdx.z * ld * ld;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t a = i0 + ty + 16 * u, b = k0 + tx + 16 * v;
      if (a < m && b < m) Gp[a * ld + b] = acc[u][v];
    }
}

// ------------------------------------------------------- dense eigensolver
constexpr int DC_NT = 512;         // threads of the per-part eigensolver block
constexpr int DC_NW = DC_NT / 64;  // its waves

// A22 -= v w' + w v' with w = p - K v over the rows i = wv (mod DC_NW),
// lanes along the row, four rows loaded before any is stored.  Both
// products are rounded before the sum, so A22 stays exactly symmetric.
// Returns this lane's part of the squared norm of row 0 beyond its first two
// entries (the next column below its subdiagonal).
__device__ __forceinline__ double dc_rank2(double* __restrict__ A22, int lda,
                                           const double* __restrict__ vv,
                                           const double* __restrict__ pw, double K, int n2,
                                           int wv, int lane) {
  double ps = 0.0;
  for (int jc0 = 0; jc0 < n2; jc0 += 64) {
    const int jj = jc0 + lane;
    if (jj >= n2) continue;
    const double vj = vv[jj];
    const double wj = fma(-K, vj, pw[jj]);
    for (int i0 = wv; i0 < n2; i0 += 4 * DC_NW) {
      double vi[4], wi[4], av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * DC_NW;
        vi[u] = 0.0;
        wi[u] = 0.0;
        av[u] = 0.0;
        if (i < n2) {
          vi[u] = vv[i];
          wi[u] = fma(-K, vi[u], pw[i]);
          av[u] = A22[(int64_t)i * lda + jj];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * DC_NW;
        if (i < n2) {
          const double nv = av[u] - (__dmul_rn(vi[u], wj) + __dmul_rn(wi[u], vj));
          A22[(int64_t)i * lda + jj] = nv;
          if (i == 0 && jj >= 2) ps = fma(nv, nv, ps);
        }
      }
    }
  }
  return ps;
}

// One block per part.  The symmetric matrix (dd x dd, full storage) is
// reduced to tridiagonal form by Householder reflections H_k = I - tau_k v v'
// (LAPACK's unblocked lower reduction); v_k is kept in row k, which later
// steps no longer read.  The nr largest eigenpairs of the tridiagonal matrix
// are mapped back by z <- H_0 ... H_{dd-3} z.  With IN_LDS the matrix is
// copied to LDS; otherwise it is reduced in place in global memory.
//
// Output per part j: lam[j][t]; for the feature Gram (rows_gram == 0) the
// eigenvectors U[j] (p x r, row-major); for the row Gram the coordinates
// Xs[j][i][t] = v_t[i] sqrt(lam_t) (zero where lam_t <= 0).  status[j] = 1
// when lam_1 <= 0 (all rows of the part coincide).
template <bool IN_LDS>
__global__ __launch_bounds__(DC_NT) void k_dc_eigen(double* __restrict__ G, int d, DcShape s,
                                                  int rows_gram, int64_t j0, int nr,
                                                  double* __restrict__ zg, double* __restrict__ wkg,
                                                  double* __restrict__ partg,
                                                  double* __restrict__ lam, double* __restrict__ U,
                                                  double* __restrict__ Xs, int* __restrict__ status) {
  extern __shared__ double dsm[];
  __shared__ double shw[DC_NW];
  __shared__ double theta[MDS_MAX_R];
  __shared__ double sig_next;
  const int t = threadIdx.x;
  const int64_t jc = blockIdx.x, j = j0 + jc;
  const int dd = rows_gram ? (int)dc_part_size(j, s) : d;
  const int nrr = std::min(nr, dd);
  double* Gp = G + jc * (int64_t)d * d;
  int lda, ldz;
  double *A, *al, *be, *tau, *pw, *Z, *wk;
  if (IN_LDS) {
    lda = dd;
    ldz = dd;
    A = dsm;
    al = A + (int64_t)dd * dd;
    be = al + dd;
    tau = be + dd;
    pw = tau + dd;
    Z = pw + (2 + DC_NW) * dd;  // pw, vv, one partial row per wave
    wk = Z + (int64_t)nr * dd;
    for (int64_t e = t; e < (int64_t)dd * dd; e += DC_NT) A[e] = Gp[(e / dd) * d + (e % dd)];
  } else {
    lda = d;
    ldz = d;
    A = Gp;
    al = dsm;
    be = al + dd;
    tau = be + dd;
    pw = tau + dd;
    Z = zg + jc * (int64_t)nr * d;
    wk = wkg + jc * (int64_t)4 * d * nr;
  }
  __syncthreads();

  // Reduction to tridiagonal form.  Per step: v from the column below the
  // diagonal; p = tau A22 v (wave w sums the columns jj = w mod DC_NW, lanes
  // run down the rows, the wave partials are added in order); K = tau p'v / 2;
  // A22 -= v w' + w v' with w = p - K v.  The next column's squared norm is
  // accumulated while its row is updated.
  double* vv = pw + dd;                                      // v of the current step
  double* part = IN_LDS ? vv + dd : partg + jc * DC_NW * (int64_t)d;  // DC_NW x dd partials
  const int wv = t >> 6, lane = t & 63;
  double sigma = 0.0;
  if (dd >= 3) {
    double ps = 0.0;
    for (int i = 2 + t; i < dd; i += DC_NT) ps = fma(A[i], A[i], ps);
    sigma = block_sum_n<DC_NT>(ps, shw);
  }
  for (int k = 0; k + 2 < dd; ++k) {
    const int n2 = dd - k - 1;
    double* rowk = A + (int64_t)k * lda + (k + 1);  // column k below the diagonal, by symmetry
    double* A22 = rowk + lda;                       // A[k+1][k+1]
    const double x0 = rowk[0];
    if (t == 0) al[k] = A[(int64_t)k * lda + k];
    if (sigma == 0.0) {  // already tridiagonal in this column: H_k = I
      if (t == 0) {
        tau[k] = 0.0;
        be[k] = x0;
      }
      double ps = 0.0;
      for (int i = 2 + t; i < n2; i += DC_NT) ps = fma(A22[i], A22[i], ps);
      sigma = block_sum_n<DC_NT>(ps, shw);
      continue;
    }
    const double beta = -copysign(sqrt(x0 * x0 + sigma), x0);
    const double tk = (beta - x0) / beta;
    const double scale = 1.0 / (x0 - beta);
    for (int i = t; i < n2; i += DC_NT) vv[i] = (i == 0) ? 1.0 : rowk[i] * scale;
    if (t == 0) {
      tau[k] = tk;
      be[k] = beta;
    }
    __syncthreads();
    for (int i0 = 0; i0 < n2; i0 += 64) {
      const int i = i0 + lane;
      if (i < n2) {
        double a0 = 0.0, a1 = 0.0;
        int jj = wv;
        for (; jj + DC_NW < n2; jj += 2 * DC_NW) {
          a0 = fma(A22[(int64_t)jj * lda + i], vv[jj], a0);
          a1 = fma(A22[(int64_t)(jj + DC_NW) * lda + i], vv[jj + DC_NW], a1);
        }
        if (jj < n2) a0 = fma(A22[(int64_t)jj * lda + i], vv[jj], a0);
        part[wv * dd + i] = a0 + a1;
      }
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = t; i < n2; i += DC_NT) {
      double sp = part[i];
#pragma unroll
      for (int w = 1; w < DC_NW; ++w) sp += part[w * dd + i];
      const double pi = tk * sp;
      pw[i] = pi;
      pv = fma(pi, vv[i], pv);
    }
    const double K = 0.5 * tk * block_sum_n<DC_NT>(pv, shw);
    double ps = dc_rank2(A22, lda, vv, pw, K, n2, wv, lane);
    for (int i = t; i < n2; i += DC_NT) rowk[i] = vv[i];  // v_k, kept for the back-transformation
    if (wv == 0) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) ps += __shfl_xor(ps, off, 64);
      if (lane == 0) sig_next = ps;
    }
    __syncthreads();
    sigma = sig_next;
  }
  if (t == 0) {
    if (dd >= 2) {
      al[dd - 2] = A[(int64_t)(dd - 2) * lda + (dd - 2)];
      be[dd - 2] = A[(int64_t)(dd - 1) * lda + (dd - 2)];
      tau[dd - 2] = 0.0;
    }
    al[dd - 1] = A[(int64_t)(dd - 1) * lda + (dd - 1)];
  }
  __syncthreads();

  tridiag_top<DC_NT>(al, be, dd, nrr, theta, Z, ldz, wk, pw);  // pw is free now
  __syncthreads();

  // back-transformation; wave w owns vectors w, w + DC_NW, ...
  for (int k = dd - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    const double* v = A + (int64_t)k * lda + (k + 1);
    const int n2 = dd - k - 1;
    for (int tt = wv; tt < nrr; tt += DC_NW) {
      double* z = Z + (int64_t)tt * ldz + (k + 1);
      double dot = 0.0;
      for (int i = lane; i < n2; i += 64) dot = fma(v[i], z[i], dot);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
      const double f = tk * dot;
      for (int i = lane; i < n2; i += 64) z[i] -= f * v[i];
    }
    if (!IN_LDS) __threadfence_block();
  }
  __syncthreads();

  for (int tt = t; tt < s.r; tt += DC_NT) lam[j * s.r + tt] = tt < nrr ? theta[tt] : 0.0;
  if (t == 0) status[j] = (nrr > 0 && theta[0] > 0.0) ? 0 : 1;
  if (!rows_gram) {
    for (int64_t e = t; e < (int64_t)dd * s.r; e += DC_NT) {
      const int i = (int)(e / s.r), tt = (int)(e % s.r);
      U[(j * d + i) * s.r + tt] = tt < nrr ? Z[(int64_t)tt * ldz + i] : 0.0;
    }
  } else {
    for (int64_t e = t; e < (int64_t)dd * s.r; e += DC_NT) {
      const int i = (int)(e / s.r), tt = (int)(e % s.r);
      double v = 0.0;
      if (tt < nrr && theta[tt] > 0.0) v = Z[(int64_t)tt * ldz + i] * sqrt(theta[tt]);
      Xs[(j * s.m_max + i) * s.r + tt] = v;
    }
  }
}

// ------------------------------------- register-resident eigensolver
// The same reduction, tridiagonal solver and back-transformation for
// d <= 16 NB, with the matrix held in registers instead of LDS: thread t
// (row group g = t / 16, column group c = t % 16) keeps the NB x NB entries
// A[g + 16 a][c + 16 b].  Row sums are butterflies over the 16 lanes of a
// row group (the same bits in every lane), so a Householder step needs two
// barriers; the Householder vector v_k replaces row k in the registers of
// that row's lanes, which later steps leave unchanged.  LDS holds only the
// tridiagonal matrix, the step vectors, Z and the inverse-iteration work,
// so several parts run on one compute unit.
constexpr int DCR_NT = 256;

// v from another lane of the same 16-lane row, by a DPP move of both halves
template <int CTRL>
__device__ __forceinline__ double dcr_dpp(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// the value of the wave's first active lane, in every lane
__device__ __forceinline__ double dcr_first(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// all-reduce over the 16 lanes of a row group: partner lanes 1 and 2 apart
// (quad permutations), then the other quad of the half row and the other
// half of the row (mirrors).  Each level adds the same two values in every
// lane, so all 16 lanes get the same bits.
__device__ __forceinline__ double dcr_sum16(double v) {
  v += dcr_dpp<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dcr_dpp<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dcr_dpp<0x141>(v);  // row_half_mirror
  v += dcr_dpp<0x140>(v);  // row_mirror
  return v;
}

// row ak of the register tile (ak is the same in every lane that asks)
template <int NB>
__device__ __forceinline__ void dcr_get_row(const double (&a)[NB][NB], int ak, double (&row)[NB]) {
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) row[bb] = 0.0;
#pragma unroll
  for (int aa = 0; aa < NB; ++aa)
    if (aa == ak)
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) row[bb] = a[aa][bb];
}

template <int NB>
__global__ __launch_bounds__(DCR_NT) __attribute__((amdgpu_waves_per_eu(3))) void k_dc_eigen_reg(double* __restrict__ G, int d, DcShape s,
                                                       int rows_gram, int64_t j0, int nr,
                                                       double* __restrict__ lam, double* __restrict__ U,
                                                       double* __restrict__ Xs, int* __restrict__ status) {
  constexpr int DM = 16 * NB;
  extern __shared__ double dsm[];
  // v of the step (two buffers alternating with k) and p; the first two
  // also serve the back-transformation
  __shared__ double vs[3][DM];
  __shared__ double red[DCR_NT / 64];
  __shared__ double theta[MDS_MAX_R];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int rg = 4 * wv + (lane >> 4), cg = lane & 15;
  const int64_t jc = blockIdx.x, j = j0 + jc;
  const int dd = rows_gram ? (int)dc_part_size(j, s) : d;
  const int nrr = std::min(nr, dd);
  double* Gp = G + jc * (int64_t)d * d;
  double* al = dsm;
  double* be = al + d;
  double* tau = be + d;
  double* be2 = tau + d;
  double* Z = be2 + d;
  const int ldz = d;
  double* wk = Z + (int64_t)nr * d;

  double a[NB][NB];
#pragma unroll
  for (int aa = 0; aa < NB; ++aa)
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const int i = rg + 16 * aa, jj = cg + 16 * bb;
      a[aa][bb] = (i < dd && jj < dd) ? Gp[(int64_t)i * d + jj] : 0.0;
    }

  // Reduction to tridiagonal form, H_k = I - tau_k v v' with v_{k+1} = 1.
  for (int k = 0; k + 2 < dd; ++k) {
    if (rg == (k & 15)) {  // the 16 lanes holding row k
      double row[NB];
      dcr_get_row<NB>(a, k >> 4, row);
      double x0 = 0.0, sg = 0.0, akk = 0.0;
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        const int jj = cg + 16 * bb;
        if (jj == k) akk = row[bb];
        if (jj == k + 1) x0 = row[bb];
        if (jj >= k + 2 && jj < dd) sg = fma(row[bb], row[bb], sg);
      }
      akk = dcr_sum16(akk);  // one lane holds each of these two
      x0 = dcr_sum16(x0);
      sg = dcr_sum16(sg);
      double tk = 0.0, beta = x0, scale = 0.0;
      if (sg != 0.0) {
        beta = -copysign(sqrt(x0 * x0 + sg), x0);
        tk = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        const int jj = cg + 16 * bb;
        double v = 0.0;
        if (sg != 0.0 && jj > k && jj < dd) v = (jj == k + 1) ? 1.0 : row[bb] * scale;
        vs[k & 1][jj] = v;
        if (jj > k) row[bb] = v;  // v_k kept in row k for the back-transformation
      }
#pragma unroll
      for (int aa = 0; aa < NB; ++aa)
        if (aa == (k >> 4))
#pragma unroll
          for (int bb = 0; bb < NB; ++bb) a[aa][bb] = row[bb];
      if (cg == 0) {
        al[k] = akk;
        be[k] = beta;
        tau[k] = tk;
      }
    }
    __syncthreads();
    const double tk = tau[k];
    if (tk == 0.0) continue;  // column k is already reduced: H_k = I
    // p = tau A22 v, rows k + 1 .. dd - 1 (zero elsewhere)
    double vr[NB], vc[NB], pr[NB];
#pragma unroll
    for (int aa = 0; aa < NB; ++aa) vr[aa] = vs[k & 1][rg + 16 * aa];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) vc[bb] = vs[k & 1][cg + 16 * bb];
    double pl = 0.0;
#pragma unroll
    for (int aa = 0; aa < NB; ++aa) {
      double acc = 0.0;
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) acc = fma(a[aa][bb], vc[bb], acc);
      acc = dcr_sum16(acc);
      const int i = rg + 16 * aa;
      pr[aa] = (i > k && i < dd) ? tk * acc : 0.0;
      pl = fma(pr[aa], vr[aa], pl);
    }
    // p'v: the row groups of a wave, then the waves in order
    pl += __shfl_xor(pl, 16, 64);
    pl += __shfl_xor(pl, 32, 64);
    if (lane == 0) red[wv] = pl;
    if (cg == 0)
#pragma unroll
      for (int aa = 0; aa < NB; ++aa) vs[2][rg + 16 * aa] = pr[aa];
    __syncthreads();
    const double K = 0.5 * tk * (((red[0] + red[1]) + red[2]) + red[3]);
    // A22 -= v w' + w v' with w = p - K v; both products rounded before the
    // sum, so A[i][j] and A[j][i] stay the same bits.  v and p are read
    // again from LDS (the same values), which keeps them out of registers
    // across the barrier.
    const double* vk = vs[k & 1];
    double vcb[NB], wc[NB];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      vcb[bb] = vk[cg + 16 * bb];
      wc[bb] = fma(-K, vcb[bb], vs[2][cg + 16 * bb]);
    }
#pragma unroll
    for (int aa = 0; aa < NB; ++aa) {
      const double vra = vk[rg + 16 * aa];
      const double wr = fma(-K, vra, vs[2][rg + 16 * aa]);
#pragma unroll
      for (int bb = 0; bb < NB; ++bb)
        a[aa][bb] = a[aa][bb] - (__dmul_rn(vra, wc[bb]) + __dmul_rn(wr, vcb[bb]));
    }
  }
  // the last 2 x 2 block
#pragma unroll
  for (int aa = 0; aa < NB; ++aa)
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const int i = rg + 16 * aa, jj = cg + 16 * bb;
      if (i == jj && i >= dd - 2 && i < dd) al[i] = a[aa][bb];
      if (i == dd - 1 && jj == dd - 2) be[dd - 2] = a[aa][bb];
    }
  if (t == 0 && dd >= 2) tau[dd - 2] = 0.0;
  // the tile (now holding the reflectors) waits in this part's Gram slot,
  // which nothing reads any more, while the tridiagonal solver runs: its
  // registers are free for the solver
#pragma unroll
  for (int aa = 0; aa < NB; ++aa)
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const int i = rg + 16 * aa, jj = cg + 16 * bb;
      if (i < dd && jj < dd) Gp[(int64_t)i * d + jj] = a[aa][bb];
    }
  __syncthreads();

  tridiag_top<DCR_NT>(al, be, dd, nrr, theta, Z, ldz, wk, be2);
  __syncthreads();
  asm volatile("" ::: "memory");  // reload the tile from memory
#pragma unroll
  for (int aa = 0; aa < NB; ++aa)
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      const int i = rg + 16 * aa, jj = cg + 16 * bb;
      a[aa][bb] = (i < dd && jj < dd) ? Gp[(int64_t)i * d + jj] : 0.0;
    }

  // back-transformation z <- H_k z, k descending: the lanes of row k post
  // v_k, then row group g updates vectors g, g + 16, ...; the two buffers
  // alternate over the reflections applied, so one barrier per reflection
  int ph = 0;
  for (int k = dd - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    double* vb = vs[ph];
    ph ^= 1;
    if (rg == (k & 15)) {
      double row[NB];
      dcr_get_row<NB>(a, k >> 4, row);
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        const int jj = cg + 16 * bb;
        vb[jj] = (jj > k && jj < dd) ? row[bb] : 0.0;
      }
    }
    __syncthreads();
    double v[NB];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) v[bb] = vb[cg + 16 * bb];
    for (int tt = rg; tt < nrr; tt += 16) {
      double* z = Z + (int64_t)tt * ldz;
      double dot = 0.0;
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        const int jj = cg + 16 * bb;
        if (jj < dd) dot = fma(v[bb], z[jj], dot);
      }
      const double f = tk * dcr_sum16(dot);
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        const int jj = cg + 16 * bb;
        if (jj > k && jj < dd) z[jj] -= f * v[bb];
      }
    }
  }
  __syncthreads();

  for (int tt = t; tt < s.r; tt += DCR_NT) lam[j * s.r + tt] = tt < nrr ? theta[tt] : 0.0;
  if (t == 0) status[j] = (nrr > 0 && theta[0] > 0.0) ? 0 : 1;
  if (!rows_gram) {
    for (int64_t e = t; e < (int64_t)dd * s.r; e += DCR_NT) {
      const int i = (int)(e / s.r), tt = (int)(e % s.r);
      U[(j * d + i) * s.r + tt] = tt < nrr ? Z[(int64_t)tt * ldz + i] : 0.0;
    }
  } else {
    for (int64_t e = t; e < (int64_t)dd * s.r; e += DCR_NT) {
      const int i = (int)(e / s.r), tt = (int)(e % s.r);
      double v = 0.0;
      if (tt < nrr && theta[tt] > 0.0) v = Z[(int64_t)tt * ldz + i] * sqrt(theta[tt]);
      Xs[(j * s.m_max + i) * s.r + tt] = v;
    }
  }
}

// ---------------------------------------------- coordinates X_j = B u
// Block: 64 rows of one part; features staged 32 at a time with U's rows.
// The four lanes 4 rl .. 4 rl + 3 share row rl: lane q takes features
// 8 q .. 8 q + 7 of each chunk into up to 16 independent sums (one per
// output column), and the quad adds its four partial sums in a fixed order
// (the same bits in each lane).  Row addresses are looked up once.
template <typename TX>
__global__ __launch_bounds__(256) void k_dc_coords(const TX* __restrict__ X, int64_t ldx,
                                                   const int64_t* __restrict__ order, DcShape s,
                                                   const double* __restrict__ mean,
                                                   const double* __restrict__ U,
                                                   double* __restrict__ Xs) {
  constexpr int RG = 16;  // output columns per pass
  __shared__ double Xt[64][33];
  __shared__ double Ut[32][RG + 1];
  const int t = threadIdx.x;
  const int rl = t >> 2, q = t & 3;    // row of the block, quarter of each chunk
  const int lr = t >> 5, lf = t & 31;  // staging: rows lr + 8 k, feature lf
  const int64_t j = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int64_t m = dc_part_size(j, s);
  if (i0 >= m) return;
  const double* mu = mean + j * s.p;
  const double* Uj = U + j * s.p * s.r;
  const TX* xr[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int64_t i = i0 + lr + 8 * k;
    xr[k] = (i < m) ? X + order[dc_pos(j, i, s)] * ldx : nullptr;
  }
  for (int tt0 = 0; tt0 < s.r; tt0 += RG) {
    double acc[RG];
#pragma unroll
    for (int tt = 0; tt < RG; ++tt) acc[tt] = 0.0;
    for (int64_t f0 = 0; f0 < s.p; f0 += 32) {
      const int64_t f = f0 + lf;
      const bool fin = f < s.p;
      const double muf = fin ? mu[f] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) Xt[lr + 8 * k][lf] = (xr[k] && fin) ? (double)xr[k][f] - muf : 0.0;
      for (int e = t; e < 32 * RG; e += 256) {
        const int ff = e / RG, tt = e % RG;
        Ut[ff][tt] = (f0 + ff < s.p && tt0 + tt < s.r) ? Uj[(f0 + ff) * s.r + tt0 + tt] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int ff = 8 * q + k;
        const double xv = Xt[rl][ff];
#pragma unroll
        for (int tt = 0; tt < RG; ++tt) acc[tt] = fma(xv, Ut[ff][tt], acc[tt]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int tt = 0; tt < RG; ++tt) {
      double v = acc[tt];
      v += dcr_dpp<0xB1>(v);  // quad_perm [1, 0, 3, 2]
      v += dcr_dpp<0x4E>(v);  // quad_perm [2, 3, 0, 1]
      acc[tt] = v;
    }
    if (q == 0 && i0 + rl < m) {
#pragma unroll
      for (int tt = 0; tt < RG; ++tt)
        if (tt0 + tt < s.r) Xs[(j * s.m_max + i0 + rl) * s.r + tt0 + tt] = acc[tt];
    }
  }
}

// ----------------------------------------------------- signs of part 0
// For each live column of X_0: +1 or -1 making its largest-|.| entry
// positive (first row in part order on ties).  One block; wave w scans the
// columns t = w (mod 4), lanes take rows i = lane (mod 64), and the lane
// maxima are merged by a butterfly that keeps the larger magnitude and, on
// equal magnitudes, the smaller row.
__global__ __launch_bounds__(256) void k_dc_signs(const double* __restrict__ Xs, DcShape s, int r0,
                                                  double* __restrict__ sgn) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t m0 = dc_part_size(0, s);
  for (int t = wv; t < r0; t += 4) {
    double best = -1.0, val = 0.0;
    int64_t at = INT64_MAX;
    for (int64_t i = lane; i < m0; i += 64) {
      const double v = Xs[i * s.r + t];
      if (fabs(v) > best) {
        best = fabs(v);
        val = v;
        at = i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const double ov = __shfl_xor(val, off, 64);
      const int64_t oa = __shfl_xor(at, off, 64);
      if (ob > best || (ob == best && oa < at)) {
        best = ob;
        val = ov;
        at = oa;
      }
    }
    if (lane == 0) sgn[t] = val < 0.0 ? -1.0 : 1.0;
  }
}

// ------------------------------------------------------------- alignment
// One block per part.  Part 0: its rows are written with the column signs
// from k_dc_signs.
// Part j >= 1: Procrustes fit on the c connecting rows over the r0 live
// columns: C = (B - 1b')'(A - 1a') (B: part j, A: part 0), C = U S W' by
// one-sided Jacobi (Hestenes) in one wave (column sums over the lanes as
// DPP row sums when r0 <= 16), T = U W', t = a - T' b; own rows
// become X_j T + t.  Columns r0..r-1 are zero.  status[j] = 2 when the
// smallest singular value of C is <= 1e-9 of the largest.
__global__ __launch_bounds__(256) void k_dc_align(const double* __restrict__ Xs,
                                                  const int64_t* __restrict__ order, DcShape s,
                                                  int r0, const double* __restrict__ sgn_g,
                                                  double* __restrict__ Y, int64_t ldy,
                                                  int* __restrict__ status) {
  extern __shared__ double dyn[];
  __shared__ double sgn[MDS_MAX_R];
  __shared__ double amean[MDS_MAX_R], bmean[MDS_MAX_R], tv[MDS_MAX_R], sig[MDS_MAX_R];
  // three r0 x r0 matrices, rows padded to r0 + 1:
  // CS(col, row) of C (then of C J), JS(col, row) of J, TS(a, k) = T[a][k]
  const int ldr = r0 + 1;
  double* cs_m = dyn;
  double* js_m = cs_m + (size_t)r0 * ldr;
  double* ts_m = js_m + (size_t)r0 * ldr;
#define CS(a, b) cs_m[(a) * ldr + (b)]
#define JS(a, b) js_m[(a) * ldr + (b)]
#define TS(a, b) ts_m[(a) * ldr + (b)]
  const int t = threadIdx.x;
  const int64_t j = blockIdx.x;
  const int r = s.r;
  const double* X0 = Xs;
  const double* Xj = Xs + j * s.m_max * r;
  const int64_t m0 = dc_part_size(0, s);
  if (t < r0) sgn[t] = sgn_g[t];
  __syncthreads();
  if (j == 0) {
    for (int64_t e = t; e < m0 * r; e += 256) {
      const int64_t i = e / r;
      const int k = (int)(e % r);
      Y[order[dc_pos(0, i, s)] * ldy + k] = k < r0 ? sgn[k] * X0[i * r + k] : 0.0;
    }
    return;
  }
  const int64_t c = s.c;
  if (t < r0) {
    double sa = 0.0, sb = 0.0;
    for (int64_t i = 0; i < c; ++i) {
      sa += sgn[t] * X0[i * r + t];
      sb += Xj[i * r + t];
    }
    amean[t] = sa / (double)c;
    bmean[t] = sb / (double)c;
  }
  __syncthreads();
  for (int e = t; e < r0 * r0; e += 256) {
    const int a = e / r0, b = e % r0;  // C[a][b]
    double acc = 0.0;
    for (int64_t i = 0; i < c; ++i)
      acc = fma(Xj[i * r + a] - bmean[a], sgn[b] * X0[i * r + b] - amean[b], acc);
    CS(b, a) = acc;
    JS(b, a) = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (t < 64) {
    const int lane = t;
    const bool own = lane < r0;
    for (int sweep = 0; sweep < 60; ++sweep) {
      int rotated = 0;
      for (int b1 = 0; b1 + 1 < r0; ++b1) {
        for (int b2 = b1 + 1; b2 < r0; ++b2) {
          const double x1 = own ? CS(b1, lane) : 0.0;
          const double x2 = own ? CS(b2, lane) : 0.0;
          double al = x1 * x1, be = x2 * x2, ga = x1 * x2;
          if (r0 <= 16) {  // only the first 16 lanes hold values: DPP row sums,
            // then lane 0's to every lane, so the control flow stays uniform
            al = dcr_first(dcr_sum16(al));
            be = dcr_first(dcr_sum16(be));
            ga = dcr_first(dcr_sum16(ga));
          } else {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
              al += __shfl_xor(al, off, 64);
              be += __shfl_xor(be, off, 64);
              ga += __shfl_xor(ga, off, 64);
            }
          }
          if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
          const double zeta = (be - al) / (2.0 * ga);
          const double tn = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tn * tn);
          const double sn = cs * tn;
          ++rotated;
          if (own) {
            CS(b1, lane) = cs * x1 - sn * x2;
            CS(b2, lane) = sn * x1 + cs * x2;
            const double j1 = JS(b1, lane), j2 = JS(b2, lane);
            JS(b1, lane) = cs * j1 - sn * j2;
            JS(b2, lane) = sn * j1 + cs * j2;
          }
        }
      }
      if (rotated == 0) break;
    }
    for (int b = 0; b < r0; ++b) {
      const double x = own ? CS(b, lane) : 0.0;
      double nn = x * x;
      if (r0 <= 16) {
        nn = dcr_sum16(nn);
      } else {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) nn += __shfl_xor(nn, off, 64);
      }
      if (lane == 0) sig[b] = sqrt(nn);
    }
  }
  __syncthreads();
  if (t == 0) {
    double smax = 0.0, smin = INFINITY;
    for (int b = 0; b < r0; ++b) {
      smax = fmax(smax, sig[b]);
      smin = fmin(smin, sig[b]);
    }
    status[j] = (smin > 1e-9 * smax) ? 0 : 2;
  }
  for (int e = t; e < r0 * r0; e += 256) {
    const int a = e / r0, k = e % r0;
    double acc = 0.0;
    for (int b = 0; b < r0; ++b) acc = fma(CS(b, a) / sig[b], JS(b, k), acc);
    TS(a, k) = acc;
  }
  __syncthreads();
  if (t < r0) {
    double acc = 0.0;
    for (int a = 0; a < r0; ++a) acc = fma(TS(a, t), bmean[a], acc);
    tv[t] = amean[t] - acc;
  }
  __syncthreads();
  const int64_t m = dc_part_size(j, s);
  for (int64_t e = t; e < (m - c) * r; e += 256) {
    const int64_t i = c + e / r;
    const int k = (int)(e % r);
    double y = 0.0;
    if (k < r0) {
      double acc = 0.0;
      for (int a = 0; a < r0; ++a) acc = fma(Xj[i * r + a], TS(a, k), acc);
      y = acc + tv[k];
    }
    Y[order[dc_pos(j, i, s)] * ldy + k] = y;
  }
}

#undef CS
#undef JS
#undef TS

struct DevMem {
  void* p = nullptr;
  hipStream_t st = nullptr;
  ~DevMem() {
    if (p) (void)hipFreeAsync(p, st);
  }
  template <typename T>
  T* get() const {
    return static_cast<T*>(p);
  }
};

#define DC_HIP(call)                                     \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) return hip_fail(_e, #call);    \
  } while (0)

#define DC_LAUNCH(what)                                  \
  do {                                                   \
    hipError_t _e = hipGetLastError();                   \
    if (_e != hipSuccess) return hip_fail(_e, what);     \
  } while (0)

constexpr size_t kDcLdsMax = 150 * 1024;
constexpr size_t kDcGramBudget = (size_t)1 << 30;

size_t eigen_lds_bytes(int d, int nr) {
  // A, five vectors, one partial row per wave, Z and the inverse-iteration work
  return sizeof(double) * ((size_t)d * d + (5 + DC_NW) * (size_t)d + (size_t)nr * d + 4 * (size_t)d * nr);
}

// the register-resident solver: four vectors, Z and the inverse-iteration work
constexpr int kDcRegMaxD = 112;
size_t eigen_reg_lds_bytes(int d, int nr) {
  return sizeof(double) * (size_t)d * (4 + 5 * (size_t)nr);
}

hipError_t set_eigen_reg_attrs() {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f) {
    if (e == hipSuccess) e = lds_limit_once(f, (int)kDcLdsMax);
  };
  set(reinterpret_cast<const void*>(&k_dc_eigen_reg<1>));
  set(reinterpret_cast<const void*>(&k_dc_eigen_reg<2>));
  set(reinterpret_cast<const void*>(&k_dc_eigen_reg<4>));
  set(reinterpret_cast<const void*>(&k_dc_eigen_reg<7>));
  return e;
}

// tile width NB = ceil(d / 16), rounded up to 1, 2, 4 or 7
void launch_eigen_reg(unsigned grid, size_t lds, hipStream_t st, double* G, int d, DcShape s,
                      int rows_gram, int64_t j0, int nr, double* lam, double* U, double* Xs, int* status) {
  if (d <= 16)
    k_dc_eigen_reg<1><<<grid, DCR_NT, lds, st>>>(G, d, s, rows_gram, j0, nr, lam, U, Xs, status);
  else if (d <= 32)
    k_dc_eigen_reg<2><<<grid, DCR_NT, lds, st>>>(G, d, s, rows_gram, j0, nr, lam, U, Xs, status);
  else if (d <= 64)
    k_dc_eigen_reg<4><<<grid, DCR_NT, lds, st>>>(G, d, s, rows_gram, j0, nr, lam, U, Xs, status);
  else
    k_dc_eigen_reg<7><<<grid, DCR_NT, lds, st>>>(G, d, s, rows_gram, j0, nr, lam, U, Xs, status);
}

template <typename TX>
mds_status dc_run(const TX* X, int64_t ldx, DcShape s, uint64_t seed, double* Y, int64_t ldy,
                  double* lam_bar, int32_t* r_eff, int64_t* order_out, hipStream_t st) {
  const int64_t n = s.n, p = s.p, np = s.nparts;
  const int r = s.r;
  const bool rows_gram = s.m_max < p;  // solve through the smaller Gram matrix
  const int d = (int)(rows_gram ? s.m_max : p);
  const int nr = std::min(r, d);
  const bool in_lds = eigen_lds_bytes(d, nr) <= kDcLdsMax;
  const bool in_regs = d <= kDcRegMaxD && eigen_reg_lds_bytes(d, nr) <= kDcLdsMax;
  const int64_t chunk =
      std::max<int64_t>(1, std::min<int64_t>(np, (int64_t)(kDcGramBudget / (sizeof(double) * (size_t)d * d))));

  DevMem keys_in, keys_out, vals, order_buf, tmp, mean, lam, status, U, Xs, G, zg, wkg, partg, bad, sgn;
  auto alloc = [&](DevMem& b, size_t bytes) -> hipError_t {
    b.st = st;
    return hipMallocAsync(&b.p, std::max<size_t>(bytes, 256), st);
  };
  DC_HIP(alloc(keys_in, sizeof(uint64_t) * n));
  DC_HIP(alloc(keys_out, sizeof(uint64_t) * n));
  DC_HIP(alloc(vals, sizeof(int64_t) * n));
  int64_t* order = order_out;
  if (!order) {
    DC_HIP(alloc(order_buf, sizeof(int64_t) * n));
    order = order_buf.get<int64_t>();
  }
  DC_HIP(alloc(mean, sizeof(double) * np * p));
  DC_HIP(alloc(lam, sizeof(double) * np * r));
  DC_HIP(alloc(status, sizeof(int) * np));
  if (!rows_gram) DC_HIP(alloc(U, sizeof(double) * np * p * r));
  DC_HIP(alloc(Xs, sizeof(double) * np * s.m_max * r));
  DC_HIP(alloc(G, sizeof(double) * chunk * d * d));
  if (!in_lds) {
    DC_HIP(alloc(zg, sizeof(double) * chunk * nr * d));
    DC_HIP(alloc(wkg, sizeof(double) * chunk * 4 * d * nr));
    DC_HIP(alloc(partg, sizeof(double) * chunk * DC_NW * d));
  }
  DC_HIP(alloc(bad, sizeof(int)));
  DC_HIP(alloc(sgn, sizeof(double) * MDS_MAX_R));
  DC_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));

  // partition: keys, then a stable radix sort of (key, row)
  {
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
    k_dc_keys<<<grid, 256, 0, st>>>(n, seed, keys_in.get<uint64_t>(), vals.get<int64_t>());
    DC_LAUNCH("partition keys");
    size_t tbytes = 0;
    DC_HIP(rocprim::radix_sort_pairs(nullptr, tbytes, keys_in.get<uint64_t>(), keys_out.get<uint64_t>(),
                                     vals.get<int64_t>(), order, (size_t)n, 0, 64, st));
    DC_HIP(alloc(tmp, tbytes));
    DC_HIP(rocprim::radix_sort_pairs(tmp.p, tbytes, keys_in.get<uint64_t>(), keys_out.get<uint64_t>(),
                                     vals.get<int64_t>(), order, (size_t)n, 0, 64, st));
  }
  {
    dim3 grid((unsigned)np, (unsigned)((p + 63) / 64));
    k_dc_mean<TX><<<grid, 256, 0, st>>>(X, ldx, order, s, mean.get<double>(), bad.get<int>());
    DC_LAUNCH("part means");
  }
  DC_HIP(lds_limit_once(reinterpret_cast<const void*>(&k_dc_eigen<true>), (int)kDcLdsMax));
  DC_HIP(lds_limit_once(reinterpret_cast<const void*>(&k_dc_eigen<false>), (int)kDcLdsMax));
  DC_HIP(lds_limit_once(reinterpret_cast<const void*>(&k_dc_align), (int)kDcLdsMax));
  DC_HIP(set_eigen_reg_attrs());
  for (int64_t j0 = 0; j0 < np; j0 += chunk) {
    const int64_t cnt = std::min(chunk, np - j0);
    const unsigned tiles = (unsigned)((d + 63) / 64);
    dim3 ggrid(tiles, tiles, (unsigned)cnt);
    if (rows_gram)
      k_dc_gram_rows<TX><<<ggrid, 256, 0, st>>>(X, ldx, order, s, mean.get<double>(), j0, G.get<double>());
    else if (p <= DCG_MAXP)
      k_dc_gram_mfma<TX><<<(unsigned)cnt, 256, 0, st>>>(X, ldx, order, s, mean.get<double>(), j0,
                                                         G.get<double>());
    else
      k_dc_gram_feat<TX><<<ggrid, 256, 0, st>>>(X, ldx, order, s, mean.get<double>(), j0, G.get<double>());
    DC_LAUNCH("part Gram matrices");
    if (in_regs)
      launch_eigen_reg((unsigned)cnt, eigen_reg_lds_bytes(d, nr), st, G.get<double>(), d, s,
                       rows_gram ? 1 : 0, j0, nr, lam.get<double>(), U.get<double>(), Xs.get<double>(),
                       status.get<int>());
    else if (in_lds)
      k_dc_eigen<true><<<(unsigned)cnt, DC_NT, eigen_lds_bytes(d, nr), st>>>(
          G.get<double>(), d, s, rows_gram ? 1 : 0, j0, nr, nullptr, nullptr, nullptr,
          lam.get<double>(), U.get<double>(), Xs.get<double>(), status.get<int>());
    else
      k_dc_eigen<false><<<(unsigned)cnt, DC_NT, sizeof(double) * 5 * (size_t)d, st>>>(
          G.get<double>(), d, s, rows_gram ? 1 : 0, j0, nr, zg.get<double>(), wkg.get<double>(),
          partg.get<double>(), lam.get<double>(), U.get<double>(), Xs.get<double>(),
          status.get<int>());
    DC_LAUNCH("part eigensolver");
  }
  if (!rows_gram) {
    dim3 grid((unsigned)((s.m_max + 63) / 64), (unsigned)np);
    k_dc_coords<TX><<<grid, 256, 0, st>>>(X, ldx, order, s, mean.get<double>(), U.get<double>(),
                                         Xs.get<double>());
    DC_LAUNCH("part coordinates");
  }
  std::vector<double> hlam((size_t)np * r);
  std::vector<int> hstat((size_t)np);
  int hbad = 0;
  DC_HIP(hipMemcpyAsync(hlam.data(), lam.p, sizeof(double) * np * r, hipMemcpyDeviceToHost, st));
  DC_HIP(hipMemcpyAsync(hstat.data(), status.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
  DC_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  if (hbad) return set_error(MDS_ERR_INVALID_ARG, "non-finite value in X");
  for (int64_t j = 0; j < np; ++j)
    if (hstat[j]) return set_error(MDS_ERR_DEGENERATE, "all rows of a part coincide (lambda_1 <= 0)");
  int r0 = 0;
  for (int t = 0; t < r; ++t)
    if (hlam[t] > MDS_TAU * hlam[0]) ++r0;
  k_dc_signs<<<1, 256, 0, st>>>(Xs.get<double>(), s, r0, sgn.get<double>());
  DC_LAUNCH("signs of the first part");
  const size_t align_lds = sizeof(double) * 3 * (size_t)r0 * (r0 + 1);
  k_dc_align<<<(unsigned)np, 256, align_lds, st>>>(Xs.get<double>(), order, s, r0, sgn.get<double>(),
                                                   Y, ldy, status.get<int>());
  DC_LAUNCH("alignment");
  DC_HIP(hipMemcpyAsync(hstat.data(), status.p, sizeof(int) * np, hipMemcpyDeviceToHost, st));
  DC_HIP(hipStreamSynchronize(st));
  for (int64_t j = 1; j < np; ++j)
    if (hstat[j]) return set_error(MDS_ERR_DEGENERATE, "connecting points do not fix the Procrustes rotation");
  if (lam_bar) {
    for (int t = 0; t < r; ++t) {
      double acc = 0.0;
      for (int64_t j = 0; j < np; ++j) acc += hlam[(size_t)j * r + t] / (double)dc_part_size(j, s);
      lam_bar[t] = acc / (double)np;
    }
  }
  if (r_eff) *r_eff = r0;
  return MDS_OK;
}

}  // namespace

mds_status dense_top_eigen(double* G, int d, int r, double* lam, double* U, int* status,
                           hipStream_t st) {
  DcShape s;
  s.n = d;
  s.p = d;
  s.l = d;
  s.c = 0;
  s.r = r;
  s.nparts = 1;
  s.m_max = d;
  const int nr = std::min(r, d);
  DC_HIP(lds_limit_once(reinterpret_cast<const void*>(&k_dc_eigen<true>), (int)kDcLdsMax));
  DC_HIP(lds_limit_once(reinterpret_cast<const void*>(&k_dc_eigen<false>), (int)kDcLdsMax));
  DC_HIP(set_eigen_reg_attrs());
  if (d <= kDcRegMaxD && eigen_reg_lds_bytes(d, nr) <= kDcLdsMax) {
    launch_eigen_reg(1, eigen_reg_lds_bytes(d, nr), st, G, d, s, 0, 0, nr, lam, U, nullptr, status);
  } else if (eigen_lds_bytes(d, nr) <= kDcLdsMax) {
    k_dc_eigen<true><<<1, DC_NT, eigen_lds_bytes(d, nr), st>>>(G, d, s, 0, 0, nr, nullptr, nullptr,
                                                              nullptr, lam, U, nullptr, status);
  } else {
    DevMem zg, wkg, partg;
    auto alloc = [&](DevMem& b, size_t bytes) -> hipError_t {
      b.st = st;
      return hipMallocAsync(&b.p, std::max<size_t>(bytes, 256), st);
    };
    DC_HIP(alloc(zg, sizeof(double) * nr * (size_t)d));
    DC_HIP(alloc(wkg, sizeof(double) * 4 * (size_t)d * nr));
    DC_HIP(alloc(partg, sizeof(double) * DC_NW * (size_t)d));
    k_dc_eigen<false><<<1, DC_NT, sizeof(double) * 5 * (size_t)d, st>>>(
        G, d, s, 0, 0, nr, zg.get<double>(), wkg.get<double>(), partg.get<double>(), lam, U, nullptr,
        status);
  }
  DC_LAUNCH("dense eigensolver");
  return MDS_OK;
}

mds_status dc_on_device(const void* X, int dt, int64_t n, int64_t p, int64_t ldx, int64_t l, int64_t c,
                        int r, uint64_t seed, double* Y, int64_t ldy, double* lam_bar, int32_t* r_eff,
                        int64_t* order_out, hipStream_t st) {
  DcShape s;
  s.n = n;
  s.p = p;
  s.l = l;
  s.c = c;
  s.r = r;
  s.nparts = (n <= l) ? 1 : 1 + (n - l + (l - c) - 1) / (l - c);
  s.m_max = std::min(n, l);
  if (dt == MDS_F32)
    return dc_run<float>(static_cast<const float*>(X), ldx, s, seed, Y, ldy, lam_bar, r_eff, order_out, st);
  return dc_run<double>(static_cast<const double*>(X), ldx, s, seed, Y, ldy, lam_bar, r_eff, order_out, st);
}

}  // namespace mds
