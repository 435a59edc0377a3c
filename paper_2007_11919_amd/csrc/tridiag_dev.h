// Device helpers shared by the eigensolvers of the fit and of
// divide-and-conquer MDS: a hash for start vectors, a fixed-order block
// sum, and the symmetric tridiagonal solver that returns the largest
// eigenpairs.  Every function here is called by a whole 256-thread block.
#ifndef MDS_TRIDIAG_DEV_H
#define MDS_TRIDIAG_DEV_H

#include <hip/hip_runtime.h>

#include <cfloat>
#include <stdint.h>

#include "mds.h"

namespace mds {
namespace {

__device__ inline double hash_unit(uint64_t i, uint64_t salt) {
  // SplitMix64 finaliser of (salt, i) mapped to [-1, 1); used only to seed
  // start vectors and restarts.
  uint64_t z = i * 0x9E3779B97F4A7C15ull + salt * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// fixed-order sum over a 256-thread block: butterfly within each wave, then
// the four wave partials in order
__device__ inline double block_sum4(double v, double* sh4) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
  __syncthreads();
  return r;
}

__device__ inline int sturm_count(const double* alpha, const double* beta, int k, double x,
                                  double pivmin) {
  // number of eigenvalues of T below x
  int cnt = 0;
  double d = alpha[0] - x;
  if (fabs(d) < pivmin) d = -pivmin;
  if (d < 0) ++cnt;
  for (int i = 1; i < k; ++i) {
    const double b = beta[i - 1];
    d = (alpha[i] - x) - b * b / d;
    if (fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++cnt;
  }
  return cnt;
}

// The nr largest eigenpairs of the k x k symmetric tridiagonal T with
// diagonal al[0..k) and off-diagonal be[0..k-1) (both readable by every
// thread).  Eigenvalues by bisection on Sturm counts, multisected over the
// 256 threads; eigenvectors by inverse iteration with partial pivoting,
// orthogonalised (modified Gram-Schmidt) within clusters of close
// eigenvalues.  Output: theta[t] (shared, nr entries, descending) and the
// unit vector of pair t at Z + t * ldz.  wk holds 4 * k * nr doubles.
__device__ void tridiag_top(const double* al, const double* be, int k, int nr, double* theta,
                            double* Z, int ldz, double* wk) {
  __shared__ double sh[256];
  __shared__ double sh4[4];
  __shared__ double ga[MDS_MAX_R], gb[MDS_MAX_R];
  __shared__ int flag[256];
  const int t = threadIdx.x;
  // Gershgorin interval and scale
  double lo = DBL_MAX, hi = -DBL_MAX, bmax = 0.0;
  for (int i = t; i < k; i += 256) {
    const double bl = (i > 0) ? fabs(be[i - 1]) : 0.0;
    const double br = (i < k - 1) ? fabs(be[i]) : 0.0;
    lo = fmin(lo, al[i] - bl - br);
    hi = fmax(hi, al[i] + bl + br);
    bmax = fmax(bmax, br);
  }
  sh[t] = lo;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) sh[t] = fmin(sh[t], sh[t + s2]);
    __syncthreads();
  }
  lo = sh[0];
  __syncthreads();
  sh[t] = hi;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) sh[t] = fmax(sh[t], sh[t + s2]);
    __syncthreads();
  }
  hi = sh[0];
  __syncthreads();
  sh[t] = bmax;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if (t < s2) sh[t] = fmax(sh[t], sh[t + s2]);
    __syncthreads();
  }
  bmax = sh[0];
  __syncthreads();
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = DBL_MIN * fmax(1.0, bmax * bmax);
  const double eps = DBL_EPSILON;
  lo -= 2.0 * eps * tnorm + pivmin;
  hi += 2.0 * eps * tnorm + pivmin;

  // All wanted eigenvalues at once: a group of G threads multisects each.
  int G = 256;
  while (G > 1 && G * nr > 256) G >>= 1;
  const int grp = t / G, gl = t % G;
  const bool active = grp < nr;
  if (t < nr) {
    ga[t] = lo;
    gb[t] = hi;
  }
  __syncthreads();
  const int m = k - 1 - grp;  // ascending index of eigenvalue grp (largest first)
  for (int round = 0; round < 64; ++round) {
    int more = 0;
    if (active) {
      const double a = ga[grp], b = gb[grp];
      more = (b - a > 2.0 * eps * fmax(fabs(a), fabs(b)) + pivmin) ? 1 : 0;
      if (more) {
        const double x = a + (b - a) * (double)(gl + 1) / (double)(G + 1);
        flag[t] = sturm_count(al, be, k, x, pivmin) >= m + 1;
      }
    }
    if (!__syncthreads_or(more)) break;
    if (active && gl == 0) {
      const double a = ga[grp], b = gb[grp];
      if (b - a > 2.0 * eps * fmax(fabs(a), fabs(b)) + pivmin) {
        int first = G;
        for (int q = 0; q < G; ++q)
          if (flag[grp * G + q]) {
            first = q;
            break;
          }
        const double xa = (first == 0) ? a : a + (b - a) * (double)first / (double)(G + 1);
        const double xb = (first == G) ? b : a + (b - a) * (double)(first + 1) / (double)(G + 1);
        ga[grp] = xa;
        gb[grp] = xb;
      }
    }
    __syncthreads();
  }
  if (t < nr) theta[t] = 0.5 * (ga[t] + gb[t]);
  __syncthreads();

  // eigenvectors by inverse iteration (thread tt owns vector tt)
  const double pert = eps * fmax(tnorm, DBL_MIN) + pivmin;
  const double cluster_gap = 1e-3 * tnorm;
  for (int it = 0; it < 3; ++it) {
    if (t < nr) {
      double* z = Z + (int64_t)t * ldz;
      const double th = theta[t];
      // factor T - th I with partial pivoting, applying the row operations to
      // the right-hand side on the fly; keep U (dd, u1, u2) and the
      // eliminated right-hand side y for the backward pass.
      double zc = (it == 0) ? 1.0 + 0.5 * hash_unit(0, 977 + t) : z[0];
      double cur_d = al[0] - th;
      double cur_u = (k > 1) ? be[0] : 0.0;
      double cur_u2 = 0.0;
      for (int i = 0; i < k - 1; ++i) {
        const double sub = be[i];
        const double nd = al[i + 1] - th;
        const double nu = (i + 1 < k - 1) ? be[i + 1] : 0.0;
        const double zn = (it == 0) ? 1.0 + 0.5 * hash_unit((uint64_t)(i + 1), 977 + t) : z[i + 1];
        double di, u1, u2, y;
        if (fabs(cur_d) >= fabs(sub)) {
          di = (cur_d == 0.0) ? pert : cur_d;
          const double mlt = sub / di;
          u1 = cur_u;
          u2 = cur_u2;
          y = zc;
          zc = zn - mlt * zc;
          cur_d = nd - mlt * cur_u;
          cur_u = nu - mlt * cur_u2;
        } else {
          const double mlt = cur_d / sub;
          di = sub;
          u1 = nd;
          u2 = nu;
          y = zn;
          zc = zc - mlt * zn;
          const double nd2 = cur_u - mlt * nd;
          const double nu2 = cur_u2 - mlt * nu;
          cur_d = nd2;
          cur_u = nu2;
        }
        cur_u2 = 0.0;
        wk[((int64_t)i * 4 + 0) * nr + t] = di;
        wk[((int64_t)i * 4 + 1) * nr + t] = u1;
        wk[((int64_t)i * 4 + 2) * nr + t] = u2;
        wk[((int64_t)i * 4 + 3) * nr + t] = y;
      }
      double dl = (cur_d == 0.0) ? pert : cur_d;
      if (fabs(dl) < pert) dl = (dl < 0 ? -pert : pert);
      // backward substitution with a rolling window of two values
      double z1 = zc / dl, z2 = 0.0;
      double nn = z1 * z1;
      z[k - 1] = z1;
      for (int i = k - 2; i >= 0; --i) {
        double di = wk[((int64_t)i * 4 + 0) * nr + t];
        const double u1 = wk[((int64_t)i * 4 + 1) * nr + t];
        const double u2 = wk[((int64_t)i * 4 + 2) * nr + t];
        const double y = wk[((int64_t)i * 4 + 3) * nr + t];
        if (fabs(di) < pert) di = (di < 0 ? -pert : pert);
        const double zi = (y - u1 * z1 - u2 * z2) / di;
        z2 = z1;
        z1 = zi;
        z[i] = zi;
        nn = fma(zi, zi, nn);
      }
      const double inv = 1.0 / sqrt(nn);
      for (int i = 0; i < k; ++i) z[i] *= inv;
    }
    __syncthreads();
    // modified Gram-Schmidt inside clusters of close eigenvalues
    for (int tt = 1; tt < nr; ++tt) {
      bool any = false;
      for (int ss = 0; ss < tt; ++ss) any |= fabs(theta[tt] - theta[ss]) <= cluster_gap;
      if (!any) continue;
      double* zt = Z + (int64_t)tt * ldz;
      for (int ss = 0; ss < tt; ++ss) {
        if (fabs(theta[tt] - theta[ss]) > cluster_gap) continue;
        const double* zs = Z + (int64_t)ss * ldz;
        double d = 0.0;
        for (int i = t; i < k; i += 256) d = fma(zs[i], zt[i], d);
        d = block_sum4(d, sh4);
        for (int i = t; i < k; i += 256) zt[i] -= d * zs[i];
        __syncthreads();
      }
      double nn = 0.0;
      for (int i = t; i < k; i += 256) nn = fma(zt[i], zt[i], nn);
      nn = block_sum4(nn, sh4);
      const double inv = 1.0 / sqrt(nn);
      for (int i = t; i < k; i += 256) zt[i] *= inv;
      __syncthreads();
    }
  }
}

}  // namespace
}  // namespace mds

#endif
