// Device helpers shared by the eigensolvers of the fit and of
// divide-and-conquer MDS: a hash for start vectors, fixed-order block sums,
// and the symmetric tridiagonal solver that returns the largest eigenpairs.
// The block functions are called by every thread of a block of NT threads
// (a multiple of 64).
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

// the same for a block of NT threads: NT / 64 wave partials in order
template <int NT>
__device__ inline double block_sum_n(double v, double* shw) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) shw[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = shw[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) r += shw[w];
  __syncthreads();
  return r;
}

// 1/d from the hardware reciprocal refined by two Newton steps (each
// squares the relative error), good to about an ulp; d must be a normal
// number.  Cheaper than a correctly rounded division, which the Sturm
// recurrence does not need: an O(eps) relative change of each pivot is a
// perturbation of T of the same order.
__device__ inline double rcp_refined(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  return r;
}

__device__ inline int sturm_count(const double* alpha, const double* beta2, int k, double x,
                                  double pivmin) {
  // number of eigenvalues of T below x (beta2 holds the squared
  // off-diagonal); pivots smaller than pivmin are replaced by -pivmin
  int cnt = 0;
  double d = alpha[0] - x;
  if (fabs(d) < pivmin) d = -pivmin;
  if (d < 0) ++cnt;
  for (int i = 1; i < k; ++i) {
    d = (alpha[i] - x) - beta2[i - 1] * rcp_refined(d);
    if (fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++cnt;
  }
  return cnt;
}

// One sweep of inverse iteration for the vector z (length k, replaced by
// the normalised solution of (T - th I) x = z): LU factorisation with
// partial pivoting, applied to the right-hand side on the fly, then the
// backward substitution.  U is kept as (1/pivot, u1, u2) with the
// eliminated right-hand side y in wk[i * 4 * nr + {0,1,2,3} * nr] (the
// caller's column t).  Pivots smaller than pert in magnitude are replaced by
// +-pert.  Thread-private: no barrier, no other thread's data.
__device__ __forceinline__ void inverse_sweep(const double* __restrict__ al,
                                              const double* __restrict__ be, int k, double th,
                                              double pert, double* __restrict__ z,
                                              double* __restrict__ wk, int nr) {
  double zc = z[0];
  double cur_d = al[0] - th;
  double cur_u = (k > 1) ? be[0] : 0.0;
  for (int i = 0; i < k - 1; ++i) {
    // rows i (cur_d, cur_u, 0 | zc) and i + 1 (sub, nd, nu | zn): the row
    // with the larger entry in column i is the pivot row, the other one is
    // eliminated with it (selects, so the lanes of a wave do not diverge)
    const double sub = be[i];
    const double nd = al[i + 1] - th;
    const double nu = (i + 1 < k - 1) ? be[i + 1] : 0.0;
    const double zn = z[i + 1];
    const bool swap = fabs(cur_d) < fabs(sub);
    const double pd = swap ? sub : cur_d;
    const double p1 = swap ? nd : cur_u, p2 = swap ? nu : 0.0, pz = swap ? zn : zc;
    const double od = swap ? cur_d : sub;
    const double o1 = swap ? cur_u : nd, o2 = swap ? 0.0 : nu, oz = swap ? zc : zn;
    const double rp = rcp_refined((fabs(pd) < pert) ? (pd < 0 ? -pert : pert) : pd);
    const double mlt = od * rp;
    cur_d = fma(-mlt, p1, o1);
    cur_u = fma(-mlt, p2, o2);
    zc = fma(-mlt, pz, oz);
    double* w = wk + (int64_t)i * 4 * nr;
    w[0] = rp;
    w[nr] = p1;
    w[2 * nr] = p2;
    w[3 * nr] = pz;
  }
  double dl = (fabs(cur_d) < pert) ? (cur_d < 0 ? -pert : pert) : cur_d;
  // backward substitution with a rolling window of two values
  double z1 = zc * rcp_refined(dl), z2 = 0.0;
  double nn = z1 * z1;
  z[k - 1] = z1;
  for (int i = k - 2; i >= 0; --i) {
    const double* w = wk + (int64_t)i * 4 * nr;
    const double zi = (w[3 * nr] - w[nr] * z1 - w[2 * nr] * z2) * w[0];
    z2 = z1;
    z1 = zi;
    z[i] = zi;
    nn = fma(zi, zi, nn);
  }
  const double inv = 1.0 / sqrt(nn);
  for (int i = 0; i < k; ++i) z[i] *= inv;
}

// The nr largest eigenpairs of the k x k symmetric tridiagonal T with
// diagonal al[0..k) and off-diagonal be[0..k-1) (both readable by every
// thread).  Eigenvalues by bisection on Sturm counts, multisected over the
// NT threads; eigenvectors by inverse iteration with partial pivoting,
// orthogonalised (modified Gram-Schmidt) within clusters of close
// eigenvalues.  Output: theta[t] (shared, nr entries, descending) and the
// unit vector of pair t at Z + t * ldz.  wk holds 4 * k * nr doubles and
// be2 k doubles of scratch (both visible to the whole block).
template <int NT>
__device__ void tridiag_top(const double* al, const double* be, int k, int nr, double* theta,
                            double* Z, int ldz, double* wk, double* be2) {
  __shared__ double sh[NT];
  __shared__ double shw[NT / 64];
  __shared__ double ga[MDS_MAX_R], gb[MDS_MAX_R];
  __shared__ int flag[NT];
  const int t = threadIdx.x;
  // Gershgorin interval and scale
  double lo = DBL_MAX, hi = -DBL_MAX, bmax = 0.0;
  for (int i = t; i < k; i += NT) {
    const double bl = (i > 0) ? fabs(be[i - 1]) : 0.0;
    const double br = (i < k - 1) ? fabs(be[i]) : 0.0;
    lo = fmin(lo, al[i] - bl - br);
    hi = fmax(hi, al[i] + bl + br);
    bmax = fmax(bmax, br);
    be2[i] = (i < k - 1) ? be[i] * be[i] : 0.0;
  }
  sh[t] = lo;
  __syncthreads();
  for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
    if (t < s2) sh[t] = fmin(sh[t], sh[t + s2]);
    __syncthreads();
  }
  lo = sh[0];
  __syncthreads();
  sh[t] = hi;
  __syncthreads();
  for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
    if (t < s2) sh[t] = fmax(sh[t], sh[t + s2]);
    __syncthreads();
  }
  hi = sh[0];
  __syncthreads();
  sh[t] = bmax;
  __syncthreads();
  for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
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
  const int G = (nr > 0) ? NT / nr : NT;
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
        flag[t] = sturm_count(al, be2, k, x, pivmin) >= m + 1;
      }
    }
    if (!__syncthreads_or(more)) break;
    if (active && gl == 0) {
      const double a = ga[grp], b = gb[grp];
      if (b - a > 2.0 * eps * fmax(fabs(a), fabs(b)) + pivmin) {
        // a transition false -> true of the flags (a at q = -1 counts as
        // false, b at q = G as true); binary search keeps that invariant
        int qlo = -1, first = G;
        while (first - qlo > 1) {
          const int mid = (qlo + first) >> 1;
          if (flag[grp * G + mid])
            first = mid;
          else
            qlo = mid;
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

  // eigenvectors by inverse iteration (thread tt owns vector tt); the shift
  // is accurate to a few ulps of |T|, so two sweeps from a random start
  // leave an error of order eps |T| / gap
  const double pert = eps * fmax(tnorm, DBL_MIN) + pivmin;
  const double cluster_gap = 1e-3 * tnorm;
  for (int e = t; e < k * nr; e += NT) {  // random start vectors
    const int tt = e / k, i = e % k;
    Z[(int64_t)tt * ldz + i] = 1.0 + 0.5 * hash_unit((uint64_t)i, 977 + tt);
  }
  __syncthreads();
  for (int it = 0; it < 2; ++it) {
    if (t < nr) inverse_sweep(al, be, k, theta[t], pert, Z + (int64_t)t * ldz, wk + t, nr);
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
        for (int i = t; i < k; i += NT) d = fma(zs[i], zt[i], d);
        d = block_sum_n<NT>(d, shw);
        for (int i = t; i < k; i += NT) zt[i] -= d * zs[i];
        __syncthreads();
      }
      double nn = 0.0;
      for (int i = t; i < k; i += NT) nn = fma(zt[i], zt[i], nn);
      nn = block_sum_n<NT>(nn, shw);
      const double inv = 1.0 / sqrt(nn);
      for (int i = t; i < k; i += NT) zt[i] *= inv;
      __syncthreads();
    }
  }
}

}  // namespace
}  // namespace mds

#endif
