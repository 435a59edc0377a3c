// Affine form of Gower's interpolation for squared Euclidean distances.
// Eq. (2) gives y = W'(c - |x|^2 1 + 2 M x); the columns of V sum to zero
// (Q1 1 = 0, Section 2), so the |x|^2 term vanishes and
//     y = A x + b,   A = 2 W' M (r x p),   b = W' c,
// both formed at fit time.  Per row this is 2 p r flops against 4 (p + r)
// bytes, so the kernel streams X once and is bound by memory bandwidth.
// It is exact in exact arithmetic and avoids the cancellation of the
// distance form; the distance-block path (mds_embed) remains the method's
// own computation.
//
// The contraction over p runs on the matrix cores (FP32 or FP64 MFMA),
// which keeps the kernel at the memory bound with wide row loads.  A row's
// result does not depend on the other rows.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "mds_internal.h"

namespace mds {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline f4 af_mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline d4 af_mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Four consecutive elements of a row from column k0 (zero beyond p).
template <typename TX, typename T>
__device__ inline void af_load4(const TX* __restrict__ src, int64_t k0, int64_t p, bool vec, bool ok,
                                T out[4]) {
  if (ok && vec && k0 + 3 < p) {
    if constexpr (sizeof(TX) == 4) {
      const f4 v = *reinterpret_cast<const f4*>(src + k0);
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q] = (T)v[q];
    } else {
      typedef double d2 __attribute__((ext_vector_type(2)));
      const d2 v0 = *reinterpret_cast<const d2*>(src + k0);
      const d2 v1 = *reinterpret_cast<const d2*>(src + k0 + 2);
      out[0] = (T)v0[0];
      out[1] = (T)v0[1];
      out[2] = (T)v1[0];
      out[3] = (T)v1[1];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = (ok && k0 + q < p) ? (T)src[k0 + q] : (T)0;
  }
}

// groups of 16 rows per wave: as many as the registers allow
template <typename T, int RB>
constexpr int af_groups() {
  return sizeof(T) == 8 ? (RB == 1 ? 2 : 1) : (RB <= 2 ? 4 : 2);
}

// A wave owns AF_RG groups of 16 rows and RB tiles of 16 output columns.
// Per 32 columns of X, lane l loads X[row l%16 of each group][32j + 8(l/16)
// + 0..7] (whole 128-byte lines per row) and A[col l%16][the same eight
// columns], shared by the groups; eight MFMAs (16x16x4) per group and tile
// consume them, slot l/16 of step s standing for column 32j + 8(l/16) + s
// on both operands, so the sum over the columns is unchanged by the
// permutation.  Each output is one MFMA accumulation chain over the
// columns in a fixed order.
template <typename TX, typename T, int RB>
__global__ __launch_bounds__(256) void k_embed_affine(const TX* __restrict__ X, int64_t n, int64_t ldx,
                                                      int64_t p, const T* __restrict__ A,
                                                      const T* __restrict__ b, int r,
                                                      T* __restrict__ Y, int64_t ldy, int xvec,
                                                      int avec) {
  using Acc = typename std::conditional<std::is_same<T, double>::value, d4, f4>::type;
  constexpr int AF_RG = af_groups<T, RB>();
  constexpr int ROWS = 16 * AF_RG;  // rows per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rr = lane & 15, kq = lane >> 4;
  const int64_t rowbase = ((int64_t)blockIdx.x * 4 + wave) * ROWS;
  Acc acc[AF_RG][RB];
#pragma unroll
  for (int g = 0; g < AF_RG; ++g)
#pragma unroll
    for (int tb = 0; tb < RB; ++tb) acc[g][tb] = Acc{0, 0, 0, 0};
  const TX* xs[AF_RG];
  bool rok[AF_RG];
#pragma unroll
  for (int g = 0; g < AF_RG; ++g) {
    const int64_t row = rowbase + 16 * g + rr;
    rok[g] = row < n;
    xs[g] = X + (rok[g] ? row : 0) * ldx + 8 * kq;  // rows past n read row 0, never stored
  }
  const T* as[RB];
#pragma unroll
  for (int tb = 0; tb < RB; ++tb) {
    const int col = 16 * tb + rr;
    as[tb] = A + (int64_t)(col < r ? col : 0) * p + 8 * kq;  // columns past r are never stored
  }
  // Full 32-column chunks with aligned rows: unmasked loads, the next
  // chunk's loads in flight during the current chunk's MFMAs.
  const int64_t pfull = (xvec && avec) ? (p / 32) * 32 : 0;
  if (pfull > 0) {
    T xc[AF_RG][8], ac[RB][8];
#pragma unroll
    for (int g = 0; g < AF_RG; ++g) {
      af_load4<TX, T>(xs[g], 0, 4, true, true, xc[g]);
      af_load4<TX, T>(xs[g], 4, 8, true, true, xc[g] + 4);
    }
#pragma unroll
    for (int tb = 0; tb < RB; ++tb) {
      af_load4<T, T>(as[tb], 0, 4, true, true, ac[tb]);
      af_load4<T, T>(as[tb], 4, 8, true, true, ac[tb] + 4);
    }
    for (int64_t j0 = 0; j0 < pfull; j0 += 32) {
      const int64_t jn = (j0 + 32 < pfull) ? j0 + 32 : j0;  // the last step reloads its own chunk
      T xn[AF_RG][8], an[RB][8];
#pragma unroll
      for (int g = 0; g < AF_RG; ++g) {
        af_load4<TX, T>(xs[g], jn, jn + 4, true, true, xn[g]);
        af_load4<TX, T>(xs[g], jn + 4, jn + 8, true, true, xn[g] + 4);
      }
#pragma unroll
      for (int tb = 0; tb < RB; ++tb) {
        af_load4<T, T>(as[tb], jn, jn + 4, true, true, an[tb]);
        af_load4<T, T>(as[tb], jn + 4, jn + 8, true, true, an[tb] + 4);
      }
#pragma unroll
      for (int g = 0; g < AF_RG; ++g)
#pragma unroll
        for (int tb = 0; tb < RB; ++tb)
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[g][tb] = af_mfma(xc[g][q], ac[tb][q], acc[g][tb]);
#pragma unroll
      for (int g = 0; g < AF_RG; ++g)
#pragma unroll
        for (int q = 0; q < 8; ++q) xc[g][q] = xn[g][q];
#pragma unroll
      for (int tb = 0; tb < RB; ++tb)
#pragma unroll
        for (int q = 0; q < 8; ++q) ac[tb][q] = an[tb][q];
    }
  }
  for (int64_t j0 = pfull; j0 < p; j0 += 32) {  // ragged tail or unaligned input
    const int64_t k0 = j0 + 8 * kq;
    T av[RB][8];
#pragma unroll
    for (int tb = 0; tb < RB; ++tb) {
      const int col = 16 * tb + rr;
      const T* ar = A + (int64_t)(col < r ? col : 0) * p;
      af_load4<T, T>(ar, k0, p, avec != 0, col < r, av[tb]);
      af_load4<T, T>(ar, k0 + 4, p, avec != 0, col < r, av[tb] + 4);
    }
#pragma unroll
    for (int g = 0; g < AF_RG; ++g) {
      const TX* xr = xs[g] - 8 * kq;
      T xv[8];
      af_load4<TX, T>(xr, k0, p, xvec != 0, rok[g], xv);
      af_load4<TX, T>(xr, k0 + 4, p, xvec != 0, rok[g], xv + 4);
#pragma unroll
      for (int tb = 0; tb < RB; ++tb)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[g][tb] = af_mfma(xv[q], av[tb][q], acc[g][tb]);
    }
  }
  // Write through LDS: the wave's outputs are staged as a ROWS x r tile,
  // then stored with lanes running along the rows, so a wave writes whole
  // consecutive rows of Y (one contiguous range when ldy == r).
  __shared__ T tile[4][ROWS][16 * RB + 1];
#pragma unroll
  for (int tb = 0; tb < RB; ++tb)
#pragma unroll
    for (int g = 0; g < AF_RG; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // result layout: FP32 rows 4(l/16) + v, FP64 rows l/16 + 4v
        const int i = std::is_same<T, double>::value ? kq + 4 * v : 4 * kq + v;
        tile[wave][16 * g + i][16 * tb + rr] = acc[g][tb][v];
      }
  __builtin_amdgcn_wave_barrier();
  const int64_t left = n - rowbase;
  const int nrows = (int)(left < ROWS ? (left > 0 ? left : 0) : ROWS);
  for (int e = lane; e < nrows * r; e += 64) {
    const int i = e / r, col = e - (e / r) * r;
    Y[(rowbase + i) * ldy + col] = tile[wave][i][col] + b[col];
  }
}

template <typename TX, typename T, int RB>
void launch_af_rb(const TX* x, int64_t n, int64_t ldx, int64_t p, const T* A, const T* b, int r, T* y,
                  int64_t ldy, int xvec, int avec, hipStream_t st) {
  constexpr int rows = 64 * af_groups<T, RB>();
  const int64_t blocks = (n + rows - 1) / rows;
  k_embed_affine<TX, T, RB><<<(unsigned)blocks, 256, 0, st>>>(x, n, ldx, p, A, b, r, y, ldy, xvec, avec);
}

template <typename TX, typename T>
hipError_t launch_af(const T* A, const T* b, int64_t p, int r, const void* X, int64_t n, int64_t ldx,
                     void* Y, int64_t ldy, hipStream_t st) {
  const TX* x = static_cast<const TX*>(X);
  T* y = static_cast<T*>(Y);
  const int xvec = ((reinterpret_cast<uintptr_t>(X) % 16) == 0 && (ldx * (int64_t)sizeof(TX)) % 16 == 0);
  const int avec = ((reinterpret_cast<uintptr_t>(A) % 16) == 0 && (p * (int64_t)sizeof(T)) % 16 == 0);
  switch ((r + 15) / 16) {
    case 1: launch_af_rb<TX, T, 1>(x, n, ldx, p, A, b, r, y, ldy, xvec, avec, st); break;
    case 2: launch_af_rb<TX, T, 2>(x, n, ldx, p, A, b, r, y, ldy, xvec, avec, st); break;
    case 3: launch_af_rb<TX, T, 3>(x, n, ldx, p, A, b, r, y, ldy, xvec, avec, st); break;
    default: launch_af_rb<TX, T, 4>(x, n, ldx, p, A, b, r, y, ldy, xvec, avec, st); break;
  }
  return hipGetLastError();
}

}  // namespace

mds_status launch_affine_raw(const void* A, const void* b, int prec64, int64_t p, int r, const void* X,
                             int dt, int64_t n, int64_t ldx, void* Y, int64_t ldy, hipStream_t st) {
  hipError_t e;
  if (prec64) {
    const double* a = static_cast<const double*>(A);
    const double* bb = static_cast<const double*>(b);
    e = (dt == MDS_F64) ? launch_af<double, double>(a, bb, p, r, X, n, ldx, Y, ldy, st)
                        : launch_af<float, double>(a, bb, p, r, X, n, ldx, Y, ldy, st);
  } else {
    e = launch_af<float, float>(static_cast<const float*>(A), static_cast<const float*>(b), p, r, X, n,
                                ldx, Y, ldy, st);
  }
  if (e != hipSuccess) return hip_fail(e, "affine embed");
  return MDS_OK;
}

mds_status launch_embed_affine(const Model& m, int prec64, const void* X, int dt, int64_t n,
                               int64_t ldx, void* Y, int64_t ldy, hipStream_t st) {
  return launch_affine_raw(prec64 ? m.aff64 : m.aff32, prec64 ? m.affb64 : m.affb32, prec64, m.p, m.r,
                           X, dt, n, ldx, Y, ldy, st);
}

}  // namespace mds
