// Embedding from given squared dissimilarities (Section 2 states MDS on a
// dissimilarity matrix; eq. (2) needs only A21^2 and the fitted model):
//     y = sum_j (q_j - a_j) W_j,   W = 1/2 V Lambda^{-1/2}.
// The n x l input block is read once from HBM, so this kernel is bound by
// memory bandwidth (4 or 8 bytes per element against 2 r flops).
//
// A 256-thread block owns 64 rows and walks the landmarks 64 at a time.
// Each chunk of A2 is loaded with coalesced 16-byte loads, turned into
// e = q - a on its way into LDS (double-buffered, one barrier per chunk),
// and projected with MFMA: each wave accumulates Y^T (16 columns x its 16
// rows) += W^T E^T over the chunk.  The per-row reduction order is fixed.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "mds_internal.h"

namespace mds {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int SQ_BM = 64;   // rows per block
constexpr int SQ_LC = 64;   // landmarks per chunk

__device__ inline f4 sq_mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline d4 sq_mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Element layout of the MFMA result: FP64 interleaves rows, FP32 blocks them.
template <typename T>
__device__ constexpr int sq_row(int g, int v) {
  return std::is_same<T, double>::value ? g + 4 * v : 4 * g + v;
}

// TA: element type of A2; T: arithmetic type (float or double).
// W layout: FP32 column-major (16 rb) x l_pad with leading dimension ldw;
//           FP64 row-major l_pad x (16 rb) with leading dimension ldw.
template <typename TA, typename T, int RB>
__global__ __launch_bounds__(256) void k_embed_sq(const TA* __restrict__ A2, int64_t n, int64_t lda,
                                                  int l, const T* __restrict__ q,
                                                  const T* __restrict__ W, int64_t ldw, int r,
                                                  T* __restrict__ Y, int64_t ldy) {
  using Acc = typename std::conditional<std::is_same<T, double>::value, d4, f4>::type;
  constexpr int EPS = 16 / sizeof(TA);           // A2 elements per 16-byte load
  constexpr int SEGS = SQ_BM * SQ_LC / EPS / 256; // loads per thread per chunk
  constexpr int EROW = SQ_LC + 16 / (int)sizeof(T);  // LDS row stride (elements)
  constexpr int WN = 16 * RB;                    // weight columns staged
  constexpr int WPER = SQ_LC * WN / 256;         // weights per thread per chunk
  __shared__ __align__(16) T Es[2][SQ_BM][EROW];
  __shared__ __align__(16) T Ws[2][SQ_LC][WN];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * SQ_BM;
  const int nrows = (int)((n - row0) < SQ_BM ? (n - row0) : SQ_BM);
  const TA* Ab = A2 + row0 * lda;
  const bool avec = ((((uintptr_t)A2) & 15) == 0) && ((lda * (int64_t)sizeof(TA)) % 16 == 0);
  const int nchunks = (l + SQ_LC - 1) / SQ_LC;

  // Thread t always covers the same EPS-wide column segment of a chunk and
  // rows (t / SPR) + RSTEP u; so q is one vector per chunk.
  constexpr int SPR = SQ_LC / EPS;     // segments per row
  constexpr int RSTEP = 256 / SPR;     // rows between a thread's segments
  const int cseg = t % SPR;
  const int rbase = t / SPR;
  TA ar[SEGS][EPS];
  T qr[EPS];
  T wr[WPER];
  Acc yacc[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) yacc[b] = Acc{0, 0, 0, 0};

  auto load = [&](int c) {
    const int l0 = c * SQ_LC;
    const int j0 = l0 + cseg * EPS;
#pragma unroll
    for (int i = 0; i < EPS; ++i) qr[i] = q[j0 + i];  // q is zero-padded to l_pad
#pragma unroll
    for (int u = 0; u < SEGS; ++u) {
      const int row = rbase + RSTEP * u;
      const bool rin = row < nrows;
      if (rin && avec && j0 + EPS <= l) {
        const u4 raw = *reinterpret_cast<const u4*>(Ab + (int64_t)row * lda + j0);
        __builtin_memcpy(&ar[u][0], &raw, 16);
      } else {
#pragma unroll
        for (int i = 0; i < EPS; ++i)
          ar[u][i] = (rin && j0 + i < l) ? Ab[(int64_t)row * lda + j0 + i] : (TA)0;
      }
    }
#pragma unroll
    for (int k = 0; k < WPER; ++k) {
      const int e = t + 256 * k;
      if constexpr (std::is_same<T, double>::value) {
        wr[k] = W[(int64_t)(l0 + e / WN) * ldw + e % WN];         // row-major: coalesced
      } else {
        wr[k] = W[(int64_t)(e / SQ_LC) * ldw + l0 + e % SQ_LC];  // column-major: coalesced
      }
    }
  };
  auto store = [&](int buf, int c) {
    const int l0 = c * SQ_LC;
    const int jj = cseg * EPS;
#pragma unroll
    for (int u = 0; u < SEGS; ++u) {
      const int row = rbase + RSTEP * u;
#pragma unroll
      for (int i = 0; i < EPS; ++i)
        Es[buf][row][jj + i] = (l0 + jj + i < l) ? qr[i] - (T)ar[u][i] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < WPER; ++k) {
      const int e = t + 256 * k;
      if constexpr (std::is_same<T, double>::value)
        Ws[buf][e / WN][e % WN] = wr[k];
      else
        Ws[buf][e % SQ_LC][e / SQ_LC] = wr[k];
    }
  };

  load(0);
  store(0, 0);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) load(c + 1);
#pragma unroll 4
    for (int s = 0; s < SQ_LC / 4; ++s) {
      const T b = Es[buf][16 * wave + lr][4 * s + lg];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) yacc[rb] = sq_mfma(Ws[buf][4 * s + lg][16 * rb + lr], b, yacc[rb]);
    }
    if (c + 1 < nchunks) store(buf ^ 1, c + 1);
    __syncthreads();
  }
  const int row = 16 * wave + lr;
  if (row < nrows) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * rb + sq_row<T>(lg, v);
        if (col < r) Y[(row0 + row) * ldy + col] = yacc[rb][v];
      }
  }
}

template <typename TA, typename T>
hipError_t launch_sq(const Model& m, const void* A2, int64_t n, int64_t lda, void* Y, int64_t ldy,
                     hipStream_t st) {
  const int grid = (int)((n + SQ_BM - 1) / SQ_BM);
  const T* q = reinterpret_cast<const T*>(std::is_same<T, double>::value ? m.q64 : m.q32);
  const T* W = reinterpret_cast<const T*>(std::is_same<T, double>::value ? m.w64 : m.w32);
  const int64_t ldw = std::is_same<T, double>::value ? (int64_t)16 * m.rb : m.l_pad;
  const TA* a = reinterpret_cast<const TA*>(A2);
  T* y = reinterpret_cast<T*>(Y);
  switch (m.rb) {
    case 1: k_embed_sq<TA, T, 1><<<grid, 256, 0, st>>>(a, n, lda, (int)m.l, q, W, ldw, m.r, y, ldy); break;
    case 2: k_embed_sq<TA, T, 2><<<grid, 256, 0, st>>>(a, n, lda, (int)m.l, q, W, ldw, m.r, y, ldy); break;
    default: k_embed_sq<TA, T, 4><<<grid, 256, 0, st>>>(a, n, lda, (int)m.l, q, W, ldw, m.r, y, ldy); break;
  }
  return hipGetLastError();
}

}  // namespace

mds_status launch_embed_sqdist(const Model& m, int prec64, const void* A2, int dt, int64_t n,
                               int64_t lda, void* Y, int64_t ldy, hipStream_t st) {
  hipError_t e;
  if (prec64)
    e = (dt == MDS_F64) ? launch_sq<double, double>(m, A2, n, lda, Y, ldy, st)
                        : launch_sq<float, double>(m, A2, n, lda, Y, ldy, st);
  else
    e = launch_sq<float, float>(m, A2, n, lda, Y, ldy, st);
  if (e != hipSuccess) return hip_fail(e, "embed from dissimilarities");
  return MDS_OK;
}

}  // namespace mds
