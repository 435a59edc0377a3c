// Embed: Gower's interpolation formula, eq. (2) of Section 3.1, as one
// fused kernel.  For a data row x and landmark j
//     d_j = |x|^2 + |m_j|^2 - 2 x.m_j          (squared distance, Section 2)
//     e_j = q_j - d_j = c_j - |x|^2 + 2 x.m_j  (c = q - |m|^2, fixed at fit)
//     y   = sum_j e_j W_j,   W = 1/2 V Lambda^{-1/2}
// which is eq. (2) with (1/l) X1 S1^{-1} = V Lambda^{-1/2} (Section 3.1).
// The n x l block of distances never leaves registers.
//
// Work decomposition (flash-attention shaped): a 256-thread block owns
// BM = 128 data rows and walks the landmarks BN = 128 at a time.  Four waves
// split the 128 x 128 tile into 2 x 2 quadrants of 64 rows x 64 landmarks.
// The contraction over p is staged through LDS in chunks of 128 bytes per
// row (double-buffered, one barrier per chunk):
//   FP32        32 values, v_mfma_f32_16x16x4_f32
//   FP64        16 values, v_mfma_f64_16x16x4_f64
//   split BF16  32 hi + 32 lo values, v_mfma_f32_16x16x32_bf16, four
//               products hi.hi + lo.hi + hi.lo + lo.lo with FP32
//               accumulation (a BF16 part carries 8 bits, so the lo.lo
//               term is 2^-16 of x.m, the order of what the split leaves
//               out, and worth keeping)
//   split FP16  hi.hi + lo.hi + hi.lo with FP16 operands scaled by a power
//               of two (11-bit parts: lo.lo is 2^-22 of x.m, dropped)
// The MFMA computes S^T (landmarks x rows), so its accumulator is directly
// the B operand of the projection MFMA Y^T += W^T E^T (no data movement);
// the epilogue e = c - |x|^2 + 2 S runs in between on the accumulator.
// The per-row reduction order is fixed (landmark tiles in order, then the
// two landmark halves of a block in order), so a row's result does not
// depend on the batch it arrives in.  Models with one 16-column output
// block run a 512-landmark variant further down when it pays (the choice
// is a function of the model alone): embed_tile_wide in FP32, and in the
// split precisions embed_tile_s3, which uses 32 x 32 x 16 products on
// data and landmark parts kept in separate hi and lo planes.  In FP32 the 16-value k-block holding
// value p - 1 is stored transposed in the landmark pack and in LDS, so the
// products past p can be skipped.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "mds_internal.h"

namespace mds {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

constexpr int ROW_BYTES = CHUNK_BYTES + 16;  // LDS row stride (16-byte pad)
constexpr int TILE_BYTES = BM * ROW_BYTES;
constexpr int LDS_BYTES = 4 * TILE_BYTES + BM * 8;

template <int MODE>
struct Tr {
  using T = float;   // epilogue / projection type
  using Acc = f4;
  static constexpr int E = 4;          // data elements per 16-byte segment
  static constexpr int KB = 2;         // MFMA k-blocks per chunk
  static constexpr int KBLK = 16;      // data elements per k-block
  static constexpr int CH = 32;        // data elements per chunk
};
template <>
struct Tr<MODE_F64> {
  using T = double;
  using Acc = d4;
  static constexpr int E = 2;
  static constexpr int KB = 2;
  static constexpr int KBLK = 8;
  static constexpr int CH = 16;
};
template <>
struct Tr<MODE_BF16> {
  using T = float;
  using Acc = f4;
  static constexpr int E = 4;
  static constexpr int CH = 32;
};
template <>
struct Tr<MODE_F16> : Tr<MODE_BF16> {};

// Row (within a 16-row MFMA block) held by accumulator element v of a lane
// in lane group g: the FP64 instruction interleaves rows, the others block.
template <int MODE>
__device__ constexpr int acc_row(int g, int v) {
  return MODE == MODE_F64 ? g + 4 * v : 4 * g + v;
}

__device__ inline f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename TX, int E>
struct Seg {
  TX v[E];
};

template <typename TX, int E>
__device__ inline Seg<TX, E> load_seg(const TX* __restrict__ rowp, int64_t k, int p, bool vec) {
  Seg<TX, E> s;
  if (vec && k + E <= p) {
    if constexpr (sizeof(TX) * E == 16) {
      const u4 raw = *reinterpret_cast<const u4*>(rowp + k);
      __builtin_memcpy(&s, &raw, 16);
    } else {
      const u2 raw = *reinterpret_cast<const u2*>(rowp + k);
      __builtin_memcpy(&s, &raw, 8);
    }
  } else {
#pragma unroll
    for (int i = 0; i < E; ++i) s.v[i] = (k + i < p) ? rowp[k + i] : (TX)0;
  }
  return s;
}

// One 128-row tile of data rows through every landmark tile.
//   rb_rt: 16-wide output column blocks actually used (<= RB)
template <int MODE, typename TX, int RB>
__device__ void embed_tile(const EmbedModelView& mv, const TX* __restrict__ X, int64_t ldx,
                           int nrows, void* __restrict__ Yv, int64_t ldy, char* lds) {
  using Tt = Tr<MODE>;
  using T = typename Tt::T;
  using Acc = typename Tt::Acc;
  constexpr int E = Tt::E;
  constexpr bool SPLIT = (MODE == MODE_BF16 || MODE == MODE_F16);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1;   // 64-row half
  const int wn = wave >> 1;  // 64-landmark half
  const int lr = lane & 15;
  const int lg = lane >> 4;
  const int p = mv.p;
  const int nch = mv.nchunks;
  const int ntl = mv.ntl;
  const int total = nch * ntl;
  const int rb_rt = mv.rb < RB ? mv.rb : RB;
  const int ldw = 16 * mv.rb;
  const bool xvec = ((((uintptr_t)X) & 15) == 0) && ((ldx * (int64_t)sizeof(TX)) % 16 == 0);

  char* Xs = lds;
  char* Ms = lds + 2 * TILE_BYTES;
  T* xnorm = reinterpret_cast<T*>(lds + 4 * TILE_BYTES);

  // loader mapping: segment u covers row (tid >> 3) + 32 u, 16-byte slot tid & 7
  const int lrow = tid >> 3;
  const int lseg = tid & 7;

  Acc acc[4][4];
  Acc yacc[4][RB];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < RB; ++b) yacc[a][b] = Acc{0, 0, 0, 0};
  }
  T nacc[4] = {0, 0, 0, 0};
  T xn[4] = {0, 0, 0, 0};
  Seg<TX, E> xr[4];
  u4 mr[4];
  int xlo_cur = 1;  // lo parts of the data chunk being computed are not all zero

  const char* mbase = reinterpret_cast<const char*>(mv.mpack);
  const T* cvec = reinterpret_cast<const T*>(mv.c);
  const T* wmat = reinterpret_cast<const T*>(mv.w);

  // Fast path: rows 16-byte aligned and p a multiple of the segment width, so
  // every segment is wholly inside or wholly outside the data; the loads
  // then issue without branches (clamped address, zero selected outside).
  const bool xfast = xvec && (p % E == 0) && (sizeof(TX) * E == 16);
  auto load_chunk = [&](int lt, int ch) {
    const int64_t k0 = (int64_t)ch * Tt::CH + lseg * E;
    if (xfast) {
      const bool kin = k0 < p;
      const int64_t kk = kin ? k0 : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = lrow + 32 * u;
        const bool in = kin && (row < nrows);
        const int64_t rr = (row < nrows) ? row : 0;
        const u4 raw = *reinterpret_cast<const u4*>(X + rr * ldx + kk);
        const u4 z = {0u, 0u, 0u, 0u};
        const u4 v = in ? raw : z;
        __builtin_memcpy(&xr[u], &v, 16);
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = lrow + 32 * u;
        if (row < nrows) {
          xr[u] = load_seg<TX, E>(X + (int64_t)row * ldx, k0, p, xvec);
        } else {
#pragma unroll
          for (int i = 0; i < E; ++i) xr[u].v[i] = (TX)0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t lm = (int64_t)lt * BN + lrow + 32 * u;
      mr[u] = *reinterpret_cast<const u4*>(mbase + (lm * nch + ch) * CHUNK_BYTES + lseg * 16);
    }
  };
  auto accumulate_norm = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const T x = (T)xr[u].v[i];
        nacc[u] = fma(x, x, nacc[u]);
      }
  };
  // returns 1 if any lo part of this thread's data is nonzero (split modes)
  auto store_chunk = [&](int buf, int ch) -> int {
    int lo_nz = 0;
    char* xb = Xs + buf * TILE_BYTES;
    char* mb = Ms + buf * TILE_BYTES;
    // FP32 tail k-block (the one holding value p - 1 when p is not a
    // multiple of 16) is stored transposed, as the FP32 landmark pack is
    const bool tail = (MODE == MODE_F32) && (p - (ch * 32 + (lseg >> 2) * 16) < 16);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = lrow + 32 * u;
      if constexpr (MODE == MODE_F32) {
        if (tail) {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            *reinterpret_cast<float*>(xb + row * ROW_BYTES + (lseg >> 2) * 64 + c * 16 + (lseg & 3) * 4) =
                (float)xr[u].v[c];
        } else {
          f4 v = {(float)xr[u].v[0], (float)xr[u].v[1], (float)xr[u].v[2], (float)xr[u].v[3]};
          *reinterpret_cast<f4*>(xb + row * ROW_BYTES + lseg * 16) = v;
        }
      } else if constexpr (MODE == MODE_F64) {
        d2 v = {(double)xr[u].v[0], (double)xr[u].v[1]};
        *reinterpret_cast<d2*>(xb + row * ROW_BYTES + lseg * 16) = v;
      } else {
        uint16_t hi[4], lo[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float x = (float)xr[u].v[i];
          if constexpr (MODE == MODE_BF16) {
            const __bf16 h = (__bf16)x;
            const __bf16 lw = (__bf16)(x - (float)h);
            hi[i] = __builtin_bit_cast(uint16_t, h);
            lo[i] = __builtin_bit_cast(uint16_t, lw);
            lo_nz |= ((float)lw != 0.0f);
          } else {
            x *= mv.prescale;
            const _Float16 h = (_Float16)x;
            const _Float16 lw = (_Float16)(x - (float)h);
            hi[i] = __builtin_bit_cast(uint16_t, h);
            lo[i] = __builtin_bit_cast(uint16_t, lw);
            lo_nz |= ((float)lw != 0.0f);
          }
        }
        u2 hv = {(uint32_t)hi[0] | ((uint32_t)hi[1] << 16), (uint32_t)hi[2] | ((uint32_t)hi[3] << 16)};
        u2 lv = {(uint32_t)lo[0] | ((uint32_t)lo[1] << 16), (uint32_t)lo[2] | ((uint32_t)lo[3] << 16)};
        *reinterpret_cast<u2*>(xb + row * ROW_BYTES + lseg * 8) = hv;
        *reinterpret_cast<u2*>(xb + row * ROW_BYTES + 64 + lseg * 8) = lv;
      }
      *reinterpret_cast<u4*>(mb + row * ROW_BYTES + lseg * 16) = mr[u];
    }
    return lo_nz;
  };

  auto compute_chunk = [&](int buf, int ch, bool do_xlo) {
    const char* xb = Xs + buf * TILE_BYTES;
    const char* mb = Ms + buf * TILE_BYTES;
    if constexpr (!SPLIT) {
#pragma unroll
      for (int kb = 0; kb < Tt::KB; ++kb) {
        const int rem = p - (ch * Tt::CH + kb * Tt::KBLK);
        if (rem <= 0) break;
        using V = typename std::conditional<MODE == MODE_F64, d2, f4>::type;
        V b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[j] = *reinterpret_cast<const V*>(xb + (64 * wm + 16 * j + lr) * ROW_BYTES + kb * 64 + lg * 16);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const V a = *reinterpret_cast<const V*>(mb + (64 * wn + 16 * i + lr) * ROW_BYTES + kb * 64 + lg * 16);
#pragma unroll
          for (int jj = 0; jj < 16 / (int)sizeof(T); ++jj)
            // FP32 tail k-block (transposed): product jj holds values
            // 4 jj .. 4 jj + 3, so those past p are skipped
            if (MODE == MODE_F64 || 4 * jj < rem)
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[jj], b[j][jj], acc[i][j]);
        }
      }
    } else {
      using V = typename std::conditional<MODE == MODE_BF16, bf8, h8>::type;
      V bh[4], bl[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const char* xa = xb + (64 * wm + 16 * j + lr) * ROW_BYTES + lg * 16;
        bh[j] = *reinterpret_cast<const V*>(xa);
        bl[j] = *reinterpret_cast<const V*>(xa + 64);
      }
      const bool do_mlo = !mv.m_lo_zero;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const char* ma = mb + (64 * wn + 16 * i + lr) * ROW_BYTES + lg * 16;
        const V ah = *reinterpret_cast<const V*>(ma);
        const V al = *reinterpret_cast<const V*>(ma + 64);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if constexpr (MODE == MODE_BF16) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
            if (do_mlo) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
            if (do_xlo) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
            if (do_mlo && do_xlo)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bl[j], acc[i][j], 0, 0, 0);
          } else {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[j], acc[i][j], 0, 0, 0);
            if (do_mlo) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[j], acc[i][j], 0, 0, 0);
            if (do_xlo) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }
  };

  // epilogue e = c - |x|^2 + 2 s and projection Y^T += W^T E^T for tile lt
  auto epilogue = [&](int lt) {
    const int64_t lbase = (int64_t)lt * BN + 64 * wn;
    const T two = SPLIT ? (T)(2.0f * mv.postscale) : (T)2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      T cv[4];
      if constexpr (MODE == MODE_F64) {
#pragma unroll
        for (int v = 0; v < 4; ++v) cv[v] = cvec[lbase + 16 * i + acc_row<MODE>(lg, v)];
      } else {
        // the lane's four landmarks are consecutive: one vector load
        const f4 c4 = *reinterpret_cast<const f4*>(cvec + lbase + 16 * i + 4 * lg);
#pragma unroll
        for (int v = 0; v < 4; ++v) cv[v] = c4[v];
      }
      Acc e[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) e[j][v] = (cv[v] - xn[j]) + two * acc[i][j][v];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb < rb_rt) {
          T wv[4];
          if constexpr (MODE == MODE_F64) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              wv[v] = wmat[(lbase + 16 * i + acc_row<MODE>(lg, v)) * ldw + 16 * rb + lr];
          } else {
            // FP32 weights are stored column-major (output column, landmark)
            const f4 w4 = *reinterpret_cast<const f4*>(wmat + (int64_t)(16 * rb + lr) * mv.ldwt +
                                                       lbase + 16 * i + 4 * lg);
#pragma unroll
            for (int v = 0; v < 4; ++v) wv[v] = w4[v];
          }
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int j = 0; j < 4; ++j) yacc[j][rb] = mfma(wv[v], e[j][v], yacc[j][rb]);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = Acc{0, 0, 0, 0};
    }
  };

  // ---- pipeline over (landmark tile, chunk) ----
  load_chunk(0, 0);
  accumulate_norm();
  {
    const int nz = store_chunk(0, 0);
    xlo_cur = __syncthreads_or(nz);
  }
  int lt = 0, ch = 0;
  for (int it = 0; it < total; ++it) {
    const int buf = it & 1;
    const bool has_next = it + 1 < total;
    const int nchn = (ch + 1 == nch) ? 0 : ch + 1;
    const int nlt = (ch + 1 == nch) ? lt + 1 : lt;
    if (has_next) load_chunk(nlt, nchn);
    compute_chunk(buf, ch, xlo_cur != 0);
    int nz = 0;
    if (has_next) {
      if (nlt == 0) accumulate_norm();
      nz = store_chunk(buf ^ 1, nchn);
    }
    const bool tile_end = (ch == nch - 1);
    if (tile_end && lt == 0) {
      // row norms: 8 lanes share each row; fixed butterfly order
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        T s = nacc[u];
        s += __shfl_xor(s, 4, 64);
        s += __shfl_xor(s, 2, 64);
        s += __shfl_xor(s, 1, 64);
        if (lseg == 0) xnorm[lrow + 32 * u] = s;
      }
    }
    xlo_cur = __syncthreads_or(nz);
    if (tile_end) {
      if (lt == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) xn[j] = xnorm[64 * wm + 16 * j + lr];
      }
      epilogue(lt);
    }
    lt = nlt;
    ch = nchn;
  }

  // ---- combine the two landmark halves (fixed order) and store ----
  __syncthreads();
  T* ysh = reinterpret_cast<T*>(lds);
  if (wn == 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) ysh[(((wm * 4 + j) * RB + rb) * 4 + v) * 64 + lane] = yacc[j][rb][v];
  }
  __syncthreads();
  if (wn == 0) {
    T* Y = reinterpret_cast<T*>(Yv);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 64 * wm + 16 * j + lr;
      if (row >= nrows) continue;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= rb_rt) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * rb + acc_row<MODE>(lg, v);
          const T val = yacc[j][rb][v] + ysh[(((wm * 4 + j) * RB + rb) * 4 + v) * 64 + lane];
          if (col < mv.r) Y[(int64_t)row * ldy + col] = val;
        }
      }
    }
  }
  __syncthreads();
}

// ---- FP32 with 512 landmarks per pass over the row tile ----
// The 128-landmark kernel moves one 128 x 32 data chunk and one 128 x 32
// landmark chunk through LDS per 128 x 128 x 32 block of products; its two
// blocks per CU tend to run in phase, so the copies and barriers add to the
// MFMA time instead of hiding under it.  With p in the hundreds a 128-row
// tile of X is also too large to stay in L2 while the block walks the
// landmarks, so every landmark tile re-reads it.  This variant keeps the
// 128-row tile but walks the landmarks WBN = 512 at a time: eight waves as
// 2 row halves x 4 landmark quarters, each 64 rows x 128 landmarks of
// accumulators, so a chunk copy feeds twice the products and X is read a
// quarter as often.  One chunk buffer (X 16 KB + landmarks 64 KB) is
// double-buffered, which fills the 160 KB of LDS; 16-byte segments are
// XOR-swizzled by row instead of padded, and the landmark operands are
// copied from memory straight into LDS (the FP32 pack is allocated to a
// multiple of WBN rows, zero past l_pad), as are aligned data chunks
// without a ragged k-block.  Each wave sums the row norms from the operands
// it reads.  The quarters are added in order at the end.  The landmark
// order of the sums differs from the 128-landmark variant, so each model
// always runs the same variant (plain and serving launches alike).  The
// split precisions use the same passes of 512 landmarks in embed_tile_s3.
constexpr int WBN = 512;
constexpr int WTHREADS = 512;
constexpr int WX_BYTES = BM * CHUNK_BYTES;
constexpr int WBUF_BYTES = WX_BYTES + WBN * CHUNK_BYTES;
constexpr int WLDS_BYTES = 2 * WBUF_BYTES;
static_assert(WBN == kSplitPackRows, "landmark packs are padded for this variant");

// s_waitcnt immediate for vmcnt(0) with the other counters left alone
constexpr int kWaitVm0 = 0x0F70;

// byte offset of 16-byte segment seg (0..7) in a 128-byte row of LDS: the
// XOR with bits 1..3 of the row puts the 16 rows read by 16 lanes (row
// pairs share a 256-byte line) on distinct 16-byte slots
__device__ inline int swz(int row, int seg) { return (seg ^ ((row >> 1) & 7)) << 4; }

// KTAIL: p may end inside a 16-value k-block, whose products past p are
// skipped by uniform branches.  With p a multiple of 16 those branches
// are always taken, so the form without them gives the same bits with
// fewer branches in the product loop.
template <int MODE, bool KTAIL>
__device__ void embed_tile_wide(const EmbedModelView& mv, const float* __restrict__ X, int64_t ldx,
                                int nrows, float* __restrict__ Y, int64_t ldy, char* lds) {
  static_assert(MODE == MODE_F32, "the split precisions run embed_tile_s3");
  constexpr int E = 4;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1;   // 64-row half
  const int wn = wave >> 1;  // 128-landmark quarter
  const int lr = lane & 15;
  const int lg = lane >> 4;
  const int p = mv.p;
  const int nch = mv.nchunks;
  const int64_t l_pad = (int64_t)mv.ntl * BN;
  const int nst = (int)((l_pad + WBN - 1) / WBN);
  const int total = nch * nst;
  const bool xvec = ((((uintptr_t)X) & 15) == 0) && ((ldx * (int64_t)sizeof(float)) % 16 == 0);
  const bool xfast = xvec && (p % E == 0);

  // loader mapping: X rows lrow + 64 u (u < 2), 16-byte slot lseg
  const int lrow = tid >> 3;
  const int lseg = tid & 7;

  f4 acc[8][4];  // [landmark block][row block]
  f4 yacc[4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};
#pragma unroll
  for (int b = 0; b < 4; ++b) yacc[b] = f4{0, 0, 0, 0};
  float xn[4] = {0.f, 0.f, 0.f, 0.f};
  Seg<float, E> xr[2];
  // each wave sums the squares of the data operands it reads in the
  // first pass (lane (lr, g) holds a quarter of row 16 j + lr), so the row
  // norms need no exchange, whichever way a chunk reached LDS
  float nrm[4] = {0.f, 0.f, 0.f, 0.f};

  // Landmark operands go from memory straight into LDS (16 bytes per lane,
  // no registers): wave load u of wave w fills the 1 KB of landmark rows
  // 64 u + 8 w .. + 8, lane L the physical segment L % 8 of row L / 8, so
  // it fetches the logical segment (L % 8) ^ ((row / 2) % 8).
  const int64_t mrow_bytes = (int64_t)nch * CHUNK_BYTES;
  const char* mlane = reinterpret_cast<const char*>(mv.mpack) +
                      (int64_t)(8 * wave + (lane >> 3)) * mrow_bytes +
                      (((lane & 7) ^ ((4 * (wave & 1) + (lane >> 4)) & 7)) << 4);
  auto dma_chunk = [&](int s, int ch, int buf) {
    char* mb = lds + buf * WBUF_BYTES + WX_BYTES + 8 * wave * CHUNK_BYTES;
    const char* src = mlane + (int64_t)s * WBN * mrow_bytes + (int64_t)ch * CHUNK_BYTES;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src + (int64_t)(64 * u) * mrow_bytes),
                                       (__attribute__((address_space(3))) void*)(mb + 64 * u * CHUNK_BYTES),
                                       16, 0, 0);
  };

  // Data chunks without a ragged k-block also go straight to LDS when
  // the rows are 16-byte aligned: wave copy u fills rows 64 u + 8 w .. + 8
  // with the same lane mapping as the landmark copies.  Rows past nrows
  // repeat the last row (their results are not stored); a segment that
  // starts past p re-reads the row's first segment (its k-block is never
  // computed), so every address stays inside the row.
  // (row addresses are formed at each copy: fewer live registers)
  const int xdseg = ((lane & 7) ^ ((4 * (wave & 1) + (lane >> 4)) & 7)) * E;
  // the chunk holds no computed k-block with values past p
  auto x_direct = [&](int ch) {
    if (!xfast) return false;
    const int r0 = p - ch * 32, r1 = r0 - 16;
    return !(r0 > 0 && r0 < 16) && !(r1 > 0 && r1 < 16);
  };
  auto dma_x = [&](int ch, int buf) {
    char* xb = lds + buf * WBUF_BYTES + 8 * wave * CHUNK_BYTES;
    const int k = ch * 32 + xdseg;
    const int64_t koff = k < p ? k : 0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int row = 64 * u + 8 * wave + (lane >> 3);
      const float* src = X + (int64_t)(row < nrows ? row : nrows - 1) * ldx + koff;
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                       (__attribute__((address_space(3))) void*)(xb + 64 * u * CHUNK_BYTES),
                                       16, 0, 0);
    }
  };

  auto load_chunk = [&](int ch) {
    const int64_t k0 = (int64_t)ch * 32 + lseg * E;
    if (xfast) {
      const bool kin = k0 < p;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        // the lane's 16-byte slot of row lrow + 64 u (the last row stands in
        // for rows past nrows, whose values are zeroed)
        const int row = lrow + 64 * u;
        const float* xrow = X + (int64_t)(row < nrows ? row : nrows - 1) * ldx + lseg * E;
        const bool in = kin && (row < nrows);
        const u4 raw = *reinterpret_cast<const u4*>(xrow + (kin ? (int64_t)ch * 32 : 0));
        const u4 z = {0u, 0u, 0u, 0u};
        const u4 v = in ? raw : z;
        __builtin_memcpy(&xr[u], &v, 16);
      }
    } else {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int row = lrow + 64 * u;
        if (row < nrows) {
          xr[u] = load_seg<float, E>(X + (int64_t)row * ldx, k0, p, xvec);
        } else {
#pragma unroll
          for (int i = 0; i < E; ++i) xr[u].v[i] = 0.f;
        }
      }
    }
  };
  auto store_chunk = [&](int buf, int ch) {
    char* xb = lds + buf * WBUF_BYTES;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int row = lrow + 64 * u;
      if (p - (ch * 32 + (lseg >> 2) * 16) < 16) {
        // tail k-block, transposed: value c of this segment goes to
        // segment 4 (lseg / 4) + c, slot lseg % 4
#pragma unroll
        for (int c = 0; c < 4; ++c)
          *reinterpret_cast<float*>(xb + row * CHUNK_BYTES + swz(row, 4 * (lseg >> 2) + c) + 4 * (lseg & 3)) =
              xr[u].v[c];
      } else {
        u4 v;
        __builtin_memcpy(&v, &xr[u], 16);
        *reinterpret_cast<u4*>(xb + row * CHUNK_BYTES + swz(row, lseg)) = v;
      }
    }
  };
  // Lane group g holds values 4 g .. 4 g + 3 of a k-block (the
  // tail k-block is stored transposed, so that product jj holds values
  // 4 jj .. 4 jj + 3 there and the products past p are skipped)
  auto compute_chunk_f32 = [&](int buf, int ch, bool norms) {
    const char* xb = lds + buf * WBUF_BYTES;
    const char* mb = xb + WX_BYTES;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const int rem = p - (ch * 32 + kb * 16);
      if (rem <= 0) break;
      f4 b[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 64 * wm + 16 * j + lr;
        b[j] = *reinterpret_cast<const f4*>(xb + row * CHUNK_BYTES + swz(row, 4 * kb + lg));
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int lm = 128 * wn + 16 * i + lr;
        const f4 a = *reinterpret_cast<const f4*>(mb + lm * CHUNK_BYTES + swz(lm, 4 * kb + lg));
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          if (!KTAIL || 4 * jj < rem)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[jj], b[j][jj], acc[i][j]);
      }
      // after the products, so that no branch separates the operand loads
      if (norms) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int c = 0; c < 4; ++c) nrm[j] = fma(b[j][c], b[j][c], nrm[j]);
      }
    }
  };
  // e = c - |x|^2 + 2 s and Y^T += W^T E^T for the wave's quarter of super tile s
  auto epilogue = [&](int s) {
    const float two = 2.0f;
    // (formed here rather than kept live across the chunk loop)
    const float* cb = reinterpret_cast<const float*>(mv.c) + (int64_t)s * WBN + 128 * wn + 4 * lg;
    const float* wb =
        reinterpret_cast<const float*>(mv.w) + (int64_t)lr * mv.ldwt + (int64_t)s * WBN + 128 * wn + 4 * lg;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const f4 c4 = *reinterpret_cast<const f4*>(cb + 16 * i);
      const f4 w4 = *reinterpret_cast<const f4*>(wb + 16 * i);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        f4 e;
#pragma unroll
        for (int v = 0; v < 4; ++v) e[v] = (c4[v] - xn[j]) + two * acc[i][j][v];
#pragma unroll
        for (int v = 0; v < 4; ++v) yacc[j] = mfma(w4[v], e[v], yacc[j]);
        acc[i][j] = f4{0, 0, 0, 0};
      }
    }
  };

  // ---- pipeline over (super tile, chunk) ----
  // The landmark copies of a chunk are waited for (vmcnt) before the
  // barrier that publishes the chunk.
  dma_chunk(0, 0, 0);
  if (x_direct(0)) {
    dma_x(0, 0);
  } else {
    load_chunk(0);
    store_chunk(0, 0);
  }
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  __syncthreads();
  int s = 0, ch = 0;
  for (int it = 0; it < total; ++it) {
    const int buf = it & 1;
    const bool has_next = it + 1 < total;
    const int nchn = (ch + 1 == nch) ? 0 : ch + 1;
    const int nsn = (ch + 1 == nch) ? s + 1 : s;
    // a quarter wholly past the padded landmark count does no work
    const bool live = (int64_t)s * WBN + 128 * wn < l_pad;
    const bool next_direct = has_next && x_direct(nchn);
    if (has_next) {
      dma_chunk(nsn, nchn, buf ^ 1);
      if (next_direct)
        dma_x(nchn, buf ^ 1);
      else
        load_chunk(nchn);
    }
    if (live) compute_chunk_f32(buf, ch, s == 0);
    if (has_next && !next_direct) store_chunk(buf ^ 1, nchn);
    const bool tile_end = (ch == nch - 1);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
    if (tile_end) {
      if (s == 0) {
        // fixed butterfly over the four lane groups: every lane of a row
        // gets the same bits
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float t = nrm[j];
          t += __shfl_xor(t, 16, 64);
          t += __shfl_xor(t, 32, 64);
          xn[j] = t;
        }
      }
      if (live) epilogue(s);
    }
    s = nsn;
    ch = nchn;
  }

  // ---- add the four landmark quarters in order and store ----
  __syncthreads();
  float* ysh = reinterpret_cast<float*>(lds);
  if (wn > 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) ysh[((((wn - 1) * 2 + wm) * 4 + j) * 4 + v) * 64 + lane] = yacc[j][v];
  }
  __syncthreads();
  if (wn == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 64 * wm + 16 * j + lr;
      if (row >= nrows) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 4 * lg + v;
        float val = yacc[j][v];
#pragma unroll
        for (int q = 0; q < 3; ++q) val += ysh[(((q * 2 + wm) * 4 + j) * 4 + v) * 64 + lane];
        if (col < mv.r) Y[(int64_t)row * ldy + col] = val;
      }
    }
  }
  __syncthreads();
}

// Barriers of the split kernel are raw s_barrier with an explicit wait that
// leaves the newest copies in flight; a compiler memory barrier keeps LDS
// accesses on their side of it.
__device__ inline void raw_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::: "memory");
}

// ---- split precisions with 32 x 32 x 16 matrix-core products ----
// A 512-thread block (two waves per SIMD) owns 128 data rows and walks the
// landmarks 512 at a time; wave (h, q) holds the 64 x 128 block of S^T for
// rows 64 h .. 64 h + 63 and landmarks 128 q .. 128 q + 127 of the pass
// (8 accumulators of 32 x 32).  Per 32-value chunk of the contraction:
//   * the landmark parts come from the chunk-major, pre-swizzled pack
//     straight into LDS (each wave's share is one contiguous 4 KB run), two
//     chunks ahead when the landmarks have no lo parts, else one;
//   * each thread loads 8 values of one data row of the next chunk into
//     registers before the products of this one, then splits them into 8 hi
//     and 8 lo 16-bit values and stores them in that chunk's hi and lo
//     planes (64-byte rows, 16-byte segments swizzled on row bits 2..3), so
//     a lane reads its 32 x 32 x 16 operand (8 values of one row) with one
//     16-byte read;
//   * the products with the data lo parts are skipped for a chunk in which
//     every data lo part is zero (they would add exact zeros), decided once
//     per chunk from flags the splitting waves publish;
//   * one barrier per chunk: chunk it + 1 is split while chunk it is
//     multiplied.
// The 32 x 32 accumulators feed the projection directly: for accumulator
// register v, lane quarter b holds 16 rows x 1 landmark, the B operand of
// block b of v_mfma_f32_16x16x1_4b_f32, whose A operand is the W row of
// that landmark; blocks 0 + 2 and 1 + 3 are added at the end.
constexpr int S3_THREADS = 512;
constexpr int S3_XP = BM * 64;   // one part of a data chunk: 128 rows x 32 16-bit values
constexpr int S3_M = WBN * 64;   // one part of a landmark chunk: 512 x 32 16-bit values
template <bool HI>
constexpr int s3_nbuf() { return HI ? 3 : 2; }
template <bool HI>
constexpr int s3_buf() { return 2 * S3_XP + (HI ? 1 : 2) * S3_M; }
template <bool HI>
constexpr int s3_lds() { return s3_nbuf<HI>() * s3_buf<HI>() + (HI ? 128 : 0); }
static_assert(s3_lds<true>() <= 163840 && s3_lds<false>() <= 163840, "LDS of the split kernels");

typedef float f16v __attribute__((ext_vector_type(16)));

// s_waitcnt immediate: vmcnt(vm) (6 bits, split over two fields) and
// lgkmcnt(lgkm), expcnt left alone
constexpr int wait_imm(int vm, int lgkm) { return (vm & 15) | ((vm >> 4) << 14) | (7 << 4) | (lgkm << 8); }

__device__ inline f16v mfma32(const bf8& a, const bf8& b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ inline f16v mfma32(const h8& a, const h8& b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// byte offset of 16-byte segment g (0..3) of row `row` in a plane of 64-byte rows
__device__ inline int s3_off(int row, int g) { return row * 64 + ((g ^ ((row >> 2) & 3)) << 4); }

// Data part of a buffer: 8 regions of 16 rows, each a 1 KB hi plane then a
// 1 KB lo plane; the 16 bytes holding values 8 g .. 8 g + 7 of row `row`
// sit in slot 4 (row & 15) + (g ^ ((row >> 1) & 3)) of its region's plane.
// Slot L of a region belongs to lane L of wave `region`, which is how a
// direct copy into LDS lays out 64 lanes x 16 bytes.
constexpr int S3_XLO = 1024;  // lo plane after the hi plane of a region
__device__ inline int s3_xoff(int row, int g) {
  return (row >> 4) * 2048 + ((((row & 15) << 2) + (g ^ ((row >> 1) & 3))) << 4);
}

// XDMA (landmarks without lo parts, 16-byte aligned rows, p a multiple of 4):
// the data chunks are copied straight into LDS as well, and each thread
// splits its own 32 bytes there in place, so every memory operation of the
// chunk loop is a copy into LDS and the waits count them exactly.
template <int MODE, bool HI, bool XDMA>
__device__ void embed_tile_s3(const EmbedModelView& mv, const float* __restrict__ X, int64_t ldx,
                              int nrows, float* __restrict__ Y, int64_t ldy, char* lds) {
  static_assert(!XDMA || HI, "direct data copies need the third buffer");
  using V = typename std::conditional<MODE == MODE_BF16, bf8, h8>::type;
  constexpr int NBUF = s3_nbuf<HI>();
  constexpr int BUF = s3_buf<HI>();
  constexpr int MAHEAD = NBUF - 1;  // landmark copies run this many chunks ahead
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1;   // 64-row half
  const int wn = wave >> 1;  // 128-landmark quarter of the pass
  const int l31 = lane & 31;
  const int half = lane >> 5;
  const int p = mv.p;
  const int nch = mv.nchunks;
  const int64_t l_pad = (int64_t)mv.ntl * BN;
  const int nst = (int)((l_pad + WBN - 1) / WBN);
  const int total = nch * nst;
  const bool xvec = ((((uintptr_t)X) & 15) == 0) && ((ldx * (int64_t)sizeof(float)) % 16 == 0);
  const bool xfast = xvec && (p % 4 == 0);
  int* flags = reinterpret_cast<int*>(lds + NBUF * BUF);  // HI: [NBUF][8 waves]

  f16v acc[4][2];    // [landmark block][row block]
  float ysum[2][8];  // running projection over the passes: [row block][value]
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int v = 0; v < 8; ++v) ysum[j][v] = 0.f;
  float nacc = 0.f;
  float xn[2] = {0.f, 0.f};

  // data: thread owns values 8 gx .. 8 gx + 7 of row xrow of each chunk, gx
  // chosen so that its hi and lo parts sit in slot `lane` of its wave's
  // region; byte offsets inside the tile are 32-bit, chunk offsets uniform
  const int xrow = tid >> 2;
  const int q8 = tid & 3;
  const int gx = q8 ^ ((xrow >> 1) & 3);
  const char* xbase = reinterpret_cast<const char*>(X);
  const uint32_t xrow_off = (uint32_t)((int64_t)(xrow < nrows ? xrow : nrows - 1) * ldx * 4);
  const uint32_t xoff = xrow_off + 32u * (uint32_t)gx;
  const int sw_off = s3_xoff(xrow, gx);  // = 2048 wave + 16 lane
  f4 xa[2], xb[2];                     // 8 values of two chunks in flight
  auto load_x = [&](int ch, auto slot_tag) {
    constexpr int SL = decltype(slot_tag)::value;
    f4& xa_ = xa[SL];
    f4& xb_ = xb[SL];
    if (xfast) {
      if (32 * ch + 32 <= p) {
        const char* cb = xbase + (int64_t)ch * 128;
        xa_ = *reinterpret_cast<const f4*>(cb + xoff);
        xb_ = *reinterpret_cast<const f4*>(cb + xoff + 16);
      } else {
        // last chunk: rows past nrows repeat the last row; a 16-byte piece
        // past p (p is a multiple of 4) re-reads the row's first values
        // instead (finite, zeroed by the split), so no read leaves the row
        const int k = 32 * ch + 8 * gx;
        xa_ = *reinterpret_cast<const f4*>(xbase + (k < p ? (int64_t)ch * 128 + xoff : xrow_off));
        xb_ = *reinterpret_cast<const f4*>(xbase + (k + 4 < p ? (int64_t)ch * 128 + xoff + 16 : xrow_off));
      }
    } else {
      const int k = 32 * ch + 8 * gx;
      Seg<float, 4> v0, v1;
      if (xrow < nrows) {
        v0 = load_seg<float, 4>(X + (int64_t)xrow * ldx, k, p, xvec);
        v1 = load_seg<float, 4>(X + (int64_t)xrow * ldx, k + 4, p, xvec);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v0.v[e] = v1.v[e] = 0.f;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        xa_[e] = v0.v[e];
        xb_[e] = v1.v[e];
      }
    }
  };
  // split of chunk ch's 8 values (x) into buffer b; returns whether a data
  // lo part is nonzero
  auto split_vals = [&](float (&x)[8], int ch, int b, bool norms) -> bool {
    if (32 * ch + 32 > p) {
      const int k0 = 32 * ch + 8 * gx;
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (k0 + e < p) ? x[e] : 0.f;
    }
    if (norms) {
#pragma unroll
      for (int e = 0; e < 8; ++e) nacc = fma(x[e], x[e], nacc);
    }
    uint32_t hi[4], lo[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      if constexpr (MODE == MODE_BF16) {
        typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
        typedef float fl2 __attribute__((ext_vector_type(2)));
        const fl2 xv = {x[e], x[e + 1]};
        const bf2 h = __builtin_convertvector(xv, bf2);
        const uint32_t hb = __builtin_bit_cast(uint32_t, h);
        const fl2 hf = {__builtin_bit_cast(float, hb << 16), __builtin_bit_cast(float, hb & 0xffff0000u)};
        const fl2 d = {xv[0] - hf[0], xv[1] - hf[1]};
        hi[e >> 1] = hb;
        lo[e >> 1] = __builtin_bit_cast(uint32_t, __builtin_convertvector(d, bf2));
      } else {
        typedef _Float16 hf2 __attribute__((ext_vector_type(2)));
        typedef float fl2 __attribute__((ext_vector_type(2)));
        const fl2 xv = {x[e] * mv.prescale, x[e + 1] * mv.prescale};
        const hf2 h = __builtin_convertvector(xv, hf2);
        const fl2 hf = __builtin_convertvector(h, fl2);
        const fl2 d = {xv[0] - hf[0], xv[1] - hf[1]};
        hi[e >> 1] = __builtin_bit_cast(uint32_t, h);
        lo[e >> 1] = __builtin_bit_cast(uint32_t, __builtin_convertvector(d, hf2));
      }
    }
    char* xh = lds + b * BUF + sw_off;
    *reinterpret_cast<u4*>(xh) = u4{hi[0], hi[1], hi[2], hi[3]};
    *reinterpret_cast<u4*>(xh + S3_XLO) = u4{lo[0], lo[1], lo[2], lo[3]};
    return ((lo[0] | lo[1]) | (lo[2] | lo[3])) != 0u;
  };
  // from the register slot the values were loaded into
  auto split = [&](int ch, int b, bool norms, auto slot_tag) -> bool {
    constexpr int SL = decltype(slot_tag)::value;
    float x[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x[e] = xa[SL][e];
      x[4 + e] = xb[SL][e];
    }
    return split_vals(x, ch, b, norms);
  };
  // in place, from the thread's own two copied 16-byte pieces in buffer b
  auto split_lds = [&](int ch, int b, bool norms) -> bool {
    const char* xh = lds + b * BUF + sw_off;
    const f4 va = *reinterpret_cast<const f4*>(xh);
    const f4 vb = *reinterpret_cast<const f4*>(xh + S3_XLO);
    float x[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x[e] = va[e];
      x[4 + e] = vb[e];
    }
    return split_vals(x, ch, b, norms);
  };
  // data copies of chunk ch into buffer b: lane L copies the 16-byte pieces
  // u = 0, 1 of its values (raw FP32) into slot L of its region's planes u;
  // a piece past p re-reads the row's first values (zeroed by the split)
  auto dma_x = [&](int ch, int b) {
    char* xb_ = lds + b * BUF + wave * 2048;
    const int k = 32 * ch + 8 * gx;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const char* src = xbase + (k + 4 * u < p ? (int64_t)ch * 128 + xoff + 16 * u : (int64_t)xrow_off);
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                       (__attribute__((address_space(3))) void*)(xb_ + u * S3_XLO), 16, 0, 0);
    }
  };
  // landmark copies of chunk (s, ch) into buffer b: wave w copies bytes
  // [4096 w, 4096 w + 4096) of each part
  const int64_t plane = (int64_t)nch * mv.lsplit * 64;
  const uint32_t mlane = (uint32_t)lane * 16u;
  auto dma_m = [&](int s, int ch, int b) {
    const char* src = reinterpret_cast<const char*>(mv.spack) +
                      ((int64_t)ch * mv.lsplit + (int64_t)s * WBN) * 64 + wave * 4096;
    char* mb = lds + b * BUF + 2 * S3_XP + wave * 4096;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src + mlane + u * 1024),
                                       (__attribute__((address_space(3))) void*)(mb + u * 1024), 16, 0, 0);
    if constexpr (!HI) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src + plane + mlane + u * 1024),
                                         (__attribute__((address_space(3))) void*)(mb + S3_M + u * 1024), 16, 0,
                                         0);
    }
  };

  // operand offsets: data row block j adds 4096 bytes (two regions) and
  // landmark block i 2048 (32 rows of 64 bytes); the swizzles depend on row
  // bits 1..3 only
  const int bo0 = s3_xoff(64 * wm + l31, half), bo1 = s3_xoff(64 * wm + l31, 2 + half);
  const int ao0 = s3_off(128 * wn + l31, half), ao1 = s3_off(128 * wn + l31, 2 + half);
  // products of the chunk in buffer b: first those with the data hi parts
  // (hi.hi, then lo.hi when the landmarks have lo parts) for both k-steps,
  // then, when do_xlo, those with the data lo parts (hi.lo, lo.lo)
  auto compute = [&](int b, bool do_xlo) {
    constexpr bool MLO = !HI;
    const char* base = lds + b * BUF;
    auto pass = [&](int xplane, bool lo_lo) {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const char* pb = base + (ks ? bo1 : bo0) + xplane;
        const char* pa = base + 2 * S3_XP + (ks ? ao1 : ao0);
        V bx[2], ah[4], al[4];
#pragma unroll
        for (int j = 0; j < 2; ++j) bx[j] = *reinterpret_cast<const V*>(pb + 4096 * j);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ah[i] = *reinterpret_cast<const V*>(pa + 2048 * i);
          if constexpr (MLO) al[i] = *reinterpret_cast<const V*>(pa + S3_M + 2048 * i);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(ah[i], bx[j], acc[i][j]);
        if (MLO && lo_lo) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = mfma32(al[i], bx[j], acc[i][j]);
        }
      }
    };
    pass(0, true);
    if (do_xlo) pass(S3_XLO, MODE == MODE_BF16);
  };

  // e = c - |x|^2 + 2 s and Y^T += W^T E^T for the wave's landmarks of pass
  // s; the pass's projection is then added to the running sum (lane value
  // (j, k): blocks k >> 2 and 2 + (k >> 2) of the 4-block accumulator).
  // The c and W rows of landmark block i + 2 are loaded while block i is
  // projected.
  auto epilogue = [&](int s) {
    const float two = 2.0f * mv.postscale;
    f16v yacc[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) yacc[j][v] = 0.f;
    const int64_t lb = (int64_t)s * WBN + 128 * wn + 4 * half;
    const float* cb = reinterpret_cast<const float*>(mv.c) + lb;
    const float* wb = reinterpret_cast<const float*>(mv.w) + (int64_t)(lane & 15) * mv.ldwt + lb;
    f4 cw[2][8];
    auto ld = [&](int i, int slot) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        cw[slot][a] = *reinterpret_cast<const f4*>(cb + 32 * i + 8 * a);
        cw[slot][4 + a] = *reinterpret_cast<const f4*>(wb + 32 * i + 8 * a);
      }
    };
    ld(0, 0);
    ld(1, 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int slot = i & 1;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const float e = (cw[slot][v >> 2][v & 3] - xn[j]) + two * acc[i][j][v];
          yacc[j] = __builtin_amdgcn_mfma_f32_16x16x1f32(cw[slot][4 + (v >> 2)][v & 3], e, yacc[j], 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;
      }
      if (i + 2 < 4) ld(i + 2, slot);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 8; ++q) ysum[j][q] += yacc[j][q] + yacc[j][q + 8];
  };

  // ---- pipeline ----
  // iteration it (pass s, chunk ch): landmark copies of chunk it + MAHEAD
  // (into the buffer the products of chunk it - 1 read), then data loads of
  // chunk it + 2 into the register slot chunk it used (XDMA: data copies of
  // chunk it + 2 into its buffer); products of chunk it; split of chunk
  // it + 1 (loaded two iterations back) into its buffer; wait for the
  // landmark copies of chunk it + 1; one barrier.  The loop is unrolled by
  // two so that the register slots are fixed.
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  const int cm = HI ? 4 : 8;  // landmark copies per chunk and wave
  {
    int ms = 0, mc = 0;
    for (int q = 0; q < MAHEAD && q < total; ++q) {
      dma_m(ms, mc, q);
      if (++mc == nch) {
        mc = 0;
        ++ms;
      }
    }
  }
  bool nz0;
  if constexpr (XDMA) {
    dma_x(0, 0);
    if (total > 1) dma_x(1 % nch, 1);
    __builtin_amdgcn_s_waitcnt(wait_imm(0, 15));
    __builtin_amdgcn_sched_barrier(0);
    nz0 = split_lds(0, 0, true);
  } else {
    load_x(0, S0{});
    if (total > 1) load_x(1 % nch, S1{});
    nz0 = split(0, 0, true, S0{});
  }
  {
    const bool nz = nz0;
    if constexpr (HI) {
      const bool any = __builtin_amdgcn_ballot_w64(nz) != 0;
      if (lane == 0) flags[wave] = any ? 1 : 0;
    }
  }
  __builtin_amdgcn_s_waitcnt(wait_imm(0, 0));
  raw_barrier();
  // (s, ch): chunk it; (ns, nc): chunk it + 1; (ms, mc): chunk it + MAHEAD;
  // lc: the chunk (within its pass) of chunk it + 2
  int s = 0, ch = 0, b = 0;
  int ns = (nch == 1) ? 1 : 0, nc = (nch == 1) ? 0 : 1;
  int ms = MAHEAD / nch, mc = MAHEAD % nch;
  int lc = 2 % nch;
  // FULL (direct data copies only): a step with it + 2 < total, whose
  // copies are issued without a condition, so that the copies in flight
  // are the same on every path and the waits count them exactly
  auto step = [&](int it, auto cur, auto full) {
    using SC = decltype(cur);
    using SN = std::integral_constant<int, 1 - SC::value>;
    constexpr bool FULL = decltype(full)::value;
    const bool live = (int64_t)s * WBN + 128 * wn < l_pad;
    const bool next = FULL || it + 1 < total;
    const int bn = (b + 1 == NBUF) ? 0 : b + 1;
    if (FULL || it + MAHEAD < total) dma_m(ms, mc, (b + MAHEAD) % NBUF);
    if (FULL || it + 2 < total) {
      if constexpr (XDMA)
        dma_x(lc, (b + 2) % NBUF);
      else
        load_x(lc, SC{});
    }
    bool do_xlo = true;
    if constexpr (HI) {
      const int* fb = flags + b * 8;
      do_xlo = ((fb[0] | fb[1]) | (fb[2] | fb[3]) | (fb[4] | fb[5]) | (fb[6] | fb[7])) != 0;
    }
    if (live) compute(b, do_xlo);
    if (next) {
      bool nz;
      if constexpr (XDMA) {
        // the data copies of chunk it + 1 (one step back) have landed once
        // at most this step's copies remain
        if (FULL || it + 2 < total)
          __builtin_amdgcn_s_waitcnt(wait_imm(cm + 2, 15));
        else
          __builtin_amdgcn_s_waitcnt(wait_imm(0, 15));
        __builtin_amdgcn_sched_barrier(0);
        nz = split_lds(nc, bn, ns == 0);
      } else {
        nz = split(nc, bn, ns == 0, SN{});
      }
      if constexpr (HI) {
        const bool any = __builtin_amdgcn_ballot_w64(nz) != 0;
        if (lane == 0) flags[bn * 8 + wave] = any ? 1 : 0;
      }
    }
    // the landmark copies of chunk it + 1 have landed once at most the
    // later memory operations remain: (three buffers) data loads or copies
    // of chunks it + 1 and it + 2 and landmark copies of chunk it + 2, (two
    // buffers) data loads of chunk it + 2; the split's stores are done
    if (HI && (FULL || it + 2 < total)) __builtin_amdgcn_s_waitcnt(wait_imm(cm + 4, 0));
    else if (!HI && (FULL || it + 2 < total)) __builtin_amdgcn_s_waitcnt(wait_imm(2, 0));
    else __builtin_amdgcn_s_waitcnt(wait_imm(0, 0));
    raw_barrier();
    if (ch == nch - 1) {
      if (s == 0) {
        // row norms (4 threads per row, fixed butterfly) through buffer b,
        // which nothing touches again before the next iteration's copies
        float* xnorm = reinterpret_cast<float*>(lds + b * BUF);
        float t = nacc;
        t += __shfl_xor(t, 2, 64);
        t += __shfl_xor(t, 1, 64);
        if (q8 == 0) xnorm[xrow] = t;
        __builtin_amdgcn_s_waitcnt(wait_imm(63, 0));
        raw_barrier();
#pragma unroll
        for (int j = 0; j < 2; ++j) xn[j] = xnorm[64 * wm + 32 * j + l31];
        __builtin_amdgcn_s_waitcnt(wait_imm(63, 0));
        raw_barrier();
      }
      if (live) epilogue(s);
    }
    // advance the chunk counters
    s = ns;
    ch = nc;
    b = bn;
    if (++nc == nch) {
      nc = 0;
      ++ns;
    }
    if (++mc == nch) {
      mc = 0;
      ++ms;
    }
    if (++lc == nch) lc = 0;
  };
  using FullStep = std::true_type;
  using TailStep = std::false_type;
  int it = 0;
  if constexpr (XDMA) {
    for (; it + 3 < total; it += 2) {
      step(it, S0{}, FullStep{});
      step(it + 1, S1{}, FullStep{});
    }
  }
  for (; it < total; it += 2) {
    step(it, S0{}, TailStep{});
    if (it + 1 < total) step(it + 1, S1{}, TailStep{});
  }

  // ---- add the four landmark quarters in order and store ----
  // lane value (j, k): row 64 h + 32 j + 16 (k >> 2) + (lane & 15), column
  // 4 (lane >> 4) + (k & 3)
  __syncthreads();
  float* ysh = reinterpret_cast<float*>(lds);
  if (wn > 0) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 8; ++k) ysh[((((wn - 1) * 2 + wm) * 2 + j) * 8 + k) * 64 + lane] = ysum[j][k];
  }
  __syncthreads();
  if (wn == 0) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int row = 64 * wm + 32 * j + 16 * (k >> 2) + (lane & 15);
        const int col = 4 * (lane >> 4) + (k & 3);
        float val = ysum[j][k];
#pragma unroll
        for (int w = 0; w < 3; ++w) val += ysh[(((w * 2 + wm) * 2 + j) * 8 + k) * 64 + lane];
        if (row < nrows && col < mv.r) Y[(int64_t)row * ldy + col] = val;
      }
  }
  __syncthreads();
}

// Two waves per SIMD (two blocks per CU) where the registers fit without
// spilling; the FP64 and wide-output variants keep one.
template <int MODE, int RB>
constexpr int waves_per_simd() {
  return (MODE != MODE_F64 && (RB == 1 || (RB == 2 && MODE == MODE_F32))) ? 2 : 1;
}

template <int MODE, typename TX, int RB>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(waves_per_simd<MODE, RB>(), waves_per_simd<MODE, RB>()))) void k_embed(EmbedModelView mv, const TX* __restrict__ X,
                                                   int64_t n, int64_t ldx, void* __restrict__ Y,
                                                   int64_t ldy) {
  extern __shared__ __align__(16) char lds[];
  using T = typename Tr<MODE>::T;
  const int64_t ntiles = (n + BM - 1) / BM;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * BM;
    const int nrows = (int)((n - row0) < BM ? (n - row0) : BM);
    embed_tile<MODE, TX, RB>(mv, X + row0 * ldx, ldx, nrows,
                             reinterpret_cast<T*>(Y) + row0 * ldy, ldy, lds);
  }
}

// Persistent serving kernel: blocks stride over a device table of tiles,
// each naming its model; every tile runs the same embed_tile code as the
// plain kernel (same template arguments), so results are identical alone
// and in a mix.  One launch serves models of one 16-column block class.
template <int MODE, int RB>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(waves_per_simd<MODE, RB>(), waves_per_simd<MODE, RB>()))) void k_embed_work(
    const EmbedModelView* __restrict__ views, const TileWork* __restrict__ work,
    const int32_t* __restrict__ nwork) {
  extern __shared__ __align__(16) char lds[];
  using T = typename Tr<MODE>::T;
  const int nw = nwork[0];
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
    const TileWork tw = work[w];
    const EmbedModelView mv = views[tw.model];
    const float* X = reinterpret_cast<const float*>(tw.x) + tw.row0 * tw.ldx;
    T* Y = reinterpret_cast<T*>(tw.y) + tw.row0 * tw.ldy;
    embed_tile<MODE, float, RB>(mv, X, tw.ldx, tw.nrows, Y, tw.ldy, lds);
  }
}

template <int MODE, bool KTAIL>
__global__ __launch_bounds__(WTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_embed_wide(
    EmbedModelView mv, const float* __restrict__ X, int64_t n, int64_t ldx, float* __restrict__ Y,
    int64_t ldy) {
  extern __shared__ __align__(16) char lds[];
  const int64_t ntiles = (n + BM - 1) / BM;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * BM;
    const int nrows = (int)((n - row0) < BM ? (n - row0) : BM);
    embed_tile_wide<MODE, KTAIL>(mv, X + row0 * ldx, ldx, nrows, Y + row0 * ldy, ldy, lds);
  }
}

// serving form of the same variant (one tile table entry per 128 rows)
template <int MODE>
__global__ __launch_bounds__(WTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_embed_work_wide(
    const EmbedModelView* __restrict__ views, const TileWork* __restrict__ work,
    const int32_t* __restrict__ nwork) {
  extern __shared__ __align__(16) char lds[];
  const int nw = nwork[0];
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
    const TileWork tw = work[w];
    const EmbedModelView mv = views[tw.model];
    const float* X = reinterpret_cast<const float*>(tw.x) + tw.row0 * tw.ldx;
    float* Y = reinterpret_cast<float*>(tw.y) + tw.row0 * tw.ldy;
    embed_tile_wide<MODE, true>(mv, X, tw.ldx, tw.nrows, Y, tw.ldy, lds);  // models of any p
  }
}

// split precisions: the 32 x 32 variant (one 512-thread block per CU)
template <int MODE, bool HI, bool XDMA>
__global__ __launch_bounds__(S3_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_embed_s3(
    EmbedModelView mv, const float* __restrict__ X, int64_t n, int64_t ldx, float* __restrict__ Y,
    int64_t ldy) {
  extern __shared__ __align__(16) char lds[];
  const int64_t ntiles = (n + BM - 1) / BM;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * BM;
    const int nrows = (int)((n - row0) < BM ? (n - row0) : BM);
    embed_tile_s3<MODE, HI, XDMA>(mv, X + row0 * ldx, ldx, nrows, Y + row0 * ldy, ldy, lds);
  }
}

template <int MODE, bool HI>
__global__ __launch_bounds__(S3_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_embed_work_s3(
    const EmbedModelView* __restrict__ views, const TileWork* __restrict__ work,
    const int32_t* __restrict__ nwork) {
  extern __shared__ __align__(16) char lds[];
  const int nw = nwork[0];
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
    const TileWork tw = work[w];
    const EmbedModelView mv = views[tw.model];
    const float* X = reinterpret_cast<const float*>(tw.x) + tw.row0 * tw.ldx;
    float* Y = reinterpret_cast<float*>(tw.y) + tw.row0 * tw.ldy;
    // the register path for every request (the same arithmetic, bit for bit)
    embed_tile_s3<MODE, HI, false>(mv, X, tw.ldx, tw.nrows, Y, tw.ldy, lds);
  }
}

template <int MODE, typename TX, int RB>
hipError_t launch_t(const EmbedModelView& mv, const void* X, int64_t n, int64_t ldx, void* Y,
                    int64_t ldy, hipStream_t st) {
  {
    hipError_t e = lds_limit_once(reinterpret_cast<const void*>(&k_embed<MODE, TX, RB>), LDS_BYTES);
    if (e != hipSuccess) return e;
  }
  const int64_t ntiles = (n + BM - 1) / BM;
  const int64_t cap = (int64_t)num_cu() * 2 * 64;
  const int grid = (int)(ntiles < cap ? ntiles : cap);
  k_embed<MODE, TX, RB><<<grid, THREADS, LDS_BYTES, st>>>(mv, reinterpret_cast<const TX*>(X), n, ldx,
                                                           Y, ldy);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_wide_v(const EmbedModelView& mv, const void* X, int64_t n, int64_t ldx, void* Y,
                         int64_t ldy, hipStream_t st) {
  for (const void* f : {reinterpret_cast<const void*>(&k_embed_wide<MODE, true>),
                        reinterpret_cast<const void*>(&k_embed_wide<MODE, false>)}) {
    hipError_t e = lds_limit_once(f, WLDS_BYTES);
    if (e != hipSuccess) return e;
  }
  const int64_t ntiles = (n + BM - 1) / BM;
  // persistent: one block per CU (the LDS holds one), each walking tiles
  // gridDim apart; lane constants are computed (and spilled) once per block
  const int64_t cap = (int64_t)num_cu();
  const int grid = (int)(ntiles < cap ? ntiles : cap);
  if (mv.p % 16 != 0)
    k_embed_wide<MODE, true><<<grid, WTHREADS, WLDS_BYTES, st>>>(
        mv, reinterpret_cast<const float*>(X), n, ldx, reinterpret_cast<float*>(Y), ldy);
  else
    k_embed_wide<MODE, false><<<grid, WTHREADS, WLDS_BYTES, st>>>(
        mv, reinterpret_cast<const float*>(X), n, ldx, reinterpret_cast<float*>(Y), ldy);
  return hipGetLastError();
}

template <int MODE, bool HI, bool XDMA>
hipError_t launch_s3(const EmbedModelView& mv, const void* X, int64_t n, int64_t ldx, void* Y,
                     int64_t ldy, hipStream_t st) {
  {
    hipError_t e = lds_limit_once(reinterpret_cast<const void*>(&k_embed_s3<MODE, HI, XDMA>), s3_lds<HI>());
    if (e != hipSuccess) return e;
  }
  const int64_t ntiles = (n + BM - 1) / BM;
  const int64_t cap = (int64_t)num_cu();
  const int grid = (int)(ntiles < cap ? ntiles : cap);
  k_embed_s3<MODE, HI, XDMA><<<grid, S3_THREADS, s3_lds<HI>(), st>>>(
      mv, reinterpret_cast<const float*>(X), n, ldx, reinterpret_cast<float*>(Y), ldy);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_wide(const EmbedModelView& mv, const void* X, int64_t n, int64_t ldx, void* Y,
                       int64_t ldy, hipStream_t st) {
  if constexpr (MODE == MODE_F32)
    return launch_wide_v<MODE>(mv, X, n, ldx, Y, ldy, st);
  else
  {
    // data copies straight into LDS need 16-byte aligned rows and p a
    // multiple of 4 (whole 16-byte pieces), and the third buffer
    const bool xdma = mv.m_lo_zero && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                      ((ldx * (int64_t)sizeof(float)) % 16 == 0) && (mv.p % 4 == 0);
    if (xdma) return launch_s3<MODE, true, true>(mv, X, n, ldx, Y, ldy, st);
    return mv.m_lo_zero ? launch_s3<MODE, true, false>(mv, X, n, ldx, Y, ldy, st)
                        : launch_s3<MODE, false, false>(mv, X, n, ldx, Y, ldy, st);
  }
}

template <int MODE, typename TX>
hipError_t launch_rb(const EmbedModelView& mv, const void* X, int64_t n, int64_t ldx, void* Y,
                     int64_t ldy, hipStream_t st) {
  if (mv.rb <= 1) return launch_t<MODE, TX, 1>(mv, X, n, ldx, Y, ldy, st);
  if (mv.rb == 2) return launch_t<MODE, TX, 2>(mv, X, n, ldx, Y, ldy, st);
  return launch_t<MODE, TX, 4>(mv, X, n, ldx, Y, ldy, st);
}

}  // namespace

static int g_num_cu = 0;

int num_cu() {
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
    g_num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  }
  return g_num_cu;
}

int embed_max_rb() { return 4; }

EmbedModelView Model::view(int mode) const {
  EmbedModelView v{};
  v.p = (int)p;
  v.ntl = (int)(l_pad / BN);
  v.r = r;
  v.rb = rb;
  v.prescale = 1.f;
  v.postscale = 1.f;
  switch (mode) {
    case MODE_F64:
      v.mpack = m64;
      v.w = w64;
      v.c = c64;
      v.nchunks = (int)((p + 15) / 16);
      break;
    case MODE_F32:
      v.mpack = m32;
      v.w = w32;
      v.ldwt = l_pad;
      v.c = c32;
      v.nchunks = (int)((p + 31) / 32);
      break;
    case MODE_BF16:
      v.mpack = mbf;
      v.spack = sbf;
      v.lsplit = l_split;
      v.w = w32;
      v.ldwt = l_pad;
      v.c = c32;
      v.nchunks = (int)((p + 31) / 32);
      v.m_lo_zero = bf_lo_zero;
      break;
    default:
      v.mpack = mh;
      v.spack = sh;
      v.lsplit = l_split;
      v.w = w32;
      v.ldwt = l_pad;
      v.c = c32;
      v.nchunks = (int)((p + 31) / 32);
      v.m_lo_zero = h_lo_zero;
      v.prescale = h_prescale;
      v.postscale = h_postscale;
      break;
  }
  return v;
}

mds_status launch_embed(const Model& m, int mode, const void* X, int dt, int64_t n, int64_t ldx,
                        void* Y, int64_t ldy, hipStream_t st) {
  const EmbedModelView mv = m.view(mode);
  hipError_t e;
  switch (mode) {
    case MODE_F64:
      e = (dt == MDS_F64) ? launch_rb<MODE_F64, double>(mv, X, n, ldx, Y, ldy, st)
                          : launch_rb<MODE_F64, float>(mv, X, n, ldx, Y, ldy, st);
      break;
    case MODE_F32:
      e = embed_wide(mode, m.p, m.rb, m.l_pad) ? launch_wide<MODE_F32>(mv, X, n, ldx, Y, ldy, st)
                                      : launch_rb<MODE_F32, float>(mv, X, n, ldx, Y, ldy, st);
      break;
    case MODE_BF16:
      e = embed_wide(mode, m.p, m.rb, m.l_pad) ? launch_wide<MODE_BF16>(mv, X, n, ldx, Y, ldy, st)
                                      : launch_rb<MODE_BF16, float>(mv, X, n, ldx, Y, ldy, st);
      break;
    default:
      e = embed_wide(mode, m.p, m.rb, m.l_pad) ? launch_wide<MODE_F16>(mv, X, n, ldx, Y, ldy, st)
                                      : launch_rb<MODE_F16, float>(mv, X, n, ldx, Y, ldy, st);
      break;
  }
  if (e != hipSuccess) return hip_fail(e, "embed launch");
  return MDS_OK;
}

namespace {
template <int MODE>
const void* worklist_fn_rb(int rbc) {
  switch (rbc) {
    case 0: return reinterpret_cast<const void*>(&k_embed_work<MODE, 1>);
    case 1: return reinterpret_cast<const void*>(&k_embed_work<MODE, 2>);
    case 2: return reinterpret_cast<const void*>(&k_embed_work<MODE, 4>);
    case kWideClass:
      if constexpr (MODE == MODE_F32) return reinterpret_cast<const void*>(&k_embed_work_wide<MODE>);
      else return reinterpret_cast<const void*>(&k_embed_work_s3<MODE, false>);
    default:
      if constexpr (MODE == MODE_F32) return nullptr;
      else return reinterpret_cast<const void*>(&k_embed_work_s3<MODE, true>);
  }
}
const void* worklist_fn(int mode, int rbc) {
  switch (mode) {
    case MODE_F32: return worklist_fn_rb<MODE_F32>(rbc);
    case MODE_BF16: return worklist_fn_rb<MODE_BF16>(rbc);
    case MODE_F16: return worklist_fn_rb<MODE_F16>(rbc);
    default: return nullptr;
  }
}

template <int MODE>
void launch_work_rb(int rbc, int grid, hipStream_t st, const EmbedModelView* v, const TileWork* w,
                    const int32_t* nw) {
  switch (rbc) {
    case 0: k_embed_work<MODE, 1><<<grid, THREADS, LDS_BYTES, st>>>(v, w, nw); break;
    case 1: k_embed_work<MODE, 2><<<grid, THREADS, LDS_BYTES, st>>>(v, w, nw); break;
    case 2: k_embed_work<MODE, 4><<<grid, THREADS, LDS_BYTES, st>>>(v, w, nw); break;
    case kWideClass:
      if constexpr (MODE == MODE_F32)
        k_embed_work_wide<MODE><<<grid, WTHREADS, WLDS_BYTES, st>>>(v, w, nw);
      else
        k_embed_work_s3<MODE, false><<<grid, S3_THREADS, s3_lds<false>(), st>>>(v, w, nw);
      break;
    default:
      if constexpr (MODE != MODE_F32)
        k_embed_work_s3<MODE, true><<<grid, S3_THREADS, s3_lds<true>(), st>>>(v, w, nw);
      break;
  }
}
}  // namespace

int rb_class(int rb) { return rb <= 1 ? 0 : (rb == 2 ? 1 : 2); }

int embed_class(int mode, int64_t p, int rb, int64_t l_pad, int m_lo_zero) {
  if (!embed_wide(mode, p, rb, l_pad)) return rb_class(rb);
  return (m_lo_zero && mode != MODE_F32) ? kWideHiClass : kWideClass;
}

int embed_blocks_per_cu(int mode, int rbc) {
  if (mode == MODE_F64 || rbc >= 2) return 1;
  if (rbc == 0) return 2;
  return mode == MODE_F32 ? 2 : 1;
}

// Sets the kernel's LDS limit outside any stream capture.
mds_status prepare_embed_worklist(int mode, int rbc) {
  const void* fn = worklist_fn(mode, rbc);
  if (!fn) return set_error(MDS_ERR_INVALID_ARG, "serving supports FP32 and split precisions");
  const int bytes = rbc < kWideClass ? LDS_BYTES
                    : mode == MODE_F32 ? WLDS_BYTES
                    : rbc == kWideHiClass ? s3_lds<true>() : s3_lds<false>();
  hipError_t e = lds_limit_once(fn, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  return MDS_OK;
}

mds_status launch_embed_worklist(int mode, int rbc, const EmbedModelView* views_dev,
                                 const TileWork* work_dev, const int32_t* nwork_dev, int grid,
                                 hipStream_t st) {
  mds_status s = prepare_embed_worklist(mode, rbc);
  if (s != MDS_OK) return s;
  if (grid <= 0) grid = num_cu() * embed_blocks_per_cu(mode, rbc);
  switch (mode) {
    case MODE_F32: launch_work_rb<MODE_F32>(rbc, grid, st, views_dev, work_dev, nwork_dev); break;
    case MODE_BF16: launch_work_rb<MODE_BF16>(rbc, grid, st, views_dev, work_dev, nwork_dev); break;
    default: launch_work_rb<MODE_F16>(rbc, grid, st, views_dev, work_dev, nwork_dev); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "serving launch");
  return MDS_OK;
}

}  // namespace mds
