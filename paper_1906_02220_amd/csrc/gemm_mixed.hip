// Reduced-precision contractions with FP64 inputs and outputs.
//
// CTM_PREC_F32: one FP32 product.  Operands are rounded to FP32 while they
// are staged into LDS, v_mfma_f32_16x16x4_f32 accumulates in FP32, and the
// FP32 result is widened to FP64.
//
// CTM_PREC_BF16X3 / X4: split-precision products on the BF16 matrix cores.
// Every row of A (and every column of B) is scaled by a power of two 2^-e
// with e chosen so that the row's largest entry falls below 1 in magnitude,
// then cut into S slices of 8 bits each:
//     y = x 2^(8 - e),  q_0 = rint(y),  q_i = rint(256 (y_(i-1) - q_(i-1))),
// stored as the BF16 numbers q_i 2^(-8 i) (|q_0| <= 256, |q_i| <= 128 for
// i >= 1, so every slice is exact in BF16's 8-bit significand).  Then
//     A B = 2^(eA + eB - 16) sum_{i + j < S} A_i B_j
// up to the dropped levels i + j >= S and the residual of the S-th slice,
// both about 2^(-8 S) relative to the row and column scales.
//
// The products run on v_mfma_f32_16x16x32_bf16 with FP32 accumulation over
// K chunks of 128:
//   * level 0 (A_0 B_0) has its own accumulator: products are integers below
//     2^16 in magnitude and a chunk sum stays below 2^23, so the FP32 sum is
//     exact;
//   * all other pairs share a second accumulator, whose FP32 rounding is at
//     most about 2^-32 relative to the level-0 scale.
// After every chunk both accumulators are added into an FP64 accumulator
// held in registers, and the epilogue applies the row and column scales
// exactly (ldexp).
//
// The slices are built by two memory-bound kernels (a max-abs reduction and
// the split itself).  Both operands are stored K-step-major,
// Q[k / 32][r][i][k % 32]: the S slices of a row's 32-wide K step are
// contiguous, and so are all rows of one step.  The GEMM's K step then reads
// whole 128-byte lines (a row-major slice would use half of each line per
// step and fetch the other half again on the next), and a lane's MFMA
// operand (8 consecutive k) is one 16-byte LDS read.
//
// MFMA operand fragments (checked on the device with an in-bounds probe):
//   16x16x32 BF16: lane l holds A[l % 16][8 (l / 16) + e] and
//                  B[8 (l / 16) + e][l % 16], e < 8;
//   16x16x4 F32:   lane l holds A[l % 16][l / 16] and B[l / 16][l % 16];
//   accumulator register r of lane l holds C[4 (l / 16) + r][l % 16] (unlike
//   the FP64 MFMA, whose register r holds row 4 r + l / 16).
#include <climits>
#include <cmath>
#include <cstdint>

#include "ctm.h"
#include "internal.hpp"

namespace ctm {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int kChunk = 128;  // K chunk of exact FP32 accumulation (BF16 path)

// ------------------------------------------------------------ slicing

// max |x| over each row r of the R x K view (element (r, k) at p[r rs + k]),
// one wave per row and four rows per workgroup; rows are 16-byte aligned (the
// dispatcher checks p and an even rs).  Each lane keeps eight 16-byte loads
// in flight; a workgroup per row, with five loads per thread, streamed only
// 4.3 TB/s.  A NaN wins, so the maximum does not depend on the order.  It
// also clears zero_out[0..nzero) for the column maxima that follow on the
// same stream.
constexpr int kRowmaxRows = 4;
__global__ __launch_bounds__(64 * kRowmaxRows) void rowmax_contig_kernel(
    const double* __restrict__ p, long long rs, int R, int K, double* __restrict__ mx,
    double* __restrict__ zero_out, int nzero) {
  const int t = threadIdx.x, lane = t & 63;
  for (int i = blockIdx.x * blockDim.x + t; i < nzero; i += gridDim.x * blockDim.x) zero_out[i] = 0.0;
  const int r = blockIdx.x * kRowmaxRows + (t >> 6);
  if (r >= R) return;  // whole waves; no barrier follows
  auto take = [](double m, double v) { return (v > m || v != v) ? v : m; };  // a NaN wins
  const double* row = p + r * rs;
  double m0 = 0.0, m1 = 0.0;
  constexpr int kBatch = 8;
  for (int k0 = 2 * lane; k0 + 1 < K; k0 += 128 * kBatch) {
    d2v v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int k = k0 + 128 * u;
      v[u] = k + 1 < K ? *(const d2v*)(row + k) : d2v{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      m0 = take(m0, fabs(v[u].x));
      m1 = take(m1, fabs(v[u].y));
    }
  }
  if ((K & 1) && lane == 0) m0 = take(m0, fabs(row[K - 1]));
  double m = take(m0, m1);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = take(m, __shfl_xor(m, off, 64));
  if (lane == 0) mx[r] = m;
}

// max |x| over each column n of a K x N row-major matrix (row stride ld):
// thread = column, blockIdx.y = K slab, combined with an integer atomic max
// on the bit pattern (non-negative doubles order like their bits; a NaN's
// pattern is above every finite one).  mx must start at +0.
__global__ __launch_bounds__(256) void colmax_kernel(const double* __restrict__ p, long long ld,
                                                     int K, int N, int kslab,
                                                     unsigned long long* __restrict__ mx) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int k0 = blockIdx.y * kslab, k1 = min(K, k0 + kslab);
  auto take = [](double m, double v) { return (v > m || v != v) ? v : m; };  // a NaN wins
  // four independent loads in flight per step
  double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
  int k = k0;
  for (; k + 3 < k1; k += 4) {
    const double v0 = fabs(p[(long long)k * ld + n]), v1 = fabs(p[(long long)(k + 1) * ld + n]);
    const double v2 = fabs(p[(long long)(k + 2) * ld + n]), v3 = fabs(p[(long long)(k + 3) * ld + n]);
    m0 = take(m0, v0);
    m1 = take(m1, v1);
    m2 = take(m2, v2);
    m3 = take(m3, v3);
  }
  for (; k < k1; ++k) m0 = take(m0, fabs(p[(long long)k * ld + n]));
  const double m = take(take(m0, m1), take(m2, m3));
  atomicMax(mx + n, (unsigned long long)__double_as_longlong(m));
}

__device__ inline int scale_exponent(double m) {
  // smallest e with m < 2^e (0 for an all-zero or non-finite row)
  if (!(m > 0.0) || !(m < INFINITY)) return 0;
  return ilogb(m) + 1;
}

// Cut one value into S slices (see the file comment); a non-finite value
// gives a NaN first slice so that the product row turns NaN.
template <int S>
__device__ inline void cut(double x, int e, __bf16* out) {
  if (!isfinite(x)) {
    out[0] = (__bf16)NAN;
#pragma unroll
    for (int i = 1; i < S; ++i) out[i] = (__bf16)0.0f;
    return;
  }
  double y = ldexp(x, 8 - e);
  double w = 1.0;
#pragma unroll
  for (int i = 0; i < S; ++i) {
    const double q = rint(y);
    out[i] = (__bf16)(float)(q * w);
    y = (y - q) * 256.0;
    w *= 1.0 / 256.0;
  }
}

// Slices of the R x K view (element (r, k) at p[r rs + k cs]) into the
// K-step-major Q[k / 32][r][i][k % 32] (zero for K <= k < Kp).  A 64 x 64 tile per
// workgroup goes through LDS so that the global reads are coalesced along
// whichever index is contiguous and the slice writes along k.
template <int S>
__global__ __launch_bounds__(256) void split_kernel(const double* __restrict__ p, long long rs,
                                                    long long cs, int R, int K, int Kp,
                                                    const double* __restrict__ mx,
                                                    __bf16* __restrict__ Q) {
  __shared__ double tile[64][65];
  const int r0 = blockIdx.y * 64, k0 = blockIdx.x * 64;
  const int t = threadIdx.x;
  // 16-byte loads of two neighbours along the contiguous index (the caller
  // passes a 16-byte aligned p and an even stride).  All eight loads of a
  // thread are issued before any LDS write, so they are in flight together
  // (a loop that wrote each value before the next load kept one in flight).
  // A tile inside both bounds (all but the last along each axis) loads
  // without branches; the bounds checks' joins would make the compiler wait
  // for each load before the next.
  constexpr int kLoads = 64 * 32 / 256;
  double v0[kLoads], v1[kLoads];
  const bool interior = r0 + 64 <= R && k0 + 64 <= K;
  if (cs == 1 && interior) {
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int idx = t + 256 * j;
      const int r = r0 + (idx >> 5), k = k0 + (idx & 31) * 2;
      const d2v v = *(const d2v*)(p + r * rs + k);
      v0[j] = v.x;
      v1[j] = v.y;
    }
  } else if (interior) {
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int idx = t + 256 * j;
      const int k = k0 + (idx >> 5), r = r0 + (idx & 31) * 2;
      const d2v v = *(const d2v*)(p + r + k * cs);
      v0[j] = v.x;
      v1[j] = v.y;
    }
  } else if (cs == 1) {
    // rows contiguous along k: consecutive threads walk k
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int idx = t + 256 * j;
      const int r = r0 + (idx >> 5), k = k0 + (idx & 31) * 2;
      v0[j] = 0.0;
      v1[j] = 0.0;
      if (r < R) {
        if (k + 1 < K) {
          const d2v v = *(const d2v*)(p + r * rs + k);
          v0[j] = v.x;
          v1[j] = v.y;
        } else if (k < K) {
          v0[j] = p[r * rs + k];
        }
      }
    }
  } else {
    // contiguous along r (rs == 1): consecutive threads walk r
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int idx = t + 256 * j;
      const int k = k0 + (idx >> 5), r = r0 + (idx & 31) * 2;
      v0[j] = 0.0;
      v1[j] = 0.0;
      if (k < K) {
        if (r + 1 < R) {
          const d2v v = *(const d2v*)(p + r + k * cs);
          v0[j] = v.x;
          v1[j] = v.y;
        } else if (r < R) {
          v0[j] = p[r + k * cs];
        }
      }
    }
  }
  // the scales of this thread's two rows (see below), fetched while the tile
  // loads are in flight
  double mrow[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = r0 + (t >> 3) + 32 * h;
    mrow[h] = r < R ? mx[r] : 0.0;
  }
  if (cs == 1) {
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int idx = t + 256 * j;
      const int rr = idx >> 5, kk = (idx & 31) * 2;
      tile[rr][kk] = v0[j];
      tile[rr][kk + 1] = v1[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int idx = t + 256 * j;
      const int kk = idx >> 5, rr = (idx & 31) * 2;
      tile[rr][kk] = v0[j];
      tile[rr + 1][kk] = v1[j];
    }
  }
  __syncthreads();
  // each thread: 8 consecutive k of one row, for two rows; 8 lanes cover a
  // row's 64 k, so each slice store writes whole 64-byte runs (a thread with
  // 16 k wrote two separate 16-byte pieces of every run per store; the split
  // went 3 % faster)
  const int c8 = t & 7;
  const long long step = (long long)R * S * 32;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int rr = (t >> 3) + 32 * h;
    const int r = r0 + rr;
    if (r >= R) break;
    const int kb = k0 + 8 * c8;
    if (kb >= Kp) continue;
    const int e = scale_exponent(mrow[h]);
    __bf16 v[S][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      __bf16 o[S];
      cut<S>(tile[rr][8 * c8 + u], e, o);
#pragma unroll
      for (int i = 0; i < S; ++i) v[i][u] = o[i];
    }
#pragma unroll
    for (int i = 0; i < S; ++i) {
      bf8 w;
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = v[i][u];
      *(bf8*)(Q + (kb >> 5) * step + (long long)r * (S * 32) + i * 32 + (kb & 31)) = w;
    }
  }
}

}  // namespace

// ------------------------------------------------------------ BF16 slice GEMM

// 16 bytes per lane from global memory straight into LDS, lane l's bytes at
// LDS address lds + 16 l (lds wave-uniform, through M0).  Written as inline
// asm so that the compiler, which cannot tell these LDS writes from the
// fragment reads of the other stage, does not wait for them before every LDS
// read; the kernel waits for them itself (vmcnt) before its barriers.  The
// instruction has no register result.
__device__ inline void load_to_lds16(const void* g, unsigned lds) {
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds)
               : "memory", "m0");
}

// LDS position (in BF16 units) of the 16-byte chunk c (8 consecutive k) of
// row r in a 32-wide K step: rows are 64 bytes, unpadded, and the chunk index
// is XORed with ((r >> 1) ^ (r >> 2)) & 3.  Both the operand reads (16
// consecutive rows, one chunk) and the tile stores (4 consecutive rows, all
// four chunks) then touch 16 distinct 16-byte bank groups, whether LDS serves
// a 128-bit access 8 or 16 lanes at a time; a padded 80-byte row left the
// stores 2-way conflicted (half of all LDS cycles in the counters).
__device__ inline int slice_pos(int r, int c) { return r * 32 + ((c ^ (((r >> 1) ^ (r >> 2)) & 3)) << 3); }

// C (M x N, row stride ldc, FP64) = A B from the K-step-major slices of A
// (Aq[Kp / 32][M][S][32]) and of B^T (Bq[Kp / 32][N][S][32]) and the row /
// column maxima.  128 x 128
// tile, 8 waves as 4 x 2, each wave 32 x 64 (2 x 4 MFMA tiles); K steps of
// 32 through two LDS stages, the next step loaded straight into the other
// stage while this one is multiplied.  Wave w moves rows 16 w .. 16 w + 15 of
// every slice of both operands (1 KB per slice and operand): lane l fetches
// the chunk whose swizzled LDS slot is byte 16 l of the wave's kilobyte.
// Rows past M (N) repeat row M - 1 (N - 1); they only reach accumulator rows
// (columns) that are not stored.
template <int S, int TAG, int XG = 8>
__global__ __launch_bounds__(512) void gemm_bf16s_kernel(
    int M, int N, int Kp, const __bf16* __restrict__ Aq, const __bf16* __restrict__ Bq,
    const double* __restrict__ amax, const double* __restrict__ bmax, double* __restrict__ C,
    OutMap om) {
  constexpr int BM = 128, BN = 128, BK = 32;
  constexpr int TI = 2, TJ = 4;
  // LDS stages: three at S = 3 (144 KB), loaded two K steps ahead; two at
  // S = 4 (128 KB), one step ahead
  constexpr int NS = S == 3 ? 3 : 2;
  __shared__ __attribute__((aligned(1024))) __bf16 As[NS][S][BM * BK];
  __shared__ __attribute__((aligned(1024))) __bf16 Bs[NS][S][BN * BK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  int tm, tn;
  xcd_tile<XG>(blockIdx.x, (M + BM - 1) / BM, (N + BN - 1) / BN, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const long long astep = (long long)M * S * BK, bstep = (long long)N * S * BK;
  const int lr = 16 * wave + (lane >> 2);                     // tile row this lane moves
  const int lc = (lane & 3) ^ (((lr >> 1) ^ (lr >> 2)) & 3);  // its chunk at LDS slot lane & 3
  const __bf16* ag = Aq + (long long)min(m0 + lr, M - 1) * (S * BK) + 8 * lc;
  const __bf16* bg = Bq + (long long)min(n0 + lr, N - 1) * (S * BK) + 8 * lc;
  const unsigned a_lds = __builtin_amdgcn_readfirstlane(
      (unsigned)(uintptr_t)(__attribute__((address_space(3))) __bf16*)&As[0][0][16 * wave * BK]);
  const unsigned b_lds = __builtin_amdgcn_readfirstlane(
      (unsigned)(uintptr_t)(__attribute__((address_space(3))) __bf16*)&Bs[0][0][16 * wave * BK]);
  constexpr unsigned slice_bytes = BM * BK * 2, stage_bytes = S * slice_bytes;
  static_assert(BM == BN, "A and B stages share the byte strides");
  auto load = [&](int kt, int buf) {
    const long long st = kt / BK;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      load_to_lds16(ag + st * astep + i * BK, a_lds + buf * stage_bytes + i * slice_bytes);
      load_to_lds16(bg + st * bstep + i * BK, b_lds + buf * stage_bytes + i * slice_bytes);
    }
  };
  // the loads of the stage needed next have landed (a wave issues 2 S loads
  // per stage and they complete in order, so vmcnt(2 S) leaves only the
  // stage issued in this step in flight; vmcnt(0) when none was issued),
  // every LDS read has returned, then all waves meet
  constexpr int kVmStage = 0xF70 | (2 * S);  // s_waitcnt vmcnt(2 S)
  static_assert(2 * S < 16, "vmcnt field");
  auto step_barrier = [&](bool stage_in_flight) {
    if (stage_in_flight) __builtin_amdgcn_s_waitcnt(kVmStage);
    else __builtin_amdgcn_s_waitcnt(0xF70);  // vmcnt(0)
    __builtin_amdgcn_s_waitcnt(0xC07F);      // lgkmcnt(0)
    asm volatile("s_barrier" ::: "memory");
  };
  f4 acc0[TI][TJ], accr[TI][TJ];
  double acc[TI][TJ][4];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      acc0[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      accr[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
    }
  const int fr = lane & 15, fc = lane >> 4;
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[i][j][r] += (double)acc0[i][j][r] + (double)accr[i][j][r];
        acc0[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        accr[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      }
  };
  // One K step: all fragments first, slice by slice, so that the level-0
  // products can start while the other slices' reads are in flight; then the
  // products level by level across the TI x TJ tiles.  Consecutive MFMAs then
  // write different accumulators (8 apart on the same one), where issuing
  // each tile's five lower-level products back to back made every one wait
  // for the previous result (the launch took 9 % longer).  Each accumulator
  // still receives its products in the same order.
  bf8 a[TI][S], b[TJ][S];
  auto read_fragments = [&](int bb) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int i = 0; i < TI; ++i) a[i][s] = *(const bf8*)(&As[bb][s][slice_pos(wm + 16 * i + fr, fc)]);
#pragma unroll
      for (int j = 0; j < TJ; ++j) b[j][s] = *(const bf8*)(&Bs[bb][s][slice_pos(wn + 16 * j + fr, fc)]);
    }
  };
  auto multiply = [&]() {
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int i = 0; i < TI; ++i)
        acc0[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], acc0[i][j], 0, 0, 0);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S; ++q)
        if (p + q >= 1 && p + q < S) {
#pragma unroll
          for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int i = 0; i < TI; ++i)
              accr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][p], b[j][q], accr[i][j], 0, 0, 0);
        }
  };
  load(0, 0);
  if (NS == 3 && BK < Kp) load(BK, 1);
  step_barrier(NS == 3 && BK < Kp);
  int buf = 0;
  for (int kt = 0; kt < Kp; kt += BK) {
    // the stage loaded here was last read NS - 1 steps ago, behind a barrier
    const int ahead = (NS - 1) * BK;
    const bool issue = kt + ahead < Kp;
    if (issue) load(kt + ahead, buf + NS - 1 < NS ? buf + NS - 1 : buf - 1);
    read_fragments(buf);
    multiply();
    if (((kt + BK) % kChunk) == 0 || kt + BK >= Kp) flush();
    step_barrier(issue && NS == 3);
    buf = buf + 1 < NS ? buf + 1 : 0;
  }
  // epilogue: C = acc 2^(eA + eB - 16), placed by om (the row and column
  // parts of the offset are computed once per row and per column)
  const int lq = lane >> 4;
  long long coff[TJ];
  int eb[TJ];
  bool bbad[TJ];
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    const int gn = n0 + wn + 16 * j + fr;
    const int g = gn < N ? gn : 0;
    coff[j] = (long long)(g / om.c2) * om.sc1 + g % om.c2;
    eb[j] = scale_exponent(bmax[g]);
    bbad[j] = !(bmax[g] < INFINITY);
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + wm + 16 * i + 4 * lq + r;
      if (gm >= M) continue;
      const int ea = scale_exponent(amax[gm]);
      const bool abad = !(amax[gm] < INFINITY);
      const long long roff = (long long)(gm / om.r2) * om.sr1 + (long long)(gm % om.r2) * om.sr2;
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const int gn = n0 + wn + 16 * j + fr;
        if (gn < N) {
          const double v = ldexp(acc[i][j][r], ea + eb[j] - 16);
          C[roff + coff[j]] = (abad || bbad[j]) ? NAN : v;
        }
      }
    }
}

// ------------------------------------------------------------ FP32 GEMM

// C = A B with FP64 operands rounded to FP32 on the way into LDS, FP32 MFMA
// and FP32 accumulation; same staging as the FP64 row-major kernel (96 x 96
// tile, 2 x 2 waves, 16-byte global loads, double-buffered LDS).
// One BM x BN tile of the FP32 product at (m0, n0), for gemm_f32x1_kernel
// and the grouped kernel.
template <int BM, int BN, int WGM, int WGN>
__device__ __forceinline__ void f32_tile(int M, int N, int K, const double* __restrict__ A, int lda,
                                         const double* __restrict__ B, int ldb,
                                         double* __restrict__ C, int ldc, int m0, int n0,
                                         float (*As)[BM * 17], float (*Bs)[16 * (BN + 1)]) {
  constexpr int BK = 16, NT = WGM * WGN * 64;
  constexpr int WM = BM / WGM, WN = BN / WGN, TI = WM / 16, TJ = WN / 16;
  static_assert(TI * 16 == WM && TJ * 16 == WN, "wave tile must be a multiple of 16");
  static_assert((BM * BK / 2) % NT == 0 && (BK * BN / 2) % NT == 0, "pair mapping");
  constexpr int SA = BK + 1, SB = BN + 1;
  constexpr int AV = BM * BK / 2 / NT, BV = BK * BN / 2 / NT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WGN) * WM, wn = (wave % WGN) * WN;
  const bool full_m = (m0 + BM <= M), full_n = (n0 + BN <= N);
  d2v ra[AV], rb[BV];
  auto load = [&](int kt) {
#pragma unroll
    for (int e = 0; e < AV; ++e) {
      const int p = tid + e * NT;
      const int r = p / (BK / 2), k = (p % (BK / 2)) * 2;
      const int gm = m0 + r, gk = kt + k;
      if ((full_m || gm < M) && gk + 1 < K) {
        ra[e] = *(const d2v*)(A + gm * lda + gk);
      } else {
        ra[e].x = (gm < M && gk < K) ? A[gm * lda + gk] : 0.0;
        ra[e].y = (gm < M && gk + 1 < K) ? A[gm * lda + gk + 1] : 0.0;
      }
    }
#pragma unroll
    for (int e = 0; e < BV; ++e) {
      const int p = tid + e * NT;
      const int k = p / (BN / 2), c = (p % (BN / 2)) * 2;
      const int gk = kt + k, gn = n0 + c;
      if (gk < K && (full_n || gn + 1 < N)) {
        rb[e] = *(const d2v*)(B + gk * ldb + gn);
      } else {
        rb[e].x = (gk < K && gn < N) ? B[gk * ldb + gn] : 0.0;
        rb[e].y = (gk < K && gn + 1 < N) ? B[gk * ldb + gn + 1] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AV; ++e) {
      const int p = tid + e * NT;
      float* d = &As[buf][(p / (BK / 2)) * SA + (p % (BK / 2)) * 2];
      d[0] = (float)ra[e].x;
      d[1] = (float)ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < BV; ++e) {
      const int p = tid + e * NT;
      float* d = &Bs[buf][(p / (BN / 2)) * SB + (p % (BN / 2)) * 2];
      d[0] = (float)rb[e].x;
      d[1] = (float)rb[e].y;
    }
  };
  f4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int lr = lane & 15, lk = lane >> 4;
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int kt = 0; kt < K; kt += BK) {
    const bool more = kt + BK < K;
    if (more) load(kt + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      float av[TI], bv[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) av[i] = As[buf][(wm + i * 16 + lr) * SA + kk + lk];
#pragma unroll
      for (int j = 0; j < TJ; ++j) bv[j] = Bs[buf][(kk + lk) * SB + wn + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + 4 * lk + r, gn = n0 + wn + j * 16 + lr;
        if (gm < M && gn < N) C[gm * ldc + gn] = (double)acc[i][j][r];
      }
}

template <int BM, int BN, int WGM, int WGN, int TAG>
__global__ __launch_bounds__(WGM * WGN * 64) void gemm_f32x1_kernel(int M, int N, int K,
                                                                    const double* __restrict__ A,
                                                                    int lda,
                                                                    const double* __restrict__ B,
                                                                    int ldb,
                                                                    double* __restrict__ C,
                                                                    int ldc) {
  __shared__ float As[2][BM * 17];
  __shared__ float Bs[2][16 * (BN + 1)];
  const int ntn = (N + BN - 1) / BN;
  f32_tile<BM, BN, WGM, WGN>(M, N, K, A, lda, B, ldb, C, ldc, (blockIdx.x / ntn) * BM,
                             (blockIdx.x % ntn) * BN, As, Bs);
}

// Grouped FP32 products: the persistent tile queue of dgemm_rr_grouped
// over f32_tile.
__global__ __launch_bounds__(256) void gemm_f32x1_grouped(GroupTable tab, int* __restrict__ counter) {
  __shared__ float As[2][96 * 17];
  __shared__ float Bs[2][16 * 97];
  __shared__ int claim;
  for (;;) {
    if (threadIdx.x == 0) claim = atomicAdd(counter, 1);
    __syncthreads();
    const int t = claim;
    __syncthreads();
    if (t >= tab.total) break;
    int p = 0;
    while (p + 1 < tab.count && tab.tile_start[p + 1] <= t) ++p;
    const GroupProblem& q = tab.p[p];
    const int local = t - tab.tile_start[p];
    const int ntn = (q.N + 95) / 96;
    f32_tile<96, 96, 2, 2>(q.M, q.N, q.K, q.A, q.lda, q.B, q.ldb, q.C, q.ldc, (local / ntn) * 96,
                           (local % ntn) * 96, As, Bs);
  }
}

namespace {

template <int S>
void run_bf16s(Context& ctx, int M, int N, int K, const double* A, long long lda,
               const double* B, long long ldb, double* C, const OutMap& om, int cls,
               SliceCache* bc = nullptr) {
  const int tag = cls == 0 ? 0 : 1;
  const int Kp = (K + 31) / 32 * 32;
  const size_t aq = (size_t)S * M * Kp, bq = (size_t)S * N * Kp;
  const size_t need = (aq + bq) * sizeof(__bf16) + (size_t)(M + N) * sizeof(double) + 256;
  if (ctx.mixed_ws.bytes < need) {
    CTM_HIP(hipStreamSynchronize(ctx.stream));
    ctx.mixed_ws.alloc(need);
  }
  char* base = (char*)ctx.mixed_ws.p;
  __bf16* Aq = (__bf16*)base;
  __bf16* Bq = Aq + aq;
  double* amax = (double*)(((uintptr_t)(Bq + bq) + 255) & ~(uintptr_t)255);
  double* bmax = amax + M;
  // a cached B is sliced once, into the cache, and reused while valid
  bool slice_b = true;
  if (bc) {
    if (bc->valid && bc->S == S && bc->N == N && bc->K == K && bc->src == B) {
      slice_b = false;
    } else {
      if (bc->q.bytes < bq * sizeof(__bf16) || bc->mx.bytes < (size_t)N * sizeof(double)) {
        CTM_HIP(hipStreamSynchronize(ctx.stream));
        bc->q.alloc(bq * sizeof(__bf16));
        bc->mx.alloc((size_t)N * sizeof(double));
      }
      bc->S = S;
      bc->N = N;
      bc->K = K;
      bc->src = B;
      bc->valid = true;
    }
    Bq = (__bf16*)bc->q.p;
    bmax = (double*)bc->mx.p;
  }
  // maxima: rows of A (contiguous; that kernel also clears bmax when B is
  // sliced here), columns of B (atomic max over K slabs)
  hipLaunchKernelGGL(rowmax_contig_kernel, dim3((M + kRowmaxRows - 1) / kRowmaxRows),
                     dim3(64 * kRowmaxRows), 0, ctx.stream, A, lda, M, K, amax,
                     bmax, slice_b ? N : 0);
  const int kslab = 32;
  if (slice_b)
    hipLaunchKernelGGL(colmax_kernel, dim3((N + 255) / 256, (K + kslab - 1) / kslab), dim3(256), 0,
                       ctx.stream, B, ldb, K, N, kslab, (unsigned long long*)bmax);
  CTM_HIP(hipGetLastError());
  // slices, K-step-major: A by rows, B^T (the columns of B)
  hipLaunchKernelGGL((split_kernel<S>), dim3(Kp / 64 + (Kp % 64 ? 1 : 0), (M + 63) / 64),
                     dim3(256), 0, ctx.stream, A, lda, 1LL, M, K, Kp, amax, Aq);
  if (slice_b)
    hipLaunchKernelGGL((split_kernel<S>), dim3(Kp / 64 + (Kp % 64 ? 1 : 0), (N + 63) / 64),
                       dim3(256), 0, ctx.stream, B, 1LL, ldb, N, K, Kp, bmax, Bq);
  CTM_HIP(hipGetLastError());
  const long long tiles = (long long)((M + 127) / 128) * ((N + 127) / 128);
  CTM_REQUIRE(tiles <= INT_MAX, "gemm_mixed: grid too large");
  // timing class 0 covers the slice product only (the slicing is class 1)
  ScopedTimer t0(ctx, cls == 0 ? 0 : -1, 2.0 * M * N * (double)K);
  if (tag == 0)
    hipLaunchKernelGGL((gemm_bf16s_kernel<S, 0>), dim3((unsigned)tiles), dim3(512), 0, ctx.stream,
                       M, N, Kp, Aq, Bq, amax, bmax, C, om);
  else
    hipLaunchKernelGGL((gemm_bf16s_kernel<S, 1>), dim3((unsigned)tiles), dim3(512), 0, ctx.stream,
                       M, N, Kp, Aq, Bq, amax, bmax, C, om);
  CTM_HIP(hipGetLastError());
}

}  // namespace

bool mixed_mode_supported(int mode) {
  return mode == CTM_PREC_F64 || mode == CTM_PREC_F32 || mode == CTM_PREC_BF16X3 ||
         mode == CTM_PREC_BF16X4;
}

// The reduced-precision kernels cover plain row-major products C = A B with
// 16-byte aligned operands and 32-bit offsets.
static bool mixed_plain(int mode, int M, int N, int K, double alpha, View A, View B, double beta,
                        ViewOut C, int batch) {
  const long long i32 = INT_MAX;
  return mode != CTM_PREC_F64 && alpha == 1.0 && beta == 0.0 && batch == 1 && A.cs == 1 &&
         B.cs == 1 && C.cs == 1 && M >= 1 && N >= 1 && K >= 1 && (long long)M * A.rs + K < i32 &&
         (long long)K * B.rs + N < i32 && (long long)M * C.rs + N < i32 &&
         ((reinterpret_cast<uintptr_t>(A.p) | reinterpret_cast<uintptr_t>(B.p)) & 15) == 0 &&
         A.rs % 2 == 0 && B.rs % 2 == 0;
}

int grouped_kind(const Context& ctx, int mode, int M, int N, int K, View A, View B, ViewOut C) {
  if (mixed_plain(mode, M, N, K, 1.0, A, B, 0.0, C, 1)) return mode == CTM_PREC_F32 ? 2 : 0;
  return rr_grouped_ok(ctx, M, N, K, A, B, C) ? 1 : 0;
}

void gemm_grouped(Context& ctx, int kind, const GroupProblem* probs, int count, int* counter) {
  CTM_REQUIRE(kind == 1 || kind == 2, "gemm_grouped: unknown kernel kind");
  for (int s = 0; s < count; s += kGroupMax) {
    GroupTable tab{};
    tab.count = std::min(kGroupMax, count - s);
    long long total = 0;
    for (int i = 0; i < tab.count; ++i) {
      const GroupProblem& q = probs[s + i];
      CTM_REQUIRE(q.M >= 1 && q.N >= 1 && q.K >= 1, "gemm_grouped: empty problem");
      tab.p[i] = q;
      tab.tile_start[i] = (int)total;
      total += (long long)((q.M + 95) / 96) * ((q.N + 95) / 96);
      CTM_REQUIRE(total < INT_MAX / 2, "gemm_grouped: too many tiles");
    }
    tab.tile_start[tab.count] = (int)total;
    tab.total = (int)total;
    if (kind == 1) {
      gemm_grouped_f64(ctx, tab, counter);
    } else {
      fill_zero_int(ctx, counter, 1);
      const int grid = (int)std::min<long long>(total, 3LL * ctx.num_cus);
      hipLaunchKernelGGL(gemm_f32x1_grouped, dim3(grid), dim3(256), 0, ctx.stream, tab, counter);
      CTM_HIP(hipGetLastError());
    }
  }
}

void gemm_mixed(Context& ctx, int mode, int M, int N, int K, double alpha, View A, View B,
                double beta, ViewOut C, int batch, int cls) {
  CTM_REQUIRE(mixed_mode_supported(mode), "precision mode not available");
  const long long i32 = INT_MAX;
  const bool plain = mixed_plain(mode, M, N, K, alpha, A, B, beta, C, batch);
  if (!plain) {
    // FP64 for every contraction the reduced-precision kernels do not cover
    gemm_f64(ctx, M, N, K, alpha, A, B, beta, C, batch, cls);
    return;
  }
  const double flops = 2.0 * M * N * (double)K;
  ScopedTimer t1(ctx, 1, flops);
  const int tag = cls == 0 ? 0 : 1;
  if (mode == CTM_PREC_F32) {
    ScopedTimer t0(ctx, cls == 0 ? 0 : -1, flops);
    CTM_REQUIRE((long long)((M + 63) / 64) * ((N + 63) / 64) <= i32, "gemm_mixed: grid too large");
    // tile candidates: 96 x 96 (2 x 2 waves), 128 x 128 (4 x 2), 64 x 64 (2 x 2), all with the
    // same K order; the autotuner (when on) keeps the fastest per shape
    auto run = [&](int v) {
      const int bm = v == 1 ? 128 : (v == 2 ? 64 : 96);
      const dim3 g((unsigned)(((M + bm - 1) / bm) * ((N + bm - 1) / bm)));
#define CTM_F32(BM_, WGM_, WGN_)                                                                   \
  do {                                                                                            \
    if (tag == 0)                                                                                 \
      hipLaunchKernelGGL((gemm_f32x1_kernel<BM_, BM_, WGM_, WGN_, 0>), g, dim3(WGM_ * WGN_ * 64), 0, \
                         ctx.stream, M, N, K, A.p, (int)A.rs, B.p, (int)B.rs, C.p, (int)C.rs);     \
    else                                                                                          \
      hipLaunchKernelGGL((gemm_f32x1_kernel<BM_, BM_, WGM_, WGN_, 1>), g, dim3(WGM_ * WGN_ * 64), 0, \
                         ctx.stream, M, N, K, A.p, (int)A.rs, B.p, (int)B.rs, C.p, (int)C.rs);     \
  } while (0)
      if (v == 1) CTM_F32(128, 4, 2);
      else if (v == 2) CTM_F32(64, 2, 2);
      else CTM_F32(96, 2, 2);
#undef CTM_F32
      CTM_HIP(hipGetLastError());
    };
    run(pick_variant(ctx, 1, M, N, K, cls, 3, run));
  } else if (mode == CTM_PREC_BF16X3) {
    run_bf16s<3>(ctx, M, N, K, A.p, A.rs, B.p, B.rs, C.p, OutMap::plain(M, N, C.rs), cls);
  } else {
    run_bf16s<4>(ctx, M, N, K, A.p, A.rs, B.p, B.rs, C.p, OutMap::plain(M, N, C.rs), cls);
  }
}

bool gemm_slices_split_out(Context& ctx, int mode, int M, int N, int K, View A, View B, double* C,
                           const OutMap& om, int cls, SliceCache* bc) {
  if (mode != CTM_PREC_BF16X3 && mode != CTM_PREC_BF16X4) return false;
  // the operand conditions of the slice path; C's placement is om's
  if (!mixed_plain(mode, M, N, K, 1.0, A, B, 0.0, ViewOut{C, (long long)N, 1, 0}, 1)) return false;
  CTM_REQUIRE(om.r2 >= 1 && om.c2 >= 1, "gemm_slices_split_out: bad output map");
  ScopedTimer t1(ctx, 1, 2.0 * M * N * (double)K);
  if (mode == CTM_PREC_BF16X3) run_bf16s<3>(ctx, M, N, K, A.p, A.rs, B.p, B.rs, C, om, cls, bc);
  else run_bf16s<4>(ctx, M, N, K, A.p, A.rs, B.p, B.rs, C, om, cls, bc);
  return true;
}

}  // namespace ctm
