// FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
// C = alpha * A * B + beta * C for strided (optionally batched) operands.
// One workgroup computes a BM x BN tile of C; its waves are arranged
// WGM x WGN, each owning a (BM/WGM) x (BN/WGN) block made of 16x16 MFMA
// tiles.  K advances in steps of BK through a double-buffered LDS stage:
// while the MFMAs consume one stage, the next K tile is already loaded into
// registers and written to the other stage, so one barrier per K tile
// suffices.  LDS tiles are stored k-major (As[k][m], Bs[k][n]) so that the
// 16 lanes reading one MFMA operand column touch 16 consecutive doubles.
//
// Operand fragments (checked on the device with an in-bounds probe):
//   A: lane l holds A[l % 16][k0 + l / 16], B: lane l holds B[k0 + l / 16][l % 16],
//   accumulator register r of lane l holds C[4 r + l / 16][l % 16].
//
// Split-K: for skinny outputs the K range is cut into `ksplit` chunks; each
// chunk writes its partial tile to a workspace and a second kernel sums the
// chunks in a fixed order (deterministic) and applies alpha and beta.
//
// Large products of two row-major operands (the half-system products, the
// cut matrix and the site-tensor absorption) take a separate kernel,
// dgemm_rr: 16-byte global loads, A staged [m][k] and B [k][n] in LDS, and a
// 96 x 96 tile with 2 x 2 waves, so three workgroups share a CU (53 KB LDS
// each) and an n = 2592 product (27 x 27 tiles) runs as one pass over the
// 256 CUs.  Tiles are assigned XCD by XCD (see xcd_tile), which cuts the L2
// misses on re-read operand panels.  Its template tag only separates the cut-matrix products from
// the other users in kernel traces.
#include "internal.hpp"

#include <cstdint>
#include <functional>

namespace ctm {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

// C = A B with A (row stride lda) and B (row stride ldb) both
// contiguous along their second index, lda and ldb even and both base
// pointers 16-byte aligned (checked by the dispatcher).  blockIdx.x is the
// tile (row-major over the tile grid), blockIdx.y the batch.
// Offsets within one matrix are 32-bit (the dispatcher checks that they
// fit), which keeps the address arithmetic of the loads short.
//
// Split-K: blockIdx.z selects the K chunk [z kchunk, (z + 1) kchunk).  With
// a workspace W (ksplit > 1, or a product with alpha != 1, beta != 0 or a
// strided C) each chunk's partial product goes to W (row stride N, one M x N
// slab per (batch, chunk)) for the fixed-order reduction, which also applies
// alpha and beta.
// One BM x BN tile of C = A B at (m0, n0) over the K range [kbeg, kend),
// for dgemm_rr and the grouped kernel: 16-byte global loads into registers
// (two 8-byte loads for an operand whose rows are not 16-byte aligned, VA /
// VB false),
// A staged [m][k] and B [k][n] in double-buffered LDS (one barrier per K
// tile), and a plain store of the accumulators.  An alpha / beta epilogue
// here costs enough registers to drop the occupancy to two workgroups per
// CU, so the dispatchers send only C = A B products to it.
template <int BM, int BN, int BK, int WGM, int WGN, bool VA = true, bool VB = true>
__device__ __forceinline__ void rr_tile(int M, int N, const double* __restrict__ A, int lda,
                                        const double* __restrict__ B, int ldb,
                                        double* __restrict__ C, int ldc, int m0, int n0, int kbeg,
                                        int kend, double (*As)[BM * (BK + 2)],
                                        double (*Bs)[BK * (BN + 2)]) {
  constexpr int NT = WGM * WGN * 64;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TI = WM / 16, TJ = WN / 16;
  constexpr int SA = BK + 2, SB = BN + 2;
  constexpr int AV = BM * BK / 2 / NT;  // 16-byte loads of A per thread per K tile
  constexpr int BV = BK * BN / 2 / NT;
  static_assert(AV >= 1 && BV >= 1 && (BM * BK / 2) % NT == 0 && (BK * BN / 2) % NT == 0,
                "tile does not split evenly into 16-byte loads");
  static_assert(TI * 16 == WM && TJ * 16 == WN, "wave tile must be a multiple of 16");
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
      if (VA && (full_m || gm < M) && gk + 1 < kend) {
        ra[e] = *(const d2v*)(A + gm * lda + gk);
      } else {
        ra[e].x = (gm < M && gk < kend) ? A[gm * lda + gk] : 0.0;
        ra[e].y = (gm < M && gk + 1 < kend) ? A[gm * lda + gk + 1] : 0.0;
      }
    }
#pragma unroll
    for (int e = 0; e < BV; ++e) {
      const int p = tid + e * NT;
      const int k = p / (BN / 2), c = (p % (BN / 2)) * 2;
      const int gk = kt + k, gn = n0 + c;
      if (VB && gk < kend && (full_n || gn + 1 < N)) {
        rb[e] = *(const d2v*)(B + gk * ldb + gn);
      } else {
        rb[e].x = (gk < kend && gn < N) ? B[gk * ldb + gn] : 0.0;
        rb[e].y = (gk < kend && gn + 1 < N) ? B[gk * ldb + gn + 1] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AV; ++e) {
      const int p = tid + e * NT;
      *(d2v*)(&As[buf][(p / (BK / 2)) * SA + (p % (BK / 2)) * 2]) = ra[e];
    }
#pragma unroll
    for (int e = 0; e < BV; ++e) {
      const int p = tid + e * NT;
      *(d2v*)(&Bs[buf][(p / (BN / 2)) * SB + (p % (BN / 2)) * 2]) = rb[e];
    }
  };

  d4v acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
  const int lr = lane & 15, lk = lane >> 4;
  load(kbeg);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int kt = kbeg; kt < kend; kt += BK) {
    const bool more = kt + BK < kend;
    if (more) load(kt + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double av[TI], bv[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) av[i] = As[buf][(wm + i * 16 + lr) * SA + kk + lk];
#pragma unroll
      for (int j = 0; j < TJ; ++j) bv[j] = Bs[buf][(kk + lk) * SB + wn + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
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
        const int gm = m0 + wm + i * 16 + 4 * r + lk, gn = n0 + wn + j * 16 + lr;
        if (gm < M && gn < N) C[gm * ldc + gn] = acc[i][j][r];
      }
}

template <int BM, int BN, int BK, int WGM, int WGN, int TAG, bool VA = true, bool VB = true>
__global__ __launch_bounds__(WGM * WGN * 64) void dgemm_rr(
    int M, int N, int K, const double* __restrict__ A, int lda, long long abs_,
    const double* __restrict__ B, int ldb, long long bbs, double* __restrict__ C, int ldc,
    long long cbs, int ksplit, int kchunk, double* __restrict__ W) {
  __shared__ double As[2][BM * (BK + 2)];
  __shared__ double Bs[2][BK * (BN + 2)];
  int tm, tn;
  xcd_tile<8>(blockIdx.x, (M + BM - 1) / BM, (N + BN - 1) / BN, tm, tn);
  A += blockIdx.y * abs_;
  B += blockIdx.y * bbs;
  if (W) {
    C = W + ((long long)blockIdx.y * ksplit + blockIdx.z) * ((long long)M * N);
    ldc = N;
  } else {
    C += blockIdx.y * cbs;
  }
  const int kbeg = blockIdx.z * kchunk;
  rr_tile<BM, BN, BK, WGM, WGN, VA, VB>(M, N, A, lda, B, ldb, C, ldc, tm * BM, tn * BN, kbeg,
                                        min(K, kbeg + kchunk), As, Bs);
}

// Grouped products: one persistent launch over a table of independent
// C = A B problems (row-major, the dgemm_rr conditions), tiles numbered
// problem by problem and claimed one at a time from a device counter, which
// the host clears before the launch.  Every tile is computed exactly as
// dgemm_rr computes it without split-K, so the results do not depend on which
// workgroup takes which tile.  Each workgroup leaves once a claim passes the
// last tile.
template <int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(WGM * WGN * 64) void dgemm_rr_grouped(GroupTable tab,
                                                                    int* __restrict__ counter) {
  __shared__ double As[2][BM * (BK + 2)];
  __shared__ double Bs[2][BK * (BN + 2)];
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
    const int ntn = (q.N + BN - 1) / BN;
    rr_tile<BM, BN, BK, WGM, WGN>(q.M, q.N, q.A, q.lda, q.B, q.ldb, q.C, q.ldc, (local / ntn) * BM,
                                  (local % ntn) * BN, 0, q.K, As, Bs);
  }
}

template <int BM, int BN, int BK, int WGM, int WGN, bool A_KC, bool B_NC>
__global__ __launch_bounds__(WGM * WGN * 64) void dgemm_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, long long ars,
    long long acs, long long abs_, const double* __restrict__ B, long long brs, long long bcs,
    long long bbs, double beta, double* __restrict__ C, long long crs, long long ccs,
    long long cbs, int ksplit, int kchunk, double* __restrict__ W) {
  constexpr int NT = WGM * WGN * 64;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TI = WM / 16, TJ = WN / 16;
  constexpr int PAD = 2;
  constexpr int LDA = BM + PAD, LDB = BN + PAD;
  constexpr int LA = BM * BK / NT;  // A elements loaded per thread per K tile
  constexpr int LB = BK * BN / NT;
  static_assert(LA >= 1 && LB >= 1, "tile too small for the thread count");
  static_assert(TI >= 1 && TJ >= 1, "wave tile must hold a 16x16 MFMA tile");
  __shared__ double As[2][BK][LDA];
  __shared__ double Bs[2][BK][LDB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave / WGN) * WM;
  const int wn = (wave % WGN) * WN;
  const int bz = blockIdx.z;
  const int batch = bz / ksplit;
  const int split = bz - batch * ksplit;
  const int m0 = blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  A += batch * abs_;
  B += batch * bbs;

  // thread -> element mapping of the global loads (coalesced along the
  // contiguous dimension of each operand)
  int a_r, a_k;  // first element handled: row within tile, k within tile
  if (A_KC) {
    constexpr int TPR = BK / LA;
    a_r = tid / TPR;
    a_k = (tid % TPR) * LA;
  } else {
    constexpr int TPK = BM / LA;
    a_k = tid / TPK;
    a_r = (tid % TPK) * LA;
  }
  int b_k, b_c;
  if (B_NC) {
    constexpr int TPK = BN / LB;
    b_k = tid / TPK;
    b_c = (tid % TPK) * LB;
  } else {
    constexpr int TPC = BK / LB;
    b_c = tid / TPC;
    b_k = (tid % TPC) * LB;
  }

  double ra[LA], rb[LB];
  auto load_tiles = [&](int kt) {
#pragma unroll
    for (int e = 0; e < LA; ++e) {
      const int r = A_KC ? a_r : a_r + e;
      const int k = A_KC ? a_k + e : a_k;
      const int gm = m0 + r, gk = kt + k;
      ra[e] = (gm < M && gk < kend) ? A[(long long)gm * ars + (long long)gk * acs] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      const int k = B_NC ? b_k : b_k + e;
      const int c = B_NC ? b_c + e : b_c;
      const int gk = kt + k, gn = n0 + c;
      rb[e] = (gk < kend && gn < N) ? B[(long long)gk * brs + (long long)gn * bcs] : 0.0;
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int e = 0; e < LA; ++e) {
      const int r = A_KC ? a_r : a_r + e;
      const int k = A_KC ? a_k + e : a_k;
      As[buf][k][r] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      const int k = B_NC ? b_k : b_k + e;
      const int c = B_NC ? b_c + e : b_c;
      Bs[buf][k][c] = rb[e];
    }
  };

  d4v acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};

  const int lr = lane & 15;
  const int lk = lane >> 4;
  int buf = 0;
  if (kbeg < kend) {
    load_tiles(kbeg);
    store_tiles(0);
  }
  __syncthreads();
  for (int kt = kbeg; kt < kend; kt += BK) {
    const bool more = kt + BK < kend;
    if (more) load_tiles(kt + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double av[TI], bv[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) av[i] = As[buf][kk + lk][wm + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < TJ; ++j) bv[j] = Bs[buf][kk + lk][wn + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (more) store_tiles(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // epilogue
  if (ksplit > 1) {
    double* Wp = W + (long long)bz * M * N;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wm + i * 16 + 4 * r + lk;
          const int gn = n0 + wn + j * 16 + lr;
          if (gm < M && gn < N) Wp[(long long)gm * N + gn] = acc[i][j][r];
        }
  } else {
    double* Cp = C + batch * cbs;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wm + i * 16 + 4 * r + lk;
          const int gn = n0 + wn + j * 16 + lr;
          if (gm < M && gn < N) {
            double* c = Cp + (long long)gm * crs + (long long)gn * ccs;
            const double v = alpha * acc[i][j][r];
            *c = (beta == 0.0) ? v : v + beta * (*c);
          }
        }
  }
}

// Sum of the split-K partial tiles in split order, then alpha / beta.
__global__ void splitk_reduce_kernel(int M, int N, int ksplit, int batch, double alpha,
                                     const double* __restrict__ W, double beta,
                                     double* __restrict__ C, long long crs, long long ccs,
                                     long long cbs) {
  const long long MN = (long long)M * N;
  const long long total = MN * batch;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long bt = idx / MN;
    const long long rem = idx - bt * MN;
    const int m = (int)(rem / N), n = (int)(rem - (long long)(rem / N) * N);
    const double* w = W + bt * ksplit * MN + rem;
    // eight loads in flight, then the sums in split order
    double s = 0.0;
    int z = 0;
    for (; z + 8 <= ksplit; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = w[(z + u) * MN];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; z < ksplit; ++z) s += w[z * MN];
    double* c = C + bt * cbs + (long long)m * crs + (long long)n * ccs;
    const double v = alpha * s;
    *c = (beta == 0.0) ? v : v + beta * (*c);
  }
}

__global__ void scale_matrix_kernel(int M, int N, int batch, double beta, double* C,
                                    long long crs, long long ccs, long long cbs) {
  const long long MN = (long long)M * N;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < MN * batch;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long bt = idx / MN;
    const long long rem = idx - bt * MN;
    const int m = (int)(rem / N), n = (int)(rem % N);
    double* c = C + bt * cbs + (long long)m * crs + (long long)n * ccs;
    *c = (beta == 0.0) ? 0.0 : beta * (*c);
  }
}

namespace {

struct Cfg {
  int BM, BN;
};

template <int BM, int BN, int BK, int WGM, int WGN>
void launch_cfg(Context& ctx, bool akc, bool bnc, dim3 grid, int M, int N, int K, double alpha,
                View A, View B, double beta, ViewOut C, int ksplit, int kchunk, double* W) {
  const dim3 block(WGM * WGN * 64);
#define CTM_LAUNCH(AK, BN_)                                                                  \
  hipLaunchKernelGGL((dgemm_kernel<BM, BN, BK, WGM, WGN, AK, BN_>), grid, block, 0,          \
                     ctx.stream, M, N, K, alpha, A.p, A.rs, A.cs, A.bs, B.p, B.rs, B.cs, B.bs, \
                     beta, C.p, C.rs, C.cs, C.bs, ksplit, kchunk, W)
  if (akc && bnc) CTM_LAUNCH(true, true);
  else if (akc && !bnc) CTM_LAUNCH(true, false);
  else if (!akc && bnc) CTM_LAUNCH(false, true);
  else CTM_LAUNCH(false, false);
#undef CTM_LAUNCH
  CTM_HIP(hipGetLastError());
}

}  // namespace

int pick_variant(Context& ctx, int kind, int M, int N, int K, int cls, int nvariants,
                 const std::function<void(int)>& run) {
  if (!ctx.autotune || nvariants <= 1) return 0;
  const auto key = std::make_tuple(kind, M, N, K, cls);
  auto it = ctx.tuned.find(key);
  if (it != ctx.tuned.end()) return it->second;
  hipEvent_t e0 = ctx.get_event(), e1 = ctx.get_event();
  int best = 0;
  float best_ms = 0.0f;
  for (int v = 0; v < nvariants; ++v) {
    run(v);
    CTM_HIP(hipEventRecord(e0, ctx.stream));
    run(v);
    run(v);
    CTM_HIP(hipEventRecord(e1, ctx.stream));
    CTM_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    CTM_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (v == 0 || ms < best_ms) { best = v; best_ms = ms; }
  }
  ctx.event_pool.push_back(e0);
  ctx.event_pool.push_back(e1);
  ctx.tuned[key] = best;
  return best;
}

// Large products of two row-major operands take dgemm_rr.
static bool rr_eligible(int M, int N, int K, View A, View B) {
  const long long i32 = 0x7fffffffLL;
  const bool fits32 = (long long)M * A.rs + K < i32 && (long long)K * B.rs + N < i32 &&
                      (long long)M * N < i32;
  return A.cs == 1 && B.cs == 1 && fits32 && M >= 384 && N >= 384 && K >= 16;
}

// dgemm_rr writes C itself (otherwise through the split-K workspace).
static bool rr_direct(int M, int N, double alpha, double beta, ViewOut C) {
  return alpha == 1.0 && beta == 0.0 && C.cs == 1 && (long long)M * C.rs + N < 0x7fffffffLL;
}

// Every row of every batch entry starts 16-byte aligned: the operand takes
// 16-byte loads.
static bool rr_vec(const View& X) {
  return ((reinterpret_cast<uintptr_t>(X.p) & 15) == 0) && (X.rs % 2 == 0) && (X.bs % 2 == 0);
}

// K chunks of a dgemm_rr product: three workgroups fit on a CU; K is split
// when the tiles fill less than one pass and every chunk keeps at least 32 K
// tiles.
// Device memory for `need` bytes of partial products: the caller's fixed
// scratch when the context has one (refused if too small), otherwise the
// context's workspace, grown when needed.
static double* splitk_space(Context& ctx, size_t need) {
  if (ctx.fixed_splitk) {
    CTM_REQUIRE(need <= ctx.fixed_splitk_bytes,
                "the product's partial sums do not fit the fixed scratch");
    return ctx.fixed_splitk;
  }
  if (ctx.splitk_ws.bytes < need) {
    CTM_HIP(hipStreamSynchronize(ctx.stream));
    ctx.splitk_ws.alloc(need);
  }
  return ctx.splitk_ws.d();
}

static int rr_ksplit(const Context& ctx, int M, int N, int K, int batch, int& kchunk) {
  constexpr int BM = 96, BN = 96, BK = 16;
  const long long tiles = (long long)((M + BM - 1) / BM) * ((N + BN - 1) / BN) * batch;
  const long long slots = 3LL * ctx.num_cus;
  int ksplit = 1;
  if (tiles < slots && K >= 64 * BK) {
    ksplit = (int)std::min<long long>(slots / tiles, K / (32 * BK));
    ksplit = std::max(1, std::min(ksplit, 16));
  }
  kchunk = K;
  if (ksplit > 1) {
    kchunk = ((K + ksplit - 1) / ksplit + BK - 1) / BK * BK;
    ksplit = (K + kchunk - 1) / kchunk;
  }
  return ksplit;
}

bool rr_grouped_ok(const Context& ctx, int M, int N, int K, View A, View B, ViewOut C) {
  int kchunk = 0;
  return rr_eligible(M, N, K, A, B) && rr_direct(M, N, 1.0, 0.0, C) && rr_vec(A) && rr_vec(B) &&
         A.bs == 0 && B.bs == 0 && rr_ksplit(ctx, M, N, K, 1, kchunk) == 1;
}

void gemm_grouped_f64(Context& ctx, const GroupTable& tab, int* counter) {
  if (tab.total <= 0) return;
  fill_zero_int(ctx, counter, 1);
  const int grid = (int)std::min<long long>(tab.total, 3LL * ctx.num_cus);
  hipLaunchKernelGGL((dgemm_rr_grouped<96, 96, 16, 2, 2>), dim3(grid), dim3(256), 0, ctx.stream,
                     tab, counter);
  CTM_HIP(hipGetLastError());
}

void gemm_f64(Context& ctx, int M, int N, int K, double alpha, View A, View B, double beta,
              ViewOut C, int batch, int cls) {
  CTM_REQUIRE(M >= 0 && N >= 0 && K >= 0 && batch >= 1, "gemm: negative size");
  if (M == 0 || N == 0) return;
  const double flops = 2.0 * M * N * (double)K * batch;
  ScopedTimer t1(ctx, 1, flops);
  ScopedTimer t0(ctx, cls == 0 ? 0 : -1, flops);
  if (K == 0) {
    const long long total = (long long)M * N * batch;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_matrix_kernel, dim3(blocks), dim3(256), 0, ctx.stream, M, N, batch,
                       beta, C.p, C.rs, C.cs, C.bs);
    CTM_HIP(hipGetLastError());
    return;
  }
  if (rr_eligible(M, N, K, A, B)) {
    constexpr int BM = 96, BN = 96, BK = 16;
    const long long i32 = 0x7fffffffLL;
    const long long tiles = (long long)((M + BM - 1) / BM) * ((N + BN - 1) / BN) * batch;
    CTM_REQUIRE(tiles <= i32 && batch <= 65535, "gemm: grid too large");
    int kchunk = K;
    int ksplit = rr_ksplit(ctx, M, N, K, batch, kchunk);
    const bool direct = rr_direct(M, N, alpha, beta, C);
    double* W = nullptr;
    if (ksplit > 1 || !direct) W = splitk_space(ctx, (size_t)ksplit * batch * M * N * sizeof(double));
    const int lda = (int)A.rs, ldb = (int)B.rs, ldc = (int)C.rs;
    const bool va = rr_vec(A), vb = rr_vec(B);
    if (ksplit == 1 && direct && ctx.autotune && va && vb) {
      // tile candidates: 96 x 96 (2 x 2 waves), 128 x 128 (4 x 2), 64 x 64 (2 x 2);
      // all accumulate K in the same order, so the choice never changes C
      auto run = [&](int v) {
        const int bm = v == 1 ? 128 : (v == 2 ? 64 : 96);
        const dim3 g((unsigned)(((M + bm - 1) / bm) * ((N + bm - 1) / bm)), batch, 1);
#define CTM_RR(BM_, WGM_, WGN_)                                                                   \
  do {                                                                                           \
    if (cls == 0)                                                                                \
      hipLaunchKernelGGL((dgemm_rr<BM_, BM_, BK, WGM_, WGN_, 0>), g, dim3(WGM_ * WGN_ * 64), 0,    \
                         ctx.stream, M, N, K, A.p, lda, A.bs, B.p, ldb, B.bs, C.p, ldc, C.bs, 1, K, \
                         nullptr);                                                              \
    else                                                                                         \
      hipLaunchKernelGGL((dgemm_rr<BM_, BM_, BK, WGM_, WGN_, 1>), g, dim3(WGM_ * WGN_ * 64), 0,    \
                         ctx.stream, M, N, K, A.p, lda, A.bs, B.p, ldb, B.bs, C.p, ldc, C.bs, 1, K, \
                         nullptr);                                                              \
  } while (0)
        if (v == 1) CTM_RR(128, 4, 2);
        else if (v == 2) CTM_RR(64, 2, 2);
        else CTM_RR(96, 2, 2);
#undef CTM_RR
        CTM_HIP(hipGetLastError());
      };
      run(pick_variant(ctx, 0, M, N, K, cls, 3, run));
      return;
    }
    const dim3 grid((unsigned)(tiles / batch), batch, ksplit), block(256);
#define CTM_RRV(TAG_, VA_, VB_)                                                                 \
  hipLaunchKernelGGL((dgemm_rr<BM, BN, BK, 2, 2, TAG_, VA_, VB_>), grid, block, 0, ctx.stream, M, N, \
                     K, A.p, lda, A.bs, B.p, ldb, B.bs, C.p, ldc, C.bs, ksplit, kchunk, W)
    const int tag = cls == 0 ? 0 : 1;
    const int v = (va ? 2 : 0) + (vb ? 1 : 0);
    if (tag == 0) {
      if (v == 3) CTM_RRV(0, true, true);
      else if (v == 2) CTM_RRV(0, true, false);
      else if (v == 1) CTM_RRV(0, false, true);
      else CTM_RRV(0, false, false);
    } else {
      if (v == 3) CTM_RRV(1, true, true);
      else if (v == 2) CTM_RRV(1, true, false);
      else if (v == 1) CTM_RRV(1, false, true);
      else CTM_RRV(1, false, false);
    }
#undef CTM_RRV
    CTM_HIP(hipGetLastError());
    if (W) {
      const long long total = (long long)M * N * batch;
      const int blocks = (int)std::min<long long>((total + 255) / 256, 8192);
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, ctx.stream, M, N,
                         ksplit, batch, alpha, W, beta, C.p, C.rs, C.cs, C.bs);
      CTM_HIP(hipGetLastError());
    }
    return;
  }
  // Contiguity of the operands decides the load mapping (correct either way).
  const bool akc = (A.cs == 1);
  const bool bnc = (B.cs == 1);
  int BM, BN;
  if (M >= 1024 && N >= 1024) { BM = 128; BN = 128; }
  else if (N <= 48) { BM = 64; BN = 32; }
  else { BM = 64; BN = 64; }
  // The split-K factor follows from the tile count of this choice.  A skinny
  // side of at most 96 then takes a narrower tile (64 x 32, or 32 x 64 when
  // only M is small): less of the tile is padding, and since the K chunks do
  // not change, neither does C.
  const long long tiles = (long long)((M + BM - 1) / BM) * ((N + BN - 1) / BN) * batch;
  if (BM == 64 && BN == 64) {
    if (N <= 96) BN = 32;
    else if (M <= 96) BM = 32;
  }
  const int BK = 16;
  int ksplit = 1;
  const long long target = 2LL * ctx.num_cus;
  if (tiles < target && K >= 8 * BK) {
    ksplit = (int)std::min<long long>((target + tiles - 1) / tiles, K / (4 * BK));
    ksplit = std::max(1, std::min(ksplit, 64));
  }
  int kchunk = K;
  double* W = nullptr;
  if (ksplit > 1) {
    kchunk = (K + ksplit - 1) / ksplit;
    kchunk = (kchunk + BK - 1) / BK * BK;
    ksplit = (K + kchunk - 1) / kchunk;
    W = splitk_space(ctx, (size_t)ksplit * batch * M * N * sizeof(double));
  }
  const dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch * ksplit);
  CTM_REQUIRE(grid.y <= 65535 && grid.z <= 65535, "gemm: grid too large");
  if (BM == 128) launch_cfg<128, 128, 16, 2, 2>(ctx, akc, bnc, grid, M, N, K, alpha, A, B, beta, C, ksplit, kchunk, W);
  else if (BN == 32) launch_cfg<64, 32, 16, 2, 2>(ctx, akc, bnc, grid, M, N, K, alpha, A, B, beta, C, ksplit, kchunk, W);
  else if (BM == 32) launch_cfg<32, 64, 16, 2, 2>(ctx, akc, bnc, grid, M, N, K, alpha, A, B, beta, C, ksplit, kchunk, W);
  else launch_cfg<64, 64, 16, 2, 2>(ctx, akc, bnc, grid, M, N, K, alpha, A, B, beta, C, ksplit, kchunk, W);
  if (ksplit > 1) {
    const long long total = (long long)M * N * batch;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, ctx.stream, M, N,
                       ksplit, batch, alpha, W, beta, C.p, C.rs, C.cs, C.bs);
    CTM_HIP(hipGetLastError());
  }
}

}  // namespace ctm
