// Small and memory-bound kernels of the CTMRG path: fills, normalisation,
// reductions, the counter-based generator, the Gram-Cholesky factor used to
// orthonormalise the subspace of the truncated projector SVD, the one-sided
// Jacobi SVD of small square matrices, and column scalings.
#include <cfloat>
#include <mutex>
#include <utility>
#include <vector>
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace ctm {

namespace {

constexpr int kRedBlocks = 512;  // fixed partition of the two-stage reductions
// arrays up to this size are max-abs normalised by one workgroup (a chi = 96
// corner has 9216 elements); 1024 threads x 16 elements
constexpr int kNormaliseOneGroup = 16384;

__device__ inline unsigned long long splitmix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Standard normal number k of the stream `seed` (SplitMix64 outputs 2k+1 and
// 2k+2 of the sequence seed + i * golden-gamma, then Box-Muller).
__device__ inline double normal_at(unsigned long long seed, unsigned long long k) {
  const unsigned long long g = 0x9e3779b97f4a7c15ULL;
  const unsigned long long x1 = splitmix64(seed + (2 * k + 1) * g);
  const unsigned long long x2 = splitmix64(seed + (2 * k + 2) * g);
  const double u1 = ((double)(x1 >> 11) + 1.0) * (1.0 / 9007199254740992.0);  // (0, 1]
  const double u2 = (double)(x2 >> 11) * (1.0 / 9007199254740992.0);          // [0, 1)
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Reciprocal and reciprocal square root of a normal, finite double: the
// hardware estimate refined by two Newton steps (full double precision).
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * r, r, 0.5);
  r = fma(r, e, r);
  e = fma(-h * r, r, 0.5);
  return fma(r, e, r);
}

template <typename T>
__global__ void fill_kernel(T* p, size_t n, T v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void copy_kernel(double* __restrict__ d, const double* __restrict__ s, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

__global__ void copy_block_kernel(double* __restrict__ dst, long long ldd,
                                  const double* __restrict__ src, long long lds, int rows,
                                  int cols) {
  const long long total = (long long)rows * cols;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long i = idx / cols;
    const long long j = idx - i * cols;
    dst[i * ldd + j] = src[i * lds + j];
  }
}

__global__ void fill_normal_kernel(double* p, size_t n, unsigned long long seed,
                                   unsigned long long ctr) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = normal_at(seed, ctr + i);
}

// block-wide reductions over 256 threads
__device__ inline double block_max256(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
__device__ inline double block_sum256(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// max |p| per block; a non-finite entry makes the block's value +inf
__global__ void maxabs_partial_kernel(const double* __restrict__ p, size_t n, double* partial) {
  __shared__ double sh[256];
  double m = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double v = p[i];
    m = isfinite(v) ? fmax(m, fabs(v)) : INFINITY;
  }
  m = block_max256(m, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// 1 / m for the max-abs m of a normalised array (1 when m is 0 or not
// finite: the array is left as it is and the flag raised).  One thread of the
// launch records the flag, the log scale and the factor.
__device__ inline double normalise_factor(double m, bool record, double* log_slot, int* flag,
                                          double* inv_keep) {
  const bool bad = !(m < INFINITY) || m == 0.0;
  const double inv = bad ? 1.0 : 1.0 / m;
  if (record) {
    if (bad)
      *flag = 1;
    else
      *log_slot += log(m);
    if (inv_keep) *inv_keep = inv;
  }
  return inv;
}

// Second stage: every workgroup takes the maximum over the nb partial maxima
// itself (the same value in each) and scales its share of p.
__global__ void scale_by_max_kernel(double* p, size_t n, const double* __restrict__ partial,
                                    int nb, double* log_slot, int* flag, double* inv_keep) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, partial[i]);
  m = block_max256(m, sh);
  const double f = normalise_factor(m, blockIdx.x == 0 && threadIdx.x == 0, log_slot, flag,
                                    inv_keep);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] *= f;
}

// An array of at most kNormaliseOneGroup elements (a corner) in one workgroup
// of 1024 threads: every thread loads its (at most 16) elements at once into
// registers, the maximum goes through wave shuffles and LDS, and the scaled
// values are written from the registers; one launch, one read.
constexpr int kNormaliseThreads = 1024;
constexpr int kNormalisePerThread = 16;
static_assert(kNormaliseOneGroup <= kNormaliseThreads * kNormalisePerThread,
              "one workgroup holds a whole small array in registers");
__global__ __launch_bounds__(kNormaliseThreads) void normalise_one_group_kernel(
    double* p, int n, double* log_slot, int* flag, double* inv_keep) {
  __shared__ double wmax[kNormaliseThreads / 64];
  const int t = threadIdx.x;
  double v[kNormalisePerThread];
#pragma unroll
  for (int u = 0; u < kNormalisePerThread; ++u) {
    const int i = t + u * kNormaliseThreads;
    v[u] = i < n ? p[i] : 0.0;
  }
  double m = 0.0;
#pragma unroll
  for (int u = 0; u < kNormalisePerThread; ++u) m = isfinite(v[u]) ? fmax(m, fabs(v[u])) : INFINITY;
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((t & 63) == 0) wmax[t >> 6] = m;
  __syncthreads();
  m = 0.0;
#pragma unroll
  for (int w = 0; w < kNormaliseThreads / 64; ++w) m = fmax(m, wmax[w]);
  const double f = normalise_factor(m, t == 0, log_slot, flag, inv_keep);
#pragma unroll
  for (int u = 0; u < kNormalisePerThread; ++u) {
    const int i = t + u * kNormaliseThreads;
    if (i < n) p[i] = v[u] * f;
  }
}

__global__ void dot_partial_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                   size_t n, double* partial) {
  __shared__ double sh[256];
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void sum_final_kernel(const double* partial, int nb, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------------------------ Gram-Cholesky

// 64-bit value of lane `lane` (wave-uniform) of a wave.
__device__ inline double readlane64(double x, int lane) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Second pass of a CholeskyQR: for the Gram matrix G = Q^T Q of columns that
// the first pass left orthonormal up to E = G - I with max |E_ij| <= tau,
// W = (3 I - G) / 2 = I - E / 2 makes Q W orthonormal up to W G W - I =
// -(3/4) E^2 + O(E^3) (one step of the Newton-Schulz iteration for the polar
// factor), with no dependent column.  Called by all threads of the Cholesky
// kernel's workgroup: writes W and dep and returns true, or returns false
// (a larger or non-finite E, e.g. after refilled columns) having written
// nothing, and the Cholesky inverse runs as usual.
__device__ bool near_identity_inverse(const double* __restrict__ G, int b, double tau,
                                      double* __restrict__ Wout, int* __restrict__ dep) {
  __shared__ double red[16];
  __shared__ int ok;
  const int t = threadIdx.x, nt = blockDim.x;
  double e = 0.0;
  for (int idx = t; idx < b * b; idx += nt) {
    const int i = idx / b, j = idx - (idx / b) * b;
    const double g = G[idx] - (i == j ? 1.0 : 0.0);
    e = (g == g) ? fmax(e, fabs(g)) : INFINITY;  // fmax would drop a NaN
  }
  for (int o = 32; o > 0; o >>= 1) e = fmax(e, __shfl_xor(e, o));
  if ((t & 63) == 0) red[t >> 6] = e;
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int w = 0; w < (nt + 63) / 64; ++w) m = fmax(m, red[w]);
    ok = m <= tau;
  }
  __syncthreads();
  if (!ok) return false;
  for (int idx = t; idx < b * b; idx += nt) {
    const int i = idx / b, j = idx - (idx / b) * b;
    Wout[idx] = (i == j ? 1.5 : 0.0) - 0.5 * G[idx];
  }
  for (int j = t; j < b; j += nt) dep[j] = 0;
  return true;
}

// Cholesky factor and its inverse in one pass, register-tiled: TG x TG
// threads, thread (ti, tj) owning entries (ti + TG r, tj + TG c), r, c < NR =
// NB / TG, of the symmetric Schur complement S and of X (both NB x NB, zero
// beyond b so that no row or column needs a guard).  Pivot k eliminates
// column k below the pivot (S -= s_k s_k^T / piv on the trailing block; only
// the upper triangle of S is ever read, so blocks below the diagonal are not
// updated) and applies the same row operation to X, which stays lower
// triangular; then row k of X is scaled by 1/sqrt(piv).  At the end
// X = R^-T, where R^T R is the column-scaled Gram matrix, so W = D^-1 X^T has
// Z W orthonormal.  Columns whose pivot falls below dep_tol (numerically
// dependent) are skipped: no elimination, flag set.
//
// The pivots are taken PB at a time.  The panel of rows k0 .. k0 + PB - 1 of
// S and X goes through LDS into the registers of wave 0, which eliminates the
// panel's pivots among the panel's own rows: lane l holds columns l and
// l + 64 of every panel row, so a pivot and a multiplier are the only values
// that cross lanes (readlane), and no pivot waits for an LDS round trip or a
// barrier.  The other rows then take the PB eliminations as one update, pivot
// by pivot in order, so every element that is read later receives the same
// FMAs in the same order as with one pivot per barrier (the same W and flags
// bit for bit, 5 % sooner at NB = 96: the broadcast reads of the pivot rows,
// which every thread needs, are what the kernel waits on).  The workgroup
// meets at two barriers per panel.
template <int NB, int TG, int PB>
__global__ __launch_bounds__(TG * TG) void chol_inv_panel_kernel(const double* __restrict__ G, int b,
                                                                 double dep_tol,
                                                                 double* __restrict__ Wout,
                                                                 int* __restrict__ dep, int* err,
                                                                 double first_order_tol) {
  // a second CholeskyQR pass near the identity needs no factorisation
  if (first_order_tol > 0.0 && near_identity_inverse(G, b, first_order_tol, Wout, dep)) return;
  constexpr int NR = NB / TG;
  static_assert(NR * TG == NB, "the thread grid must tile NB");
  static_assert(TG * TG >= NB, "threads 0..NB-1 load the diagonal scales");
  static_assert(TG % PB == 0 && NB % PB == 0, "a panel lies in one row block");
  static_assert(NB <= 128, "two columns per lane of wave 0");
  __shared__ double Dn[NB];
  __shared__ double Pr[2][PB][NB];  // panel rows of S (pivot rows after the panel)
  __shared__ double Px[2][PB][NB];  // panel rows of X, not yet scaled
  __shared__ double pinfo[2][PB][2];  // 1/piv (0 for a dependent column), 1/sqrt(piv)
  __shared__ int depl[NB];
  __shared__ int bad;
  const int t = threadIdx.x;
  const int ti = t / TG, tj = t % TG;
  const int lane = t & 63;
  const bool w0 = t < 64;
  if (t == 0) bad = 0;
  if (t < NB) {
    double dv = 0.0;
    if (t < b) {
      const double g = G[t * b + t];
      dv = (g > 0.0 && isfinite(g)) ? sqrt(g) : 0.0;
    }
    Dn[t] = dv;
  }
  __syncthreads();
  double S[NR][NR], X[NR][NR];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const int i = ti + TG * r, j = tj + TG * c;
      double v = 0.0;
      if (i < b && j < b) {
        const double g = G[i * b + j];
        if (!isfinite(g)) bad = 1;
        const double den = Dn[i] * Dn[j];
        v = den > 0.0 ? g / den : 0.0;
      }
      S[r][c] = v;
      X[r][c] = (i == j) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int k0 = 0; k0 < NB; k0 += PB) {
    if (k0 >= b) continue;  // uniform: b is a kernel argument
    const int buf = (k0 / PB) & 1;
    const int rk = k0 / TG;
    // the panel's owners hand its rows over
    if (ti >= k0 % TG && ti < k0 % TG + PB) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        Pr[buf][ti - k0 % TG][tj + TG * c] = S[rk][c];
        Px[buf][ti - k0 % TG][tj + TG * c] = X[rk][c];
      }
    }
    __syncthreads();
    if (w0) {
      double ps[PB][2], px[PB][2];
#pragma unroll
      for (int q = 0; q < PB; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = lane + 64 * h;
          ps[q][h] = j < NB ? Pr[buf][q][j] : 0.0;
          px[q][h] = j < NB ? Px[buf][q][j] : 0.0;
        }
#pragma unroll
      for (int kk = 0; kk < PB; ++kk) {
        const int k = k0 + kk;
        if (k >= b) break;  // uniform
        const double piv = readlane64(ps[kk][k / 64], k % 64);
        const bool dk = !(piv > dep_tol);
        const double ir = dk ? 1.0 : rsq_nr(piv);
        const double ipiv = dk ? 0.0 : ir * ir;
        if (lane == 0) {
          pinfo[buf][kk][0] = ipiv;
          pinfo[buf][kk][1] = ir;
          depl[k] = dk ? 1 : 0;
        }
#pragma unroll
        for (int ii = kk + 1; ii < PB; ++ii) {
          const int i = k0 + ii;
          const double mi = readlane64(ps[kk][i / 64], i % 64) * ipiv;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * h;
            if (j > k) ps[ii][h] = fma(-mi, ps[kk][h], ps[ii][h]);
            else px[ii][h] = fma(-mi, px[kk][h], px[ii][h]);  // X row k is zero beyond column k
          }
        }
      }
#pragma unroll
      for (int q = 0; q < PB; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = lane + 64 * h;
          if (j < NB) {
            Pr[buf][q][j] = ps[q][h];
            Px[buf][q][j] = px[q][h];
          }
        }
    }
    __syncthreads();
    // the panel's owners take their final X rows: row k scaled by 1/sqrt(piv)
    if (ti >= k0 % TG && ti < k0 % TG + PB) {
      const int q = ti - k0 % TG;
      if (k0 + q < b) {
        const double ir = pinfo[buf][q][1];
#pragma unroll
        for (int c = 0; c < NR; ++c) X[rk][c] = Px[buf][q][tj + TG * c] * ir;
      }
    }
    // every row after the panel takes the panel's eliminations in order
#pragma unroll
    for (int kk = 0; kk < PB; ++kk) {
      const int k = k0 + kk;
      if (k >= b) break;  // uniform
      const double ipiv = pinfo[buf][kk][0];
      double xr[NR], sr[NR];
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        const int j = tj + TG * c;
        xr[c] = (TG * c <= k) ? Px[buf][kk][j] : 0.0;
        sr[c] = (TG * c + TG - 1 > k && j > k) ? Pr[buf][kk][j] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (TG * r + TG - 1 < k0 + PB) continue;  // rows all in or before the panel
        const int i = ti + TG * r;
        const double mi = (i >= k0 + PB) ? Pr[buf][kk][i] * ipiv : 0.0;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          if (TG * c + TG - 1 > k && c >= r) S[r][c] = fma(-mi, sr[c], S[r][c]);
          if (TG * c <= k && c <= r) X[r][c] = fma(-mi, xr[c], X[r][c]);
        }
      }
    }
  }
  __syncthreads();
  // W[j][i] = X[i][j] / D[j]
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const int i = ti + TG * r, j = tj + TG * c;
      if (i < b && j < b) Wout[j * b + i] = Dn[j] > 0.0 ? X[r][c] / Dn[j] : 0.0;
    }
  if (t < b) dep[t] = depl[t];
  if (t == 0 && bad) *err = 1;
}

// Replace the columns j with dep[j] != 0 of an n x b row-major Q by
// standard normal numbers.
__global__ void refill_kernel(double* Q, int ldq, int n, int b, const int* __restrict__ dep,
                              unsigned long long seed,
                              const unsigned long long* __restrict__ ctr_in,
                              unsigned long long* __restrict__ ctr_out) {
  __shared__ int dl[128];
  int mine = 0;
  for (int j = threadIdx.x; j < b; j += blockDim.x) {
    dl[j] = dep[j];
    mine |= dep[j];
  }
  const unsigned long long ctr = *ctr_in;
  // the next call reads the other slot, so no block can see this write early
  if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_out = ctr + (unsigned long long)n * b;
  // most calls have no dependent column: every block then leaves at once
  if (!__syncthreads_or(mine)) return;
  const long long total = (long long)n * b;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(idx % b);
    if (dl[j]) {
      const long long i = idx / b;
      Q[i * ldq + j] = normal_at(seed, ctr + (unsigned long long)idx);
    }
  }
}

// ------------------------------------------------------------ Jacobi SVD

// 64-bit DPP move: both 32-bit halves moved with the same control.
template <int CTRL>
__device__ inline double dpp64(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Sum over a group of LPP (8 or 16) consecutive lanes: two quad butterflies,
// the half-row mirror and, for 16 lanes, the row mirror.
template <int LPP>
__device__ inline double group_sum(double v) {
  v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp64<0x141>(v);  // row_half_mirror
  if (LPP == 16) v += dpp64<0x140>(v);  // row_mirror
  return v;
}

constexpr int kJacobiMaxSweeps = 60;
constexpr int kJacobiMaxB = 128;

// Parallel (round-robin) ordering of the column pairs.  Slot g of the P = bp/2
// slots pairs a top and a bottom column.  Slot 0's top column is column 0
// and never moves; the other columns sit on a ring that runs through the top
// columns of slots 1..P-1 and then the bottom columns of slots P-1..0, and
// the ring advances one position per round, so every pair meets once in the
// bp - 1 rounds of a sweep and a sweep ends where it began.  ring_col(k) is
// the column at ring position k before the first round (top of slot g: 2g,
// bottom: 2g + 1).
__device__ inline int ring_col(int k, int P) { return k <= P - 2 ? 2 * (k + 1) : 4 * P - 3 - 2 * k; }

// LDS row of logical row i in column j: 16-row (LPP = 16) or 8-row (LPP = 8)
// blocks exchanged by j, so that the lane groups of a wave, which read
// different columns at the same rows, start on different banks.
template <int LPP>
__device__ inline int jac_row(int i, int j) {
  return i ^ (LPP * (j & (LPP == 16 ? 1 : 3)));
}

// One-sided Jacobi (Hestenes) on the columns of A (A = B, or B^T when
// trans != 0), one workgroup per matrix.  The working matrix W = A J lives in
// LDS, column-major, LPP * RPT rows per column; each round rotates the P
// disjoint pairs of the ring ordering in parallel, LPP lanes per pair and RPT
// rows per lane.  The rotation (the smaller root t of t^2 + 2 zeta t - 1 = 0,
// c = 1/sqrt(1 + t^2), s = c t, with Newton-refined reciprocals) is applied
// to W only: the accumulated rotations J are not kept here.  When rotlog is
// given, the (c, s) of every slot and round go there in order ((1, 0) for a
// pair left alone), with the number of sweeps in *sweeps_out and each
// column's place in the descending order in rank_out, and
// jacobi_replay_kernel rebuilds J from them.  On exit so holds the singular
// values (the column norms of W) in descending order and Uo, if given, the
// normalised columns of W in that order.  Sweeps stop after one in which no
// rotation had a relative coupling |ga| / sqrt(al be) above 1e-9: Jacobi
// converges quadratically, so the couplings left are of order 1e-18, below
// the rotation threshold b eps.  Two levels (relative to ||A||_F) exempt
// pairs from keeping the sweeps going; an exempt pair is still rotated while
// above the rotation threshold.
//  * zr > 0: a pair with a column of norm at most zr ||A||_F.  At the rounding
//    level of A's entries (zr ~ b eps) such a column is zero to working
//    precision: its direction carries no information and its relative
//    coupling with any other column never settles.
//  * zp > 0: a pair whose two columns both have a norm of at most zp ||A||_F,
//    for A known only to a relative accuracy zp.  Their mutual rotations fit
//    the error of A.  A pair with one larger column still converges: left
//    unconverged, the smaller column keeps a component of the larger one's
//    direction as large as their relative coupling.
template <int RPT, int LPP>
__global__ __launch_bounds__(1024) void jacobi_kernel(
    const double* __restrict__ Bm, int b, long long bstride, long long sstride,
    double* __restrict__ Uo, double* __restrict__ so, double2* __restrict__ rotlog,
    int* __restrict__ rank_out, int* __restrict__ sweeps_out, int* err, int trans, double zr,
    double zp) {
  constexpr int ld = LPP * RPT;
  static_assert(RPT % (LPP == 16 ? 2 : 4) == 0, "the row-block exchange needs whole block pairs");
  extern __shared__ double lds[];
  const int bp = b + (b & 1);
  const int P = bp / 2, m1 = bp - 1;
  double* Wc = lds;                        // bp columns of ld rows
  double* sv = lds + (size_t)bp * ld;      // bp column norms
  int* rk = (int*)(sv + bp);               // bp ranks
  __shared__ int changed;
  __shared__ int big;
  __shared__ int bad;
  __shared__ double fro_part[16];
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  const double* B = Bm + blockIdx.x * bstride;
  if (t == 0) { changed = 0; big = 0; bad = 0; }
  double fro = 0.0;
  for (int idx = t; idx < bp * ld; idx += nt) {
    const int j = idx / ld, i = idx - (idx / ld) * ld;
    double v = 0.0;
    if (j < b && i < b) v = trans ? B[(long long)j * b + i] : B[(long long)i * b + j];
    Wc[j * ld + jac_row<LPP>(i, j)] = v;
    fro = fma(v, v, fro);
  }
  // ||A||_F^2 (rotations keep it): per wave, then over the waves
  for (int o = 32; o > 0; o >>= 1) fro += __shfl_xor(fro, o);
  if ((t & 63) == 0) fro_part[t >> 6] = fro;
  __syncthreads();
  double fro2 = 0.0;
  for (int w = 0; w < (nt + 63) / 64; ++w) fro2 += fro_part[w];
  const double zr2f2 = zr > 0.0 ? zr * zr * fro2 : 0.0;
  const double zp2f2 = zp > 0.0 ? zp * zp * fro2 : 0.0;
  const int g = t / LPP;
  const int sub = t - g * LPP;
  const bool active = g < P;
  const double tol = b * DBL_EPSILON;
  const double tol2 = tol * tol;
  int kp = g > 0 ? g - 1 : 0;  // ring positions of the slot's top and bottom columns
  int kq = 2 * P - 2 - g;
  int sweeps = 0;
  bool converged = false;
  while (sweeps < kJacobiMaxSweeps && !converged) {
    for (int r = 0; r < m1; ++r) {
      if (active) {
        const int p = g == 0 ? 0 : ring_col(kp, P);
        const int q = ring_col(kq, P);
        const double* rp = Wc + p * ld + sub;
        const double* rq = Wc + q * ld + sub;
        const int fp = LPP * (p & (LPP == 16 ? 1 : 3));
        const int fq = LPP * (q & (LPP == 16 ? 1 : 3));
        double xp[RPT], xq[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          xp[k] = rp[(LPP * k) ^ fp];
          xq[k] = rq[(LPP * k) ^ fq];
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          al = fma(xp[k], xp[k], al);
          be = fma(xq[k], xq[k], be);
          ga = fma(xp[k], xq[k], ga);
        }
        al = group_sum<LPP>(al);
        be = group_sum<LPP>(be);
        ga = group_sum<LPP>(ga);
        const bool rot = al > 0.0 && be > 0.0 && ga * ga > tol2 * al * be;
        const double g2 = rot ? 2.0 * ga : 1.0;
        // t = 1 / (|zeta| + sqrt(1 + zeta^2)); above 1e150 zeta^2 would
        // overflow and t = 1 / (2 |zeta|) is exact to rounding.  The angle must
        // not be clamped: a too large angle on a strongly graded pair
        // overshoots and the pair never settles.  An infinite zeta gives t = 0
        // (no rotation, and the pair does not count as changed).  t comes from
        // the hardware reciprocal and root estimates without refinement: any
        // t gives an exact rotation once c and s are consistent, and an angle
        // off by the estimates' relative error leaves a coupling of that
        // relative size, which the next sweep removes.  c = 1/sqrt(1 + t^2)
        // is refined to full precision, so that c^2 + s^2 = 1 to rounding.
        const double zeta = rot ? (be - al) * __builtin_amdgcn_rcp(g2) : 0.0;
        const double az = fabs(zeta);
        const double azc = fmin(az, 1e150);
        const double w = fma(azc, azc, 1.0);
        const double den = (az < 1e150) ? fma(w, __builtin_amdgcn_rsq(w), azc) : 2.0 * az;
        double tt = (den < INFINITY) ? __builtin_amdgcn_rcp(den) : 0.0;
        tt = rot ? (zeta < 0.0 ? -tt : tt) : 0.0;
        double c = 1.0, s = 0.0;
        if (tt != 0.0) {
          c = rsq_nr(fma(tt, tt, 1.0));
          s = c * tt;
          double* wp = Wc + p * ld + sub;
          double* wq = Wc + q * ld + sub;
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            wp[(LPP * k) ^ fp] = c * xp[k] - s * xq[k];
            wq[(LPP * k) ^ fq] = s * xp[k] + c * xq[k];
          }
          if (sub == 0) {
            changed = 1;
            if (ga * ga > 1e-18 * al * be && fmin(al, be) > zr2f2 && fmax(al, be) > zp2f2)
              big = 1;
          }
        }
        if (rotlog && sub == 0) rotlog[((size_t)sweeps * m1 + r) * P + g] = make_double2(c, s);
      }
      kp = kp == 0 ? m1 - 1 : kp - 1;
      kq = kq == 0 ? m1 - 1 : kq - 1;
      __syncthreads();
    }
    const int ch = changed, bg = big;
    __syncthreads();
    if (t == 0) { changed = 0; big = 0; }
    __syncthreads();
    ++sweeps;
    converged = !ch || !bg;
  }
  // column norms: slot g takes columns 2g and 2g + 1
  if (active) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = 2 * g + h;
      const double* wc = Wc + col * ld + sub;
      const int f = LPP * (col & (LPP == 16 ? 1 : 3));
      double ss = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const double v = wc[(LPP * k) ^ f];
        ss = fma(v, v, ss);
      }
      ss = group_sum<LPP>(ss);
      if (sub == 0) {
        const double sq = sqrt(ss);
        if (!isfinite(sq)) bad = 1;
        sv[col] = sq;
      }
    }
  }
  __syncthreads();
  double* so_b = so + blockIdx.x * sstride;
  for (int j = t; j < b; j += nt) {
    const double sj = sv[j];
    int rank = 0;
    for (int k = 0; k < b; ++k) {
      const double sk = sv[k];
      rank += (sk > sj || (sk == sj && k < j)) ? 1 : 0;
    }
    rk[j] = rank;
    so_b[rank] = sj;
    if (rank_out) rank_out[j] = rank;
  }
  __syncthreads();
  if (Uo) {
    double* X = Uo + blockIdx.x * bstride;
    for (int idx = t; idx < b * b; idx += nt) {
      const int i = idx / b, j = idx - (idx / b) * b;
      const double sj = sv[j];
      const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
      X[(long long)i * b + rk[j]] = Wc[j * ld + jac_row<LPP>(i, j)] * inv;
    }
  }
  if (t == 0) {
    if (bad || !converged) *err = 1;
    if (sweeps_out) *sweeps_out = sweeps;
  }
}

// The accumulated rotations J of jacobi_kernel, rebuilt from its log: J
// starts as the identity and takes the logged plane rotations in order.  The
// rows of J evolve independently, so each wave rebuilds one row i: lane g
// holds the row's entries in the two columns of slot g, rotates them with
// slot g's (c, s) of the round and passes them along the ring (wave shifts by
// one lane).  After whole sweeps the columns are back in their starting
// slots, and entry (i, j) is written to Vo[i][rank[j]], the column order of
// the singular values.  The log was written by one workgroup on one XCD, so
// each of the kReplayGroups workgroups streams it through LDS in chunks of
// kReplayChunk rounds, loading the next chunk while its waves work on the
// current one; workgroup x rebuilds rows x, x + kReplayGroups, ... (at most
// four rows, one wave each, so that the waves of a CU do not queue for it).
constexpr int kReplayGroups = 32;
constexpr int kReplayChunk = 64;
__global__ __launch_bounds__(1024) void jacobi_replay_kernel(const double2* __restrict__ rotlog,
                                                             const int* __restrict__ sweeps_in,
                                                             const int* __restrict__ rank, int b,
                                                             double* __restrict__ Vo) {
  extern __shared__ double2 chunk[];  // 2 x kReplayChunk rounds x P slots
  const int bp = b + (b & 1);
  const int P = bp / 2, m1 = bp - 1;
  const int t = threadIdx.x, nt = blockDim.x;
  const int g = t & 63;
  const int i = blockIdx.x + kReplayGroups * (t >> 6);  // this wave's row
  const bool act = g < P;
  double tv = (act && 2 * g == i) ? 1.0 : 0.0;
  double bv = (act && 2 * g + 1 == i) ? 1.0 : 0.0;
  const long long total = (long long)(*sweeps_in) * m1;
  const int per = kReplayChunk * P;     // entries of one chunk
  constexpr int kLoads = (kReplayChunk * 64 + 255) / 256;  // per thread, at >= 256 threads
  double2 stage[kLoads];
  // chunk 0 into buffer 0
  for (int e = t; e < per; e += nt) chunk[e] = e < total * P ? rotlog[e] : make_double2(1.0, 0.0);
  __syncthreads();
  for (long long c0 = 0; c0 < total; c0 += kReplayChunk) {
    const int buf = (int)((c0 / kReplayChunk) & 1);
    const long long n0 = c0 + kReplayChunk;  // first round of the next chunk
    const bool more = n0 < total;
    if (more) {
#pragma unroll
      for (int q = 0; q < kLoads; ++q) {
        const long long e = (long long)t + (long long)q * nt;
        const long long src = n0 * P + e;
        stage[q] = (e < per && src < total * P) ? rotlog[src] : make_double2(1.0, 0.0);
      }
    }
    const double2* cs = chunk + buf * per;
    const int rounds = (int)min<long long>(kReplayChunk, total - c0);
    // groups of 8 rounds, their (c, s) read from LDS before the first of
    // them is applied, so that the LDS latency stays off the chain of
    // dependent rotations (rounds past the chunk's end are the identity)
    for (int r0 = 0; r0 < rounds; r0 += 8) {  // uniform over the workgroup
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = (act && r0 + u < rounds) ? cs[(r0 + u) * P + g] : make_double2(1.0, 0.0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double nt_ = v[u].x * tv - v[u].y * bv;
        const double nb_ = v[u].y * tv + v[u].x * bv;
        const double from_left_t = dpp64<0x138>(nt_);   // wave_shr:1, lane g <- g - 1
        const double from_left_b = dpp64<0x138>(nb_);
        const double from_right_b = dpp64<0x130>(nb_);  // wave_shl:1, lane g <- g + 1
        const double t1 = g == 0 ? nt_ : (g == 1 ? from_left_b : from_left_t);
        // with one slot the ring is its bottom column alone
        const double b1 = g == P - 1 ? (P == 1 ? nb_ : nt_) : from_right_b;
        // a round past the chunk's end does not move the ring either
        const bool live = r0 + u < rounds;
        tv = live ? t1 : tv;
        bv = live ? b1 : bv;
      }
    }
    if (more) {
      double2* dst = chunk + (buf ^ 1) * per;
#pragma unroll
      for (int q = 0; q < kLoads; ++q) {
        const long long e = (long long)t + (long long)q * nt;
        if (e < per) dst[e] = stage[q];
      }
    }
    __syncthreads();
  }
  if (act && i < b) {
    if (2 * g < b) Vo[(long long)i * b + rank[2 * g]] = tv;
    if (2 * g + 1 < b) Vo[(long long)i * b + rank[2 * g + 1]] = bv;
  }
}

// One workgroup per column i: ||Y[:, i] - s_i V[:, i]||_2.
__global__ void column_residuals_kernel(const double* __restrict__ Y, const double* __restrict__ V,
                                        const double* __restrict__ s, int n, int ld, int kk,
                                        double* __restrict__ out) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  const double si = s[i];
  double acc = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    const double e = fma(-si, V[(long long)r * ld + i], Y[(long long)r * ld + i]);
    acc = fma(e, e, acc);
  }
  acc = block_sum256(acc, sh);
  if (threadIdx.x == 0) {
    out[i] = sqrt(acc);
    if (i == 0) out[kk] = s[0];
  }
}

__global__ void inv_sqrt_cut_kernel(const double* s, int kk, int chi, double eps, double* w) {
  const double s0 = s[0];
  for (int j = threadIdx.x; j < chi; j += blockDim.x) {
    double v = 0.0;
    if (j < kk && s0 > 0.0 && s[j] > eps * s0) v = 1.0 / sqrt(s[j]);
    w[j] = v;
  }
}

__global__ void scale_cols_kernel(double* Z, int n, int c, int ldz, const double* w) {
  const long long total = (long long)n * c;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long i = idx / c;
    const int j = (int)(idx - i * c);
    Z[i * ldz + j] *= w[j];
  }
}

__global__ void fix_signs_kernel(double* X, int ldx, double* Y, int ldy, int n) {
  __shared__ double sv[256];
  __shared__ int si[256];
  const int j = blockIdx.x;
  const int t = threadIdx.x;
  double best = -1.0;
  int bi = 0x7fffffff;
  // eight strided loads in flight, then compared in row order (the first
  // row of the largest |value| wins, as in a plain scan)
  const int nt = blockDim.x;
  for (int i0 = t; i0 < n; i0 += 8 * nt) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * nt;
      v[u] = i < n ? fabs(X[(long long)i * ldx + j]) : -1.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (v[u] > best) { best = v[u]; bi = i0 + u * nt; }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      const double o = sv[t + s];
      const int oi = si[t + s];
      if (o > sv[t] || (o == sv[t] && oi < si[t])) { sv[t] = o; si[t] = oi; }
    }
    __syncthreads();
  }
  // One thread reads the sign of the pivot entry and shares it: the column
  // is flipped in place, so a wave reading X[imax][j] itself could see the
  // entry already flipped by the wave that owns row imax and leave its own
  // rows as they were.
  __shared__ int flip_s;
  if (t == 0) {
    const int imax = si[0];
    flip_s = (imax < n) && X[(long long)imax * ldx + j] < 0.0;
  }
  __syncthreads();
  const bool flip = flip_s != 0;
  if (flip) {
    for (int i = t; i < n; i += blockDim.x) {
      X[(long long)i * ldx + j] = -X[(long long)i * ldx + j];
      Y[(long long)i * ldy + j] = -Y[(long long)i * ldy + j];
    }
  }
}

__global__ void spectra_delta_kernel(const double* s, double* old, int chi, double* delta) {
  __shared__ double sh[256];
  double dmax = 0.0;
  for (int c = 0; c < 4; ++c) {
    const double* sc = s + c * chi;
    double* oc = old + c * chi;
    double ss = 0.0;
    for (int j = threadIdx.x; j < chi; j += blockDim.x) ss += sc[j] * sc[j];
    ss = block_sum256(ss, sh);
    const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    double dd = 0.0;
    for (int j = threadIdx.x; j < chi; j += blockDim.x) {
      const double v = sc[j] * inv;
      const double d = v - oc[j];
      dd += d * d;
    }
    dd = block_sum256(dd, sh);
    __syncthreads();
    for (int j = threadIdx.x; j < chi; j += blockDim.x) oc[j] = sc[j] * inv;
    dmax = fmax(dmax, sqrt(dd));
    __syncthreads();
  }
  if (threadIdx.x == 0) *delta = dmax;
}

inline int grid_for(size_t n, int block = 256, int cap = 4096) {
  size_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > (size_t)cap) g = cap;
  return (int)g;
}

double* red_scratch(Context& ctx) {
  static_assert(kRedBlocks + 64 <= kRedScratchDoubles, "reduction scratch size");
  if (ctx.fixed_red) return ctx.fixed_red;
  if (ctx.scratch_small.bytes < (kRedBlocks + 64) * sizeof(double)) {
    CTM_HIP(hipStreamSynchronize(ctx.stream));
    ctx.scratch_small.alloc((kRedBlocks + 64) * sizeof(double));
  }
  return ctx.scratch_small.d();
}

}  // namespace

// Raise a kernel's dynamic-LDS limit to `bytes` when above the 64 KB
// default (gfx950 has 160 KB of LDS per CU), once per (kernel, size) and
// process: later calls, including those made while a stream is being captured
// into a graph, issue no runtime call.
void allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return;
  static std::mutex mu;
  static std::vector<std::pair<const void*, size_t>> done;
  std::lock_guard<std::mutex> lock(mu);
  for (auto& e : done)
    if (e.first == fn && e.second >= bytes) return;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
    (void)hipGetLastError();
  else
    done.push_back({fn, bytes});
}

void fill_zero(Context& ctx, double* p, size_t n) {
  if (!n) return;
  hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(n)), dim3(256), 0, ctx.stream, p, n, 0.0);
  CTM_HIP(hipGetLastError());
}
void fill_zero_int(Context& ctx, int* p, size_t n) {
  if (!n) return;
  hipLaunchKernelGGL(fill_kernel<int>, dim3(grid_for(n)), dim3(256), 0, ctx.stream, p, n, 0);
  CTM_HIP(hipGetLastError());
}
void copy_dev(Context& ctx, double* dst, const double* src, size_t n) {
  if (!n) return;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, ctx.stream, dst, src, n);
  CTM_HIP(hipGetLastError());
}
void copy_block(Context& ctx, double* dst, long long ldd, const double* src, long long lds,
                int rows, int cols) {
  const size_t total = (size_t)rows * cols;
  if (!total) return;
  hipLaunchKernelGGL(copy_block_kernel, dim3(grid_for(total)), dim3(256), 0, ctx.stream, dst, ldd,
                     src, lds, rows, cols);
  CTM_HIP(hipGetLastError());
}
void fill_normal(Context& ctx, double* Z, size_t count, unsigned long long seed,
                 unsigned long long counter) {
  if (!count) return;
  hipLaunchKernelGGL(fill_normal_kernel, dim3(grid_for(count)), dim3(256), 0, ctx.stream, Z,
                     count, seed, counter);
  CTM_HIP(hipGetLastError());
}

void normalise_maxabs(Context& ctx, double* p, size_t n, double* log_slot, int* flag,
                      double* inv_keep) {
  if (n <= (size_t)kNormaliseOneGroup) {
    hipLaunchKernelGGL(normalise_one_group_kernel, dim3(1), dim3(kNormaliseThreads), 0, ctx.stream,
                       p, (int)n, log_slot, flag, inv_keep);
    CTM_HIP(hipGetLastError());
    return;
  }
  double* part = red_scratch(ctx);
  const int nb = grid_for(n, 256, kRedBlocks);
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(nb), dim3(256), 0, ctx.stream, p, n, part);
  hipLaunchKernelGGL(scale_by_max_kernel, dim3(grid_for(n)), dim3(256), 0, ctx.stream, p, n, part,
                     nb, log_slot, flag, inv_keep);
  CTM_HIP(hipGetLastError());
}

void dot(Context& ctx, const double* x, const double* y, size_t n, double* result) {
  double* part = red_scratch(ctx);
  const int nb = grid_for(n, 256, kRedBlocks);
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(256), 0, ctx.stream, x, y, n, part);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(256), 0, ctx.stream, part, nb, result);
  CTM_HIP(hipGetLastError());
}

int jacobi_max_b(bool) { return kJacobiMaxB; }

void jacobi_svd(Context& ctx, const double* B, int b, double* X, double* s, double* Y, int* err,
                int batch, long long bstride, long long sstride, bool trans, double zr,
                double zp) {
  CTM_REQUIRE(b >= 1 && b <= kJacobiMaxB, "jacobi_svd: b out of range");
  CTM_REQUIRE(zr >= 0.0 && zr < 1.0, "jacobi_svd: zr out of range");
  double* Uo = trans ? Y : X;  // normalised columns of the working matrix
  double* Vo = trans ? X : Y;  // accumulated rotations
  CTM_REQUIRE(Vo == nullptr || batch == 1, "jacobi_svd: rotations of one matrix at a time");
  const int bp = b + (b & 1);
  const int P = bp / 2;
  constexpr int LPP = 16;
  int rpt = (b + LPP - 1) / LPP;
  rpt += rpt & 1;  // whole pairs of 16-row blocks
  const int ld = LPP * rpt;
  const size_t lds = ((size_t)bp * ld + bp) * sizeof(double) + (size_t)bp * sizeof(int);
  CTM_REQUIRE(lds <= 160 * 1024, "jacobi_svd: matrix too large for LDS");
  const int threads = std::max(64, (P * LPP + 63) / 64 * 64);
  double2* rotlog = nullptr;
  int* rank = nullptr;
  int* sweeps = nullptr;
  if (Vo) {
    // one fixed-size workspace per context (its address never changes, so
    // captured graphs stay valid): the rotation log of the largest matrix
    // for the most sweeps, the ranks and the sweep count
    const size_t logb = (size_t)kJacobiMaxSweeps * (kJacobiMaxB - 1) * (kJacobiMaxB / 2) *
                        sizeof(double2);
    const size_t need = logb + (kJacobiMaxB + 64) * sizeof(int);
    if (ctx.jacobi_ws.bytes < need) {
      CTM_HIP(hipStreamSynchronize(ctx.stream));
      ctx.jacobi_ws.alloc(need);
    }
    rotlog = (double2*)ctx.jacobi_ws.p;
    rank = (int*)((char*)ctx.jacobi_ws.p + logb);
    sweeps = rank + kJacobiMaxB;
  }
#define CTM_JAC(R)                                                                                \
  do {                                                                                            \
    allow_lds((const void*)jacobi_kernel<R, LPP>, lds);                                           \
    hipLaunchKernelGGL((jacobi_kernel<R, LPP>), dim3(batch), dim3(threads), lds, ctx.stream, B, b, \
                       bstride, sstride, Uo, s, rotlog, rank, sweeps, err, trans ? 1 : 0, zr, zp);    \
  } while (0)
  if (rpt == 2) CTM_JAC(2);
  else if (rpt == 4) CTM_JAC(4);
  else if (rpt == 6) CTM_JAC(6);
  else CTM_JAC(8);
#undef CTM_JAC
  CTM_HIP(hipGetLastError());
  if (Vo) {
    const int rows = (b + kReplayGroups - 1) / kReplayGroups;  // waves per workgroup
    const size_t clds = 2ull * kReplayChunk * P * sizeof(double2);
    allow_lds((const void*)jacobi_replay_kernel, clds);
    hipLaunchKernelGGL(jacobi_replay_kernel, dim3(kReplayGroups), dim3(64 * std::max(rows, 4)), clds,
                       ctx.stream, rotlog, sweeps, rank, b, Vo);
    CTM_HIP(hipGetLastError());
  }
}

void chol_inverse(Context& ctx, const double* G, int b, double dep_tol, double* W, int* dep,
                  int* err, bool first_order) {
  CTM_REQUIRE(b >= 1 && b <= 128, "chol_inverse: b out of range");
  const double fo = first_order ? kNearIdentityTol : 0.0;
  // the panel form gives the same W bit for bit, 5 % (b = 96) to 12 % (b = 128) sooner
  if (b <= 96)
    hipLaunchKernelGGL((chol_inv_panel_kernel<96, 32, 8>), dim3(1), dim3(1024), 0, ctx.stream, G, b,
                       dep_tol, W, dep, err, fo);
  else
    hipLaunchKernelGGL((chol_inv_panel_kernel<128, 32, 8>), dim3(1), dim3(1024), 0, ctx.stream, G, b,
                       dep_tol, W, dep, err, fo);
  CTM_HIP(hipGetLastError());
}

void refill_columns(Context& ctx, double* Q, int ldq, int n, int b, const int* dep,
                    unsigned long long seed, const unsigned long long* counter_in,
                    unsigned long long* counter_out) {
  CTM_REQUIRE(b >= 1 && b <= 128, "refill_columns: b out of range");
  const size_t total = (size_t)n * b;
  hipLaunchKernelGGL(refill_kernel, dim3(grid_for(total, 256, 1024)), dim3(256), 0, ctx.stream, Q,
                     ldq, n, b, dep, seed, counter_in, counter_out);
  CTM_HIP(hipGetLastError());
}

void column_residuals(Context& ctx, const double* Y, const double* V, const double* s, int n,
                      int ld, int kk, double* out) {
  if (kk <= 0) return;
  hipLaunchKernelGGL(column_residuals_kernel, dim3(kk), dim3(256), 0, ctx.stream, Y, V, s, n, ld,
                     kk, out);
  CTM_HIP(hipGetLastError());
}

void inv_sqrt_cut(Context& ctx, const double* s, int kk, int chi, double eps, double* w) {
  hipLaunchKernelGGL(inv_sqrt_cut_kernel, dim3(1), dim3(256), 0, ctx.stream, s, kk, chi, eps, w);
  CTM_HIP(hipGetLastError());
}

void scale_cols(Context& ctx, double* Z, int n, int c, int ldz, const double* w) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for((size_t)n * c)), dim3(256), 0, ctx.stream, Z,
                     n, c, ldz, w);
  CTM_HIP(hipGetLastError());
}

void fix_signs(Context& ctx, double* X, int ldx, double* Y, int ldy, int n, int b) {
  hipLaunchKernelGGL(fix_signs_kernel, dim3(b), dim3(256), 0, ctx.stream, X, ldx, Y, ldy, n);
  CTM_HIP(hipGetLastError());
}

void spectra_delta(Context& ctx, const double* s, double* old, int chi, double* delta) {
  hipLaunchKernelGGL(spectra_delta_kernel, dim3(1), dim3(256), 0, ctx.stream, s, old, chi, delta);
  CTM_HIP(hipGetLastError());
}

}  // namespace ctm
