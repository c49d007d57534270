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

__global__ void maxabs_final_kernel(const double* partial, int nb, double* log_slot, int* flag,
                                    double* inv_out, double* inv_keep) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, partial[i]);
  m = block_max256(m, sh);
  if (threadIdx.x == 0) {
    double inv = 1.0;
    if (!(m < INFINITY) || m == 0.0) {
      *flag = 1;
    } else {
      inv = 1.0 / m;
      *log_slot += log(m);
    }
    *inv_out = inv;
    if (inv_keep) *inv_keep = inv;
  }
}

__global__ void scale_by_dev_kernel(double* p, size_t n, const double* s) {
  const double f = *s;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] *= f;
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

// Cholesky factor and its inverse in one pass, register-tiled: TG x TG
// threads, thread (ti, tj) owning entries (ti + TG r, tj + TG c),
// r, c < NR = 96 / TG, of the symmetric Schur complement S and of X (both 96 x 96,
// zero beyond b so that no row or column needs a guard).  Step k eliminates
// column k below the pivot (S -= s_k s_k^T / piv on the trailing block) and
// applies the same row operation to X, then scales row k of X by 1/sqrt(piv).
// At the end X = R^-T, where R^T R is the column-scaled Gram matrix, so
// W = D^-1 X^T has Z W orthonormal.  Columns whose pivot falls below dep_tol
// (numerically dependent) are skipped: no elimination, flag set.  All
// updates are unconditional FMAs with masked multipliers.
template <int TG>
__global__ __launch_bounds__(TG * TG) void chol_inv_kernel(const double* __restrict__ G, int b,
                                                           double dep_tol, double* __restrict__ Wout,
                                                           int* __restrict__ dep, int* err) {
  constexpr int NR = 96 / TG;
  static_assert(NR * TG == 96, "the thread grid must tile 96");
  static_assert(TG * TG >= 96, "threads 0..95 load the diagonal scales");
  __shared__ double Dn[96];
  __shared__ double rowk[2][96];
  __shared__ double xrow[2][96];
  __shared__ int depl[96];
  __shared__ int bad;
  const int t = threadIdx.x;
  const int ti = t / TG, tj = t % TG;
  if (t == 0) bad = 0;
  if (t < 96) {
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
  // The 96 steps are unrolled so that k, and with it the register row
  // k / TG that holds row k and the blocks the step can touch, are
  // compile-time constants: no select chains, and register blocks that lie
  // entirely before the pivot are skipped.  Row k is broadcast through a
  // double-buffered LDS row, so one barrier per step suffices (a buffer is
  // rewritten two steps later, after every reader has passed the barrier in
  // between).
#pragma unroll 96
  for (int k = 0; k < 96; ++k) {
    if (k >= b) continue;                                     // uniform: b is a kernel argument
    const int rk = k / TG;
    const int buf = k & 1;
    if (ti == (k % TG)) {
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        rowk[buf][tj + TG * c] = S[rk][c];
        xrow[buf][tj + TG * c] = X[rk][c];
      }
    }
    __syncthreads();
    const double piv = rowk[buf][k];
    const bool dk = !(piv > dep_tol);
    const double ir = dk ? 1.0 : rsq_nr(piv);
    const double ipiv = dk ? 0.0 : ir * ir;
    double xr[NR], sr[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const int j = tj + TG * c;
      xr[c] = (TG * c <= k) ? xrow[buf][j] : 0.0;          // X row k is zero beyond column k
      sr[c] = (TG * c + TG - 1 > k && j > k) ? rowk[buf][j] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (TG * r + TG - 1 < k) continue;                     // rows all before the pivot
      const int i = ti + TG * r;
      const double mi = (i > k) ? rowk[buf][i] * ipiv : 0.0;
      const double sc = (i == k) ? ir : 1.0;
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        if (TG * c + TG - 1 > k) S[r][c] = fma(-mi, sr[c], S[r][c]);
        if (TG * c <= k) X[r][c] = fma(-mi, xr[c], X[r][c]) * sc;
      }
    }
    if (t == 0) depl[k] = dk ? 1 : 0;
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
  for (int j = threadIdx.x; j < b; j += blockDim.x) dl[j] = dep[j];
  const unsigned long long ctr = *ctr_in;
  // the next call reads the other slot, so no block can see this write early
  if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_out = ctr + (unsigned long long)n * b;
  __syncthreads();
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

// Sum over a group of 8 consecutive lanes (half a DPP row): butterflies
// with quad permutations, then the half-row mirror.
__device__ inline double dpp_step(double x, int ctrl) {
  const long long u = __double_as_longlong(x);
  int lo = (int)(u & 0xffffffffLL), hi = (int)(u >> 32);
  if (ctrl == 0) {
    lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
  } else if (ctrl == 1) {
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
  }
  return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline double lane8_sum(double v) {
  v += dpp_step(v, 0);
  v += dpp_step(v, 1);
  v += dpp_step(v, 2);
  return v;
}

// One workgroup per matrix, one-sided Jacobi (Hestenes) on the columns of A
// (A = B, or B^T when trans != 0).  Columns of the working matrix and of V
// are kept column-major in LDS, 8 RPT rows each, with the 8-row blocks of
// column j permuted by block ^ (j & 3): the 8-lane groups of a wave read
// columns whose indices differ by one, so the groups hit different banks;
// each round of the circle
// schedule (precomputed in LDS) rotates the bp/2 disjoint column pairs in
// parallel, 8 lanes per pair, each lane holding RPT rows of the pair in
// registers.  The rotation (the smaller root t of t^2 + 2 zeta t - 1 = 0,
// c = 1/sqrt(1 + t^2), s = c t) uses Newton-refined reciprocals.  On exit
// A = U diag(s) V^T with s descending; with trans == 0 X = U, Y = V, with
// trans != 0 X = V, Y = U (so that always B = X diag(s) Y^T).
// LDS row of logical row i in column j (a permutation of the 8-row blocks
// inside each aligned group of 4 blocks).
__device__ inline int jac_row(int i, int j) { return i ^ (8 * (j & 3)); }

template <int RPT>
__global__ __launch_bounds__(512) void jacobi_svd_kernel(const double* __restrict__ Bm, int b,
                                                         long long bstride, long long sstride,
                                                         double* __restrict__ Xo,
                                                         double* __restrict__ so,
                                                         double* __restrict__ Yo, int* err,
                                                         int want_vec, int trans) {
  extern __shared__ double lds[];
  const int bp = b + (b & 1);
  constexpr int ld = 8 * RPT;  // rows b..8*RPT-1 stay zero
  static_assert(RPT % 4 == 0, "the block permutation needs groups of 4 blocks");
  double* Wc = lds;                                  // bp columns
  double* Vc = want_vec ? lds + bp * ld : nullptr;   // bp columns
  double* sv = lds + (want_vec ? 2 : 1) * bp * ld;   // bp singular values
  unsigned char* sched = (unsigned char*)(sv + bp);  // (bp-1) rounds x bp entries
  __shared__ int changed;
  __shared__ int big;  // a rotated pair had |cos| of its angle above 1e-9
  __shared__ int bad;
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  const double* B = Bm + blockIdx.x * bstride;
  if (t == 0) { changed = 0; big = 0; bad = 0; }
  for (int idx = t; idx < bp * ld; idx += nt) {
    const int j = idx / ld, i = idx - (idx / ld) * ld;
    double v = 0.0;
    if (j < b && i < b) v = trans ? B[(long long)j * b + i] : B[(long long)i * b + j];
    const int ph = j * ld + jac_row(i, j);
    Wc[ph] = v;
    if (Vc) Vc[ph] = (i == j && i < b) ? 1.0 : 0.0;
  }
  const int P = bp / 2;
  const int m = bp - 1;
  for (int idx = t; idx < m * P; idx += nt) {
    const int r = idx / P, pi = idx - (idx / P) * P;
    int p, q;
    if (pi == 0) { p = m; q = r; }
    else { p = (r + pi) % m; q = (r - pi + m) % m; }
    sched[2 * idx] = (unsigned char)p;
    sched[2 * idx + 1] = (unsigned char)q;
  }
  __syncthreads();
  const int pi = t >> 3;
  const int sub = t & 7;
  const bool active = pi < P;
  const double tol = b * DBL_EPSILON;
  const double tol2 = tol * tol;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    for (int r = 0; r < m; ++r) {
      if (active) {
        const int p = sched[2 * (r * P + pi)];
        const int q = sched[2 * (r * P + pi) + 1];
        double* wp = Wc + p * ld + sub;
        double* wq = Wc + q * ld + sub;
        // offsets of the logical rows sub + 8k, k = 4g + e: 32 g + op[e]
        int op[4], oq[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          op[e] = 8 * (e ^ (p & 3));
          oq[e] = 8 * (e ^ (q & 3));
        }
        double xp[RPT], xq[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          xp[k] = wp[32 * (k >> 2) + op[k & 3]];
          xq[k] = wq[32 * (k >> 2) + oq[k & 3]];
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          al = fma(xp[k], xp[k], al);
          be = fma(xq[k], xq[k], be);
          ga = fma(xp[k], xq[k], ga);
        }
        al = lane8_sum(al);
        be = lane8_sum(be);
        ga = lane8_sum(ga);
        const bool rot = al > 0.0 && be > 0.0 && ga * ga > tol2 * al * be;
        // rotation parameters, computed unconditionally (c = 1, s = 0 when idle)
        const double g2 = rot ? 2.0 * ga : 1.0;
        const double zeta = rot ? (be - al) * rcp_nr(g2) : 0.0;
        // t = 1 / (|zeta| + sqrt(1 + zeta^2)); above 1e150 zeta^2 would
        // overflow and t = 1 / (2 |zeta|) is exact to rounding.  The angle must
        // not be clamped: a too large angle on a strongly graded pair
        // overshoots and the pair never settles.  An infinite zeta gives t = 0
        // (no rotation, and the pair does not count as changed).
        const double az = fabs(zeta);
        const double azc = fmin(az, 1e150);
        const double w = fma(azc, azc, 1.0);
        const double den = (az < 1e150) ? azc + w * rsq_nr(w) : 2.0 * az;
        double tt = (den < INFINITY) ? rcp_nr(den) : 0.0;
        tt = rot ? (zeta < 0.0 ? -tt : tt) : 0.0;
        if (tt != 0.0) {
          const double c = rsq_nr(fma(tt, tt, 1.0));
          const double s = c * tt;
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            wp[32 * (k >> 2) + op[k & 3]] = c * xp[k] - s * xq[k];
            wq[32 * (k >> 2) + oq[k & 3]] = s * xp[k] + c * xq[k];
          }
          if (Vc) {
            double* vp = Vc + p * ld + sub;
            double* vq = Vc + q * ld + sub;
            double yp[RPT], yq[RPT];
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
              yp[k] = vp[32 * (k >> 2) + op[k & 3]];
              yq[k] = vq[32 * (k >> 2) + oq[k & 3]];
            }
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
              vp[32 * (k >> 2) + op[k & 3]] = c * yp[k] - s * yq[k];
              vq[32 * (k >> 2) + oq[k & 3]] = s * yp[k] + c * yq[k];
            }
          }
          if (sub == 0) {
            changed = 1;
            if (ga * ga > 1e-18 * al * be) big = 1;
          }
        }
      }
      __syncthreads();
    }
    const int ch = changed, bg = big;
    __syncthreads();
    if (t == 0) { changed = 0; big = 0; }
    __syncthreads();
    // Cyclic Jacobi converges quadratically: after a sweep whose largest
    // relative coupling |ga| / sqrt(al be) was below 1e-9 the couplings left
    // are of order 1e-18, below tol, so the rotation-free check sweep is
    // skipped.
    if (!ch || !bg) break;
  }
  // singular values and ordering
  for (int j = t; j < bp; j += nt) {
    double s = 0.0;
    for (int i = 0; i < b; ++i) {
      const double w = Wc[j * ld + jac_row(i, j)];
      s += w * w;
    }
    s = sqrt(s);
    if (!isfinite(s)) bad = 1;
    sv[j] = s;
  }
  __syncthreads();
  double* so_b = so + blockIdx.x * sstride;
  double* Uo = trans ? Yo : Xo;   // normalised columns of the working matrix
  double* Vo = trans ? Xo : Yo;   // accumulated rotations
  for (int j = t; j < b; j += nt) {
    const double sj = sv[j];
    int rank = 0;
    for (int k = 0; k < b; ++k) {
      const double sk = sv[k];
      rank += (sk > sj || (sk == sj && k < j)) ? 1 : 0;
    }
    so_b[rank] = sj;
    if (Uo) {
      double* X = Uo + blockIdx.x * bstride;
      const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
      for (int i = 0; i < b; ++i) X[(long long)i * b + rank] = Wc[j * ld + jac_row(i, j)] * inv;
    }
    if (Vo && Vc) {
      double* Y = Vo + blockIdx.x * bstride;
      for (int i = 0; i < b; ++i) Y[(long long)i * b + rank] = Vc[j * ld + jac_row(i, j)];
    }
  }
  if (t == 0 && (bad || sweep >= 60)) *err = 1;
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
  for (int i = t; i < n; i += blockDim.x) {
    const double v = fabs(X[(long long)i * ldx + j]);
    if (v > best) { best = v; bi = i; }
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
  const int imax = si[0];
  const bool flip = (imax < n) && X[(long long)imax * ldx + j] < 0.0;
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

// Raise the dynamic-LDS limit of a kernel to `bytes` when above the 64 KB
// default (gfx950 has 160 KB of LDS per CU).
// Raise a kernel's dynamic-LDS limit once per (kernel, size) and process:
// later calls, including those made while a stream is being captured into a
// graph, issue no runtime call.
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

inline int grid_for(size_t n, int block = 256, int cap = 4096) {
  size_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > (size_t)cap) g = cap;
  return (int)g;
}

double* red_scratch(Context& ctx) {
  if (ctx.scratch_small.bytes < (kRedBlocks + 64) * sizeof(double)) {
    CTM_HIP(hipStreamSynchronize(ctx.stream));
    ctx.scratch_small.alloc((kRedBlocks + 64) * sizeof(double));
  }
  return ctx.scratch_small.d();
}

}  // namespace

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
  double* part = red_scratch(ctx);
  double* inv = part + kRedBlocks;
  const int nb = grid_for(n, 256, kRedBlocks);
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(nb), dim3(256), 0, ctx.stream, p, n, part);
  hipLaunchKernelGGL(maxabs_final_kernel, dim3(1), dim3(256), 0, ctx.stream, part, nb, log_slot,
                     flag, inv, inv_keep);
  hipLaunchKernelGGL(scale_by_dev_kernel, dim3(grid_for(n)), dim3(256), 0, ctx.stream, p, n, inv);
  CTM_HIP(hipGetLastError());
}

void dot(Context& ctx, const double* x, const double* y, size_t n, double* result) {
  double* part = red_scratch(ctx);
  const int nb = grid_for(n, 256, kRedBlocks);
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(256), 0, ctx.stream, x, y, n, part);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(256), 0, ctx.stream, part, nb, result);
  CTM_HIP(hipGetLastError());
}

int jacobi_max_b(bool vectors) { return vectors ? 96 : 128; }

void jacobi_svd(Context& ctx, const double* B, int b, double* X, double* s, double* Y, int* err,
                int batch, long long bstride, long long sstride, bool trans) {
  const bool vec = (X != nullptr || Y != nullptr);
  CTM_REQUIRE(b >= 1 && b <= jacobi_max_b(vec), "jacobi_svd: b out of range");
  const int bp = b + (b & 1);
  int rpt = (b + 7) / 8;
  rpt = rpt <= 4 ? 4 : (rpt <= 8 ? 8 : (rpt <= 12 ? 12 : 16));
  const int ld = 8 * rpt;
  const size_t lds = ((vec ? 2 : 1) * (size_t)bp * ld + bp) * sizeof(double) +
                     (size_t)(bp - 1) * bp + 16;
  CTM_REQUIRE(lds <= 160 * 1024, "jacobi_svd: matrix too large for LDS");
  const int threads = std::max(64, (bp / 2) * 8);
  CTM_REQUIRE(threads <= 512, "jacobi_svd: too many column pairs");
#define CTM_JAC(R)                                                                            \
  do {                                                                                        \
    allow_lds((const void*)jacobi_svd_kernel<R>, lds);                                        \
    hipLaunchKernelGGL(jacobi_svd_kernel<R>, dim3(batch), dim3(threads), lds, ctx.stream, B, b, \
                       bstride, sstride, X, s, Y, err, vec ? 1 : 0, trans ? 1 : 0);          \
  } while (0)
  if (rpt == 4) CTM_JAC(4);
  else if (rpt == 8) CTM_JAC(8);
  else if (rpt == 12) CTM_JAC(12);
  else CTM_JAC(16);
#undef CTM_JAC
  CTM_HIP(hipGetLastError());
}

void chol_inverse(Context& ctx, const double* G, int b, double dep_tol, double* W, int* dep,
                  int* err) {
  CTM_REQUIRE(b >= 1 && b <= 96, "chol_inverse: b out of range");
  hipLaunchKernelGGL((chol_inv_kernel<32>), dim3(1), dim3(1024), 0, ctx.stream, G, b, dep_tol, W,
                     dep, err);
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
