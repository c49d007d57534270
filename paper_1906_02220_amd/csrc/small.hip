// Small and memory-bound kernels of the CTMRG path: fills, normalisation,
// reductions, the counter-based generator, the Gram-Cholesky factor used to
// orthonormalise the subspace of the truncated projector SVD, the one-sided
// Jacobi SVD of small square matrices, and column scalings.
#include <cfloat>
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
                                    double* inv_out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = fmax(m, partial[i]);
  m = block_max256(m, sh);
  if (threadIdx.x == 0) {
    if (!(m < INFINITY) || m == 0.0) {
      *flag = 1;
      *inv_out = 1.0;
    } else {
      *inv_out = 1.0 / m;
      *log_slot += log(m);
    }
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

__global__ __launch_bounds__(1024) void gram_cholesky_kernel(const double* __restrict__ G, int b,
                                                             double dep_tol,
                                                             double* __restrict__ Wout,
                                                             int* __restrict__ dep, int* err) {
  extern __shared__ double lds[];
  double* R = lds;              // b x b, row-major; upper part R, lower part X^T
  double* D = lds + b * b;      // column scales
  double* Xd = D + b;           // diagonal of X = R^{-1}
  int* depl = (int*)(Xd + b);   // dependency flags
  __shared__ int bad;
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  if (t == 0) bad = 0;
  for (int i = t; i < b; i += nt) {
    const double g = G[i * b + i];
    D[i] = (g > 0.0 && isfinite(g)) ? sqrt(g) : 0.0;
    if (!isfinite(g)) bad = 1;
  }
  __syncthreads();
  for (int idx = t; idx < b * b; idx += nt) {
    const int i = idx / b, j = idx - (idx / b) * b;
    const double g = G[idx];
    if (!isfinite(g)) bad = 1;
    const double den = D[i] * D[j];
    R[idx] = (den > 0.0) ? g / den : 0.0;
  }
  __syncthreads();
  // right-looking upper Cholesky of the unit-diagonal Gram with dependency
  // detection (a pivot below dep_tol marks the column as dependent)
  for (int k = 0; k < b; ++k) {
    const double piv = R[k * b + k];
    const bool dk = !(piv > dep_tol);
    const double r = dk ? 1.0 : sqrt(piv);
    __syncthreads();
    if (t == 0) depl[k] = dk ? 1 : 0;
    for (int j = k + 1 + t; j < b; j += nt) R[k * b + j] = dk ? 0.0 : R[k * b + j] / r;
    if (t == 0) R[k * b + k] = r;
    __syncthreads();
    const int m = b - k - 1;
    if (!dk && m > 0) {
      for (int idx = t; idx < m * m; idx += nt) {
        const int i = k + 1 + idx / m, j = k + 1 + (idx - (idx / m) * m);
        if (j >= i) R[i * b + j] -= R[k * b + i] * R[k * b + j];
      }
    }
    __syncthreads();
  }
  // X = R^{-1}: thread j computes column j; X[i][j] (i < j) is kept at R[j][i]
  for (int j = t; j < b; j += nt) {
    const double xjj = 1.0 / R[j * b + j];
    Xd[j] = xjj;
    for (int i = j - 1; i >= 0; --i) {
      double s = R[i * b + j] * xjj;
      for (int k = i + 1; k < j; ++k) s += R[i * b + k] * R[j * b + k];
      R[j * b + i] = -s / R[i * b + i];
    }
  }
  __syncthreads();
  // W = D^{-1} X (row i scaled by 1/D_i; zero column scale -> zero row)
  for (int idx = t; idx < b * b; idx += nt) {
    const int i = idx / b, j = idx - (idx / b) * b;
    double x = 0.0;
    if (i == j) x = Xd[i];
    else if (i < j) x = R[j * b + i];
    Wout[idx] = (D[i] > 0.0) ? x / D[i] : 0.0;
  }
  for (int i = t; i < b; i += nt) dep[i] = depl[i];
  if (t == 0 && bad) *err = 1;
}

// Q = Z W with W staged in LDS; dependent columns refilled with normals.
__global__ __launch_bounds__(256) void apply_right_kernel(const double* __restrict__ Z, int ldz,
                                                          const double* __restrict__ Wm, int n,
                                                          int b, double* __restrict__ Q, int ldq,
                                                          const int* __restrict__ dep,
                                                          unsigned long long seed,
                                                          unsigned long long ctr) {
  extern __shared__ double Ws[];
  const int t = threadIdx.x;
  for (int idx = t; idx < b * b; idx += blockDim.x) Ws[idx] = Wm[idx];
  __syncthreads();
  constexpr int TPR = 16;  // threads per row
  const int row = blockIdx.x * (256 / TPR) + t / TPR;
  const int cg = t % TPR;
  if (row >= n) return;
  const double* z = Z + (long long)row * ldz;
  double acc[8];
  for (int c0 = 0; c0 < b; c0 += 8 * TPR) {
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = 0.0;
    for (int k = 0; k < b; ++k) {
      const double zk = z[k];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = c0 + cg + e * TPR;
        if (j < b) acc[e] += zk * Ws[k * b + j];
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int j = c0 + cg + e * TPR;
      if (j < b) {
        double v = acc[e];
        if (dep && dep[j]) v = normal_at(seed, ctr + (unsigned long long)row * b + j);
        Q[(long long)row * ldq + j] = v;
      }
    }
  }
}

// ------------------------------------------------------------ Jacobi SVD

// One workgroup per matrix.  Columns of the working matrix and of V are kept
// column-major in LDS; each round of the circle schedule rotates bp/2
// disjoint column pairs in parallel, a group of TP lanes per pair.
__global__ __launch_bounds__(1024) void jacobi_svd_kernel(const double* __restrict__ Bm, int b,
                                                          long long bstride, long long sstride,
                                                          double* __restrict__ Xo,
                                                          double* __restrict__ so,
                                                          double* __restrict__ Yo, int* err,
                                                          int want_vec, int TP) {
  extern __shared__ double lds[];
  const int bp = b + (b & 1);
  double* Wc = lds;                                 // bp columns of length b
  double* Vc = want_vec ? lds + bp * b : nullptr;   // bp columns of length b
  double* sv = lds + (want_vec ? 2 : 1) * bp * b;   // bp singular values
  __shared__ int changed;
  __shared__ int bad;
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  const double* B = Bm + blockIdx.x * bstride;
  if (t == 0) { changed = 0; bad = 0; }
  for (int idx = t; idx < bp * b; idx += nt) {
    const int j = idx / b, i = idx - (idx / b) * b;
    Wc[idx] = (j < b) ? B[(long long)i * b + j] : 0.0;
    if (Vc) Vc[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int P = bp / 2;
  const int m = bp - 1;
  const int pi = t / TP;
  const int sub = t - pi * TP;
  const double tol = fmax(1e-15, sqrt((double)b) * DBL_EPSILON);
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    for (int r = 0; r < m; ++r) {
      if (pi < P) {
        int p, q;
        if (pi == 0) { p = m; q = r; }
        else { p = (r + pi) % m; q = (r - pi + m) % m; }
        double* wp = Wc + p * b;
        double* wq = Wc + q * b;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = sub; i < b; i += TP) {
          const double x = wp[i], y = wq[i];
          al += x * x; be += y * y; ga += x * y;
        }
        for (int o = TP / 2; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, TP);
          be += __shfl_xor(be, o, TP);
          ga += __shfl_xor(ga, o, TP);
        }
        double tt = 0.0;
        if (al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
          // tangent of the rotation angle, the smaller root of t^2 + 2 zeta t - 1 = 0
          const double zeta = (be - al) / (2.0 * ga);
          tt = (fabs(zeta) < 1e150)
                   ? (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta))
                   : 0.5 / zeta;
        }
        if (tt != 0.0) {
          const double c = 1.0 / sqrt(1.0 + tt * tt);
          const double s = c * tt;
          for (int i = sub; i < b; i += TP) {
            const double x = wp[i], y = wq[i];
            wp[i] = c * x - s * y;
            wq[i] = s * x + c * y;
          }
          if (Vc) {
            double* vp = Vc + p * b;
            double* vq = Vc + q * b;
            for (int i = sub; i < b; i += TP) {
              const double x = vp[i], y = vq[i];
              vp[i] = c * x - s * y;
              vq[i] = s * x + c * y;
            }
          }
          if (sub == 0) changed = 1;
        }
      }
      __syncthreads();
    }
    const int ch = changed;
    __syncthreads();
    if (t == 0) changed = 0;
    __syncthreads();
    if (!ch) break;
  }
  // singular values and ordering
  for (int j = t; j < bp; j += nt) {
    double s = 0.0;
    for (int i = 0; i < b; ++i) s += Wc[j * b + i] * Wc[j * b + i];
    s = sqrt(s);
    if (!isfinite(s)) bad = 1;
    sv[j] = s;
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
    so_b[rank] = sj;
    if (Xo) {
      double* X = Xo + blockIdx.x * bstride;
      const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
      for (int i = 0; i < b; ++i) X[(long long)i * b + rank] = Wc[j * b + i] * inv;
    }
    if (Yo && Vc) {
      double* Y = Yo + blockIdx.x * bstride;
      for (int i = 0; i < b; ++i) Y[(long long)i * b + rank] = Vc[j * b + i];
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
void allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
    (void)hipGetLastError();
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
void fill_normal(Context& ctx, double* Z, size_t count, unsigned long long seed,
                 unsigned long long counter) {
  if (!count) return;
  hipLaunchKernelGGL(fill_normal_kernel, dim3(grid_for(count)), dim3(256), 0, ctx.stream, Z,
                     count, seed, counter);
  CTM_HIP(hipGetLastError());
}

void normalise_maxabs(Context& ctx, double* p, size_t n, double* log_slot, int* flag) {
  double* part = red_scratch(ctx);
  double* inv = part + kRedBlocks;
  const int nb = grid_for(n, 256, kRedBlocks);
  hipLaunchKernelGGL(maxabs_partial_kernel, dim3(nb), dim3(256), 0, ctx.stream, p, n, part);
  hipLaunchKernelGGL(maxabs_final_kernel, dim3(1), dim3(256), 0, ctx.stream, part, nb, log_slot,
                     flag, inv);
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

void gram_cholesky(Context& ctx, const double* G, int b, double dep_tol, double* W, int* dep,
                   int* err) {
  CTM_REQUIRE(b >= 1 && b <= 128, "gram_cholesky: b out of range");
  const size_t lds = (size_t)b * b * sizeof(double) + 2 * b * sizeof(double) + b * sizeof(int);
  allow_lds((const void*)gram_cholesky_kernel, lds);
  hipLaunchKernelGGL(gram_cholesky_kernel, dim3(1), dim3(1024), lds, ctx.stream, G, b, dep_tol, W,
                     dep, err);
  CTM_HIP(hipGetLastError());
}

void apply_right(Context& ctx, const double* Z, int ldz, const double* W, int n, int b, double* Q,
                 int ldq, const int* dep, unsigned long long seed, unsigned long long counter) {
  CTM_REQUIRE(b >= 1 && b <= 128, "apply_right: b out of range");
  const size_t lds = (size_t)b * b * sizeof(double);
  allow_lds((const void*)apply_right_kernel, lds);
  const int blocks = (n + 15) / 16;
  hipLaunchKernelGGL(apply_right_kernel, dim3(blocks), dim3(256), lds, ctx.stream, Z, ldz, W, n, b,
                     Q, ldq, dep, seed, counter);
  CTM_HIP(hipGetLastError());
}

int jacobi_max_b(bool vectors) { return vectors ? 96 : 128; }

void jacobi_svd(Context& ctx, const double* B, int b, double* X, double* s, double* Y, int* err,
                int batch, long long bstride, long long sstride) {
  const bool vec = (X != nullptr || Y != nullptr);
  CTM_REQUIRE(b >= 1 && b <= jacobi_max_b(vec), "jacobi_svd: b out of range");
  const int bp = b + (b & 1);
  const size_t lds = ((vec ? 2 : 1) * (size_t)bp * b + bp) * sizeof(double);
  allow_lds((const void*)jacobi_svd_kernel, lds);
  const int P = bp / 2;
  int TP = 64;
  while (TP > 1 && P * TP > 1024) TP >>= 1;
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(batch), dim3(1024), lds, ctx.stream, B, b, bstride,
                     sstride, X, s, Y, err, vec ? 1 : 0, TP);
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
