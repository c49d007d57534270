// Leading eigenvalues of the column (or row) transfer matrix of a CTMRG
// environment, for the correlation length xi = -1 / ln |lambda_2 / lambda_1|
// in lattice constants of the rhombic lattice (Sec. IV quotes xi in those
// units).
//
// Horizontal transfer matrix of one column (the top edge, the site row, the
// bottom edge), acting on a vector v[x][l][y] of the vertical cut:
//   v'[x', r, y'] = sum T1[x, m, x'] a[m, l, n, r] T3[y', n, y] v[x, l, y],
// applied as three GEMMs and two permutations (4 chi^3 d^2 + 2 chi^2 d^4
// flops); without the site row the inner legs of T1 and T3 are joined.  The
// vertical one is the same in the frame rotated once (T2, a rotated, T4).
//
// The spectrum comes from k steps of Arnoldi on the GPU (classical
// Gram-Schmidt applied twice, by bandwidth-bound projection and update
// kernels), enqueued without waiting for the device, and the eigenvalues of
// the k x k Hessenberg matrix by a complex shifted QR iteration (Wilkinson
// shifts, Givens rotations, deflation at a relative subdiagonal of 2^-52) in
// one wave.  The 2 chi^2 d^4 product of the site row runs in the
// environment's precision mode; the rest is FP64.

#include <algorithm>
#include <cmath>
#include <vector>

#include "transfer.hpp"

namespace ctm {

namespace {

struct cx {
  double r, i;
};
__device__ inline cx cadd(cx a, cx b) { return {a.r + b.r, a.i + b.i}; }
__device__ inline cx csub(cx a, cx b) { return {a.r - b.r, a.i - b.i}; }
__device__ inline cx cmul(cx a, cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline cx cconj(cx a) { return {a.r, -a.i}; }
__device__ inline double cabs_(cx a) { return hypot(a.r, a.i); }
__device__ inline cx cscale(cx a, double s) { return {a.r * s, a.i * s}; }
__device__ inline cx csqrt_(cx a) {
  const double m = cabs_(a);
  if (m == 0.0) return {0.0, 0.0};
  const double re = sqrt(0.5 * (m + fabs(a.r)));
  if (a.r >= 0.0) return {re, a.i / (2.0 * re)};
  return {fabs(a.i) / (2.0 * re), a.i >= 0.0 ? re : -re};
}

// Eigenvalues of the leading k x k block of the upper Hessenberg matrix H
// (row-major, leading dimension ldh, kmax columns), where k is kmax or the
// first j + 1 with H[j + 1][j] exactly zero (an Arnoldi breakdown), into wr,
// wi, and k into *count.  *err = 1 if some eigenvalue did not converge in 200
// steps.  One wave: the matrix lives in LDS (k^2 complex entries), every
// lane takes the same shift and rotation decisions, and each plane rotation
// updates its two rows (or columns) across the lanes, element by element in
// the same arithmetic as a serial sweep.
constexpr int kHessThreads = 64;
__global__ __launch_bounds__(kHessThreads) void hessenberg_eigen_kernel(
    const double* __restrict__ H, int kmax, int ldh, double* wr, double* wi, int* err, int* count) {
  extern __shared__ cx Z[];  // k x k, then the rotations of one QR step
  const int t = threadIdx.x;
  int k = kmax;
  for (int j = 0; j + 1 < kmax; ++j)
    if (H[(j + 1) * ldh + j] == 0.0) { k = j + 1; break; }
  cx* cs = Z + (size_t)kmax * kmax;
  cx* sn = cs + kmax;
  for (int idx = t; idx < k * k; idx += kHessThreads) {
    const int i = idx / k, j = idx - (idx / k) * k;
    Z[idx] = {j >= i - 1 ? H[i * ldh + j] : 0.0, 0.0};
  }
  if (t == 0) *count = k;
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  int hi = k - 1, iter = 0;
  while (hi >= 0) {
    int l = hi;
    while (l > 0) {
      const double s = cabs_(Z[(l - 1) * k + l - 1]) + cabs_(Z[l * k + l]);
      const double sub = cabs_(Z[l * k + l - 1]);
      if (sub <= eps * s || sub == 0.0) break;
      --l;
    }
    __syncthreads();  // every lane has read what decided l
    if (l > 0 && t == 0) Z[l * k + l - 1] = {0.0, 0.0};
    if (l == hi) {
      if (t == 0) {
        wr[hi] = Z[hi * k + hi].r;
        wi[hi] = Z[hi * k + hi].i;
      }
      --hi;
      iter = 0;
      __syncthreads();
      continue;
    }
    if (++iter > 200) {
      if (t == 0) {
        *err = 1;
        for (int i = 0; i <= hi; ++i) {
          wr[i] = Z[i * k + i].r;
          wi[i] = Z[i * k + i].i;
        }
      }
      return;
    }
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer to
    // its last diagonal entry; every 10th step an exceptional shift
    const cx a = Z[(hi - 1) * k + hi - 1], b = Z[(hi - 1) * k + hi], c = Z[hi * k + hi - 1],
             d = Z[hi * k + hi];
    cx mu;
    if (iter % 10 == 0) {
      mu = cadd(d, {0.75 * cabs_(c), 0.0});
    } else {
      const cx half = cscale(csub(a, d), 0.5);
      const cx disc = csqrt_(cadd(cmul(half, half), cmul(b, c)));
      const cx m0 = cadd(cscale(cadd(a, d), 0.5), disc), m1 = csub(cscale(cadd(a, d), 0.5), disc);
      mu = cabs_(csub(m0, d)) <= cabs_(csub(m1, d)) ? m0 : m1;
    }
    __syncthreads();  // the shift is read before the diagonal moves
    for (int i = l + t; i <= hi; i += kHessThreads) Z[i * k + i] = csub(Z[i * k + i], mu);
    __syncthreads();
    // Z - mu = Q R by Givens rotations G_i = [[conj c, conj s], [-s, c]] on
    // rows i, i+1; then R Q by G_i^H on columns i, i+1.
    for (int i = l; i < hi; ++i) {
      const cx x = Z[i * k + i], y = Z[(i + 1) * k + i];
      const double r = hypot(cabs_(x), cabs_(y));
      cx cc = {1.0, 0.0}, ss = {0.0, 0.0};
      if (r > 0.0) {
        cc = cscale(x, 1.0 / r);
        ss = cscale(y, 1.0 / r);
      }
      if (t == 0) {
        cs[i - l] = cc;
        sn[i - l] = ss;
      }
      __syncthreads();  // x and y are read before lane i rewrites them
      for (int j = i + t; j <= hi; j += kHessThreads) {
        const cx u = Z[i * k + j], v = Z[(i + 1) * k + j];
        Z[i * k + j] = cadd(cmul(cconj(cc), u), cmul(cconj(ss), v));
        Z[(i + 1) * k + j] = csub(cmul(cc, v), cmul(ss, u));
      }
      __syncthreads();
    }
    for (int i = l; i < hi; ++i) {
      const cx cc = cs[i - l], ss = sn[i - l];
      const int rmax = min(i + 1, hi);
      for (int r = l + t; r <= rmax; r += kHessThreads) {
        const cx u = Z[r * k + i], v = Z[r * k + i + 1];
        Z[r * k + i] = cadd(cmul(u, cc), cmul(v, ss));
        Z[r * k + i + 1] = csub(cmul(v, cconj(cc)), cmul(u, cconj(ss)));
      }
      __syncthreads();
    }
    for (int i = l + t; i <= hi; i += kHessThreads) Z[i * k + i] = cadd(Z[i * k + i], mu);
    __syncthreads();
  }
}

// Arnoldi bookkeeping of step j: H[0..j][j] = h1 + h2 (the two Gram-Schmidt
// passes), H[j+1][j] = ||w|| from nrm2 = w.w, inv = 1 / ||w||.  At a
// breakdown (||w|| <= 1e-14 or not finite: an invariant subspace) H[j+1][j]
// is set to exactly 0 and inv to 0, so that every later basis vector, and
// with it every later column of H, is exactly zero and the eigenvalue kernel
// stops at the zero subdiagonal.
__global__ void arnoldi_step_kernel(double* H, int ldh, int j, const double* h1,
                                    const double* h2, const double* nrm2, double* inv) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i <= j; ++i) H[i * ldh + j] = h1[i] + h2[i];
  const double nv = sqrt(fmax(*nrm2, 0.0));
  const bool ok = nv > 1e-14 && nv < INFINITY;
  H[(j + 1) * ldh + j] = ok ? nv : 0.0;
  *inv = ok ? 1.0 / nv : 0.0;
}

// Classical Gram-Schmidt against the rows V[0..rows) (each dim long, row
// stride ld) of the Krylov basis, in two kernels each reading V once.
// Projection: block b writes part[b * 64 + i] = sum over its chunk of
// V[i][t] w[t] for every row at once (one accumulator per row, one
// reduction per block); gs_sum_kernel adds the blocks' parts in a fixed
// order (the result does not depend on scheduling).
constexpr int kGsMaxRows = 64;
__global__ __launch_bounds__(256) void gs_project_kernel(const double* __restrict__ V, size_t ld,
                                                         size_t dim, int rows,
                                                         const double* __restrict__ w,
                                                         double* __restrict__ part) {
  __shared__ double red[4][kGsMaxRows];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t chunk = (dim + gridDim.x - 1) / gridDim.x;
  const size_t t0 = (size_t)blockIdx.x * chunk;
  const size_t t1 = t0 + chunk < dim ? t0 + chunk : dim;
  double a[kGsMaxRows];
#pragma unroll
  for (int i = 0; i < kGsMaxRows; ++i) a[i] = 0.0;
  for (size_t t = t0 + tid; t < t1; t += 256) {
    const double wt = w[t];
#pragma unroll
    for (int i = 0; i < kGsMaxRows; ++i)
      if (i < rows) a[i] = fma(V[(size_t)i * ld + t], wt, a[i]);
  }
#pragma unroll
  for (int i = 0; i < kGsMaxRows; ++i) {
    if (i < rows) {
      double v = a[i];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wave][i] = v;
    }
  }
  __syncthreads();
  if (tid < rows)
    part[(size_t)blockIdx.x * kGsMaxRows + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// h[i] = sum over the nblk blocks' parts of row i, one workgroup of
// kGsSumGroups groups of 64 threads (one thread per row): group q adds parts
// q, q + G, q + 2 G, ... in batches of kGsSumBatch loads in flight, into four
// running sums, and the groups' sums then meet in a fixed tree, so the result
// does not depend on scheduling.  (A serial chain of dependent loads took
// 43 us per call.)
constexpr int kGsSumGroups = 16;
constexpr int kGsSumBatch = 8;
__global__ __launch_bounds__(64 * kGsSumGroups) void gs_sum_kernel(const double* __restrict__ part,
                                                                  int nblk, int rows,
                                                                  double* __restrict__ h) {
  __shared__ double sh[kGsSumGroups][kGsMaxRows];
  const int i = threadIdx.x & (kGsMaxRows - 1), q = threadIdx.x >> 6;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < rows) {
    constexpr int G = kGsSumGroups;
    for (int b0 = q; b0 < nblk; b0 += G * kGsSumBatch) {
      double v[kGsSumBatch];
#pragma unroll
      for (int u = 0; u < kGsSumBatch; ++u) {
        const int b = b0 + u * G;
        v[u] = b < nblk ? part[(size_t)b * kGsMaxRows + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kGsSumBatch; ++u) s[u & 3] += v[u];
    }
  }
  sh[q][i] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  for (int w = kGsSumGroups / 2; w > 0; w >>= 1) {
    if (q < w) sh[q][i] += sh[q + w][i];
    __syncthreads();
  }
  if (q == 0 && i < rows) h[i] = sh[0][i];
}

// w[t] -= sum_i V[i][t] h[i] for i < rows.
__global__ __launch_bounds__(256) void gs_update_kernel(const double* __restrict__ V, size_t ld,
                                                        size_t dim, int rows,
                                                        const double* __restrict__ h,
                                                        double* __restrict__ w) {
  __shared__ double hs[kGsMaxRows];
  if (threadIdx.x < rows) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < dim; t += (size_t)gridDim.x * 256) {
    double s = 0.0;
    for (int i = 0; i < rows; ++i) s = fma(V[(size_t)i * ld + t], hs[i], s);
    w[t] -= s;
  }
}

// inv = 1 / sqrt(nrm2) (0 if nrm2 is 0)
__global__ void inv_norm_kernel(const double* nrm2, double* inv) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double nv = sqrt(fmax(*nrm2, 0.0));
  *inv = nv > 0.0 ? 1.0 / nv : 0.0;
}

__global__ void scale_dev_kernel(double* p, size_t n, const double* s) {
  const double f = *s;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] *= f;
}

inline int nblk(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

void mm(Context& c, int M, int N, int K, const double* A, long long lda, bool ta, const double* B,
        long long ldb, bool tb, double* C, long long ldc, double beta = 0.0, double alpha = 1.0) {
  gemm_f64(c, M, N, K, alpha, ta ? colmajor(A, lda) : rowmajor(A, lda),
           tb ? colmajor(B, ldb) : rowmajor(B, ldb), beta, out_rowmajor(C, ldc));
}

}  // namespace

Transfer::Transfer(Env& env, int direction_, bool site_)
    : e(env), ctx(env.ctx), direction(direction_), site(site_), chi(env.chi), d(env.d) {
  CTM_REQUIRE(direction == 0 || direction == 1, "direction must be 0 (columns) or 1 (rows)");
  dim = (size_t)chi * chi * (site ? d : 1);
  const size_t w = (size_t)chi * d * chi * (site ? d : 1);
  w1.alloc(w * sizeof(double));
  w2.alloc(w * sizeof(double));
  if (site) {
    // a[m, l, n, r] -> [(l n), (m r)] of the frame's site tensor
    aT.alloc((size_t)d * d * d * d * sizeof(double));
    const long long f4[4] = {d, d, d, d};
    const int p1203[4] = {1, 2, 0, 3};
    permute(ctx, e.arot[direction].d(), aT.d(), 4, f4, p1203);
  }
}

void Transfer::apply(const double* v, double* out) {
  const int dc = d * chi;
  const double* Tt = e.Tp(direction);      // T1 (or T2)
  const double* Tb = e.Tp(direction + 2);  // T3 (or T4)
  if (site) {
    // w1[(x l)][(y' n)] = v[(x l)][y] T[(y' n)][y]
    mm(ctx, dc, dc, chi, v, chi, false, Tb, chi, true, w1.d(), dc);
    const long long q4[4] = {chi, d, chi, d};
    const int p0213[4] = {0, 2, 1, 3};
    permute(ctx, w1.d(), w2.d(), 4, q4, p0213);  // [x][y'][l][n]
    // the 2 chi^2 d^4 product in the environment's precision mode (the site
    // tensor's slices are cut once per Transfer)
    const int M = chi * chi, N = d * d, K = d * d;
    if (!gemm_slices_split_out(ctx, e.opt.precision, M, N, K, rowmajor(w2.d(), K),
                               rowmajor(aT.d(), N), w1.d(), OutMap::plain(M, N, N), -1, &aslices))
      gemm_mixed(ctx, e.opt.precision, M, N, K, 1.0, rowmajor(w2.d(), K), rowmajor(aT.d(), N), 0.0,
                 out_rowmajor(w1.d(), N));
    const int p0231[4] = {0, 2, 3, 1};
    const long long r4[4] = {chi, chi, d, d};
    permute(ctx, w1.d(), w2.d(), 4, r4, p0231);  // [x][m][r][y']
    mm(ctx, chi, dc, dc, Tt, chi, true, w2.d(), dc, false, out, dc);
  } else {
    mm(ctx, chi, dc, chi, v, chi, false, Tb, chi, true, w1.d(), dc);  // [x][(y' m)]
    const long long q3[3] = {chi, chi, d};
    const int p021[3] = {0, 2, 1};
    permute(ctx, w1.d(), w2.d(), 3, q3, p021);  // [x][m][y']
    mm(ctx, chi, chi, dc, Tt, chi, true, w2.d(), chi, false, out, chi);
  }
}

int Transfer::spectrum(int krylov, unsigned long long seed, double* wr_out, double* wi_out) {
  const int k = (int)std::min<size_t>((size_t)std::max(krylov, 2), std::min<size_t>(dim, 64));
  static_assert(kGsMaxRows >= 64, "Gram-Schmidt rows");
  DevBuf V((size_t)(k + 1) * dim * sizeof(double));
  DevBuf H((size_t)(k + 1) * k * sizeof(double));
  DevBuf h(2 * (size_t)(k + 1) * sizeof(double));
  const int gblk = (int)std::min<size_t>((dim + 255) / 256, 512);
  DevBuf part((size_t)gblk * kGsMaxRows * sizeof(double));
  DevBuf sc(4 * sizeof(double));
  DevBuf wr(k * sizeof(double)), wi(k * sizeof(double));
  DevBuf flags(2 * sizeof(int));  // error, number of Ritz values
  fill_zero(ctx, H.d(), (size_t)(k + 1) * k);
  fill_zero_int(ctx, (int*)flags.p, 2);
  double* v0 = V.d();
  fill_normal(ctx, v0, dim, seed, 0);
  dot(ctx, v0, v0, dim, sc.d());
  hipLaunchKernelGGL(inv_norm_kernel, dim3(1), dim3(1), 0, ctx.stream, sc.d(), sc.d() + 1);
  hipLaunchKernelGGL(scale_dev_kernel, dim3(nblk(dim)), dim3(256), 0, ctx.stream, v0, dim,
                     sc.d() + 1);
  CTM_HIP(hipGetLastError());
  // k steps without waiting for the device: a breakdown zeroes the rest of
  // the basis (arnoldi_step_kernel) instead of stopping the loop
  for (int j = 0; j < k; ++j) {
    double* vj = V.d() + (size_t)j * dim;
    double* w = V.d() + (size_t)(j + 1) * dim;
    apply(vj, w);
    // two passes of classical Gram-Schmidt against v_0..v_j
    double* h1 = h.d();
    double* h2 = h.d() + (k + 1);
    for (int pass = 0; pass < 2; ++pass) {
      double* hp = pass == 0 ? h1 : h2;
      hipLaunchKernelGGL(gs_project_kernel, dim3(gblk), dim3(256), 0, ctx.stream, V.d(), dim, dim,
                         j + 1, w, part.d());
      hipLaunchKernelGGL(gs_sum_kernel, dim3(1), dim3(64 * kGsSumGroups), 0, ctx.stream, part.d(),
                         gblk, j + 1, hp);
      hipLaunchKernelGGL(gs_update_kernel, dim3(nblk(dim)), dim3(256), 0, ctx.stream, V.d(), dim,
                         dim, j + 1, hp, w);
    }
    dot(ctx, w, w, dim, sc.d());
    hipLaunchKernelGGL(arnoldi_step_kernel, dim3(1), dim3(1), 0, ctx.stream, H.d(), k, j, h1, h2,
                       sc.d(), sc.d() + 1);
    hipLaunchKernelGGL(scale_dev_kernel, dim3(nblk(dim)), dim3(256), 0, ctx.stream, w, dim,
                       sc.d() + 1);
    CTM_HIP(hipGetLastError());
  }
  const size_t hlds = ((size_t)k * k + 2 * (size_t)k) * sizeof(cx);
  allow_lds((const void*)hessenberg_eigen_kernel, hlds);
  hipLaunchKernelGGL(hessenberg_eigen_kernel, dim3(1), dim3(kHessThreads), hlds, ctx.stream, H.d(),
                     k, k, wr.d(), wi.d(), (int*)flags.p, (int*)flags.p + 1);
  CTM_HIP(hipGetLastError());
  int hf[2] = {0, 0};
  CTM_HIP(hipMemcpyAsync(hf, flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  const int steps = hf[1];
  CTM_REQUIRE(steps >= 1 && steps <= k, "transfer spectrum: bad Ritz value count");
  CTM_HIP(hipMemcpy(wr_out, wr.p, steps * sizeof(double), hipMemcpyDeviceToHost));
  CTM_HIP(hipMemcpy(wi_out, wi.p, steps * sizeof(double), hipMemcpyDeviceToHost));
  if (hf[0]) throw Error(-4, "transfer spectrum: Hessenberg QR did not converge");
  return steps;
}

}  // namespace ctm
