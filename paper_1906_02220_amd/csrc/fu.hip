// One bond update of the exact-environment full update (arXiv:1906.02220,
// Sec. III, Fig. 3(b) and Fig. 4), and the second-order Trotter step built
// from it.
//
//  1. gate G = exp(-tau H / 2) of the real 4 x 4 bond Hamiltonian, by scaling
//     and squaring of its Taylor series in one small kernel;
//  2. G[(s t), (s' t')] regrouped as [(s s'), (t t')] and split by SVD into
//     two gate tensors joined by an index r of dimension 4;
//  3. A'[s, a, .., (g r), ..] = sum_s' gL[(s s'), r] A[s', a, .., g, ..] and
//     B' likewise: the gamma bond grows to 4D;
//  4. the environment of the composite A'-B' (gamma bond inside it) by the
//     engine's CTMRG, as the metric E[ket outer legs][bra outer legs];
//  5. A'', B'' with a D gamma bond minimising
//       d = sum_p <K'_p - K''_p, E (K'_p - K''_p)>,  K = composite,
//     by alternating exact least-squares solves (A'' with B'' fixed, then
//     B'' with A'' fixed) from A'' = A, B'' = B; E is symmetrised and each
//     normal matrix gets a ridge of 1e-12 tr(N) / dim(N).
//
// Step 5 in fused layouts Ap[s,a,l,u,g], Bp[t,c,r,d,g] (l, u: A's alpha and
// beta legs; r, d: B's), K[(s a t c)][(u l d r)]:
//   N_A = sum_tc M_tc^T E M_tc,   b_A = sum_tc (K' E)_tc M_tc,
//   M_tc[(u l d r)][(l' u' g)] = [u = u'][l = l'] Bp[t,c,r,d,g],
// one batched GEMM for E M, one GEMM each for N_A and b_A, and a Cholesky
// solve with the four (s a) right-hand sides; B'' symmetrically.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fu.hpp"

namespace ctm {

namespace {

inline int nblk(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

// G = exp(-tau H / 2) for a 4 x 4 matrix: X = -tau H / 2 scaled by 2^-k so
// that its 1-norm is at most 1/2, a Taylor series to 24 terms, then k
// squarings.
__global__ void gate_exp_kernel(const double* __restrict__ H, double tau, double* __restrict__ G) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double X[16], T[16], S[16], W[16];
  double nrm = 0.0;
  for (int j = 0; j < 4; ++j) {
    double c = 0.0;
    for (int i = 0; i < 4; ++i) c += fabs(H[i * 4 + j]);
    nrm = fmax(nrm, c);
  }
  nrm *= 0.5 * fabs(tau);
  int k = 0;
  while (nrm > 0.5 && k < 60) {
    nrm *= 0.5;
    ++k;
  }
  const double sc = -0.5 * tau * ldexp(1.0, -k);
  for (int i = 0; i < 16; ++i) {
    X[i] = sc * H[i];
    T[i] = (i % 5 == 0) ? 1.0 : 0.0;  // identity
    S[i] = T[i];
  }
  for (int m = 1; m <= 24; ++m) {
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double v = 0.0;
        for (int q = 0; q < 4; ++q) v += T[i * 4 + q] * X[q * 4 + j];
        W[i * 4 + j] = v / m;
      }
    for (int i = 0; i < 16; ++i) {
      T[i] = W[i];
      S[i] += W[i];
    }
  }
  for (int r = 0; r < k; ++r) {
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        double v = 0.0;
        for (int q = 0; q < 4; ++q) v += S[i * 4 + q] * S[q * 4 + j];
        W[i * 4 + j] = v;
      }
    for (int i = 0; i < 16; ++i) S[i] = W[i];
  }
  for (int i = 0; i < 16; ++i) G[i] = S[i];
}

// g[(s s'), (t t')] = G[(s t), (s' t')]
__global__ void regroup_gate_kernel(const double* __restrict__ G, double* __restrict__ g) {
  const int i = threadIdx.x;
  if (i >= 16) return;
  const int s = i >> 3, sp = (i >> 2) & 1, t = (i >> 1) & 1, tp = i & 1;
  g[((s * 2 + sp) * 2 + t) * 2 + tp] = G[((s * 2 + t) * 2 + sp) * 2 + tp];
}

// A'[s, a, i0, i1, i2] with the gamma index i_gamma = g * 4 + r:
//   side 0: sum_s' X[(s s'), r] sqrt(sv_r) A[s', a, .., g, ..]
//   side 1: sum_s' Y[(s s'), r] sqrt(sv_r) B[s', a, .., g, ..]
// (g = X diag(sv) Y^T, gL = X sqrt(sv), gR^T = Y sqrt(sv)).
__global__ void apply_gate_kernel(const double* __restrict__ in, double* __restrict__ out, int D,
                                  int gamma, const double* __restrict__ XY,
                                  const double* __restrict__ sv) {
  const int D3 = D * D * D;
  const long long total = 4LL * D3 * 4;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    // out dims [2][2][o0][o1][o2], o_gamma = 4 D
    int rem = (int)idx;
    int o[3];
    for (int ax = 2; ax >= 0; --ax) {
      const int dim = ax == gamma ? 4 * D : D;
      o[ax] = rem % dim;
      rem /= dim;
    }
    const int a = rem & 1, s = rem >> 1;
    const int g = o[gamma] >> 2, r = o[gamma] & 3;
    int ii[3] = {o[0], o[1], o[2]};
    ii[gamma] = g;
    const long long inner = ((long long)ii[0] * D + ii[1]) * D + ii[2];
    const double w = sqrt(fmax(sv[r], 0.0));
    double v = 0.0;
    for (int sp = 0; sp < 2; ++sp)
      v += XY[(s * 2 + sp) * 4 + r] * w * in[(long long)(sp * 2 + a) * D3 + inner];
    out[idx] = v;
  }
}

// Dense selection products of the least-squares maps.
//  side 0 (from B''p[t,c,r,d,g]): M[tc][(u l d r)][(l' u' g)] = [u=u'][l=l'] Bp[tc][r][d][g]
//  side 1 (from A''p[s,a,l,u,g]): M[sa][(u l d r)][(r' d' g)] = [d=d'][r=r'] Ap[sa][l][u][g]
__global__ void selection_kernel(const double* __restrict__ T, double* __restrict__ M, int D,
                                 int side) {
  const long long D3 = (long long)D * D * D, D4 = D3 * D;
  const long long total = 4 * D4 * D3;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long q = idx / (D4 * D3);
    long long rem = idx - q * D4 * D3;
    const int col = (int)(rem % D3);
    const int row = (int)(rem / D3);
    const int r = row % D, dd = (row / D) % D, l = (row / (D * D)) % D, u = row / (D * D * D);
    const int g = col % D, c1 = (col / D) % D, c0 = col / (D * D);
    double v = 0.0;
    if (side == 0) {
      if (c0 == l && c1 == u) v = T[q * D3 + ((long long)r * D + dd) * D + g];
    } else {
      if (c0 == r && c1 == dd) v = T[q * D3 + ((long long)l * D + u) * D + g];
    }
    M[idx] = v;
  }
}

__device__ inline double bsum1024(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Solve (N + ridge tr(N)/n I) x_j = r_j for a symmetric positive definite
// n x n row-major N (its lower triangle becomes the Cholesky factor L) and m
// right-hand sides stored as the rows of R (m x n, overwritten by the
// solutions).  One workgroup of 1024 threads; column k of L is staged in LDS
// for the trailing update.  A pivot that is not positive sets *err = 1 and
// drops its direction (the factor's column becomes zero, x_k = 0).
__global__ __launch_bounds__(1024) void chol_solve_kernel(double* __restrict__ N, int n,
                                                          double* __restrict__ R, int m,
                                                          double ridge, int* err) {
  __shared__ double sh[1024];
  __shared__ double colk[512];
  const int tid = threadIdx.x;
  double t = 0.0;
  for (int i = tid; i < n; i += 1024) t += N[(long long)i * n + i];
  t = bsum1024(t, sh);
  const double shift = ridge * t / n;
  for (int i = tid; i < n; i += 1024) N[(long long)i * n + i] += shift;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double p = N[(long long)k * n + k];
    const bool ok = p > 0.0 && p < INFINITY;
    const double piv = ok ? sqrt(p) : INFINITY;
    __syncthreads();
    if (tid == 0) {
      N[(long long)k * n + k] = piv;
      if (!ok) *err = 1;
    }
    for (int i = k + 1 + tid; i < n; i += 1024) {
      const double l = N[(long long)i * n + k] / piv;
      N[(long long)i * n + k] = l;
      colk[i] = l;
    }
    __syncthreads();
    const int w = n - k - 1;
    for (long long idx = tid; idx < (long long)w * w; idx += 1024) {
      const int ii = (int)(idx / w), jj = (int)(idx - (long long)ii * w);
      if (jj > ii) continue;
      const int i = k + 1 + ii, j = k + 1 + jj;
      N[(long long)i * n + j] -= colk[i] * colk[j];
    }
    __syncthreads();
  }
  // L y = r
  for (int k = 0; k < n; ++k) {
    const double lk = N[(long long)k * n + k];
    for (int r = tid; r < m; r += 1024) R[(long long)r * n + k] /= lk;
    __syncthreads();
    const int w = n - k - 1;
    for (int idx = tid; idx < m * w; idx += 1024) {
      const int r = idx / w, i = k + 1 + (idx - r * w);
      R[(long long)r * n + i] -= N[(long long)i * n + k] * R[(long long)r * n + k];
    }
    __syncthreads();
  }
  // L^T x = y
  for (int k = n - 1; k >= 0; --k) {
    const double lk = N[(long long)k * n + k];
    for (int r = tid; r < m; r += 1024) R[(long long)r * n + k] /= lk;
    __syncthreads();
    for (int idx = tid; idx < m * k; idx += 1024) {
      const int r = idx / k, i = idx - r * k;
      R[(long long)r * n + i] -= N[(long long)k * n + i] * R[(long long)r * n + k];
    }
    __syncthreads();
  }
}

__global__ void axpby2_kernel(double* y, const double* x, size_t n, double a, double b) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

void axpby2(Context& c, double* y, const double* x, size_t n, double a, double b) {
  hipLaunchKernelGGL(axpby2_kernel, dim3(nblk(n)), dim3(256), 0, c.stream, y, x, n, a, b);
  CTM_HIP(hipGetLastError());
}

void mm(Context& c, int M, int N, int K, const double* A, long long lda, bool ta, const double* B,
        long long ldb, bool tb, double* C, long long ldc, double beta = 0.0, double alpha = 1.0) {
  gemm_f64(c, M, N, K, alpha, ta ? colmajor(A, lda) : rowmajor(A, lda),
           tb ? colmajor(B, ldb) : rowmajor(B, ldb), beta, out_rowmajor(C, ldc));
}

}  // namespace

FullUpdate::FullUpdate(Context& c, int D_, int gamma_) : ctx(c), D(D_), gamma(gamma_) {
  CTM_REQUIRE(D >= 1 && D <= 8, "full update: D must be 1..8");
  CTM_REQUIRE(gamma >= 0 && gamma <= 2, "gamma must be 0, 1 or 2");
  const size_t D3 = (size_t)D * D * D, D4 = D3 * D;
  const size_t sz = 4 * D3;
  for (DevBuf* x : {&A0, &B0, &Ap, &Bp, &Acur, &Bcur}) x->alloc(sz * sizeof(double));
  Ag.alloc(4 * sz * sizeof(double));
  Bg.alloc(4 * sz * sizeof(double));
  Hd.alloc(16 * sizeof(double));
  Gd.alloc(16 * sizeof(double));
  gs.alloc(16 * sizeof(double));
  X.alloc(16 * sizeof(double));
  Y.alloc(16 * sizeof(double));
  sv.alloc(4 * sizeof(double));
  E.alloc(D4 * D4 * sizeof(double));
  Es.alloc(D4 * D4 * sizeof(double));
  Kg.alloc(16 * D4 * sizeof(double));
  KE.alloc(16 * D4 * sizeof(double));
  KEt.alloc(16 * D4 * sizeof(double));
  dK.alloc(16 * D4 * sizeof(double));
  M.alloc(4 * D4 * D3 * sizeof(double));
  P.alloc(4 * D4 * D3 * sizeof(double));
  Nm.alloc(D3 * D3 * sizeof(double));
  rhs.alloc(4 * D3 * sizeof(double));
  Kraw.alloc(16 * D4 * sizeof(double));
  scal.alloc(8 * sizeof(double));
  flag.alloc(2 * sizeof(int));
}

void FullUpdate::fused(const double* in, double* out, bool back) {
  const int al = (gamma + 1) % 3, be = (gamma + 2) % 3;
  const int perm5[5] = {0, 1, 2 + al, 2 + be, 2 + gamma};
  const long long dims[5] = {2, 2, D, D, D};
  if (!back) {
    permute(ctx, in, out, 5, dims, perm5);
  } else {
    int inv[5];
    for (int a = 0; a < 5; ++a) inv[perm5[a]] = a;
    permute(ctx, in, out, 5, dims, inv);
  }
}

void FullUpdate::composite(const double* Afused, const double* Bfused, double* K) {
  const int m4 = 4 * D * D;
  mm(ctx, m4, m4, D, Afused, D, false, Bfused, D, true, Kraw.d(), m4);
  const long long kd[8] = {2, 2, D, D, 2, 2, D, D};
  const int kperm[8] = {0, 1, 4, 5, 3, 2, 7, 6};  // -> [s,a,t,c,u,l,d,r]
  permute(ctx, Kraw.d(), K, 8, kd, kperm);
}

double FullUpdate::error(const double* Afused, const double* Bfused) {
  const int D4 = D * D * D * D;
  composite(Afused, Bfused, dK.d());
  axpby2(ctx, dK.d(), Kg.d(), 16ull * D4, -1.0, 1.0);  // K'' - K'
  mm(ctx, 16, D4, D4, dK.d(), D4, false, Es.d(), D4, false, P.d(), D4);
  dot(ctx, dK.d(), P.d(), 16ull * D4, scal.d() + 1);
  double v = 0.0;
  CTM_HIP(hipMemcpyAsync(&v, scal.d() + 1, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  return v / normK;
}

// Least-squares update of one tensor: side 0 solves for A'' from B''
// (Bcur), side 1 for B'' from A'' (Acur).
void FullUpdate::solve(int side) {
  const int D3 = D * D * D, D4 = D3 * D;
  const double* T = side == 0 ? Bcur.d() : Acur.d();
  const long long tot = 4LL * D4 * D3;
  hipLaunchKernelGGL(selection_kernel, dim3(nblk((size_t)tot)), dim3(256), 0, ctx.stream, T, M.d(),
                     D, side);
  CTM_HIP(hipGetLastError());
  // P_q = E M_q (batch of 4), N = M^T P, b = (K'E)-rows M
  gemm_f64(ctx, D4, D3, D4, 1.0, rowmajor(Es.d(), D4, 0), rowmajor(M.d(), D3, (long long)D4 * D3),
           0.0, out_rowmajor(P.d(), D3, (long long)D4 * D3), 4);
  mm(ctx, D3, D3, 4 * D4, M.d(), D3, true, P.d(), D3, false, Nm.d(), D3);
  mm(ctx, 4, D3, 4 * D4, side == 0 ? KE.d() : KEt.d(), 4 * D4, false, M.d(), D3, false, rhs.d(),
     D3);
  hipLaunchKernelGGL(chol_solve_kernel, dim3(1), dim3(1024), 0, ctx.stream, Nm.d(), D3, rhs.d(), 4,
                     1e-12, (int*)flag.p);
  CTM_HIP(hipGetLastError());
  copy_dev(ctx, side == 0 ? Acur.d() : Bcur.d(), rhs.d(), 4ull * D3);
}

void FullUpdate::run(const double* A, const double* B, const double* H, double tau, int chi,
                     const EnvOptions& opt, int sweeps, int als_iters, double* A_out,
                     double* B_out, double* errors) {
  CTM_REQUIRE(chi >= 1 && sweeps >= 0 && als_iters >= 0, "full update: bad chi, sweeps or rounds");
  const int D3 = D * D * D, D4 = D3 * D;
  const size_t sz = 4ull * D3;
  CTM_HIP(hipMemcpyAsync(A0.p, A, sz * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  CTM_HIP(hipMemcpyAsync(B0.p, B, sz * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  CTM_HIP(hipMemcpyAsync(Hd.p, H, 16 * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  fill_zero_int(ctx, (int*)flag.p, 2);
  // 1-3: gate, split, gated tensors
  hipLaunchKernelGGL(gate_exp_kernel, dim3(1), dim3(64), 0, ctx.stream, Hd.d(), tau, Gd.d());
  hipLaunchKernelGGL(regroup_gate_kernel, dim3(1), dim3(64), 0, ctx.stream, Gd.d(), gs.d());
  CTM_HIP(hipGetLastError());
  jacobi_svd(ctx, gs.d(), 4, X.d(), sv.d(), Y.d(), (int*)flag.p + 1);
  const long long tg = 16LL * D3;
  hipLaunchKernelGGL(apply_gate_kernel, dim3(nblk((size_t)tg)), dim3(256), 0, ctx.stream, A0.d(),
                     Ag.d(), D, gamma, X.d(), sv.d());
  hipLaunchKernelGGL(apply_gate_kernel, dim3(nblk((size_t)tg)), dim3(256), 0, ctx.stream, B0.d(),
                     Bg.d(), D, gamma, Y.d(), sv.d());
  CTM_HIP(hipGetLastError());
  // 4: environment of the gated composite
  {
    Env env(ctx, D * D, chi, opt);
    env.build_purification_dev(Ag.d(), Bg.d(), D, 4 * D, gamma);
    env.init_boundary();
    int done = 0;
    double delta = 0.0;
    env.sweep(sweeps, 0.0, &done, &delta);
    env.ring_ket_bra_dev(E.d());
    copy_dev(ctx, Kg.d(), env.composite_dev(), 16ull * D4);
    CTM_HIP(hipStreamSynchronize(ctx.stream));
  }
  // symmetrised metric, K' E, and its (t c)-major copy for the B'' solves
  const long long ee[2] = {D4, D4};
  const int p10[2] = {1, 0};
  permute(ctx, E.d(), Es.d(), 2, ee, p10);
  axpby2(ctx, Es.d(), E.d(), (size_t)D4 * D4, 0.5, 0.5);
  mm(ctx, 16, D4, D4, Kg.d(), D4, false, Es.d(), D4, false, KE.d(), D4);
  const long long k3[3] = {4, 4, D4};
  const int p102[3] = {1, 0, 2};
  permute(ctx, KE.d(), KEt.d(), 3, k3, p102);
  dot(ctx, Kg.d(), KE.d(), 16ull * D4, scal.d());
  CTM_HIP(hipMemcpyAsync(&normK, scal.d(), sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  CTM_REQUIRE(normK > 0.0 && std::isfinite(normK), "full update: <K', E K'> is not positive");
  // 5: alternating least squares from the old tensors
  fused(A0.d(), Acur.d(), false);
  fused(B0.d(), Bcur.d(), false);
  if (errors) errors[0] = error(Acur.d(), Bcur.d());
  for (int it = 0; it < als_iters; ++it) {
    solve(0);
    solve(1);
    if (errors) errors[it + 1] = error(Acur.d(), Bcur.d());
  }
  int hf[2];
  CTM_HIP(hipMemcpyAsync(hf, flag.p, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  if (hf[1]) throw Error(-4, "full update: gate SVD failed");
  if (hf[0]) throw Error(-4, "full update: a normal matrix is not positive definite");
  fused(Acur.d(), Ap.d(), true);
  fused(Bcur.d(), Bp.d(), true);
  CTM_HIP(hipMemcpyAsync(A_out, Ap.p, sz * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipMemcpyAsync(B_out, Bp.p, sz * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
}

}  // namespace ctm
