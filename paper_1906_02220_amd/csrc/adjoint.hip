// Reverse-mode derivative of the CTMRG environment on the rhombic lattice
// (the contraction of Sec. III, Fig. 4 of arXiv:1906.02220, differentiated
// through a fixed number of sweeps).
//
// The forward pass is the engine's own: fixed sweeps of Env::move, with the
// state checkpointed every few sweeps.  Going backwards segment by segment,
// a segment is re-run from its checkpoint (bit-identically: the checkpoint
// holds the warm starts and generator counters of the projector SVD too)
// while every move writes a tape record: the environment before the move, the
// kept singular triplets of the cut matrix and the three normalisation
// factors.  The moves of the segment are then differentiated in reverse:
//
//  * the enlarged corners, halves and cut matrix are recomputed from the
//    recorded environment (FP64 GEMMs);
//  * every product, permutation and absorption step has its plain adjoint;
//  * a max-abs normalisation multiplies the adjoint by the recorded factor:
//    the loss is invariant under a rescaling of any single environment
//    tensor, so the factor acts as a constant;
//  * the truncated SVD Mt = U S V^T (top chi) has the adjoint
//      Mt_bar = U (J S + S K + diag(s_bar)) V^T
//             + X S V^T + U X^T Mt + U S Y^T + Mt Y V^T,
//    F_ij = 1 / (s_j^2 - s_i^2) (Lorentzian-broadened at relative width
//    1e-12), J = F o (U^T U_bar - U_bar^T U), K = F o (V^T V_bar - V_bar^T V),
//    and the columns x_i, y_i solve the shifted systems
//      (s_i^2 - P' Mt Mt^T P') x_i = P' u_bar_i,  P' = 1 - U U^T,
//      (s_i^2 - Q' Mt^T Mt Q') y_i = Q' v_bar_i,  Q' = 1 - V V^T
//    on the complement of the kept subspace, where they are positive
//    definite when s_chi > s_{chi+1}.  They are solved by conjugate gradients,
//    all columns of both systems at once, projecting every iterate again.
//    Without these terms the adjoint of a truncated SVD of a full-rank matrix
//    is wrong.
//
// The loss is w_k ln kappa + w_o <O>, kappa = Z_site Z_0 / (Z_row Z_col) and
// <O> from the ring E as in the engine; their adjoints seed the environment
// adjoint, and the site-tensor adjoint is carried back through the rotated
// copies, the double layer and the composite to A and B.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "adjoint.hpp"

namespace ctm {

namespace {

inline int nblk(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

__device__ inline double bsum(double v, double* sh) {
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

// dst = src * (*f)
__global__ void scale_copy_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                  size_t n, const double* __restrict__ f) {
  const double a = *f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = a * src[i];
}

// y = a x + b y (x may alias y)
__global__ void axpby_kernel(double* y, const double* x, size_t n, double a, double b) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// Y[i][j] = (acc ? Y[i][j] : 0) + X[i][j] * s_j^p, p = 1 or 2
__global__ void col_scale_kernel(double* __restrict__ Y, long long ldy,
                                 const double* __restrict__ X, long long ldx, int rows, int cols,
                                 const double* __restrict__ s, int p, int acc) {
  const long long total = (long long)rows * cols;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long i = idx / cols;
    const int j = (int)(idx - i * cols);
    const double f = p == 2 ? s[j] * s[j] : s[j];
    const double v = X[i * ldx + j] * f;
    double* y = Y + i * ldy + j;
    *y = acc ? *y + v : v;
  }
}

// out[j] = (acc ? out[j] : 0) + sum_i X[i][j] Y[i][j]; one block per column
__global__ __launch_bounds__(256) void coldot_kernel(const double* __restrict__ X,
                                                     const double* __restrict__ Y, int rows,
                                                     int cols, double* out, int acc) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  double v = 0.0;
  for (int i = threadIdx.x; i < rows; i += 256) v += X[(long long)i * cols + j] * Y[(long long)i * cols + j];
  v = bsum(v, sh);
  if (threadIdx.x == 0) out[j] = acc ? out[j] + v : v;
}

// The chi x chi core of the SVD adjoint: Z = J S + S K + diag(s_bar), with
// s_bar_i = -w_bar_i w_i^3 / 2 from w = s^-1/2 (zero where the cutoff made
// w_i = 0).
__global__ void svd_core_kernel(const double* __restrict__ Gu, const double* __restrict__ Gv,
                                const double* __restrict__ s, const double* __restrict__ w,
                                const double* __restrict__ wbar, int chi, double eps_b,
                                double* __restrict__ Z, double* __restrict__ sbar) {
  for (int idx = threadIdx.x; idx < chi * chi; idx += blockDim.x) {
    const int i = idx / chi, j = idx - (idx / chi) * chi;
    const double si = s[i], sj = s[j];
    double z;
    if (i != j) {
      const double del = sj * sj - si * si;
      const double br = eps_b * fmax(si * si, sj * sj);
      const double den = del * del + br * br;
      const double F = den > 0.0 ? del / den : 0.0;
      z = F * ((Gu[i * chi + j] - Gu[j * chi + i]) * sj + si * (Gv[i * chi + j] - Gv[j * chi + i]));
    } else {
      const double wi = w[i];
      z = wi > 0.0 ? -0.5 * wbar[i] * wi * wi * wi : 0.0;
      sbar[i] = z;
    }
    Z[idx] = z;
  }
}

struct CgArgs {
  double* X[2];
  double* R[2];
  double* P[2];
  const double* AP[2];
  double* Xb[2];
  double* rr;
  double* bn;
  double* best;
  int* stall;
  int* active;
  int* count;
  int n, chi;
  double tol;
};

// Column j of system sys (block sys * chi + j): X = 0, Xb = 0, norms of the
// right-hand side already in R.
__global__ __launch_bounds__(256) void cg_init_kernel(CgArgs a) {
  __shared__ double sh[256];
  const int c = blockIdx.x, sys = c / a.chi, j = c - sys * a.chi;
  double v = 0.0;
  for (int i = threadIdx.x; i < a.n; i += 256) {
    const long long o = (long long)i * a.chi + j;
    const double r = a.R[sys][o];
    v += r * r;
    a.X[sys][o] = 0.0;
    a.Xb[sys][o] = 0.0;
  }
  v = bsum(v, sh);
  if (threadIdx.x == 0) {
    a.rr[c] = v;
    a.bn[c] = sqrt(v);
    a.best[c] = v;
    a.stall[c] = 0;
    a.active[c] = v > 0.0 ? 1 : 0;
  }
}

// One conjugate-gradient step of every active column (AP = A P given).  The
// iterate with the smallest recursive residual is kept in Xb; a column stops
// when its residual is below tol times its right-hand side, when the step
// length vanishes, or when the residual has not improved for 5 steps (the
// rounding floor).
__global__ __launch_bounds__(256) void cg_step_kernel(CgArgs a) {
  __shared__ double sh[256];
  const int c = blockIdx.x, sys = c / a.chi, j = c - sys * a.chi;
  if (!a.active[c]) return;
  double* X = a.X[sys];
  double* R = a.R[sys];
  double* P = a.P[sys];
  const double* AP = a.AP[sys];
  double v = 0.0;
  for (int i = threadIdx.x; i < a.n; i += 256) {
    const long long o = (long long)i * a.chi + j;
    v += P[o] * AP[o];
  }
  const double pap = bsum(v, sh);
  const double rr = a.rr[c];
  const double alpha = pap > 0.0 ? rr / pap : 0.0;
  v = 0.0;
  for (int i = threadIdx.x; i < a.n; i += 256) {
    const long long o = (long long)i * a.chi + j;
    X[o] += alpha * P[o];
    const double r = R[o] - alpha * AP[o];
    R[o] = r;
    v += r * r;
  }
  const double rr2 = bsum(v, sh);
  const bool improved = rr2 < a.best[c];
  if (improved)
    for (int i = threadIdx.x; i < a.n; i += 256) {
      const long long o = (long long)i * a.chi + j;
      a.Xb[sys][o] = X[o];
    }
  const int st = improved ? 0 : a.stall[c] + 1;
  const bool go = alpha != 0.0 && sqrt(rr2) > a.tol * a.bn[c] && st < 5;
  if (go) {
    const double beta = rr2 / rr;
    for (int i = threadIdx.x; i < a.n; i += 256) {
      const long long o = (long long)i * a.chi + j;
      P[o] = R[o] + beta * P[o];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.rr[c] = rr2;
    if (improved) a.best[c] = rr2;
    a.stall[c] = st;
    a.active[c] = go ? 1 : 0;
    if (go) atomicAdd(a.count, 1);
  }
}

// C(M x N) = alpha op(A) op(B) + beta C with row-major operands; ta / tb
// select the transpose of an operand stored row-major as K x M / N x K.
void mm(Context& c, int M, int N, int K, const double* A, long long lda, bool ta, const double* B,
        long long ldb, bool tb, double* C, long long ldc, double beta = 0.0, double alpha = 1.0) {
  gemm_f64(c, M, N, K, alpha, ta ? colmajor(A, lda) : rowmajor(A, lda),
           tb ? colmajor(B, ldb) : rowmajor(B, ldb), beta, out_rowmajor(C, ldc));
}

void axpby(Context& c, double* y, const double* x, size_t n, double a, double b) {
  if (!n) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(nblk(n)), dim3(256), 0, c.stream, y, x, n, a, b);
  CTM_HIP(hipGetLastError());
}

void col_scale(Context& c, double* Y, long long ldy, const double* X, long long ldx, int rows,
               int cols, const double* s, int p, bool acc) {
  hipLaunchKernelGGL(col_scale_kernel, dim3(nblk((size_t)rows * cols)), dim3(256), 0, c.stream, Y,
                     ldy, X, ldx, rows, cols, s, p, acc ? 1 : 0);
  CTM_HIP(hipGetLastError());
}

void col_scale(Context& c, double* Y, const double* X, int rows, int cols, const double* s, int p,
               bool acc) {
  col_scale(c, Y, cols, X, cols, rows, cols, s, p, acc);
}

void coldot(Context& c, const double* X, const double* Y, int rows, int cols, double* out,
            bool acc) {
  hipLaunchKernelGGL(coldot_kernel, dim3(cols), dim3(256), 0, c.stream, X, Y, rows, cols, out,
                     acc ? 1 : 0);
  CTM_HIP(hipGetLastError());
}

void scale_copy(Context& c, double* dst, const double* src, size_t n, const double* f) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3(nblk(n)), dim3(256), 0, c.stream, dst, src, n, f);
  CTM_HIP(hipGetLastError());
}

// Z_z <- (1 - B_z B_z^T) Z_z for two n x chi blocks Z_z and orthonormal
// n x chi B_z, z = 0, 1, each pair stored nc = n chi apart.
void project_out2(Context& c, const double* B, double* Z, int n, int chi, double* tmp) {
  const long long nc = (long long)n * chi, cc = (long long)chi * chi;
  gemm_f64(c, chi, chi, n, 1.0, colmajor(B, chi, nc), rowmajor(Z, chi, nc), 0.0,
           out_rowmajor(tmp, chi, cc), 2);
  gemm_f64(c, n, chi, chi, -1.0, rowmajor(B, chi, nc), rowmajor(tmp, chi, cc), 1.0,
           out_rowmajor(Z, chi, nc), 2);
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

Grad::Grad(Env& env, int sweeps_, int ckpt_every)
    : e(env), ctx(env.ctx), sweeps(sweeps_), chi(env.chi), d(env.d), n(env.n),
      tl(env.chi, env.d) {
  CTM_REQUIRE(sweeps >= 0, "sweeps must be >= 0");
  CTM_REQUIRE(e.opt.precision == 0, "gradients need precision mode CTM_PREC_F64");
  CTM_REQUIRE(e.b >= chi, "gradients need a projector subspace of at least chi columns");
  every = (ckpt_every <= 0 || ckpt_every > sweeps) ? std::max(sweeps, 1) : ckpt_every;
  nseg = sweeps == 0 ? 0 : (sweeps + every - 1) / every;
  const size_t dd4 = (size_t)d * d * d * d;
  const size_t big = std::max((size_t)n * n, dd4);
  const size_t nc = (size_t)n * chi, cc = (size_t)chi * chi, ct = (size_t)chi * d * chi;
  tape.alloc((size_t)every * 4 * tl.total * sizeof(double));
  stats.tape_bytes = (double)tape.bytes;
  Cb.alloc(4 * cc * sizeof(double));
  Tb.alloc(4 * ct * sizeof(double));
  for (auto& x : arb) x.alloc(dd4 * sizeof(double));
  abar.alloc(dd4 * sizeof(double));
  for (DevBuf* x : {&Qbar, &wA, &wB}) x->alloc(big * sizeof(double));
  Mt3.alloc(3ull * n * n * sizeof(double));
  for (DevBuf* x : {&PuU, &PlU, &Pub, &Plb, &UAw, &VAw, &UAb, &VAb, &x1e, &G1T, &G2, &pb, &sm1b, &X1b})
    x->alloc(nc * sizeof(double));
  for (DevBuf* x : {&LU, &RU, &LL, &RL, &Wf}) x->alloc(2 * nc * sizeof(double));
  for (DevBuf* x : {&cgX, &cgR, &cgP, &cgAP, &cgXb, &cgT}) x->alloc(2 * nc * sizeof(double));
  for (DevBuf* x : {&ckb, &cq3b, &Gu, &Gv, &Zm, &tmpB}) x->alloc(cc * sizeof(double));
  tmpA.alloc(2 * cc * sizeof(double));
  for (int f = 0; f < 4; ++f) {
    arotT[f].alloc(dd4 * sizeof(double));
    const long long dd2[2] = {(long long)d * d, (long long)d * d};
    const int p10[2] = {1, 0};
    permute(ctx, e.arot[f].d(), arotT[f].d(), 2, dd2, p10);
  }
  tq3b.alloc(ct * sizeof(double));
  sm2b.alloc(ct * sizeof(double));
  wbar.alloc(chi * sizeof(double));
  sbar.alloc(chi * sizeof(double));
  for (DevBuf* x : {&rr, &bn, &best}) x->alloc(2 * chi * sizeof(double));
  stall.alloc(2 * chi * sizeof(int));
  active.alloc(2 * chi * sizeof(int));
  count.alloc(sizeof(int));
  CTM_HIP(hipHostMalloc((void**)&hcount, sizeof(int), hipHostMallocDefault));
  fill_zero(ctx, Cb.d(), 4 * cc);
  fill_zero(ctx, Tb.d(), 4 * ct);
  for (auto& x : arb) fill_zero(ctx, x.d(), dd4);
  fill_zero(ctx, abar.d(), dd4);
  if (e.D > 0) {
    const size_t D4 = (size_t)e.D * e.D * e.D * e.D;
    Kcb.alloc(16 * D4 * sizeof(double));
    fill_zero(ctx, Kcb.d(), 16 * D4);
  }
  ck.resize(nseg);
}

void Grad::save(Ckpt& c) {
  const size_t nb = (size_t)n * e.b;
  if (!c.C.p) {
    c.C.alloc(e.Call.bytes);
    c.T.alloc(e.Tall.bytes);
    c.logs.alloc(8 * sizeof(double));
    c.warm.alloc(4 * nb * sizeof(double));
    c.rng.alloc(2 * sizeof(double));
    stats.checkpoint_bytes += (double)(c.C.bytes + c.T.bytes + c.logs.bytes + c.warm.bytes + c.rng.bytes);
  }
  copy_dev(ctx, c.C.d(), e.Call.d(), 4ull * chi * chi);
  copy_dev(ctx, c.T.d(), e.Tall.d(), 4ull * chi * d * chi);
  copy_dev(ctx, c.logs.d(), e.logs.d(), 8);
  for (int k = 0; k < 4; ++k) copy_dev(ctx, c.warm.d() + k * nb, e.warm[k].d(), nb);
  copy_dev(ctx, c.rng.d(), (const double*)e.rngc.p, 2);  // bit copy of two counters
  for (int k = 0; k < 4; ++k) {
    c.warm_ok[k] = e.warm_ok[k];
    c.warm_moves[k] = e.warm_moves[k];
  }
  c.rng_slot = e.rng_slot;
  c.rng_ctr = e.rng_ctr;
}

void Grad::restore(const Ckpt& c) {
  const size_t nb = (size_t)n * e.b;
  copy_dev(ctx, e.Call.d(), c.C.d(), 4ull * chi * chi);
  copy_dev(ctx, e.Tall.d(), c.T.d(), 4ull * chi * d * chi);
  copy_dev(ctx, e.logs.d(), c.logs.d(), 8);
  for (int k = 0; k < 4; ++k) copy_dev(ctx, e.warm[k].d(), c.warm.d() + k * nb, nb);
  copy_dev(ctx, (double*)e.rngc.p, c.rng.d(), 2);
  for (int k = 0; k < 4; ++k) {
    e.warm_ok[k] = c.warm_ok[k];
    e.warm_moves[k] = c.warm_moves[k];
    e.qvalid[k] = false;
  }
  e.rng_slot = c.rng_slot;
  e.rng_ctr = c.rng_ctr;
  e.e_valid = false;
}

void Grad::run_segment(int sg, bool record) {
  const int s0 = sg * every, s1 = std::min(sweeps, s0 + every);
  int m = 0;
  for (int s = s0; s < s1; ++s) {
    for (int i = 0; i < 4; ++i) {
      e.tape_slot = record ? tape.d() + (size_t)m * tl.total : nullptr;
      e.move(e.opt.move_order[i]);
      ++m;
    }
    e.tape_slot = nullptr;
    e.check_flags("ctm_grad");
  }
}

void Grad::forward() {
  const double t0 = now_ms();
  e.drop_graph();
  for (int sg = 0; sg < nseg; ++sg) {
    save(ck[sg]);
    run_segment(sg, sg == nseg - 1);
  }
  e.sweeps_done += sweeps;
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  stats.ms_forward = now_ms() - t0;
  stats.moves = 4 * sweeps;
}

double Grad::seed(double wk, double wo, const double* op, int op_dim, const double* a_imp,
                  double* log_kappa, double* expect) {
  const int dc = d * chi;
  const long long d2 = (long long)d * d, c2 = (long long)chi * chi;
  const size_t d4 = (size_t)d * d * d * d;
  const double* C[4] = {e.Cp(0), e.Cp(1), e.Cp(2), e.Cp(3)};
  const double* T[4] = {e.Tp(0), e.Tp(1), e.Tp(2), e.Tp(3)};
  double* Cbar[4];
  double* Tbar[4];
  for (int i = 0; i < 4; ++i) {
    Cbar[i] = Cb.d() + (size_t)i * chi * chi;
    Tbar[i] = Tb.d() + (size_t)i * chi * d * chi;
  }
  const double* a = e.arot[0].d();
  // ring (as Env::ring), keeping the halves
  double* u1 = PuU.d();   // C1 T1        [a][u,g]
  double* u2 = PlU.d();   // (C1 T1) C2   [a,u][e]
  double* l1 = Pub.d();   // C3 T3        [h][x,c]
  double* l2 = Plb.d();   // (C3 T3) C4   [h,x][d']
  DevBuf sUh((size_t)d2 * c2 * sizeof(double)), sLh((size_t)d2 * c2 * sizeof(double)),
      sE(d4 * sizeof(double));
  double* Uh = sUh.d();  // [u,r][a,h]
  double* Lh = sLh.d();  // [a,h][x,l]
  double* E = sE.d();    // [u,l,x,r]
  const long long d4c[4] = {chi, d, d, chi};
  mm(ctx, chi, dc, chi, C[0], chi, false, T[0], dc, false, u1, dc);
  mm(ctx, dc, chi, chi, u1, chi, false, C[1], chi, false, u2, chi);
  mm(ctx, dc, dc, chi, u2, chi, false, T[1], dc, false, wA.d(), dc);
  const int p1203[4] = {1, 2, 0, 3};
  permute(ctx, wA.d(), Uh, 4, d4c, p1203);
  mm(ctx, chi, dc, chi, C[2], chi, false, T[2], dc, false, l1, dc);
  mm(ctx, dc, chi, chi, l1, chi, false, C[3], chi, false, l2, chi);
  mm(ctx, dc, dc, chi, l2, chi, false, T[3], dc, false, wA.d(), dc);
  const int p3012[4] = {3, 0, 1, 2};
  permute(ctx, wA.d(), Lh, 4, d4c, p3012);
  mm(ctx, d2, d2, c2, Uh, c2, false, Lh, d2, false, wA.d(), d2);
  const long long f4[4] = {d, d, d, d};
  const int p0321[4] = {0, 3, 2, 1};
  permute(ctx, wA.d(), E, 4, f4, p0321);
  // closed rings: Z_row over R1 = u2, R2 = l2; Z_col over V1 = (C1 C2) T2, V2 = (C3 C4) T4
  double* P01 = Gu.d();
  double* P23 = Gv.d();
  double* V1 = UAw.d();
  double* V2 = VAw.d();
  mm(ctx, chi, chi, chi, C[0], chi, false, C[1], chi, false, P01, chi);
  mm(ctx, chi, chi, chi, C[2], chi, false, C[3], chi, false, P23, chi);
  mm(ctx, chi, dc, chi, P01, chi, false, T[1], dc, false, V1, dc);
  mm(ctx, chi, dc, chi, P23, chi, false, T[3], dc, false, V2, dc);
  const long long g3[3] = {chi, d, chi};
  const int p210[3] = {2, 1, 0};
  const long long g2[2] = {chi, chi};
  const int p10[2] = {1, 0};
  double* sc = e.scal.d() + 16;
  dot(ctx, E, a, d4, sc + 0);                          // Z_site
  permute(ctx, P23, tmpA.d(), 2, g2, p10);
  dot(ctx, P01, tmpA.d(), (size_t)chi * chi, sc + 1);  // Z_0
  permute(ctx, l2, UAb.d(), 3, g3, p210);
  dot(ctx, u2, UAb.d(), (size_t)dc * chi, sc + 2);     // Z_row
  permute(ctx, V2, VAb.d(), 3, g3, p210);
  dot(ctx, V1, VAb.d(), (size_t)dc * chi, sc + 3);     // Z_col
  double z[4];
  CTM_HIP(hipMemcpyAsync(z, sc, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  const double zs = z[0], z0 = z[1], zr = z[2], zc = z[3];
  const double kap = zs * z0 / (zr * zc);
  CTM_REQUIRE(std::isfinite(kap) && kap > 0.0, "ctm_grad: kappa is not positive and finite");
  const double lk = std::log(kap);
  double ex = 0.0;
  // E_bar accumulates in Qbar
  double* Eb = Qbar.d();
  fill_zero(ctx, Eb, d4);
  if (wk != 0.0) {
    axpby(ctx, Eb, a, d4, wk / zs, 1.0);
    axpby(ctx, abar.d(), E, d4, wk / zs, 1.0);
    const double a0 = wk / z0;
    mm(ctx, chi, chi, chi, P23, chi, true, C[1], chi, true, Cbar[0], chi, 1.0, a0);
    mm(ctx, chi, chi, chi, C[0], chi, true, P23, chi, true, Cbar[1], chi, 1.0, a0);
    mm(ctx, chi, chi, chi, P01, chi, true, C[3], chi, true, Cbar[2], chi, 1.0, a0);
    mm(ctx, chi, chi, chi, C[2], chi, true, P01, chi, true, Cbar[3], chi, 1.0, a0);
    // Z_row: R1_bar = ar R2^(210), R2_bar = ar R1^(210)
    const double ar = -wk / zr;
    double* R1b = UAb.d();  // holds l2 permuted
    double* R2b = VAb.d();
    permute(ctx, u2, R2b, 3, g3, p210);
    axpby(ctx, R1b, R1b, (size_t)dc * chi, 0.0, ar);  // R1b *= ar
    axpby(ctx, R2b, R2b, (size_t)dc * chi, 0.0, ar);
    for (int h = 0; h < 2; ++h) {
      const double* Rb = h ? R2b : R1b;
      const double* S = h ? l1 : u1;   // C T
      const double* Ca = C[2 * h];
      const double* Cn = C[2 * h + 1];
      const double* Ta = T[2 * h];
      mm(ctx, chi, chi, dc, S, chi, true, Rb, chi, false, Cbar[2 * h + 1], chi, 1.0);
      mm(ctx, dc, chi, chi, Rb, chi, false, Cn, chi, true, pb.d(), chi);  // S_bar
      mm(ctx, chi, chi, dc, pb.d(), dc, false, Ta, dc, true, Cbar[2 * h], chi, 1.0);
      mm(ctx, chi, dc, chi, Ca, chi, true, pb.d(), dc, false, Tbar[2 * h], dc, 1.0);
    }
    // Z_col: V1_bar = ac V2^(210), V2_bar = ac V1^(210)
    const double ac = -wk / zc;
    double* V1b = G1T.d();
    double* V2b = G2.d();
    permute(ctx, V2, V1b, 3, g3, p210);
    permute(ctx, V1, V2b, 3, g3, p210);
    axpby(ctx, V1b, V1b, (size_t)dc * chi, 0.0, ac);
    axpby(ctx, V2b, V2b, (size_t)dc * chi, 0.0, ac);
    for (int h = 0; h < 2; ++h) {
      const double* Vb = h ? V2b : V1b;
      const double* Pp = h ? P23 : P01;
      const double* Ca = C[2 * h];
      const double* Cn = C[2 * h + 1];
      const double* Tn = T[2 * h + 1];
      mm(ctx, chi, chi, dc, Vb, dc, false, Tn, dc, true, tmpB.d(), chi);  // P_bar
      mm(ctx, chi, dc, chi, Pp, chi, true, Vb, dc, false, Tbar[2 * h + 1], dc, 1.0);
      mm(ctx, chi, chi, chi, tmpB.d(), chi, false, Cn, chi, true, Cbar[2 * h], chi, 1.0);
      mm(ctx, chi, chi, chi, Ca, chi, true, tmpB.d(), chi, false, Cbar[2 * h + 1], chi, 1.0);
    }
  }
  if (e.D > 0 && op) {
    CTM_REQUIRE(op_dim == 4 || op_dim == 16, "op_dim must be 4 or 16");
    std::vector<double> O(256, 0.0);
    if (op_dim == 16) {
      std::memcpy(O.data(), op, 256 * sizeof(double));
    } else {
      for (int sA = 0; sA < 2; ++sA) for (int aA = 0; aA < 2; ++aA)
      for (int sB = 0; sB < 2; ++sB) for (int aB = 0; aB < 2; ++aB)
      for (int tA = 0; tA < 2; ++tA) for (int tB = 0; tB < 2; ++tB) {
        const int p = ((sA * 2 + aA) * 2 + sB) * 2 + aB;
        const int q = ((tA * 2 + aA) * 2 + tB) * 2 + aB;
        O[p * 16 + q] = op[(sA * 2 + sB) * 4 + (tA * 2 + tB)];
      }
    }
    const int D = e.D;
    const int D4 = D * D * D * D;
    const long long dd[8] = {D, D, D, D, D, D, D, D};
    const int pp[8] = {0, 2, 4, 6, 1, 3, 5, 7};
    double* E8 = wB.d();
    permute(ctx, E, E8, 8, dd, pp);
    const double* Kc = e.Kc.d();
    DevBuf F((size_t)D4 * 16 * sizeof(double)), Fb((size_t)D4 * 16 * sizeof(double));
    DevBuf rhoT(256 * sizeof(double)), Rb(256 * sizeof(double));
    mm(ctx, D4, 16, D4, E8, D4, false, Kc, D4, true, F.d(), 16);
    mm(ctx, 16, 16, D4, F.d(), 16, true, Kc, D4, true, rhoT.d(), 16);
    std::vector<double> hr(256);
    CTM_HIP(hipMemcpyAsync(hr.data(), rhoT.p, 256 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    CTM_HIP(hipStreamSynchronize(ctx.stream));
    double num = 0.0, tr = 0.0;
    for (int i = 0; i < 256; ++i) num += O[i] * hr[i];
    for (int i = 0; i < 16; ++i) tr += hr[i * 17];
    CTM_REQUIRE(tr != 0.0, "ctm_grad: <E, a> vanishes");
    ex = num / tr;
    if (wo != 0.0) {
      std::vector<double> hb(256);
      for (int p = 0; p < 16; ++p)
        for (int q = 0; q < 16; ++q)
          hb[p * 16 + q] = wo * (O[p * 16 + q] - (p == q ? ex : 0.0)) / tr;
      CTM_HIP(hipMemcpyAsync(Rb.p, hb.data(), 256 * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
      // rhoT = F^T Kc^T, F = E8 Kc^T
      mm(ctx, D4, 16, 16, Kc, D4, true, Rb.d(), 16, true, Fb.d(), 16);
      mm(ctx, 16, D4, 16, Rb.d(), 16, true, F.d(), 16, true, Kcb.d(), D4, 1.0);
      mm(ctx, D4, D4, 16, Fb.d(), 16, false, Kc, D4, false, wA.d(), D4);  // E8_bar
      mm(ctx, 16, D4, D4, Fb.d(), 16, true, E8, D4, false, Kcb.d(), D4, 1.0);
      const int ip[8] = {0, 4, 1, 5, 2, 6, 3, 7};
      permute(ctx, wA.d(), wB.d(), 8, dd, ip);
      axpby(ctx, Eb, wB.d(), d4, 1.0, 1.0);
    }
    CTM_HIP(hipStreamSynchronize(ctx.stream));  // F, Fb, rhoT, Rb go out of scope
  } else if (a_imp) {
    DevBuf ai(d4 * sizeof(double));
    CTM_HIP(hipMemcpyAsync(ai.p, a_imp, d4 * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
    dot(ctx, E, ai.d(), d4, sc + 4);
    double zi = 0.0;
    CTM_HIP(hipMemcpyAsync(&zi, sc + 4, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    CTM_HIP(hipStreamSynchronize(ctx.stream));
    ex = zi / zs;
    if (wo != 0.0) {
      axpby(ctx, Eb, ai.d(), d4, wo / zs, 1.0);
      axpby(ctx, Eb, a, d4, -wo * ex / zs, 1.0);
      axpby(ctx, abar.d(), E, d4, -wo * ex / zs, 1.0);
    }
    CTM_HIP(hipStreamSynchronize(ctx.stream));
  } else {
    CTM_REQUIRE(wo == 0.0, "ctm_grad: w_expect needs an operator");
  }
  // ring adjoint: E_bar -> the eight environment tensors
  double* t2b = wA.d();
  permute(ctx, Eb, t2b, 4, f4, p0321);
  double* Uhb = wB.d();
  mm(ctx, d2, c2, d2, t2b, d2, false, Lh, d2, true, Uhb, c2);
  double* Lhb = Qbar.d();  // E_bar no longer needed
  mm(ctx, c2, d2, d2, Uh, c2, true, t2b, d2, false, Lhb, d2);
  const long long e4[4] = {d, d, chi, chi};
  const int i1203[4] = {2, 0, 1, 3};
  permute(ctx, Uhb, wA.d(), 4, e4, i1203);  // u3_bar [a,u][r,h]
  const long long h4[4] = {chi, chi, d, d};
  const int i3012[4] = {1, 2, 3, 0};
  permute(ctx, Lhb, wB.d(), 4, h4, i3012);  // l3_bar [h,x][l,a]
  for (int h = 0; h < 2; ++h) {
    const double* x3b = h ? wB.d() : wA.d();
    const double* x1 = h ? l1 : u1;
    const double* x2 = h ? l2 : u2;
    const double* Ca = C[2 * h];
    const double* Cn = C[2 * h + 1];
    const double* Ta = T[2 * h];
    const double* Tn = T[2 * h + 1];
    mm(ctx, chi, dc, dc, x2, chi, true, x3b, dc, false, Tbar[2 * h + 1], dc, 1.0);
    mm(ctx, dc, chi, dc, x3b, dc, false, Tn, dc, true, pb.d(), chi);  // x2_bar
    mm(ctx, chi, chi, dc, x1, chi, true, pb.d(), chi, false, Cbar[2 * h + 1], chi, 1.0);
    mm(ctx, dc, chi, chi, pb.d(), chi, false, Cn, chi, true, sm1b.d(), chi);  // x1_bar
    mm(ctx, chi, chi, dc, sm1b.d(), dc, false, Ta, dc, true, Cbar[2 * h], chi, 1.0);
    mm(ctx, chi, dc, chi, Ca, chi, true, sm1b.d(), dc, false, Tbar[2 * h], dc, 1.0);
  }
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  if (log_kappa) *log_kappa = lk;
  if (expect) *expect = ex;
  return wk * lk + wo * ex;
}

// Complement solves of the SVD adjoint, both systems at once (system 0 on
// the left vectors with Mt Mt^T, system 1 on the right vectors with
// Mt^T Mt; VA = UA + n chi in the tape): returns the number of iterations.
// Right-hand sides in UAb, VAb; solutions in cgXb (then cgXb + n chi).
int Grad::cg(const double* UA, const double* s) {
  const size_t nc = (size_t)n * chi, nn = (size_t)n * n;
  const double* MtT = Mt3.d();  // [Mt^T | Mt | Mt^T]
  double* R = cgR.d();
  copy_dev(ctx, R, UAb.d(), nc);
  copy_dev(ctx, R + nc, VAb.d(), nc);
  project_out2(ctx, UA, R, n, chi, tmpA.d());
  project_out2(ctx, UA, R, n, chi, tmpA.d());
  copy_dev(ctx, cgP.d(), R, 2 * nc);
  CgArgs a;
  for (int sy = 0; sy < 2; ++sy) {
    a.X[sy] = cgX.d() + sy * nc;
    a.R[sy] = cgR.d() + sy * nc;
    a.P[sy] = cgP.d() + sy * nc;
    a.AP[sy] = cgAP.d() + sy * nc;
    a.Xb[sy] = cgXb.d() + sy * nc;
  }
  a.rr = rr.d();
  a.bn = bn.d();
  a.best = best.d();
  a.stall = (int*)stall.p;
  a.active = (int*)active.p;
  a.count = (int*)count.p;
  a.n = n;
  a.chi = chi;
  a.tol = 1e-13;
  hipLaunchKernelGGL(cg_init_kernel, dim3(2 * chi), dim3(256), 0, ctx.stream, a);
  CTM_HIP(hipGetLastError());
  double* P = cgP.d();
  double* AP = cgAP.d();
  double* T1 = cgT.d();
  const int maxit = 300;
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    project_out2(ctx, UA, P, n, chi, tmpA.d());
    // AP = s^2 P - G P:  T1 = (Mt^T | Mt) P,  AP -= (Mt | Mt^T) T1
    gemm_f64(ctx, n, chi, n, 1.0, rowmajor(MtT, n, nn), rowmajor(P, chi, nc), 0.0,
             out_rowmajor(T1, chi, nc), 2);
    col_scale(ctx, AP, P, 2 * n, chi, s, 2, false);
    gemm_f64(ctx, n, chi, n, -1.0, rowmajor(MtT + nn, n, nn), rowmajor(T1, chi, nc), 1.0,
             out_rowmajor(AP, chi, nc), 2);
    project_out2(ctx, UA, AP, n, chi, tmpA.d());
    fill_zero_int(ctx, (int*)count.p, 1);
    hipLaunchKernelGGL(cg_step_kernel, dim3(2 * chi), dim3(256), 0, ctx.stream, a);
    CTM_HIP(hipGetLastError());
    if ((it & 3) == 0 || it == maxit) {
      CTM_HIP(hipMemcpyAsync(hcount, count.p, sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
      CTM_HIP(hipStreamSynchronize(ctx.stream));
      if (*hcount == 0) break;
    }
  }
  return std::min(it, maxit);
}

// Adjoint of the truncated SVD in factored form: from UAb, VAb, the
// singular values s and w = s^-1/2 (wbar holds the adjoint of w),
//   Mt_bar = UA G1 + G2 VA^T,  G1^T = Mt^T Xc + Yc S + VA Z^T,  G2 = Mt Yc + Xc S.
void Grad::svd_bwd(const double* UA, const double* VA, const double* s, const double* w) {
  const size_t nc = (size_t)n * chi, nn = (size_t)n * n;
  const double* MtT = Mt3.d();
  const double* Mt = Mt3.d() + nn;
  mm(ctx, chi, chi, n, UA, chi, true, UAb.d(), chi, false, Gu.d(), chi);
  mm(ctx, chi, chi, n, VA, chi, true, VAb.d(), chi, false, Gv.d(), chi);
  hipLaunchKernelGGL(svd_core_kernel, dim3(1), dim3(256), 0, ctx.stream, Gu.d(), Gv.d(), s, w,
                     wbar.d(), chi, 1e-12, Zm.d(), sbar.d());
  CTM_HIP(hipGetLastError());
  const int its = cg(UA, s);
  stats.cg_iters_max = std::max(stats.cg_iters_max, its);
  stats.cg_iters_total += its;
  const double* Xc = cgXb.d();
  const double* Yc = cgXb.d() + nc;
  mm(ctx, n, chi, n, MtT, n, false, Xc, chi, false, G1T.d(), chi);
  col_scale(ctx, G1T.d(), Yc, n, chi, s, 1, true);
  mm(ctx, n, chi, chi, VA, chi, false, Zm.d(), chi, true, G1T.d(), chi, 1.0);
  mm(ctx, n, chi, n, Mt, n, false, Yc, chi, false, G2.d(), chi);
  col_scale(ctx, G2.d(), Xc, n, chi, s, 1, true);
}

void Grad::move_bwd(int k, const double* rec) {
  const int dc = d * chi;
  const long long d2 = (long long)d * d, c2 = (long long)chi * chi;
  const size_t cc = (size_t)chi * chi, ct = (size_t)chi * d * chi, nc = (size_t)n * chi;
  const size_t nn = (size_t)n * n;
  const int q0 = k, q1 = (k + 1) & 3, q2 = (k + 2) & 3, q3 = (k + 3) & 3;
  const double* UA = rec + tl.ua;
  const double* VA = rec + tl.va;
  const double* s = rec + tl.s;
  const double* w = rec + tl.w;
  const double* inv = rec + tl.inv;
  double* Cbar[4];
  double* Tbar[4];
  for (int i = 0; i < 4; ++i) {
    Cbar[i] = Cb.d() + (size_t)i * cc;
    Tbar[i] = Tb.d() + (size_t)i * ct;
  }
  // the environment before the move
  copy_dev(ctx, e.Call.d(), rec + tl.c, 4 * cc);
  copy_dev(ctx, e.Tall.d(), rec + tl.t, 4 * ct);
  const double* C[4] = {e.Cp(0), e.Cp(1), e.Cp(2), e.Cp(3)};
  const double* T[4] = {e.Tp(0), e.Tp(1), e.Tp(2), e.Tp(3)};
  // adjoints of the three outputs before normalisation
  scale_copy(ctx, ckb.d(), Cbar[q0], cc, inv + 0);
  scale_copy(ctx, tq3b.d(), Tbar[q3], ct, inv + 1);
  scale_copy(ctx, cq3b.d(), Cbar[q3], cc, inv + 2);
  fill_zero(ctx, Cbar[q0], cc);
  fill_zero(ctx, Tbar[q3], ct);
  fill_zero(ctx, Cbar[q3], cc);
  // corners, halves, cut matrix (and its transpose, twice), projectors
  for (int f = 0; f < 4; ++f) e.corner(f);
  const double* Q[4] = {e.Qb[0].d(), e.Qb[1].d(), e.Qb[2].d(), e.Qb[3].d()};
  double* U = e.U.d();
  double* Lt = e.Lt.d();
  double* Mt = Mt3.d() + nn;
  mm(ctx, n, n, n, Q[q0], n, false, Q[q1], n, false, U, n);
  mm(ctx, n, n, n, Q[q2], n, false, Q[q3], n, false, Lt, n);
  mm(ctx, n, n, n, Lt, n, false, U, n, false, Mt, n);
  const long long nd[2] = {n, n};
  const int p10[2] = {1, 0};
  permute(ctx, Mt, Mt3.d(), 2, nd, p10);
  copy_dev(ctx, Mt3.d() + 2 * nn, Mt3.d(), nn);
  mm(ctx, n, chi, n, Lt, n, true, UA, chi, false, PuU.d(), chi);
  mm(ctx, n, chi, n, U, n, false, VA, chi, false, PlU.d(), chi);
  double* Pu = e.Pu.d();
  double* Pl = e.Pl.d();
  col_scale(ctx, Pu, PuU.d(), n, chi, w, 1, false);
  col_scale(ctx, Pl, PlU.d(), n, chi, w, 1, false);
  // T_{k+3}' = perm(Pu^T t2b), t2b = perm(perm(T_{k+3} Pl) a_k)
  const long long e3[3] = {chi, d, chi};
  const int p021[3] = {0, 2, 1};
  permute(ctx, tq3b.d(), sm2b.d(), 3, e3, p021);  // [k1][k2][r]
  const long long d4c[4] = {chi, d, d, chi};
  const int p0321[4] = {0, 3, 2, 1};
  const int p2103[4] = {2, 1, 0, 3};
  const long long e4[4] = {chi, chi, d, d};
  const long long e4b[4] = {chi, d, chi, d};
  const int p0213[4] = {0, 2, 1, 3};
  double* t2 = e.t2.d();
  double* t2T = e.t1.d();
  const double* ar = e.arot[q0].d();
  mm(ctx, dc, dc, chi, T[q3], chi, false, Pl, dc, false, wA.d(), dc);  // [de,l][u,k2]
  permute(ctx, wA.d(), t2, 4, d4c, p0321);                              // [de,k2][u,l]
  permute(ctx, wA.d(), t2T, 4, d4c, p2103);                             // [u,l][de,k2]
  mm(ctx, c2, d2, d2, t2, d2, false, ar, d2, false, wA.d(), d2);          // [de,k2][dd,r]
  permute(ctx, wA.d(), wB.d(), 4, e4, p0213);                           // [de,dd][k2,r]
  mm(ctx, n, chi, dc, wB.d(), dc, false, sm2b.d(), dc, true, Pub.d(), chi);
  mm(ctx, n, dc, chi, Pu, chi, false, sm2b.d(), dc, false, wA.d(), dc);   // t2b_bar
  permute(ctx, wA.d(), wB.d(), 4, e4b, p0213);                          // [de,k2][dd,r]
  mm(ctx, d2, d2, c2, t2T, c2, false, wB.d(), d2, false, Qbar.d(), d2);
  axpby(ctx, arb[q0].d(), Qbar.d(), (size_t)d2 * d2, 1.0, 1.0);
  mm(ctx, c2, d2, d2, wB.d(), d2, false, arotT[q0].d(), d2, false, wA.d(), d2);  // t2_bar
  permute(ctx, wA.d(), wB.d(), 4, e4, p0321);                           // t1_bar [de,l][u,k2]
  mm(ctx, dc, chi, dc, wB.d(), dc, false, Pl, dc, true, Tbar[q3], chi, 1.0);
  mm(ctx, chi, dc, dc, T[q3], chi, true, wB.d(), dc, false, Plb.d(), dc);
  // C_{k+3}' = sm1 Pl, sm1[io][de][dd] = sum_ka C_{k+3}[ka][de] T_{k+2}[io][dd][ka]
  double* sm1 = e.sm1.d();
  gemm_f64(ctx, chi, d, chi, 1.0, View{C[q3], 1, chi, 0}, View{T[q2], 1, chi, dc}, 0.0,
           ViewOut{sm1, d, 1, dc}, chi);
  mm(ctx, chi, n, chi, cq3b.d(), chi, false, Pl, chi, true, sm1b.d(), n);
  mm(ctx, n, chi, chi, sm1, n, true, cq3b.d(), chi, false, Plb.d(), chi, 1.0);
  const long long s3[3] = {chi, chi, d};
  permute(ctx, sm1b.d(), pb.d(), 3, s3, p021);  // [io][dd][de]
  mm(ctx, n, chi, chi, pb.d(), chi, false, C[q3], chi, true, Tbar[q2], chi, 1.0);
  mm(ctx, chi, chi, n, T[q2], chi, true, pb.d(), chi, false, Cbar[q3], chi, 1.0);
  // C_k' = Pu^T X1
  const double* X1 = e.X1[q0].d();
  mm(ctx, n, chi, chi, X1, chi, false, ckb.d(), chi, true, Pub.d(), chi, 1.0);
  mm(ctx, n, chi, chi, Pu, chi, false, ckb.d(), chi, false, x1e.d(), chi);
  // projectors Pu = Lt^T UA w, Pl = U VA w: adjoints of UA, VA and w
  mm(ctx, n, chi, n, Lt, n, false, Pub.d(), chi, false, UAb.d(), chi);
  scale_cols(ctx, UAb.d(), n, chi, chi, w);
  coldot(ctx, Pub.d(), PuU.d(), n, chi, wbar.d(), false);
  mm(ctx, n, chi, n, U, n, true, Plb.d(), chi, false, VAb.d(), chi);
  scale_cols(ctx, VAb.d(), n, chi, chi, w);
  coldot(ctx, Plb.d(), PlU.d(), n, chi, wbar.d(), true);
  // cut matrix: Mt_bar = UA G1 + G2 VA^T
  svd_bwd(UA, VA, s, w);
  // Halves in factored form (rank 2 chi):
  //   U_bar  = Pl_bar w VA^T + Lt^T Mt_bar = [Pl_bar w + Lt^T G2 | Lt^T UA] [VA | G1^T]^T
  //   Lt_bar = UA w Pu_bar^T + Mt_bar U^T  = [UA | G2] [Pu_bar w + U G1^T | U VA]^T
  const int c2x = 2 * chi;
  col_scale(ctx, LU.d(), c2x, Plb.d(), chi, n, chi, w, 1, false);
  gemm_f64(ctx, n, chi, n, 1.0, colmajor(Lt, n), rowmajor(G2.d(), chi), 1.0,
           out_rowmajor(LU.d(), c2x));
  copy_block(ctx, LU.d() + chi, c2x, PuU.d(), chi, n, chi);
  copy_block(ctx, RU.d(), c2x, VA, chi, n, chi);
  copy_block(ctx, RU.d() + chi, c2x, G1T.d(), chi, n, chi);
  copy_block(ctx, LL.d(), c2x, UA, chi, n, chi);
  copy_block(ctx, LL.d() + chi, c2x, G2.d(), chi, n, chi);
  col_scale(ctx, RL.d(), c2x, Pub.d(), chi, n, chi, w, 1, false);
  gemm_f64(ctx, n, chi, n, 1.0, rowmajor(U, n), rowmajor(G1T.d(), chi), 1.0,
           out_rowmajor(RL.d(), c2x));
  copy_block(ctx, RL.d() + chi, c2x, PlU.d(), chi, n, chi);
  // enlarged corners: Q_bar of each, then its adjoint
  for (int r = 0; r < 4; ++r) {
    const int f = (k + r) & 3;
    double* Qb = Qbar.d();
    if (r == 0) {  // U_bar Q1^T = LU (Q1 RU)^T
      mm(ctx, n, c2x, n, Q[q1], n, false, RU.d(), c2x, false, Wf.d(), c2x);
      mm(ctx, n, n, c2x, LU.d(), c2x, false, Wf.d(), c2x, true, Qb, n);
    } else if (r == 1) {  // Q0^T U_bar = (Q0^T LU) RU^T
      mm(ctx, n, c2x, n, Q[q0], n, true, LU.d(), c2x, false, Wf.d(), c2x);
      mm(ctx, n, n, c2x, Wf.d(), c2x, false, RU.d(), c2x, true, Qb, n);
    } else if (r == 2) {  // Lt_bar Q3^T = LL (Q3 RL)^T
      mm(ctx, n, c2x, n, Q[q3], n, false, RL.d(), c2x, false, Wf.d(), c2x);
      mm(ctx, n, n, c2x, LL.d(), c2x, false, Wf.d(), c2x, true, Qb, n);
    } else {  // Q2^T Lt_bar = (Q2^T LL) RL^T
      mm(ctx, n, c2x, n, Q[q2], n, true, LL.d(), c2x, false, Wf.d(), c2x);
      mm(ctx, n, n, c2x, Wf.d(), c2x, false, RL.d(), c2x, true, Qb, n);
    }
    const int g = (f + 3) & 3;
    const double* Xf = e.X1[f].d();
    permute(ctx, Qb, wA.d(), 4, e4b, p0213);  // [de,ga][dd,r]
    mm(ctx, dc, dc, chi, T[g], chi, false, Xf, dc, false, wB.d(), dc);
    permute(ctx, wB.d(), t2T, 4, d4c, p2103);  // [u,l][de,ga]
    mm(ctx, d2, d2, c2, t2T, c2, false, wA.d(), d2, false, Qb, d2);
    axpby(ctx, arb[f].d(), Qb, (size_t)d2 * d2, 1.0, 1.0);
    mm(ctx, c2, d2, d2, wA.d(), d2, false, arotT[f].d(), d2, false, wB.d(), d2);
    permute(ctx, wB.d(), wA.d(), 4, e4, p0321);  // t1_bar [de,l][u,ga]
    mm(ctx, dc, chi, dc, wA.d(), dc, false, Xf, dc, true, Tbar[g], chi, 1.0);
    mm(ctx, chi, dc, dc, T[g], chi, true, wA.d(), dc, false, X1b.d(), dc);
    if (f == q0) axpby(ctx, X1b.d(), x1e.d(), nc, 1.0, 1.0);
    mm(ctx, chi, chi, dc, X1b.d(), dc, false, T[f], dc, true, Cbar[f], chi, 1.0);
    mm(ctx, chi, dc, chi, C[f], chi, true, X1b.d(), dc, false, Tbar[f], dc, 1.0);
  }
}

void Grad::backward() {
  const double t0 = now_ms();
  double trec = 0.0;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    if (sg != nseg - 1) {
      const double r0 = now_ms();
      restore(ck[sg]);
      run_segment(sg, true);
      CTM_HIP(hipStreamSynchronize(ctx.stream));
      trec += now_ms() - r0;
    }
    const int s0 = sg * every, s1 = std::min(sweeps, s0 + every);
    const int nm = 4 * (s1 - s0);
    for (int m = nm - 1; m >= 0; --m) move_bwd(e.opt.move_order[m & 3], tape.d() + (size_t)m * tl.total);
  }
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  stats.ms_recompute = trec;
  stats.ms_backward = now_ms() - t0 - trec;
}

// abar += adjoints of the four rotated copies, rotated back: a_f is
// a_{f-1} with axes (3, 0, 1, 2), whose adjoint is the axis order (1, 2, 3, 0).
void Grad::site_total() {
  if (site_done) return;
  const size_t d4 = (size_t)d * d * d * d;
  const long long f4[4] = {d, d, d, d};
  const int un[4] = {1, 2, 3, 0};
  double* g = wA.d();
  copy_dev(ctx, g, arb[3].d(), d4);
  for (int f = 2; f >= 0; --f) {
    permute(ctx, g, wB.d(), 4, f4, un);
    axpby(ctx, wB.d(), arb[f].d(), d4, 1.0, 1.0);
    copy_dev(ctx, g, wB.d(), d4);
  }
  axpby(ctx, abar.d(), g, d4, 1.0, 1.0);
  site_done = true;
}

void Grad::grad_site(double* ga_dev) {
  site_total();
  const size_t d4 = (size_t)d * d * d * d;
  copy_dev(ctx, ga_dev, abar.d(), d4);
}

void Grad::grad_purification(const double* A_dev, const double* B_dev, int D, int Dg, int gamma,
                             double* gA_dev, double* gB_dev) {
  CTM_REQUIRE(e.D == D && D * D == d, "grad_purification: not this environment's purification");
  site_total();
  const int D4 = D * D * D * D;
  const long long dd[8] = {D, D, D, D, D, D, D, D};
  const int pp[8] = {0, 2, 4, 6, 1, 3, 5, 7};
  const double* Kc = e.Kc.d();
  // a8 = Kc^T Kc, a = interleave(a8)
  permute(ctx, abar.d(), wA.d(), 8, dd, pp);
  mm(ctx, 16, D4, D4, Kc, D4, false, wA.d(), D4, true, Kcb.d(), D4, 1.0);
  mm(ctx, 16, D4, D4, Kc, D4, false, wA.d(), D4, false, Kcb.d(), D4, 1.0);
  // Kc = perm(Kraw), Kraw = A' B'^T
  const long long kd[8] = {2, 2, 2, 2, D, D, D, D};
  const int ik[8] = {0, 1, 5, 4, 2, 3, 7, 6};
  const int m4 = 4 * D * D;
  DevBuf Krb((size_t)m4 * m4 * sizeof(double));
  permute(ctx, Kcb.d(), Krb.d(), 8, kd, ik);
  const int al = (gamma + 1) % 3, be = (gamma + 2) % 3;
  int bd[3] = {D, D, D};
  bd[gamma] = Dg;
  const long long dims[5] = {2, 2, bd[0], bd[1], bd[2]};
  const int perm5[5] = {0, 1, 2 + al, 2 + be, 2 + gamma};
  int inv5[5];
  for (int a = 0; a < 5; ++a) inv5[perm5[a]] = a;
  long long pd[5];
  for (int a = 0; a < 5; ++a) pd[a] = dims[perm5[a]];
  const size_t sz = 4ull * D * D * Dg;
  DevBuf Ap(sz * sizeof(double)), Bp(sz * sizeof(double)), Apb(sz * sizeof(double)),
      Bpb(sz * sizeof(double));
  permute(ctx, A_dev, Ap.d(), 5, dims, perm5);
  permute(ctx, B_dev, Bp.d(), 5, dims, perm5);
  mm(ctx, m4, Dg, m4, Krb.d(), m4, false, Bp.d(), Dg, false, Apb.d(), Dg);
  mm(ctx, m4, Dg, m4, Krb.d(), m4, true, Ap.d(), Dg, false, Bpb.d(), Dg);
  permute(ctx, Apb.d(), gA_dev, 5, pd, inv5);
  permute(ctx, Bpb.d(), gB_dev, 5, pd, inv5);
  // the temporaries are freed on return: let the stream finish with them
  CTM_HIP(hipStreamSynchronize(ctx.stream));
}

}  // namespace ctm
