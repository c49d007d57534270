// CTMRG engine for the rhombic lattice of composite tensors (arXiv:1906.02220,
// Sec. III, Fig. 4).  All contractions are FP64 MFMA GEMMs and LDS-tiled
// permutes; the projector SVD is a warm-started subspace iteration with a
// Rayleigh-Ritz step whose small SVD is a one-sided Jacobi in one workgroup.
//
// Conventions (as in the header): a[u,l,d,r]; corners C[a][b], edges
// T[a][m][b], clockwise C1 T1 C2 T2 C3 T3 C4 T4 from the top-left.  Rotating
// the lattice by 90 degrees counter-clockwise shifts the environment by one
// slot and maps a -> a.transpose(3,0,1,2), so a move in direction k is the
// left move of the frame rotated k times:
//   Q_f       = (T_{f+3} (C_f T_f)) a_f          enlarged corner of frame f,
//               rows: cut (T_{f+3}.a, d), columns: cut (T_f.b, r)
//   U = Q_k Q_{k+1},  Lt = Q_{k+2} Q_{k+3},  Mt = Lt U  (= M^T)
//   M = X S Y^T (top chi):  Pu = Lt^T Y S^-1/2,  Pl = U X S^-1/2
//   C_k     <- Pu^T (C_k T_k)
//   T_{k+3} <- Pu^T (T_{k+3} a_k) Pl
//   C_{k+3} <- (T_{k+2} C_{k+3}) Pl
// each followed by max-abs normalisation with the log of the factor kept.
// The first three of these are the directional four-quadrant projectors of
// the square-lattice CTMRG the paper builds on (Fig. 4(c)).
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "ctm.h"
#include "engine.hpp"

namespace ctm {

namespace {

// Largest number of iterations a tolerance-controlled truncated SVD adds
// after the fixed ones.
constexpr int kSvdMaxExtraIters = 8;

__global__ void add_log_slots_kernel(double* logs, int dst0, int src0, int dst1, int src1) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    logs[dst0] += logs[src0];
    logs[dst1] += logs[src1];
  }
}

}  // namespace

Env::Env(Context& c, int d_, int chi_, const EnvOptions& o) : ctx(c), d(d_), chi(chi_), opt(o) {
  CTM_REQUIRE(d >= 1 && chi >= 1, "d and chi must be >= 1");
  CTM_REQUIRE(chi <= jacobi_max_b(false), "chi above 128 is not supported");
  n = chi * d;
  if (opt.eps_cut < 0.0) opt.eps_cut = 0.0;
  const int bmax = jacobi_max_b(true);
  if (n <= bmax) {
    b = n;  // the cut matrix is small enough for a direct Jacobi SVD
  } else if (opt.svd_block > 0) {
    CTM_REQUIRE(opt.svd_block >= chi && opt.svd_block <= bmax,
                "svd_block must lie between chi and 128");
    b = std::min(opt.svd_block, n);
  } else {
    // the chi kept directions plus a margin that separates them from the
    // rest of the spectrum during the subspace iteration: a quarter of chi,
    // at least 16 columns, at least 88 in all.  Two sweeps from the start,
    // FP64 stays within 1e-9 of the oracle's bond-metric entries at D = 6,
    // chi = 72 with 16 columns (8 columns: 4e-8) and at D = 7, chi = 96 with
    // 24 (16 columns: 1.7e-8); 8 columns also lost the FP64 parity of nearly
    // degenerate cut spectra (corner spectra 1e-5 off at D = 4, chi = 32)
    b = opt.svd_oversample > 0 ? chi + opt.svd_oversample
                               : std::max(88, chi + std::max(16, (chi + 3) / 4));
    b = std::min(b, std::min(n, bmax));
  }
  svd_iters_auto = opt.svd_iters <= 0;
  if (opt.svd_iters <= 0) opt.svd_iters = 1;
  if (opt.svd_iters_cold <= 0) opt.svd_iters_cold = 5;
  alloc();
  CTM_HIP(hipHostMalloc((void**)&hbox, 64, hipHostMallocDefault));
  CTM_HIP(hipHostMalloc((void**)&hres, (std::max(chi, b) + 2) * sizeof(double),
                        hipHostMallocDefault));
}

Env::~Env() {
  drop_graph();
  if (hbox) (void)hipHostFree(hbox);
  if (hres) (void)hipHostFree(hres);
}

void Env::drop_graph() {
  if (gexec) {
    (void)hipStreamSynchronize(ctx.stream);
    (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }
  warm_eager_done = false;
}

void Env::alloc() {
  const size_t dd4 = (size_t)d * d * d * d;
  const size_t nn = (size_t)n * n;
  for (int i = 0; i < 4; ++i) arot[i].alloc(dd4 * sizeof(double));
  Call.alloc(4ull * chi * chi * sizeof(double));
  Tall.alloc(4ull * chi * d * chi * sizeof(double));
  logs.alloc(8 * sizeof(double));
  for (int i = 0; i < 4; ++i) {
    Qb[i].alloc(nn * sizeof(double));
    X1[i].alloc((size_t)chi * d * chi * sizeof(double));
  }
  const size_t big = std::max(nn, dd4);  // n^2 = chi^2 d^2 intermediates and d^4 ring products
  U.alloc(big * sizeof(double));
  Lt.alloc(big * sizeof(double));
  Mt.alloc(big * sizeof(double));
  t1.alloc(big * sizeof(double));
  t2.alloc(big * sizeof(double));
  const size_t nb = (size_t)n * b;
  Om.alloc(nb * sizeof(double));
  Zb.alloc(nb * sizeof(double));
  Z0.alloc(nb * sizeof(double));
  Qz.alloc(nb * sizeof(double));
  Wv.alloc(nb * sizeof(double));
  UA.alloc(nb * sizeof(double));
  VA.alloc(nb * sizeof(double));
  for (int i = 0; i < 4; ++i) warm[i].alloc(nb * sizeof(double));
  G.alloc((size_t)b * b * sizeof(double));
  Wm.alloc((size_t)b * b * sizeof(double));
  Bsm.alloc((size_t)b * b * sizeof(double));
  xs.alloc((size_t)b * b * sizeof(double));
  ys.alloc((size_t)b * b * sizeof(double));
  sv.alloc((size_t)std::max(b, chi) * sizeof(double));
  winv.alloc((size_t)chi * sizeof(double));
  Pu.alloc((size_t)n * chi * sizeof(double));
  Pl.alloc((size_t)n * chi * sizeof(double));
  const size_t smallsz = std::max((size_t)chi * d * chi, (size_t)chi * chi) * sizeof(double);
  sm1.alloc(smallsz);
  sm2.alloc(smallsz);
  sm3.alloc(smallsz);
  spec_s.alloc(4ull * chi * sizeof(double));
  spec_old.alloc(4ull * chi * sizeof(double));
  scal.alloc(64 * sizeof(double));
  iflags.alloc((8 + (size_t)b) * sizeof(int));
  rngc.alloc(2 * sizeof(unsigned long long));
  fill_zero(ctx, (double*)rngc.p, 2);
  E.alloc(dd4 * sizeof(double));
  E8.alloc(dd4 * sizeof(double));
  resid.alloc((size_t)(std::max(chi, b) + 2) * sizeof(double));
  fill_zero(ctx, logs.d(), 8);
  fill_zero(ctx, scal.d(), 64);
  fill_zero_int(ctx, (int*)iflags.p, 8 + b);
}

void Env::set_site_tensor_dev(const double* a_dev) {
  drop_graph();
  copy_dev(ctx, arot[0].d(), a_dev, (size_t)d * d * d * d);
  const long long dims[4] = {d, d, d, d};
  const int rot[4] = {3, 0, 1, 2};
  for (int k = 1; k < 4; ++k) permute(ctx, arot[k - 1].d(), arot[k].d(), 4, dims, rot);
  for (int k = 0; k < 4; ++k) aslices[k].valid = false;
  e_valid = false;
}

// a1 + a2: composite of A and B fused across gamma, then the double layer.
void Env::build_purification_dev(const double* A, const double* B, int D_, int Dg, int gamma) {
  D = D_;
  CTM_REQUIRE(D * D == d, "purification: d must equal D^2");
  const int al = (gamma + 1) % 3, be = (gamma + 2) % 3;
  long long dims[8];
  dims[0] = 2; dims[1] = 2;
  int bd[3] = {D, D, D};
  bd[gamma] = Dg;
  dims[2] = bd[0]; dims[3] = bd[1]; dims[4] = bd[2];
  const int perm5[5] = {0, 1, 2 + al, 2 + be, 2 + gamma};
  const size_t szA = 4ull * D * D * Dg;
  DevBuf Ap(szA * sizeof(double)), Bp(szA * sizeof(double));
  permute(ctx, A, Ap.d(), 5, dims, perm5);  // [s,a,l,u,g]
  permute(ctx, B, Bp.d(), 5, dims, perm5);  // [t,c,r,d,g]
  const int m4 = 4 * D * D;
  DevBuf Kraw((size_t)m4 * m4 * sizeof(double));
  // Kraw[(s,a,l,u),(t,c,r,d)] = sum_g A'[(s,a,l,u), g] B'[(t,c,r,d), g]
  gemm_f64(ctx, m4, m4, Dg, 1.0, rowmajor(Ap.d(), Dg), colmajor(Bp.d(), Dg), 0.0,
           out_rowmajor(Kraw.d(), m4));
  const size_t D4 = (size_t)D * D * D * D;
  Kc.alloc(16 * D4 * sizeof(double));
  const long long kd[8] = {2, 2, D, D, 2, 2, D, D};
  const int kperm[8] = {0, 1, 4, 5, 3, 2, 7, 6};  // -> [s,a,t,c,u,l,d,r]
  permute(ctx, Kraw.d(), Kc.d(), 8, kd, kperm);
  // a8[(ket u l d r),(bra u l d r)] = sum_p K[p, ket] K[p, bra]
  DevBuf a8(D4 * D4 * sizeof(double));
  gemm_f64(ctx, (int)D4, (int)D4, 16, 1.0, colmajor(Kc.d(), (long long)D4),
           rowmajor(Kc.d(), (long long)D4), 0.0, out_rowmajor(a8.d(), (long long)D4));
  const long long ad[8] = {D, D, D, D, D, D, D, D};
  const int aperm[8] = {0, 4, 1, 5, 2, 6, 3, 7};  // -> [u_k,u_b,l_k,l_b,d_k,d_b,r_k,r_b]
  DevBuf afused(D4 * D4 * sizeof(double));
  permute(ctx, a8.d(), afused.d(), 8, ad, aperm);
  set_site_tensor_dev(afused.d());
  CTM_HIP(hipStreamSynchronize(ctx.stream));
}

// a3: C_i = [[1]], T_i[0,:,0] = boundary vector, zero-padded to chi.
void Env::init_boundary() {
  drop_graph();
  std::vector<double> bvec = opt.boundary;
  if (bvec.empty()) {
    bvec.assign(d, 0.0);
    if (D > 0) {
      for (int k = 0; k < D; ++k) bvec[k * D + k] = 1.0;  // vec(I_D)
    } else {
      bvec[0] = 1.0;  // e_0
    }
  }
  CTM_REQUIRE((int)bvec.size() == d, "boundary vector must have length d");
  std::vector<double> hc(4ull * chi * chi, 0.0), ht(4ull * chi * d * chi, 0.0);
  for (int i = 0; i < 4; ++i) {
    hc[(size_t)i * chi * chi] = 1.0;
    for (int m = 0; m < d; ++m) ht[(size_t)i * chi * d * chi + (size_t)m * chi] = bvec[m];
  }
  std::vector<double> hl(8, 0.0);
  set(hc.data(), ht.data(), hl.data());
  sweeps_done = 0;
}

void Env::check_flags(const char* where) {
  int hf[2];
  CTM_HIP(hipMemcpyAsync(hf, iflags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  if (hf[0] || hf[1]) {
    fill_zero_int(ctx, (int*)iflags.p, 2);
    throw Error(-4, std::string(where) + (hf[0] ? ": non-finite or vanishing environment tensor"
                                               : ": projector SVD failed"));
  }
}

// a4: enlarged corner of frame f.
void Env::corner(int f) {
  f &= 3;
  const int dc = d * chi;
  // X1 = C_f T_f : [al][u][ga]
  gemm_f64(ctx, chi, dc, chi, 1.0, rowmajor(Cp(f), chi), rowmajor(Tp(f), dc), 0.0,
           out_rowmajor(X1[f].d(), dc));
  // t1 = T_{f+3} X1 : [de,l][u,ga]
  gemm_f64(ctx, dc, dc, chi, 1.0, rowmajor(Tp(f + 3), chi), rowmajor(X1[f].d(), dc), 0.0,
           out_rowmajor(t1.d(), dc));
  const long long d4[4] = {chi, d, d, chi};
  const int p0321[4] = {0, 3, 2, 1};
  permute(ctx, t1.d(), t2.d(), 4, d4, p0321);  // [de,ga,u,l]
  // Q_f = (t2 a_f) [(de,ga),(u,l)] x [(u,l),(dd,r)], stored [de,dd,ga,r]: the
  // slice modes write that order from the product itself
  const OutMap to_q{chi, (long long)d * chi * d, d, d, (long long)chi * d};
  if (!gemm_slices_split_out(ctx, opt.precision, chi * chi, d * d, d * d, rowmajor(t2.d(), d * d),
                             rowmajor(arot[f].d(), d * d), Qb[f].d(), to_q, -1, &aslices[f])) {
    gemm_mixed(ctx, opt.precision, chi * chi, d * d, d * d, 1.0, rowmajor(t2.d(), d * d),
               rowmajor(arot[f].d(), d * d), 0.0, out_rowmajor(t1.d(), d * d));
    const long long e4[4] = {chi, chi, d, d};
    const int p0213[4] = {0, 2, 1, 3};
    permute(ctx, t1.d(), Qb[f].d(), 4, e4, p0213);  // [de,dd,ga,r]
  }
  qvalid[f] = true;
}

// Column-scaled CholeskyQR in `passes` passes (Z is n x b row-major): the
// Gram matrix by GEMM, its Cholesky inverse in one workgroup, Q = Z W by
// GEMM, numerically dependent columns refilled with random vectors (which the
// next pass orthogonalises).  Q gets orthonormal columns spanning Z.
void Env::orth(double* Z, double* Q, int passes) {
  int* dep = (int*)iflags.p + 8;
  int* err = (int*)iflags.p + 1;
  const double* src = Z;
  for (int pass = 0; pass < passes; ++pass) {
    double* dst = (pass == passes - 1) ? Q : ((pass & 1) ? Zb.d() : Wv.d());
    if (dst == src) dst = (src == Wv.d()) ? Zb.d() : Wv.d();
    gemm_f64(ctx, b, b, n, 1.0, colmajor(src, b), rowmajor(src, b), 0.0, out_rowmajor(G.d(), b));
    // A second pass usually starts from columns that the first left
    // orthonormal to rounding; the first-order correction (3 I - G) / 2 then
    // replaces the one-workgroup Cholesky inverse, which still runs when the
    // first pass refilled dependent columns or left more than 1e-10 (decided
    // on the device).
    chol_inverse(ctx, G.d(), b, 1e-12, Wm.d(), dep, err, pass > 0);
    gemm_f64(ctx, n, b, b, 1.0, rowmajor(src, b), rowmajor(Wm.d(), b), 0.0, out_rowmajor(dst, b));
    unsigned long long* rc = (unsigned long long*)rngc.p;
    refill_columns(ctx, dst, b, n, b, dep, opt.seed ^ 0x5deece66dULL, rc + rng_slot,
                   rc + (rng_slot ^ 1));
    rng_slot ^= 1;
    src = dst;
  }
}

// Column norm (relative to the Frobenius norm) below which the Rayleigh-Ritz
// Jacobi takes a column of its k x k matrix for zero: k eps, the rounding
// level of its k-term dot products.  The adjoint's calls (svd_tol > 0)
// converge every pair instead, and so does the full SVD of a small cut
// matrix, which the adjoint shares with plain sweeps.
static double jacobi_zero_level(const EnvOptions& o, int k) {
  return o.svd_tol > 0.0 ? 0.0 : k * DBL_EPSILON;
}

// Relative accuracy of the cut matrix when it comes from reduced-precision
// products: the unit roundoff of their operands, 2^-24 for FP32 and three BF16
// slices, 2^-32 for four.  Those products perturb the cut matrix by about that
// fraction of its norm, which by Weyl's inequality leaves its singular values
// below that level undetermined; rotations between two such columns of B only
// fit rounding noise and do not hold the Jacobi sweeps open.  FP64 and the
// adjoint's calls return 0.
static double jacobi_noise_level(const EnvOptions& o) {
  if (o.svd_tol > 0.0 || o.precision == CTM_PREC_F64) return 0.0;
  return o.precision == CTM_PREC_BF16X4 ? 0x1p-32 : 0x1p-24;
}

// a6: top-chi singular triplets of M = Mt^T by subspace iteration on the
// warm start of the previous move in the same direction.  Left vectors of
// Mt (= Y of M) go to UA, right vectors (= X of M) to VA, values to sv;
// n x b row-major.  One iteration: Z = orth(Mt Om), Om <- orth(Mt^T Z);
// then the Rayleigh-Ritz step: Z = Mt Om, Qz = orth(Z),
// B = Qz^T Z (upper triangular), B = x s y^T by one-sided Jacobi on B^T,
// UA = Qz x, VA = Om y.
void Env::svd_top(const double* MtP, int k) {
  int* err = (int*)iflags.p + 1;
  if (n <= jacobi_max_b(true)) {
    jacobi_svd(ctx, MtP, n, UA.d(), sv.d(), VA.d(), err);
    fix_signs(ctx, UA.d(), b, VA.d(), b, n, b);
    return;
  }
  int iters = opt.svd_iters;
  if (warm_ok[k]) {
    copy_dev(ctx, Om.d(), warm[k].d(), (size_t)n * b);
    // Automatic count: two iterations while the environment is still far
    // from its fixed point and the cut matrix changes a lot between moves,
    // one afterwards.  At D = 3, chi = 20 one iteration from the second
    // sweep on left <H> 1.5e-10 from the exact-SVD result after 6 sweeps
    // (two: 3e-12) and 1e-12 after 10.
    if (svd_iters_auto && warm_moves[k] < kSettleWarmMoves) iters = 2;
    if (warm_moves[k] < kSettleWarmMoves) ++warm_moves[k];
  } else {
    fill_normal(ctx, Z0.d(), (size_t)n * b, opt.seed, rng_ctr);
    rng_ctr += (unsigned long long)n * b;
    orth(Z0.d(), Om.d(), 2);
    iters = opt.svd_iters_cold;
    warm_moves[k] = 0;
  }
  // Every right basis gets two CholeskyQR passes: with one pass on the
  // intermediate ones the orthogonality error of each pass accumulates over
  // the iterations (12 iterations from the boundary start at D = 6, chi = 72
  // then left kappa 8e-9 from the full SVD's instead of 1e-10).
  if (opt.svd_tol > 0.0) {
    for (int it = 0; it < iters; ++it) subspace_iteration(MtP);
    rayleigh_ritz(MtP);
  } else {
    for (int it = 0; it + 1 < iters; ++it) subspace_iteration(MtP);
    final_iteration_ritz(MtP);
  }
  ++svd_calls;
  svd_iterations += iters;
  if (opt.svd_tol > 0.0) {
    // continue from the Ritz vectors until the kept triplets' residual meets
    // the tolerance (each check waits for the device)
    for (int extra = 0; extra < kSvdMaxExtraIters; ++extra) {
      if (svd_residual(MtP) <= opt.svd_tol) break;
      copy_dev(ctx, Om.d(), VA.d(), (size_t)n * b);
      subspace_iteration(MtP);
      rayleigh_ritz(MtP);
      ++svd_iterations;
    }
  }
  copy_dev(ctx, warm[k].d(), VA.d(), (size_t)n * b);
  warm_ok[k] = true;
}

// One subspace iteration on Om: Z = Mt Om must be orthogonalised (not only
// normalised) before Mt^T is applied: a column carrying a small contamination
// of a leading direction would otherwise lose its own small-singular-value
// component.
void Env::subspace_iteration(const double* MtP) {
  gemm_f64(ctx, n, b, n, 1.0, rowmajor(MtP, n), rowmajor(Om.d(), b), 0.0, out_rowmajor(Z0.d(), b));
  orth(Z0.d(), Qz.d(), 1);
  gemm_f64(ctx, n, b, n, 1.0, colmajor(MtP, n), rowmajor(Qz.d(), b), 0.0, out_rowmajor(Z0.d(), b));
  orth(Z0.d(), Om.d(), 2);
}

// Rayleigh-Ritz on the subspace Om: Z = Mt Om = Qz B with B upper triangular,
// B = x s y^T, so Mt Om = (Qz x) s y^T: UA = Qz x, VA = Om y, sv = s.
//
// Columns of B below b eps ||B||_F (a subspace wider than the numerical rank
// of Mt) are zero to working precision and do not hold the Jacobi sweeps
// open, and neither do pairs of two columns below the accuracy of a
// reduced-precision Mt; the adjoint's calls (svd_tol > 0) converge every
// pair.
//
// The Ritz vectors keep the signs the warm start carries through the Jacobi
// rotations; no canonical sign is imposed.  Triplets on the near-degenerate
// tail of the cut spectrum change by a few percent per move, so a rule such
// as "largest entry positive" flips some of them from one move to the next.
// Each flip changes the sign of an environment bond direction, the next cut
// matrix then differs from the one the warm start was taken from by 1e-6 to
// 1e-3 of s_1 along its leading directions, and about half of the warm
// columns come out numerically dependent every move (they are refilled at
// random, and the tail never converges).
void Env::rayleigh_ritz(const double* MtP) {
  int* err = (int*)iflags.p + 1;
  gemm_f64(ctx, n, b, n, 1.0, rowmajor(MtP, n), rowmajor(Om.d(), b), 0.0, out_rowmajor(Z0.d(), b));
  orth(Z0.d(), Qz.d(), 2);
  gemm_f64(ctx, b, b, n, 1.0, colmajor(Qz.d(), b), rowmajor(Z0.d(), b), 0.0, out_rowmajor(Bsm.d(), b));
  jacobi_svd(ctx, Bsm.d(), b, xs.d(), sv.d(), ys.d(), err, 1, 0, 0, true,
             jacobi_zero_level(opt, b), jacobi_noise_level(opt));
  gemm_f64(ctx, n, b, b, 1.0, rowmajor(Qz.d(), b), rowmajor(xs.d(), b), 0.0, out_rowmajor(UA.d(), b));
  gemm_f64(ctx, n, b, b, 1.0, rowmajor(Om.d(), b), rowmajor(ys.d(), b), 0.0, out_rowmajor(VA.d(), b));
}

// The last subspace iteration with the Rayleigh-Ritz step folded in:
// Qz = orth(Mt Om) (two passes, since Qz is the final left basis),
// Y = Mt^T Qz, Om = orth(Y).  Then Qz^T Mt Om = Y^T Om = B exactly (Om spans
// Y), and Mt^T Qz lying in the span of Om gives Qz Qz^T Mt = Qz B Om^T, so
// B = x s y^T yields UA = Qz x, VA = Om y without the product Mt Om and the
// orthogonalisation of rayleigh_ritz.  B = Y^T Om = R^T for Y = Om R is lower
// triangular, so the rotations act on its columns (the rows of R), the same
// side as rayleigh_ritz's transposed call on its upper triangular factor.
void Env::final_iteration_ritz(const double* MtP) {
  int* err = (int*)iflags.p + 1;
  gemm_f64(ctx, n, b, n, 1.0, rowmajor(MtP, n), rowmajor(Om.d(), b), 0.0, out_rowmajor(Z0.d(), b));
  orth(Z0.d(), Qz.d(), 2);
  gemm_f64(ctx, n, b, n, 1.0, colmajor(MtP, n), rowmajor(Qz.d(), b), 0.0, out_rowmajor(Z0.d(), b));
  orth(Z0.d(), Om.d(), 2);
  gemm_f64(ctx, b, b, n, 1.0, colmajor(Z0.d(), b), rowmajor(Om.d(), b), 0.0, out_rowmajor(Bsm.d(), b));
  jacobi_svd(ctx, Bsm.d(), b, xs.d(), sv.d(), ys.d(), err, 1, 0, 0, false,
             jacobi_zero_level(opt, b), jacobi_noise_level(opt));
  gemm_f64(ctx, n, b, b, 1.0, rowmajor(Qz.d(), b), rowmajor(xs.d(), b), 0.0, out_rowmajor(UA.d(), b));
  gemm_f64(ctx, n, b, b, 1.0, rowmajor(Om.d(), b), rowmajor(ys.d(), b), 0.0, out_rowmajor(VA.d(), b));
}

// max_i ||Mt^T u_i - s_i v_i|| / s_1 over the kept i < min(chi, b), read back
// to the host (waits for the stream).  Uses Z0 as scratch.
double Env::svd_residual(const double* MtP) {
  const int kk = std::min(chi, b);
  gemm_f64(ctx, n, kk, n, 1.0, colmajor(MtP, n), rowmajor(UA.d(), b), 0.0, out_rowmajor(Z0.d(), b));
  column_residuals(ctx, Z0.d(), VA.d(), sv.d(), n, b, kk, resid.d());
  CTM_HIP(hipMemcpyAsync(hres, resid.p, (kk + 1) * sizeof(double), hipMemcpyDeviceToHost,
                         ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  double r = 0.0;
  for (int i = 0; i < kk; ++i) r = std::max(r, hres[i]);
  return hres[kk] > 0.0 ? r / hres[kk] : (r > 0.0 ? INFINITY : 0.0);
}

double Env::last_svd_residual() {
  if (!moved) return 0.0;
  if (n <= jacobi_max_b(true)) {
    // full Jacobi SVD of the cut matrix: the same check on its triplets
    const int kk = std::min(chi, n);
    gemm_f64(ctx, n, kk, n, 1.0, colmajor(Mt.d(), n), rowmajor(UA.d(), b), 0.0,
             out_rowmajor(Z0.d(), b));
    column_residuals(ctx, Z0.d(), VA.d(), sv.d(), n, b, kk, resid.d());
    CTM_HIP(hipMemcpyAsync(hres, resid.p, (kk + 1) * sizeof(double), hipMemcpyDeviceToHost,
                           ctx.stream));
    CTM_HIP(hipStreamSynchronize(ctx.stream));
    double r = 0.0;
    for (int i = 0; i < kk; ++i) r = std::max(r, hres[i]);
    return hres[kk] > 0.0 ? r / hres[kk] : 0.0;
  }
  return svd_residual(Mt.d());
}

// a4 - a7: one absorption move (left move of frame k).
void Env::move(int k) {
  const double W = 2.0 * (5.0 * chi * chi * std::pow((double)d, 4) + 3.0 * std::pow((double)n, 3) +
                          8.0 * std::pow((double)chi, 3) * d * d + 6.0 * std::pow((double)chi, 3) * d);
  ScopedTimer tmove(ctx, 2, W);
  move_front(k);
  move_products(k);
  move_back(k);
}

void Env::move_front(int k) {
  k &= 3;
  const TapeLayout tl(chi, d);
  if (tape_slot) {
    copy_dev(ctx, tape_slot + tl.c, Call.d(), 4ull * chi * chi);
    copy_dev(ctx, tape_slot + tl.t, Tall.d(), 4ull * chi * d * chi);
  }
  for (int r = 0; r < 4; ++r)
    if (!qvalid[(k + r) & 3]) corner(k + r);
}

// a5: halves and the cut matrix
void Env::move_products(int k) {
  k &= 3;
  const int q0 = k, q1 = (k + 1) & 3, q2 = (k + 2) & 3, q3 = (k + 3) & 3;
  gemm_mixed(ctx, opt.precision, n, n, n, 1.0, rowmajor(Qb[q0].d(), n), rowmajor(Qb[q1].d(), n),
             0.0, out_rowmajor(U.d(), n), 1, 0);
  gemm_mixed(ctx, opt.precision, n, n, n, 1.0, rowmajor(Qb[q2].d(), n), rowmajor(Qb[q3].d(), n),
             0.0, out_rowmajor(Lt.d(), n), 1, 0);
  gemm_mixed(ctx, opt.precision, n, n, n, 1.0, rowmajor(Lt.d(), n), rowmajor(U.d(), n), 0.0,
             out_rowmajor(Mt.d(), n), 1, 0);
}

int Env::cut_products(int k, GroupProblem* probs) {
  k &= 3;
  const int q0 = k, q1 = (k + 1) & 3, q2 = (k + 2) & 3, q3 = (k + 3) & 3;
  const double* ops[3][2] = {{Qb[q0].d(), Qb[q1].d()}, {Qb[q2].d(), Qb[q3].d()}, {Lt.d(), U.d()}};
  double* outs[3] = {U.d(), Lt.d(), Mt.d()};
  int kind = -1;
  for (int i = 0; i < 3; ++i) {
    const int ki = grouped_kind(ctx, opt.precision, n, n, n, rowmajor(ops[i][0], n),
                                rowmajor(ops[i][1], n), out_rowmajor(outs[i], n));
    if (kind >= 0 && ki != kind) return 0;
    kind = ki;
    probs[i] = GroupProblem{ops[i][0], ops[i][1], outs[i], n, n, n, n, n, n};
  }
  return kind;
}

void Env::move_back(int k) {
  k &= 3;
  const int dc = d * chi;
  const TapeLayout tl(chi, d);
  const int q0 = k, q2 = (k + 2) & 3, q3 = (k + 3) & 3;
  // a6: projectors
  svd_top(Mt.d(), k);
  const int kk = std::min(chi, b);
  inv_sqrt_cut(ctx, sv.d(), kk, chi, opt.eps_cut, winv.d());
  if (tape_slot) {
    copy_block(ctx, tape_slot + tl.ua, chi, UA.d(), b, n, kk);
    copy_block(ctx, tape_slot + tl.va, chi, VA.d(), b, n, kk);
    copy_dev(ctx, tape_slot + tl.s, sv.d(), kk);
    copy_dev(ctx, tape_slot + tl.w, winv.d(), chi);
  }
  if (kk < chi) {
    fill_zero(ctx, Pu.d(), (size_t)n * chi);
    fill_zero(ctx, Pl.d(), (size_t)n * chi);
  }
  // Pu = Lt^T Y, Pl = U X (first kk columns), then S^-1/2 with the cutoff
  gemm_f64(ctx, n, kk, n, 1.0, colmajor(Lt.d(), n), rowmajor(UA.d(), b), 0.0, out_rowmajor(Pu.d(), chi));
  gemm_f64(ctx, n, kk, n, 1.0, rowmajor(U.d(), n), rowmajor(VA.d(), b), 0.0, out_rowmajor(Pl.d(), chi));
  scale_cols(ctx, Pu.d(), n, chi, chi, winv.d());
  scale_cols(ctx, Pl.d(), n, chi, chi, winv.d());
  // a7: C_k <- Pu^T (C_k T_k)
  gemm_f64(ctx, chi, chi, n, 1.0, colmajor(Pu.d(), chi), rowmajor(X1[q0].d(), chi), 0.0,
           out_rowmajor(Cw(q0), chi));
  // C_{k+3} <- (T_{k+2} C_{k+3}) Pl, with C4'[io][de][dd] = sum_ka C4[ka][de] T3[io][dd][ka]
  gemm_f64(ctx, chi, d, chi, 1.0, View{Cp(q3), 1, chi, 0}, View{Tp(q2), 1, chi, dc}, 0.0,
           ViewOut{sm1.d(), d, 1, dc}, chi);
  gemm_f64(ctx, chi, chi, n, 1.0, rowmajor(sm1.d(), n), rowmajor(Pl.d(), chi), 0.0,
           out_rowmajor(Cw(q3), chi));
  // T_{k+3} <- Pu^T (T_{k+3} a_k) Pl
  gemm_f64(ctx, dc, dc, chi, 1.0, rowmajor(Tp(q3), chi), rowmajor(Pl.d(), dc), 0.0,
           out_rowmajor(t1.d(), dc));  // [de,l][u,k2]
  const long long d4[4] = {chi, d, d, chi};
  const int p0321[4] = {0, 3, 2, 1};
  permute(ctx, t1.d(), t2.d(), 4, d4, p0321);  // [de,k2,u,l]
  // (t2 a) [de,k2,dd,r], stored [de,dd,k2,r] (by the product itself in the slice modes)
  const OutMap to_t{chi, (long long)d * chi * d, d, d, (long long)chi * d};
  const double* tq = t2.d();  // [de,dd,k2,r]
  if (gemm_slices_split_out(ctx, opt.precision, chi * chi, d * d, d * d, rowmajor(t2.d(), d * d),
                            rowmajor(arot[q0].d(), d * d), t1.d(), to_t, -1, &aslices[q0])) {
    tq = t1.d();
  } else {
    gemm_mixed(ctx, opt.precision, chi * chi, d * d, d * d, 1.0, rowmajor(t2.d(), d * d),
               rowmajor(arot[q0].d(), d * d), 0.0, out_rowmajor(t1.d(), d * d));  // [de,k2,dd,r]
    const long long e4[4] = {chi, chi, d, d};
    const int p0213[4] = {0, 2, 1, 3};
    permute(ctx, t1.d(), t2.d(), 4, e4, p0213);  // [de,dd,k2,r]
  }
  gemm_f64(ctx, chi, dc, n, 1.0, colmajor(Pu.d(), chi), rowmajor(tq, dc), 0.0,
           out_rowmajor(sm2.d(), dc));  // [k1][k2,r]
  const long long e3[3] = {chi, chi, d};
  const int p021[3] = {0, 2, 1};
  permute(ctx, sm2.d(), Tw(q3), 3, e3, p021);  // [k1][r][k2]
  // logs: the new C_k carries T_k, the new C_{k+3} carries T_{k+2}
  hipLaunchKernelGGL(add_log_slots_kernel, dim3(1), dim3(1), 0, ctx.stream, logs.d(), q0, 4 + q0,
                     q3, 4 + q2);
  CTM_HIP(hipGetLastError());
  int* nflag = (int*)iflags.p;
  double* keep = tape_slot ? tape_slot + tl.inv : nullptr;
  normalise_maxabs(ctx, Cw(q0), (size_t)chi * chi, logs.d() + q0, nflag, keep);
  normalise_maxabs(ctx, Tw(q3), (size_t)chi * d * chi, logs.d() + 4 + q3, nflag, keep ? keep + 1 : nullptr);
  normalise_maxabs(ctx, Cw(q3), (size_t)chi * chi, logs.d() + q3, nflag, keep ? keep + 2 : nullptr);
  qvalid[q0] = false;
  qvalid[q3] = false;
  e_valid = false;
  moved = true;
}

void Env::reset_spectra() {
  int* err = (int*)iflags.p + 1;
  jacobi_svd(ctx, Call.d(), chi, nullptr, spec_s.d(), nullptr, err, 4, (long long)chi * chi, chi);
  spectra_delta(ctx, spec_s.d(), spec_old.d(), chi, scal.d());
}

// a8: sweeps (left, right, up, down) with the corner-spectrum criterion.
int Env::sweep(int max_sweeps, double tol, int* done, double* delta_out) {
  CTM_REQUIRE(max_sweeps >= 0, "max_sweeps must be >= 0");
  double delta = INFINITY;
  int s = 0;
  if (tol <= 0.0 && !ctx.use_graphs) {
    // A fixed number of sweeps returns only the last sweep's delta, which
    // needs the corner spectra after the last two sweeps: the sweeps before
    // those are the four moves alone, enqueued without waiting (the error
    // flags they may raise stay set for the check after the last sweep).
    for (; s < max_sweeps - 2; ++s) {
      for (int i = 0; i < 4; ++i) move(opt.move_order[i]);
      ++sweeps_done;
    }
  }
  for (; s < max_sweeps; ++s) {
    sweep_enqueue();
    CTM_HIP(hipStreamSynchronize(ctx.stream));
    delta = sweep_finish("ctm_sweep");
    if (tol > 0.0 && delta < tol) { ++s; break; }
  }
  if (done) *done = s;
  if (delta_out) *delta_out = delta;
  if (tol > 0.0 && !(delta < tol)) return 1;
  return 0;
}

void Env::sweep_body() {
  int* err = (int*)iflags.p + 1;
  for (int i = 0; i < 4; ++i) move(opt.move_order[i]);
  jacobi_svd(ctx, Call.d(), chi, nullptr, spec_s.d(), nullptr, err, 4, (long long)chi * chi, chi);
  spectra_delta(ctx, spec_s.d(), spec_old.d(), chi, scal.d());
}

void Env::sweep_tail_eager() {
  if (gexec) drop_graph();
  int* err = (int*)iflags.p + 1;
  jacobi_svd(ctx, Call.d(), chi, nullptr, spec_s.d(), nullptr, err, 4, (long long)chi * chi, chi);
  spectra_delta(ctx, spec_s.d(), spec_old.d(), chi, scal.d());
  CTM_HIP(hipMemcpyAsync(hbox, scal.d(), sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipMemcpyAsync(hbox + 1, iflags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
}

// A sweep may be captured once every direction runs warm with its final
// iteration count (so the host takes the same branches on every sweep) and a
// warm sweep has already run eagerly
// (so every workspace the sweep needs exists and no allocation can fall into
// the capture).  Timing events are not captured.
bool Env::graph_ready() const {
  if (!ctx.use_graphs || ctx.timing || !warm_eager_done) return false;
  if (opt.svd_tol > 0.0) return false;  // its residual checks wait for the device
  if (n > jacobi_max_b(true))
    for (int k = 0; k < 4; ++k)
      if (!warm_ok[k] || (svd_iters_auto && warm_moves[k] < kSettleWarmMoves)) return false;
  return true;
}

void Env::capture_graph() {
  hipGraph_t g = nullptr;
  const int slot0 = rng_slot;
  CTM_HIP(hipStreamBeginCapture(ctx.stream, hipStreamCaptureModeThreadLocal));
  try {
    sweep_body();
    if (rng_slot != slot0) {
      // an odd number of refills: move the counter back to the slot the
      // next replay reads
      copy_dev(ctx, (double*)rngc.p + slot0, (const double*)rngc.p + rng_slot, 1);
      rng_slot = slot0;
    }
  } catch (...) {
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(ctx.stream, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    (void)hipGetLastError();
    throw;
  }
  CTM_HIP(hipStreamEndCapture(ctx.stream, &g));
  const hipError_t e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    gexec = nullptr;
    CTM_HIP(e);
  }
  g_splitk = ctx.splitk_ws.p;
  g_mixed = ctx.mixed_ws.p;
}

void Env::sweep_enqueue() {
  if (graph_ready()) {
    // the captured workspaces must still be the context's (a larger request
    // from another call reallocates them)
    if (gexec && (g_splitk != ctx.splitk_ws.p || g_mixed != ctx.mixed_ws.p)) {
      (void)hipStreamSynchronize(ctx.stream);
      (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    }
    if (!gexec) capture_graph();
    CTM_HIP(hipGraphLaunch(gexec, ctx.stream));
    e_valid = false;
  } else {
    bool warm = true;
    if (n > jacobi_max_b(true))
      for (int k = 0; k < 4; ++k) warm = warm && warm_ok[k];
    sweep_body();
    if (warm) warm_eager_done = true;
  }
  CTM_HIP(hipMemcpyAsync(hbox, scal.d(), sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipMemcpyAsync(hbox + 1, iflags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
}

double Env::sweep_finish(const char* where) {
  const int* hf = (const int*)(hbox + 1);
  if (hf[0] || hf[1]) {
    const bool nonfinite = hf[0] != 0;
    fill_zero_int(ctx, (int*)iflags.p, 2);
    throw Error(-4, std::string(where) + (nonfinite ? ": non-finite or vanishing environment tensor"
                                                    : ": projector SVD failed"));
  }
  ++sweeps_done;
  return hbox[0];
}

// a9: the ring E[u,l,x,r] of the eight environment tensors around one site,
// contracted as (C1 T1 C2 T2)[a,u,r,h] and (C3 T3 C4 T4)[h,x,l,a] joined over
// (a, h), so that no chi^2 d^3 intermediate is needed.
void Env::ring() {
  if (e_valid) return;
  const int dc = d * chi;
  // upper half
  gemm_f64(ctx, chi, dc, chi, 1.0, rowmajor(Cp(0), chi), rowmajor(Tp(0), dc), 0.0,
           out_rowmajor(sm1.d(), dc));                              // C1 T1 [a][u,g]
  gemm_f64(ctx, dc, chi, chi, 1.0, rowmajor(sm1.d(), chi), rowmajor(Cp(1), chi), 0.0,
           out_rowmajor(sm2.d(), chi));                             // [a,u][e]
  gemm_f64(ctx, dc, dc, chi, 1.0, rowmajor(sm2.d(), chi), rowmajor(Tp(1), dc), 0.0,
           out_rowmajor(t1.d(), dc));                               // [a,u][r,h]
  const long long d4[4] = {chi, d, d, chi};
  const int p1203[4] = {1, 2, 0, 3};
  permute(ctx, t1.d(), U.d(), 4, d4, p1203);                        // [u,r,a,h]
  // lower half
  gemm_f64(ctx, chi, dc, chi, 1.0, rowmajor(Cp(2), chi), rowmajor(Tp(2), dc), 0.0,
           out_rowmajor(sm1.d(), dc));                              // C3 T3 [h][x,c]
  gemm_f64(ctx, dc, chi, chi, 1.0, rowmajor(sm1.d(), chi), rowmajor(Cp(3), chi), 0.0,
           out_rowmajor(sm3.d(), chi));                             // [h,x][d']
  gemm_f64(ctx, dc, dc, chi, 1.0, rowmajor(sm3.d(), chi), rowmajor(Tp(3), dc), 0.0,
           out_rowmajor(t1.d(), dc));                               // [h,x][l,a]
  const int p3012[4] = {3, 0, 1, 2};
  permute(ctx, t1.d(), Lt.d(), 4, d4, p3012);                       // [a,h,x,l]
  // FP64 in every precision mode: the ring is contracted once per observable,
  // outside the sweeps, and its rounding is what kappa's error would follow
  gemm_f64(ctx, d * d, d * d, chi * chi, 1.0, rowmajor(U.d(), chi * chi), rowmajor(Lt.d(), d * d),
           0.0, out_rowmajor(t2.d(), d * d));  // [u,r][x,l]
  const long long f4[4] = {d, d, d, d};
  const int p0321[4] = {0, 3, 2, 1};
  permute(ctx, t2.d(), E.d(), 4, f4, p0321);                        // [u,l,x,r]
  e_valid = true;
}

// kappa = Z_site Z_0 / (Z_row Z_col) (scale-free in every tensor).
double Env::kappa() {
  ring();
  const int dc = d * chi;
  double* sc = scal.d();
  dot(ctx, E.d(), arot[0].d(), (size_t)d * d * d * d, sc + 1);           // Z_site
  // Z_row = sum (C1 T1 C2)[a,m,e] (C3 T3 C4)[e,m,a]
  gemm_f64(ctx, chi, dc, chi, 1.0, rowmajor(Cp(0), chi), rowmajor(Tp(0), dc), 0.0,
           out_rowmajor(sm1.d(), dc));
  gemm_f64(ctx, dc, chi, chi, 1.0, rowmajor(sm1.d(), chi), rowmajor(Cp(1), chi), 0.0,
           out_rowmajor(sm2.d(), chi));                                    // (C1 T1 C2)[a,m,e]
  gemm_f64(ctx, chi, dc, chi, 1.0, rowmajor(Cp(2), chi), rowmajor(Tp(2), dc), 0.0,
           out_rowmajor(sm1.d(), dc));
  gemm_f64(ctx, dc, chi, chi, 1.0, rowmajor(sm1.d(), chi), rowmajor(Cp(3), chi), 0.0,
           out_rowmajor(sm3.d(), chi));                                    // (C3 T3 C4)[e,m,a]
  const long long g3[3] = {chi, d, chi};
  const int p210[3] = {2, 1, 0};
  permute(ctx, sm3.d(), sm1.d(), 3, g3, p210);
  dot(ctx, sm2.d(), sm1.d(), (size_t)chi * d * chi, sc + 3);
  // Z_0 = Tr(C1 C2 C3 C4) = <C1 C2, (C3 C4)^T>
  gemm_f64(ctx, chi, chi, chi, 1.0, rowmajor(Cp(0), chi), rowmajor(Cp(1), chi), 0.0,
           out_rowmajor(sm1.d(), chi));                                    // C1 C2 [a][e]
  gemm_f64(ctx, chi, chi, chi, 1.0, rowmajor(Cp(2), chi), rowmajor(Cp(3), chi), 0.0,
           out_rowmajor(sm2.d(), chi));                                    // C3 C4 [h][d]
  const long long g2[2] = {chi, chi};
  const int p10[2] = {1, 0};
  permute(ctx, sm2.d(), sm3.d(), 2, g2, p10);                              // [d][h]
  dot(ctx, sm1.d(), sm3.d(), (size_t)chi * chi, sc + 2);
  // Z_col = sum (C1 C2 T2)[a,r,h] (C3 C4 T4)[h,r,a]
  gemm_f64(ctx, chi, dc, chi, 1.0, rowmajor(sm1.d(), chi), rowmajor(Tp(1), dc), 0.0,
           out_rowmajor(t1.d(), dc));                                      // [a][r,h]
  gemm_f64(ctx, chi, dc, chi, 1.0, rowmajor(sm2.d(), chi), rowmajor(Tp(3), dc), 0.0,
           out_rowmajor(t2.d(), dc));                                      // [h][r,a]
  permute(ctx, t2.d(), sm1.d(), 3, g3, p210);                              // [a][r][h]
  dot(ctx, t1.d(), sm1.d(), (size_t)chi * d * chi, sc + 4);
  double z[5];
  CTM_HIP(hipMemcpyAsync(z, sc, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  return z[1] * z[2] / (z[3] * z[4]);
}

void Env::log_z(double* log_abs, double* sign) {
  ring();
  dot(ctx, E.d(), arot[0].d(), (size_t)d * d * d * d, scal.d() + 1);
  double z = 0.0, hl[8];
  CTM_HIP(hipMemcpyAsync(&z, scal.d() + 1, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipMemcpyAsync(hl, logs.d(), 8 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  double acc = std::log(std::fabs(z));
  for (int i = 0; i < 8; ++i) acc += hl[i];
  *log_abs = acc;
  *sign = (z > 0) ? 1.0 : (z < 0 ? -1.0 : 0.0);
}

// Bond metric: E / <E, a>; for a purification reordered to (ket legs, bra legs).
void Env::bond_metric(double* out, size_t len) {
  const size_t d4 = (size_t)d * d * d * d;
  CTM_REQUIRE(len == d4, "bond_metric: len must be D^8 (purification) or d^4 (tensor)");
  ring();
  dot(ctx, E.d(), arot[0].d(), d4, scal.d() + 1);
  double z = 0.0;
  const double* src = E.d();
  if (D > 0) {
    const long long dd[8] = {D, D, D, D, D, D, D, D};
    const int pp[8] = {0, 2, 4, 6, 1, 3, 5, 7};
    permute(ctx, E.d(), E8.d(), 8, dd, pp);
    src = E8.d();
  }
  CTM_HIP(hipMemcpyAsync(&z, scal.d() + 1, sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipMemcpyAsync(out, src, d4 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  CTM_REQUIRE(z != 0.0, "bond_metric: <E, a> vanishes");
  const double inv = 1.0 / z;
  for (size_t i = 0; i < d4; ++i) out[i] *= inv;
}

void Env::ring_ket_bra_dev(double* out) {
  CTM_REQUIRE(D > 0, "ring_ket_bra_dev needs a purification environment");
  ring();
  const long long dd[8] = {D, D, D, D, D, D, D, D};
  const int pp[8] = {0, 2, 4, 6, 1, 3, 5, 7};
  permute(ctx, E.d(), out, 8, dd, pp);
}

// The operator on the composite's physical index p = (sA, aA, sB, aB): op
// itself (op_dim 16) or op on (sA, sB) times the identity on the ancillas
// (op_dim 4); O and I16 are 16 x 16 row-major.
static void composite_operator(const double* op, int op_dim, double* O, double* I16) {
  CTM_REQUIRE(op_dim == 4 || op_dim == 16, "op_dim must be 4 or 16");
  for (int i = 0; i < 256; ++i) { O[i] = 0.0; I16[i] = 0.0; }
  if (op_dim == 16) {
    std::memcpy(O, op, 256 * sizeof(double));
  } else {
    // O[(sA aA sB aB),(sA' aA' sB' aB')] = op[(sA sB),(sA' sB')] d_aA d_aB
    for (int sA = 0; sA < 2; ++sA) for (int aA = 0; aA < 2; ++aA)
    for (int sB = 0; sB < 2; ++sB) for (int aB = 0; aB < 2; ++aB)
    for (int tA = 0; tA < 2; ++tA) for (int tB = 0; tB < 2; ++tB) {
      const int p = ((sA * 2 + aA) * 2 + sB) * 2 + aB;
      const int q = ((tA * 2 + aA) * 2 + tB) * 2 + aB;
      O[p * 16 + q] = op[(sA * 2 + sB) * 4 + (tA * 2 + tB)];
    }
  }
  for (int i = 0; i < 16; ++i) I16[i * 16 + i] = 1.0;
}

// <O> = sum_pq O[p][q] rho[q][p] / tr(rho) from the 16 x 16 matrix
// rho[q][p] = sum K[q,ket] E8[ket,bra] K[p,bra], with F (D^4 x 16), rhoT,
// the operator and the identity in the given device buffers.
double Env::expect_from_ring(const double* O, const double* I16, double* F, double* rhoT,
                             double* dO, double* dI) {
  const long long dd[8] = {D, D, D, D, D, D, D, D};
  const int pp[8] = {0, 2, 4, 6, 1, 3, 5, 7};
  permute(ctx, E.d(), E8.d(), 8, dd, pp);
  const int D4 = D * D * D * D;
  // F[ket][p] = sum_bra E8[ket][bra] K[p][bra];  rho^T[p][q] = sum_ket F[ket][p] K[q][ket]
  gemm_f64(ctx, D4, 16, D4, 1.0, rowmajor(E8.d(), D4), colmajor(Kc.d(), D4), 0.0,
           out_rowmajor(F, 16));
  gemm_f64(ctx, 16, 16, D4, 1.0, colmajor(F, 16), colmajor(Kc.d(), D4), 0.0,
           out_rowmajor(rhoT, 16));  // rhoT[p][q] = rho[q][p]
  CTM_HIP(hipMemcpyAsync(dO, O, 256 * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  CTM_HIP(hipMemcpyAsync(dI, I16, 256 * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  dot(ctx, dO, rhoT, 256, scal.d() + 6);
  dot(ctx, dI, rhoT, 256, scal.d() + 7);
  CTM_HIP(hipMemcpyAsync(hres, scal.d() + 6, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  return hres[0] / hres[1];
}

double Env::expect_op(const double* op, int op_dim) {
  CTM_REQUIRE(D > 0, "ctm_expect needs a purification environment");
  double O[256], I16[256];
  composite_operator(op, op_dim, O, I16);
  ring();
  const int D4 = D * D * D * D;
  DevBuf F((size_t)D4 * 16 * sizeof(double)), rhoT(256 * sizeof(double));
  DevBuf dO(256 * sizeof(double)), dI(256 * sizeof(double));
  return expect_from_ring(O, I16, F.d(), rhoT.d(), dO.d(), dI.d());
}

size_t Env::expect_scratch_doubles() const {
  const size_t D4 = (size_t)D * D * D * D;
  return 16 * D4 + 3 * 256 + kRedScratchDoubles;
}

double Env::expect_op_fixed(const double* op, int op_dim, double* scratch, size_t scratch_doubles) {
  CTM_REQUIRE(D > 0, "ctm_expect_noalloc needs a purification environment");
  CTM_REQUIRE(e_valid, "ctm_expect_noalloc: the ring of this environment is not current (run "
                       "ctm_norm, ctm_expect or ctm_bond_metric once after the last sweep)");
  double O[256], I16[256];
  composite_operator(op, op_dim, O, I16);
  const size_t D4 = (size_t)D * D * D * D;
  const size_t fixed = expect_scratch_doubles();
  CTM_REQUIRE(fixed < scratch_doubles, "ctm_expect_noalloc: D is beyond the fixed scratch");
  double* F = scratch;
  double* rhoT = F + 16 * D4;
  double* dO = rhoT + 256;
  double* dI = dO + 256;
  double* red = dI + 256;
  // the rest takes the split-K partial sums of the two products
  struct Fixed {
    Context& c;
    bool timing;
    Fixed(Context& cc, double* red, double* part, size_t bytes) : c(cc), timing(cc.timing) {
      c.fixed_red = red;
      c.fixed_splitk = part;
      c.fixed_splitk_bytes = bytes;
      c.timing = false;  // per-launch events are not created either
    }
    ~Fixed() {
      c.fixed_red = nullptr;
      c.fixed_splitk = nullptr;
      c.fixed_splitk_bytes = 0;
      c.timing = timing;
    }
  } guard(ctx, red, scratch + fixed, (scratch_doubles - fixed) * sizeof(double));
  return expect_from_ring(O, I16, F, rhoT, dO, dI);
}

double Env::expect_tensor(const double* a_imp) {
  const size_t d4 = (size_t)d * d * d * d;
  ring();
  DevBuf da(d4 * sizeof(double));
  CTM_HIP(hipMemcpyAsync(da.p, a_imp, d4 * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  dot(ctx, E.d(), da.d(), d4, scal.d() + 6);
  dot(ctx, E.d(), arot[0].d(), d4, scal.d() + 7);
  double r[2];
  CTM_HIP(hipMemcpyAsync(r, scal.d() + 6, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  return r[0] / r[1];
}

void Env::corner_spectra(double* out, size_t len) {
  CTM_REQUIRE(len == 4ull * chi, "corner_spectra: len must be 4 chi");
  int* err = (int*)iflags.p + 1;
  jacobi_svd(ctx, Call.d(), chi, nullptr, spec_s.d(), nullptr, err, 4, (long long)chi * chi, chi);
  CTM_HIP(hipMemcpyAsync(out, spec_s.d(), len * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
  check_flags("ctm_corner_spectra");
  for (int c = 0; c < 4; ++c) {
    double s2 = 0.0;
    for (int j = 0; j < chi; ++j) s2 += out[c * chi + j] * out[c * chi + j];
    const double inv = s2 > 0.0 ? 1.0 / std::sqrt(s2) : 0.0;
    for (int j = 0; j < chi; ++j) out[c * chi + j] *= inv;
  }
}

void Env::get(double* C, double* T, double* hl) {
  if (C) CTM_HIP(hipMemcpyAsync(C, Call.p, Call.bytes, hipMemcpyDeviceToHost, ctx.stream));
  if (T) CTM_HIP(hipMemcpyAsync(T, Tall.p, Tall.bytes, hipMemcpyDeviceToHost, ctx.stream));
  if (hl) CTM_HIP(hipMemcpyAsync(hl, logs.p, 8 * sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  CTM_HIP(hipStreamSynchronize(ctx.stream));
}

void Env::set(const double* C, const double* T, const double* hl) {
  drop_graph();
  CTM_HIP(hipMemcpyAsync(Call.p, C, Call.bytes, hipMemcpyHostToDevice, ctx.stream));
  CTM_HIP(hipMemcpyAsync(Tall.p, T, Tall.bytes, hipMemcpyHostToDevice, ctx.stream));
  CTM_HIP(hipMemcpyAsync(logs.p, hl, 8 * sizeof(double), hipMemcpyHostToDevice, ctx.stream));
  for (int i = 0; i < 4; ++i) { qvalid[i] = false; warm_ok[i] = false; }
  e_valid = false;
  reset_spectra();
  CTM_HIP(hipStreamSynchronize(ctx.stream));
}

}  // namespace ctm
