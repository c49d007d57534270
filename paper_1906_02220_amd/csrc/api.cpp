// C ABI of the CTMRG library (declared in include/ctm.h).  Every entry point
// converts library errors into status codes and records the message on the
// context; no exception crosses the ABI.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <fstream>
#include <memory>
#include <string>
#include <utility>
#include <vector>
#include <cmath>

#include "ctm.h"
#include "adjoint.hpp"
#include "fu.hpp"
#include "transfer.hpp"
#include "engine.hpp"

// The context state is shared by the context handle and every environment
// created on it, so handles may be destroyed in any order.
struct ctm_context {
  std::shared_ptr<ctm::Context> sp;
  ctm::Context& c;
  ctm_context() : sp(std::make_shared<ctm::Context>()), c(*sp) {}
};

struct ctm_env {
  std::shared_ptr<ctm::Context> owner_sp;
  ctm::Context* owner_c;
  std::unique_ptr<ctm::Env> e;
};

namespace ctm {

Context::~Context() {
  (void)hipSetDevice(device);
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto& p : pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : event_pool) (void)hipEventDestroy(e);
  splitk_ws.release();
  scratch_small.release();
  if (own_stream) (void)hipStreamDestroy(own_stream);
}

hipEvent_t Context::get_event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  CTM_HIP(hipEventCreate(&e));
  return e;
}

void Context::resolve_timing() {
  if (pending.empty()) return;
  CTM_HIP(hipStreamSynchronize(stream));
  for (auto& p : pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess && p.cls >= 0 && p.cls < 3) {
      tcls[p.cls].count += 1;
      tcls[p.cls].ms += ms;
      tcls[p.cls].flops += p.flops;
    }
    event_pool.push_back(p.a);
    event_pool.push_back(p.b);
  }
  pending.clear();
}

}  // namespace ctm

// Fixed device scratch of ctm_expect_noalloc: every GPU the library runs on
// holds its own copy of this array until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device when the first context on that device is
// created, with that device current.
static constexpr size_t kNoAllocScratchDoubles = size_t(1) << 20;  // 8 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch (the device must be current).
static double* scratch_address(int device) {
  CTM_REQUIRE(device >= 0 && device < kMaxDevices, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    double* ptr = nullptr;
    CTM_HIP(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
    CTM_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned no address for the scratch");
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}


namespace {

template <typename F>
int guarded_c(ctm::Context* c, F&& f) {
  try {
    f();
    if (c) c->last_error.clear();
    return CTM_OK;
  } catch (const ctm::Error& e) {
    if (c) c->last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (c) c->last_error = "host allocation failed";
    return CTM_ENOMEM;
  } catch (const std::exception& e) {
    if (c) c->last_error = e.what();
    return CTM_EDEVICE;
  }
}

template <typename F>
int guarded(ctm_context* ctx, F&& f) {
  return guarded_c(ctx ? &ctx->c : nullptr, std::forward<F>(f));
}

ctm::EnvOptions to_options(const ctm_opts* o, int d) {
  ctm::EnvOptions r;
  if (!o) return r;
  r.precision = o->precision;
  r.eps_cut = o->eps_cut;
  r.svd_block = o->svd_block;
  r.svd_iters = o->svd_iters;
  r.svd_iters_cold = o->svd_iters_cold;
  r.svd_oversample = o->svd_oversample;
  CTM_REQUIRE(o->svd_oversample >= 0, "svd_oversample must be >= 0");
  CTM_REQUIRE(!(o->svd_tol != o->svd_tol), "svd_tol must not be NaN");
  r.svd_tol = o->svd_tol;
  const int* mo = o->move_order;
  if (mo[0] || mo[1] || mo[2] || mo[3]) {
    int seen = 0;
    for (int i = 0; i < 4; ++i) {
      CTM_REQUIRE(mo[i] >= 0 && mo[i] < 4, "move_order entries must be 0..3");
      seen |= 1 << mo[i];
    }
    CTM_REQUIRE(seen == 15, "move_order must be a permutation of 0, 1, 2, 3");
    for (int i = 0; i < 4; ++i) r.move_order[i] = mo[i];
  }
  r.seed = o->seed;
  if (o->boundary) r.boundary.assign(o->boundary, o->boundary + d);
  return r;
}

void check_precision(int p) {
  if (!ctm::mixed_mode_supported(p)) throw ctm::Error(CTM_EINVAL, "unknown precision mode");
}

// The adjoint differentiates the exact top-chi SVD of every cut matrix, so
// the forward's truncated SVD is iterated to this residual unless the caller
// sets svd_tol (a negative value keeps the fixed iteration counts).
constexpr double kGradSvdTol = 1e-12;

ctm::EnvOptions gradient_options(const ctm_opts* opts, int d) {
  ctm::EnvOptions o = to_options(opts, d);
  check_precision(o.precision);
  CTM_REQUIRE(o.precision == CTM_PREC_F64, "gradients need precision CTM_PREC_F64");
  if (o.svd_tol == 0.0) o.svd_tol = kGradSvdTol;
  return o;
}

}  // namespace

extern "C" {

void ctm_opts_default(ctm_opts* o) {
  if (!o) return;
  o->precision = CTM_PREC_F64;
  o->eps_cut = 1e-12;
  o->svd_block = 0;
  o->svd_iters = 0;
  o->svd_iters_cold = 0;
  o->seed = 0x5eedULL;
  o->boundary = nullptr;
  o->svd_oversample = 0;
  for (int i = 0; i < 4; ++i) o->move_order[i] = 0;
  o->svd_tol = 0.0;
}

int ctm_context_create(int device, ctm_context** out) {
  if (!out) return CTM_EINVAL;
  *out = nullptr;
  ctm_context* ctx = nullptr;
  try {
    ctx = new ctm_context();
  } catch (...) {
    return CTM_ENOMEM;
  }
  const int rc = guarded(ctx, [&] {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
      throw ctm::Error(CTM_EDEVICE, "no HIP device " + std::to_string(device));
    CTM_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    CTM_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      throw ctm::Error(CTM_EDEVICE, std::string("device is ") + prop.gcnArchName + ", need gfx950");
    ctx->c.device = device;
    ctx->c.num_cus = prop.multiProcessorCount;
    CTM_HIP(hipStreamCreateWithFlags(&ctx->c.own_stream, hipStreamNonBlocking));
    ctx->c.stream = ctx->c.own_stream;
    (void)scratch_address(device);  // set-up of the no-allocation entry point
  });
  if (rc != CTM_OK) {
    delete ctx;
    return rc;
  }
  *out = ctx;
  return CTM_OK;
}

void ctm_context_destroy(ctm_context* ctx) {
  // the shared state lives on while environments created on it exist
  delete ctx;
}

const char* ctm_last_error(const ctm_context* ctx) {
  return ctx ? ctx->c.last_error.c_str() : "null context";
}

int ctm_context_set_stream(ctm_context* ctx, void* s) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_HIP(hipStreamSynchronize(ctx->c.stream));
    ctx->c.stream = s ? static_cast<hipStream_t>(s) : ctx->c.own_stream;
  });
}

int ctm_context_set_autotune(ctm_context* ctx, int on) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] { ctx->c.autotune = (on != 0); });
}

int ctm_context_set_graphs(ctm_context* ctx, int on) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] { ctx->c.use_graphs = (on != 0); });
}

// A caller's device array: p must lie in one device allocation of the
// context's device that holds `bytes` from p on.
static void check_device_array(const ctm::Context& c, const void* p, size_t bytes,
                               const char* what) {
  hipPointerAttribute_t attr{};
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) (void)hipGetLastError();
  CTM_REQUIRE(e == hipSuccess && attr.type == hipMemoryTypeDevice,
              std::string(what) + " is not device memory");
  CTM_REQUIRE(attr.device == c.device,
              std::string(what) + " lives on another device than the context's");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    CTM_REQUIRE(false, std::string(what) + ": allocation range unknown");
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  CTM_REQUIRE(q >= b && (size_t)(q - b) + bytes <= size,
              std::string(what) + " is shorter than the tensor it should hold");
}

static ctm_env* new_env(ctm_context* ctx, int d, int chi, const ctm_opts* opts) {
  ctm::EnvOptions o = to_options(opts, d);
  check_precision(o.precision);
  CTM_HIP(hipSetDevice(ctx->c.device));
  auto env = std::make_unique<ctm_env>();
  env->owner_sp = ctx->sp;
  env->owner_c = ctx->sp.get();
  env->e = std::make_unique<ctm::Env>(ctx->c, d, chi, o);
  return env.release();
}

static int init_tensor(ctm_context* ctx, const double* a, int d, int chi, const ctm_opts* opts,
                       ctm_env** out, bool on_device) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_REQUIRE(a && out, "null argument");
    CTM_REQUIRE(d >= 1 && chi >= 1, "d and chi must be >= 1");
    *out = nullptr;
    const size_t d4 = (size_t)d * d * d * d;
    if (on_device) check_device_array(ctx->c, a, d4 * sizeof(double), "a");
    std::unique_ptr<ctm_env> env(new_env(ctx, d, chi, opts));
    ctm::DevBuf da;
    const double* src = a;
    if (!on_device) {
      da.alloc(d4 * sizeof(double));
      CTM_HIP(hipMemcpyAsync(da.p, a, d4 * sizeof(double), hipMemcpyHostToDevice, ctx->c.stream));
      src = da.d();
    }
    env->e->set_site_tensor_dev(src);
    env->e->init_boundary();
    CTM_HIP(hipStreamSynchronize(ctx->c.stream));
    *out = env.release();
  });
}

static int init_purification(ctm_context* ctx, const double* A, const double* B, int D,
                             int D_gamma, int gamma, int chi, const ctm_opts* opts, ctm_env** out,
                             bool on_device) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_REQUIRE(A && B && out, "null argument");
    CTM_REQUIRE(D >= 1 && D_gamma >= 1 && chi >= 1, "D, D_gamma and chi must be >= 1");
    CTM_REQUIRE(gamma >= 0 && gamma <= 2, "gamma must be 0, 1 or 2");
    CTM_REQUIRE(D <= 16, "D above 16 is not supported");
    *out = nullptr;
    const size_t sz = 4ull * D * D * D_gamma;
    if (on_device) {
      check_device_array(ctx->c, A, sz * sizeof(double), "A");
      check_device_array(ctx->c, B, sz * sizeof(double), "B");
    }
    std::unique_ptr<ctm_env> env(new_env(ctx, D * D, chi, opts));
    ctm::DevBuf dA, dB;
    const double *sA = A, *sB = B;
    if (!on_device) {
      dA.alloc(sz * sizeof(double));
      dB.alloc(sz * sizeof(double));
      CTM_HIP(hipMemcpyAsync(dA.p, A, sz * sizeof(double), hipMemcpyHostToDevice, ctx->c.stream));
      CTM_HIP(hipMemcpyAsync(dB.p, B, sz * sizeof(double), hipMemcpyHostToDevice, ctx->c.stream));
      sA = dA.d();
      sB = dB.d();
    }
    env->e->build_purification_dev(sA, sB, D, D_gamma, gamma);
    env->e->init_boundary();
    CTM_HIP(hipStreamSynchronize(ctx->c.stream));
    *out = env.release();
  });
}

int ctm_env_init_tensor(ctm_context* ctx, const double* a, int d, int chi, const ctm_opts* opts,
                        ctm_env** out) {
  return init_tensor(ctx, a, d, chi, opts, out, false);
}

int ctm_env_init_tensor_dev(ctm_context* ctx, const double* a, int d, int chi,
                            const ctm_opts* opts, ctm_env** out) {
  return init_tensor(ctx, a, d, chi, opts, out, true);
}

int ctm_env_init_purification(ctm_context* ctx, const double* A, const double* B, int D,
                              int D_gamma, int gamma, int chi, const ctm_opts* opts,
                              ctm_env** out) {
  return init_purification(ctx, A, B, D, D_gamma, gamma, chi, opts, out, false);
}

int ctm_env_init_purification_dev(ctm_context* ctx, const double* A, const double* B, int D,
                                  int D_gamma, int gamma, int chi, const ctm_opts* opts,
                                  ctm_env** out) {
  return init_purification(ctx, A, B, D, D_gamma, gamma, chi, opts, out, true);
}

void ctm_env_destroy(ctm_env* env) {
  if (!env) return;
  (void)hipSetDevice(env->owner_c->device);
  (void)hipStreamSynchronize(env->owner_c->stream);
  env->e.reset();
  delete env;  // drops the environment's share of the context state
}

int ctm_sweep(ctm_env* env, int max_sweeps, double tol, int* sweeps_done, double* delta) {
  if (!env) return CTM_EINVAL;
  int status = CTM_OK;
  const int rc = guarded_c(env->owner_c, [&] {
    CTM_HIP(hipSetDevice(env->owner_c->device));
    status = env->e->sweep(max_sweeps, tol, sweeps_done, delta);
  });
  if (rc != CTM_OK) return rc;
  if (status != CTM_OK) env->owner_c->last_error = "max_sweeps reached before tol";
  return status;
}

int ctm_sweep_batch(ctm_env* const* envs, int count, int max_sweeps, double tol, int* sweeps_done,
                    double* delta) {
  if (!envs || count < 0) return CTM_EINVAL;
  if (count == 0) return CTM_OK;
  for (int i = 0; i < count; ++i)
    if (!envs[i]) return CTM_EINVAL;
  std::vector<int> done(count, 0), active(count, 1), pending(count, 0);
  std::vector<double> dl(count, INFINITY);
  ctm::Context* errc = envs[0]->owner_c;
  int cur = -1;
  auto drain_all = [&] {
    for (int i = 0; i < count; ++i) {
      (void)hipSetDevice(envs[i]->owner_c->device);
      (void)hipStreamSynchronize(envs[i]->owner_c->stream);
    }
  };
  const int rc = guarded_c(errc, [&] {
    CTM_REQUIRE(max_sweeps >= 0, "max_sweeps must be >= 0");
    for (int i = 0; i < count; ++i)
      for (int j = 0; j < i; ++j)
        CTM_REQUIRE(envs[i] != envs[j], "an environment appears twice in the batch");
    try {
      for (int s = 0; s < max_sweeps; ++s) {
        // enqueue one sweep of every active environment, then collect them:
        // environments on different contexts run concurrently on their streams
        for (int i = 0; i < count; ++i) {
          if (!active[i]) continue;
          cur = i;
          CTM_HIP(hipSetDevice(envs[i]->owner_c->device));
          envs[i]->e->sweep_enqueue();
          pending[i] = 1;
        }
        int left = 0;
        for (int i = 0; i < count; ++i) {
          if (!pending[i]) continue;
          cur = i;
          CTM_HIP(hipSetDevice(envs[i]->owner_c->device));
          CTM_HIP(hipStreamSynchronize(envs[i]->owner_c->stream));
          pending[i] = 0;
          dl[i] = envs[i]->e->sweep_finish("ctm_sweep_batch");
          ++done[i];
          if (tol > 0.0 && dl[i] < tol) active[i] = 0;
          left += active[i];
        }
        if (left == 0) break;
      }
    } catch (const ctm::Error& e) {
      // drain every stream before reporting, so that no work is left in flight
      drain_all();
      throw ctm::Error(e.code, "environment " + std::to_string(cur) + ": " + e.what());
    } catch (...) {
      drain_all();
      throw;
    }
  });
  for (int i = 0; i < count; ++i) {
    if (sweeps_done) sweeps_done[i] = done[i];
    if (delta) delta[i] = dl[i];
  }
  if (rc != CTM_OK) return rc;
  if (tol > 0.0)
    for (int i = 0; i < count; ++i)
      if (!(dl[i] < tol)) {
        errc->last_error = "max_sweeps reached before tol";
        return CTM_ENOTCONV;
      }
  return CTM_OK;
}

namespace {

void fill_info(const ctm::GradStats& g, ctm_grad_info* info) {
  if (!info) return;
  info->moves = g.moves;
  info->cg_iters_max = g.cg_iters_max;
  info->cg_iters_total = g.cg_iters_total;
  info->ms_forward = g.ms_forward;
  info->ms_recompute = g.ms_recompute;
  info->ms_backward = g.ms_backward;
  info->tape_bytes = g.tape_bytes;
  info->checkpoint_bytes = g.checkpoint_bytes;
}

}  // namespace

static int grad_purification(ctm_context* ctx, const double* A, const double* B, int D, int D_gamma,
                             int gamma, int chi, const ctm_opts* opts, int sweeps,
                             int checkpoint_every, const double* op, int op_dim, double w_log_kappa,
                             double w_expect, double* log_kappa, double* expect, double* grad_A,
                             double* grad_B, ctm_grad_info* info, bool on_device) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_REQUIRE(A && B && grad_A && grad_B, "null argument");
    CTM_REQUIRE(D >= 1 && D_gamma >= 1 && chi >= 1, "D, D_gamma and chi must be >= 1");
    CTM_REQUIRE(gamma >= 0 && gamma <= 2, "gamma must be 0, 1 or 2");
    CTM_REQUIRE(D <= 16, "D above 16 is not supported");
    CTM_REQUIRE(sweeps >= 0, "sweeps must be >= 0");
    CTM_REQUIRE(op || w_expect == 0.0, "w_expect needs an operator");
    CTM_REQUIRE(!op || op_dim == 4 || op_dim == 16, "op_dim must be 4 or 16");
    const int d = D * D;
    const size_t sz = 4ull * D * D * D_gamma;
    if (on_device) {
      check_device_array(ctx->c, A, sz * sizeof(double), "A");
      check_device_array(ctx->c, B, sz * sizeof(double), "B");
      check_device_array(ctx->c, grad_A, sz * sizeof(double), "grad_A");
      check_device_array(ctx->c, grad_B, sz * sizeof(double), "grad_B");
    }
    ctm::EnvOptions o = gradient_options(opts, d);
    CTM_HIP(hipSetDevice(ctx->c.device));
    ctm::Env env(ctx->c, d, chi, o);
    // device copies of host inputs (and of the gradients for host outputs)
    ctm::DevBuf dA, dB, gA, gB;
    const double *sA = A, *sB = B;
    double *tA = grad_A, *tB = grad_B;
    if (!on_device) {
      dA.alloc(sz * sizeof(double));
      dB.alloc(sz * sizeof(double));
      gA.alloc(sz * sizeof(double));
      gB.alloc(sz * sizeof(double));
      CTM_HIP(hipMemcpyAsync(dA.p, A, sz * sizeof(double), hipMemcpyHostToDevice, ctx->c.stream));
      CTM_HIP(hipMemcpyAsync(dB.p, B, sz * sizeof(double), hipMemcpyHostToDevice, ctx->c.stream));
      sA = dA.d();
      sB = dB.d();
      tA = gA.d();
      tB = gB.d();
    }
    env.build_purification_dev(sA, sB, D, D_gamma, gamma);
    env.init_boundary();
    ctm::Grad g(env, sweeps, checkpoint_every);
    g.forward();
    double lk = 0.0, ex = 0.0;
    g.seed(w_log_kappa, w_expect, op, op_dim, nullptr, &lk, &ex);
    g.backward();
    g.grad_purification(sA, sB, D, D_gamma, gamma, tA, tB);
    if (!on_device) {
      CTM_HIP(hipMemcpyAsync(grad_A, gA.p, sz * sizeof(double), hipMemcpyDeviceToHost, ctx->c.stream));
      CTM_HIP(hipMemcpyAsync(grad_B, gB.p, sz * sizeof(double), hipMemcpyDeviceToHost, ctx->c.stream));
    }
    CTM_HIP(hipStreamSynchronize(ctx->c.stream));
    if (log_kappa) *log_kappa = lk;
    if (expect) *expect = ex;
    fill_info(g.stats, info);
  });
}

int ctm_grad_purification(ctm_context* ctx, const double* A, const double* B, int D, int D_gamma,
                          int gamma, int chi, const ctm_opts* opts, int sweeps,
                          int checkpoint_every, const double* op, int op_dim,
                          double w_log_kappa, double w_expect, double* log_kappa,
                          double* expect, double* grad_A, double* grad_B, ctm_grad_info* info) {
  return grad_purification(ctx, A, B, D, D_gamma, gamma, chi, opts, sweeps, checkpoint_every, op,
                           op_dim, w_log_kappa, w_expect, log_kappa, expect, grad_A, grad_B, info,
                           false);
}

int ctm_grad_purification_dev(ctm_context* ctx, const double* A, const double* B, int D,
                              int D_gamma, int gamma, int chi, const ctm_opts* opts, int sweeps,
                              int checkpoint_every, const double* op, int op_dim,
                              double w_log_kappa, double w_expect, double* log_kappa,
                              double* expect, double* grad_A, double* grad_B,
                              ctm_grad_info* info) {
  return grad_purification(ctx, A, B, D, D_gamma, gamma, chi, opts, sweeps, checkpoint_every, op,
                           op_dim, w_log_kappa, w_expect, log_kappa, expect, grad_A, grad_B, info,
                           true);
}

static int grad_tensor(ctm_context* ctx, const double* a, int d, int chi, const ctm_opts* opts,
                       int sweeps, int checkpoint_every, const double* a_imp, double w_log_kappa,
                       double w_expect, double* log_kappa, double* expect, double* grad_a,
                       ctm_grad_info* info, bool on_device) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_REQUIRE(a && grad_a, "null argument");
    CTM_REQUIRE(d >= 1 && chi >= 1, "d and chi must be >= 1");
    CTM_REQUIRE(sweeps >= 0, "sweeps must be >= 0");
    CTM_REQUIRE(a_imp || w_expect == 0.0, "w_expect needs an impurity tensor");
    const size_t d4 = (size_t)d * d * d * d;
    if (on_device) {
      check_device_array(ctx->c, a, d4 * sizeof(double), "a");
      check_device_array(ctx->c, grad_a, d4 * sizeof(double), "grad_a");
    }
    ctm::EnvOptions o = gradient_options(opts, d);
    CTM_HIP(hipSetDevice(ctx->c.device));
    ctm::Env env(ctx->c, d, chi, o);
    ctm::DevBuf da, ga;
    const double* sa = a;
    double* ta = grad_a;
    if (!on_device) {
      da.alloc(d4 * sizeof(double));
      ga.alloc(d4 * sizeof(double));
      CTM_HIP(hipMemcpyAsync(da.p, a, d4 * sizeof(double), hipMemcpyHostToDevice, ctx->c.stream));
      sa = da.d();
      ta = ga.d();
    }
    env.set_site_tensor_dev(sa);
    CTM_HIP(hipStreamSynchronize(ctx->c.stream));
    env.init_boundary();
    ctm::Grad g(env, sweeps, checkpoint_every);
    g.forward();
    double lk = 0.0, ex = 0.0;
    g.seed(w_log_kappa, w_expect, nullptr, 0, a_imp, &lk, &ex);
    g.backward();
    g.grad_site(ta);
    if (!on_device)
      CTM_HIP(hipMemcpyAsync(grad_a, ga.p, d4 * sizeof(double), hipMemcpyDeviceToHost, ctx->c.stream));
    CTM_HIP(hipStreamSynchronize(ctx->c.stream));
    if (log_kappa) *log_kappa = lk;
    if (expect) *expect = ex;
    fill_info(g.stats, info);
  });
}

int ctm_grad_tensor(ctm_context* ctx, const double* a, int d, int chi, const ctm_opts* opts,
                    int sweeps, int checkpoint_every, const double* a_imp, double w_log_kappa,
                    double w_expect, double* log_kappa, double* expect, double* grad_a,
                    ctm_grad_info* info) {
  return grad_tensor(ctx, a, d, chi, opts, sweeps, checkpoint_every, a_imp, w_log_kappa, w_expect,
                     log_kappa, expect, grad_a, info, false);
}

int ctm_grad_tensor_dev(ctm_context* ctx, const double* a, int d, int chi, const ctm_opts* opts,
                        int sweeps, int checkpoint_every, const double* a_imp, double w_log_kappa,
                        double w_expect, double* log_kappa, double* expect, double* grad_a,
                        ctm_grad_info* info) {
  return grad_tensor(ctx, a, d, chi, opts, sweeps, checkpoint_every, a_imp, w_log_kappa, w_expect,
                     log_kappa, expect, grad_a, info, true);
}

int ctm_fu_bond_update(ctm_context* ctx, const double* A, const double* B, int D, int gamma,
                       const double* H, double tau, int chi, const ctm_opts* opts, int sweeps,
                       int als_iters, double* A_out, double* B_out, double* errors) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_REQUIRE(A && B && H && A_out && B_out, "null argument");
    CTM_REQUIRE(D >= 1 && D <= 8, "D must be 1..8");
    CTM_REQUIRE(gamma >= 0 && gamma <= 2, "gamma must be 0, 1 or 2");
    CTM_REQUIRE(chi >= 1 && sweeps >= 0 && als_iters >= 0, "chi >= 1, sweeps and als_iters >= 0");
    CTM_REQUIRE(std::isfinite(tau), "tau must be finite");
    ctm::EnvOptions o = to_options(opts, D * D);
    check_precision(o.precision);
    CTM_HIP(hipSetDevice(ctx->c.device));
    ctm::FullUpdate fu(ctx->c, D, gamma);
    fu.run(A, B, H, tau, chi, o, sweeps, als_iters, A_out, B_out, errors);
  });
}

int ctm_fu_trotter_step(ctm_context* ctx, double* A, double* B, int D, const double* H,
                        double dbeta, int chi, const ctm_opts* opts, int sweeps, int als_iters,
                        double* errors) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_REQUIRE(A && B && H, "null argument");
    CTM_REQUIRE(D >= 1 && D <= 8, "D must be 1..8");
    CTM_REQUIRE(chi >= 1 && sweeps >= 0 && als_iters >= 0, "chi >= 1, sweeps and als_iters >= 0");
    CTM_REQUIRE(std::isfinite(dbeta), "dbeta must be finite");
    ctm::EnvOptions o = to_options(opts, D * D);
    check_precision(o.precision);
    CTM_HIP(hipSetDevice(ctx->c.device));
    const size_t sz = 4ull * D * D * D;
    std::vector<double> An(sz), Bn(sz);
    const int seq_gamma[5] = {0, 1, 2, 1, 0};
    const double seq_t[5] = {0.5 * dbeta, 0.5 * dbeta, dbeta, 0.5 * dbeta, 0.5 * dbeta};
    for (int i = 0; i < 5; ++i) {
      const int g = seq_gamma[i];
      ctm::FullUpdate fu(ctx->c, D, g);
      fu.run(A, B, H + 16 * g, seq_t[i], chi, o, sweeps, als_iters, An.data(), Bn.data(),
             errors ? errors + (size_t)i * (als_iters + 1) : nullptr);
      std::memcpy(A, An.data(), sz * sizeof(double));
      std::memcpy(B, Bn.data(), sz * sizeof(double));
    }
  });
}

int ctm_transfer_spectrum(ctm_env* env, int direction, int site, int nev, int krylov, double* re,
                          double* im, double* xi) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(re && im, "null argument");
    CTM_REQUIRE(krylov >= 2 && krylov <= 64, "krylov must be 2..64");
    CTM_REQUIRE(nev >= 1 && nev <= krylov, "nev must be 1..krylov");
    CTM_HIP(hipSetDevice(env->owner_c->device));
    ctm::Transfer tr(*env->e, direction, site != 0);
    std::vector<double> wr(64), wi(64);
    const int k = tr.spectrum(krylov, env->e->opt.seed ^ 0x7a5fULL, wr.data(), wi.data());
    std::vector<int> idx(k);
    for (int i = 0; i < k; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
      return std::hypot(wr[a], wi[a]) > std::hypot(wr[b], wi[b]);
    });
    for (int i = 0; i < nev; ++i) {
      re[i] = i < k ? wr[idx[i]] : 0.0;
      im[i] = i < k ? wi[idx[i]] : 0.0;
    }
    if (xi) {
      const double l1 = k > 0 ? std::hypot(wr[idx[0]], wi[idx[0]]) : 0.0;
      const double l2 = k > 1 ? std::hypot(wr[idx[1]], wi[idx[1]]) : 0.0;
      *xi = (l1 > 0.0 && l2 > 0.0) ? -1.0 / std::log(l2 / l1) : 0.0;
    }
  });
}

int ctm_sweep_batch_grouped(ctm_env* const* envs, int count, int max_sweeps, double tol,
                            int* sweeps_done, double* delta) {
  if (!envs || count < 0) return CTM_EINVAL;
  if (count == 0) return CTM_OK;
  for (int i = 0; i < count; ++i)
    if (!envs[i]) return CTM_EINVAL;
  std::vector<int> done(count, 0), active(count, 1), kind(count, 0);
  std::vector<double> dl(count, INFINITY);
  std::vector<hipEvent_t> ev(count, nullptr);
  hipEvent_t evg = nullptr;
  ctm::Context* gc = envs[0]->owner_c;
  // the grouped products run on a stream of their own (default priority), so
  // that no member's own work sits between two grouped launches
  ctm::Context grp;
  int cur = -1;
  auto drain = [&] {
    for (int i = 0; i < count; ++i) (void)hipStreamSynchronize(envs[i]->owner_c->stream);
    if (grp.stream) (void)hipStreamSynchronize(grp.stream);
  };
  auto destroy_events = [&] {
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
    if (evg) (void)hipEventDestroy(evg);
    std::fill(ev.begin(), ev.end(), nullptr);
    evg = nullptr;
  };
  const int rc = guarded_c(gc, [&] {
    CTM_REQUIRE(max_sweeps >= 0, "max_sweeps must be >= 0");
    for (int i = 0; i < count; ++i) {
      CTM_REQUIRE(envs[i]->owner_c->device == gc->device,
                  "grouped batch: every environment must live on the first one's device");
      for (int j = 0; j < i; ++j)
        CTM_REQUIRE(envs[i] != envs[j], "an environment appears twice in the batch");
    }
    CTM_HIP(hipSetDevice(gc->device));
    grp.device = gc->device;
    grp.num_cus = gc->num_cus;
    CTM_HIP(hipStreamCreateWithFlags(&grp.own_stream, hipStreamNonBlocking));
    grp.stream = grp.own_stream;
    ctm::DevBuf counter;
    counter.alloc(sizeof(int));
    try {
      for (int i = 0; i < count; ++i) CTM_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
      CTM_HIP(hipEventCreateWithFlags(&evg, hipEventDisableTiming));
      std::vector<ctm::GroupProblem> probs(3 * (size_t)count);
      std::vector<ctm::GroupProblem> first[3], second[3];  // by kernel kind 1, 2
      for (int s = 0; s < max_sweeps; ++s) {
        for (int m = 0; m < 4; ++m) {
          // move m of every environment's own sweep order
          for (auto& v : first) v.clear();
          for (auto& v : second) v.clear();
          for (int i = 0; i < count; ++i) {
            if (!active[i]) continue;
            cur = i;
            ctm::Env& e = *envs[i]->e;
            const int k = e.opt.move_order[m];
            e.move_front(k);
            kind[i] = e.cut_products(k, &probs[3 * (size_t)i]);
            if (kind[i] == 0) continue;
            first[kind[i]].push_back(probs[3 * (size_t)i]);
            first[kind[i]].push_back(probs[3 * (size_t)i + 1]);
            second[kind[i]].push_back(probs[3 * (size_t)i + 2]);
            CTM_HIP(hipEventRecord(ev[i], envs[i]->owner_c->stream));
            CTM_HIP(hipStreamWaitEvent(grp.stream, ev[i], 0));
          }
          cur = -1;
          // the half-system products of every grouped environment in one
          // launch per kernel kind, then their cut matrices
          for (int kd = 1; kd <= 2; ++kd)
            if (!first[kd].empty())
              ctm::gemm_grouped(grp, kd, first[kd].data(), (int)first[kd].size(), (int*)counter.p);
          for (int kd = 1; kd <= 2; ++kd)
            if (!second[kd].empty())
              ctm::gemm_grouped(grp, kd, second[kd].data(), (int)second[kd].size(), (int*)counter.p);
          CTM_HIP(hipEventRecord(evg, grp.stream));
          for (int i = 0; i < count; ++i) {
            if (!active[i]) continue;
            cur = i;
            ctm::Env& e = *envs[i]->e;
            const int k = e.opt.move_order[m];
            if (kind[i] == 0) e.move_products(k);
            else CTM_HIP(hipStreamWaitEvent(envs[i]->owner_c->stream, evg, 0));
            e.move_back(k);
          }
        }
        for (int i = 0; i < count; ++i)
          if (active[i]) {
            cur = i;
            envs[i]->e->sweep_tail_eager();
          }
        int left = 0;
        for (int i = 0; i < count; ++i) {
          if (!active[i]) continue;
          cur = i;
          CTM_HIP(hipStreamSynchronize(envs[i]->owner_c->stream));
          dl[i] = envs[i]->e->sweep_finish("ctm_sweep_batch_grouped");
          ++done[i];
          if (tol > 0.0 && dl[i] < tol) active[i] = 0;
          left += active[i];
        }
        if (left == 0) break;
      }
      drain();
    } catch (const ctm::Error& e) {
      drain();
      destroy_events();
      throw ctm::Error(e.code, cur >= 0 ? "environment " + std::to_string(cur) + ": " + e.what()
                                        : std::string(e.what()));
    } catch (...) {
      drain();
      destroy_events();
      throw;
    }
    destroy_events();
  });
  for (int i = 0; i < count; ++i) {
    if (sweeps_done) sweeps_done[i] = done[i];
    if (delta) delta[i] = dl[i];
  }
  if (rc != CTM_OK) return rc;
  if (tol > 0.0)
    for (int i = 0; i < count; ++i)
      if (!(dl[i] < tol)) {
        gc->last_error = "max_sweeps reached before tol";
        return CTM_ENOTCONV;
      }
  return CTM_OK;
}

int ctm_move(ctm_env* env, int direction) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(direction >= 0 && direction <= 3, "direction must be 0..3");
    CTM_HIP(hipSetDevice(env->owner_c->device));
    env->e->move(direction);
  });
}

int ctm_norm(ctm_env* env, double* kappa) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(kappa, "null argument");
    *kappa = env->e->kappa();
  });
}

int ctm_log_z(ctm_env* env, double* log_abs, double* sign) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(log_abs && sign, "null argument");
    env->e->log_z(log_abs, sign);
  });
}

int ctm_bond_metric(ctm_env* env, double* E, size_t len) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(E, "null argument");
    env->e->bond_metric(E, len);
  });
}

int ctm_expect(ctm_env* env, const double* op, int op_dim, double* value) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(op && value, "null argument");
    *value = env->e->expect_op(op, op_dim);
  });
}

int ctm_expect_noalloc(ctm_env* env, const double* op, int op_dim, double* value) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(op && value, "null argument");
    CTM_HIP(hipSetDevice(env->owner_c->device));
    double* ptr = scratch_address(env->owner_c->device);
    *value = env->e->expect_op_fixed(op, op_dim, ptr, kNoAllocScratchDoubles);
  });
}

int ctm_expect_tensor(ctm_env* env, const double* a_imp, double* value) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(a_imp && value, "null argument");
    *value = env->e->expect_tensor(a_imp);
  });
}

int ctm_corner_spectra(ctm_env* env, double* s, size_t len) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(s, "null argument");
    env->e->corner_spectra(s, len);
  });
}

int ctm_env_get(ctm_env* env, double* C, double* T, double* logs) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] { env->e->get(C, T, logs); });
}

int ctm_env_set(ctm_env* env, const double* C, const double* T, const double* logs) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(C && T && logs, "null argument");
    env->e->set(C, T, logs);
  });
}

static const char kMagic[8] = {'C', 'T', 'M', 'E', 'N', 'V', '0', '1'};

int ctm_env_save(ctm_env* env, const char* path) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(path, "null path");
    ctm::Env& e = *env->e;
    std::vector<double> C(4ull * e.chi * e.chi), T(4ull * e.chi * e.d * e.chi), L(8);
    e.get(C.data(), T.data(), L.data());
    std::ofstream f(path, std::ios::binary);
    CTM_REQUIRE(f.good(), std::string("cannot open ") + path);
    const int hdr[4] = {e.chi, e.d, e.D, e.sweeps_done};
    f.write(kMagic, 8);
    f.write(reinterpret_cast<const char*>(hdr), sizeof(hdr));
    f.write(reinterpret_cast<const char*>(L.data()), L.size() * sizeof(double));
    f.write(reinterpret_cast<const char*>(C.data()), C.size() * sizeof(double));
    f.write(reinterpret_cast<const char*>(T.data()), T.size() * sizeof(double));
    CTM_REQUIRE(f.good(), std::string("write failed: ") + path);
  });
}

int ctm_env_load(ctm_env* env, const char* path) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_REQUIRE(path, "null path");
    ctm::Env& e = *env->e;
    std::ifstream f(path, std::ios::binary);
    CTM_REQUIRE(f.good(), std::string("cannot open ") + path);
    char magic[8];
    int hdr[4];
    f.read(magic, 8);
    f.read(reinterpret_cast<char*>(hdr), sizeof(hdr));
    CTM_REQUIRE(f.good() && std::memcmp(magic, kMagic, 8) == 0, "not a checkpoint file");
    CTM_REQUIRE(hdr[0] == e.chi && hdr[1] == e.d && hdr[2] == e.D,
                "checkpoint shape does not match the environment");
    std::vector<double> C(4ull * e.chi * e.chi), T(4ull * e.chi * e.d * e.chi), L(8);
    f.read(reinterpret_cast<char*>(L.data()), L.size() * sizeof(double));
    f.read(reinterpret_cast<char*>(C.data()), C.size() * sizeof(double));
    f.read(reinterpret_cast<char*>(T.data()), T.size() * sizeof(double));
    CTM_REQUIRE(f.good(), "truncated checkpoint file");
    e.set(C.data(), T.data(), L.data());
    e.sweeps_done = hdr[3];
  });
}

int ctm_svd_stats(ctm_env* env, long long* calls, long long* iterations, double* last_residual) {
  if (!env) return CTM_EINVAL;
  return guarded_c(env->owner_c, [&] {
    CTM_HIP(hipSetDevice(env->owner_c->device));
    if (calls) *calls = env->e->svd_calls;
    if (iterations) *iterations = env->e->svd_iterations;
    if (last_residual) *last_residual = env->e->last_svd_residual();
  });
}

int ctm_debug_poison_allocations(int on, int* previous) {
  const int old = ctm::poison_allocations().exchange(on ? 1 : 0);
  if (previous) *previous = old;
  return CTM_OK;
}

int ctm_debug_guard_violations(long long* count) {
  if (!count) return CTM_EINVAL;
  *count = ctm::guard_violations();
  return CTM_OK;
}

int ctm_env_dims(const ctm_env* env, int* chi, int* d, int* D, int* sweeps) {
  if (!env) return CTM_EINVAL;
  if (chi) *chi = env->e->chi;
  if (d) *d = env->e->d;
  if (D) *D = env->e->D;
  if (sweeps) *sweeps = env->e->sweeps_done;
  return CTM_OK;
}

int ctm_timing_enable(ctm_context* ctx, int on) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    ctx->c.resolve_timing();
    ctx->c.timing = (on != 0);
  });
}

int ctm_timing_reset(ctm_context* ctx) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    ctx->c.resolve_timing();
    for (auto& t : ctx->c.tcls) t = ctm::TimingClass();
  });
}

int ctm_timing_get(ctm_context* ctx, int cls, long long* count, double* ms, double* flops) {
  if (!ctx) return CTM_EINVAL;
  return guarded(ctx, [&] {
    CTM_REQUIRE(cls >= 0 && cls < 3, "timing class must be 0, 1 or 2");
    ctx->c.resolve_timing();
    if (count) *count = ctx->c.tcls[cls].count;
    if (ms) *ms = ctx->c.tcls[cls].ms;
    if (flops) *flops = ctx->c.tcls[cls].flops;
  });
}

}  // extern "C"
