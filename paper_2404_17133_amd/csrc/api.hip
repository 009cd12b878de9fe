// C ABI of the library (declarations and contracts in include/rid.h).
// Every entry point validates its arguments, sets the context's device,
// converts internal errors into status codes and never lets an exception
// cross the boundary.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "auxint.hpp"
#include "core.hpp"
#include "engine.hpp"
#include "server.hpp"

namespace {

thread_local std::string g_create_error;

void set_error(rid_context* ctx, const std::string& msg) {
  if (ctx)
    ctx->last_error = msg;
  else
    g_create_error = msg;
}

template <typename F>
rid_status guarded(rid_context* ctx, F&& f) {
  try {
    return f();
  } catch (const rid::Error& e) {
    set_error(ctx, e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error(ctx, "host allocation failed");
    return RID_ERR_NO_MEMORY;
  } catch (const std::exception& e) {
    set_error(ctx, e.what());
    return RID_ERR_INTERNAL;
  } catch (...) {
    set_error(ctx, "unknown internal error");
    return RID_ERR_INTERNAL;
  }
}

void use_device(rid_context* ctx) { RID_HIP(hipSetDevice(ctx->device)); }

// Fixed device scratch of rid_apply_operator_noalloc.  In host code the
// array's name stands for a host-side shadow, not a device address: the
// device address of each GPU's copy is looked up once per device (in
// rid_context_create, with that device current) and only that address is
// ever handed to kernels.
__device__ __align__(256) unsigned char scratch[RID_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (the device must be current).
void* scratch_for_device(int device) {
  RID_CHECK(device >= 0 && device < kMaxDevices, RID_ERR_NO_DEVICE, "device ordinal above the library's limit");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    RID_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    RID_CHECK(ptr != nullptr, RID_ERR_HIP, "no device address for the fixed scratch");
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

const char* rid_status_string(rid_status s) {
  switch (s) {
    case RID_OK: return "ok";
    case RID_WARN_NOT_CONVERGED: return "not converged (outputs hold the last iterate)";
    case RID_ERR_INVALID_ARG: return "invalid argument";
    case RID_ERR_SHAPE: return "invalid shape";
    case RID_ERR_DTYPE: return "unsupported dtype";
    case RID_ERR_NO_MEMORY: return "out of device memory";
    case RID_ERR_HIP: return "HIP runtime error";
    case RID_ERR_INDEFINITE: return "A-B not positive definite";
    case RID_ERR_BREAKDOWN: return "subspace breakdown";
    case RID_ERR_NEAR_SINGULAR: return "frequency too close to a pole";
    case RID_ERR_NO_DEVICE: return "no usable gfx950 device";
    case RID_ERR_INTERNAL: return "internal error";
    case RID_ERR_CANCELLED: return "cancelled";
    case RID_ERR_TIMEOUT: return "timed out";
    case RID_ERR_PENDING: return "pending";
    default: return "unknown status";
  }
}

const char* rid_last_error(const rid_context* ctx) {
  return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

void rid_solve_opts_default(rid_solve_opts* o) {
  if (!o) return;
  o->precond = RID_PRECOND_RIS;
  o->precision = RID_PRECISION_FP64;
  o->tol = 1e-5;
  o->max_iter = 100;
  o->n_extra_init = -1;
  o->inner_tol = 1e-2;
  o->inner_max_iter = 20;
  o->init_tol = 1e-3;
  o->init_max_iter = 20;
  o->m_max = 0;
  o->guess_dev = nullptr;
  o->n_guess = 0;
  o->graphs = 0;
}

rid_status rid_context_create(int32_t device, void* hip_stream, const rid_allocator* alloc, rid_context** out) {
  return guarded(nullptr, [&]() -> rid_status {
    RID_CHECK(out != nullptr, RID_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    RID_CHECK(alloc && alloc->alloc && alloc->free, RID_ERR_INVALID_ARG,
              "an allocator with alloc and free callbacks is required (the library allocates device memory only "
              "through it)");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
      (void)hipGetLastError();
      throw rid::Error(RID_ERR_NO_DEVICE, "no HIP device visible");
    }
    RID_CHECK(device >= 0 && device < n, RID_ERR_NO_DEVICE, "device ordinal out of range");
    hipDeviceProp_t prop;
    RID_HIP(hipGetDeviceProperties(&prop, device));
    RID_CHECK(std::strncmp(prop.gcnArchName, "gfx950", 6) == 0, RID_ERR_NO_DEVICE,
              std::string("library built for gfx950, device is ") + prop.gcnArchName);
    RID_HIP(hipSetDevice(device));
    void* scr = scratch_for_device(device);
    rid_context* c = new rid_context();
    c->device = device;
    c->scratch = scr;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->alloc = *alloc;
    *out = c;
    return RID_OK;
  });
}

rid_status rid_context_destroy(rid_context* ctx) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return RID_OK;
}

rid_status rid_problem_create(rid_context* ctx, const rid_problem_desc* d, rid_problem** out) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(d && out, RID_ERR_INVALID_ARG, "desc or out is NULL");
    *out = nullptr;
    RID_CHECK(d->no >= 1 && d->nv >= 1 && d->naux >= 1, RID_ERR_SHAPE, "no, nv and naux must be >= 1");
    RID_CHECK((long)d->no * d->nv <= (1L << 28), RID_ERR_SHAPE, "no*nv too large");
    RID_CHECK(d->naux_ris >= 0 && d->naux_ris_k >= 0 && d->naux_ris_k <= d->naux_ris, RID_ERR_SHAPE,
              "need 0 <= naux_ris_k <= naux_ris");
    RID_CHECK(d->b_dtype == RID_F64 || d->b_dtype == RID_F32, RID_ERR_DTYPE, "tensors must be FP64 or FP32");
    RID_CHECK(d->eps_occ_host && d->eps_vir_host && d->b_ia_dev && d->b_ij_dev && d->b_ab_dev, RID_ERR_INVALID_ARG,
              "null tensor or energy pointer");
    if (d->naux_ris > 0) {
      RID_CHECK(d->bris_dtype == RID_F64 || d->bris_dtype == RID_F32, RID_ERR_DTYPE,
                "ris tensors must be FP64 or FP32");
      RID_CHECK(d->bris_ia_dev && d->bris_ij_dev && d->bris_ab_dev, RID_ERR_INVALID_ARG, "null ris tensor pointer");
    }
    RID_CHECK(std::isfinite(d->a_x), RID_ERR_INVALID_ARG, "a_x must be finite");
    RID_CHECK(std::isfinite(d->b_x), RID_ERR_INVALID_ARG, "b_x must be finite");
    RID_CHECK(d->naux_lr >= 0 && d->naux_ris_lr >= 0, RID_ERR_SHAPE, "naux_lr and naux_ris_lr must be >= 0");
    if (d->naux_lr > 0)
      RID_CHECK(d->blr_ia_dev && d->blr_ij_dev && d->blr_ab_dev, RID_ERR_INVALID_ARG, "null long-range tensor");
    if (d->naux_ris_lr > 0)
      RID_CHECK(d->naux_ris > 0 && d->brislr_ia_dev && d->brislr_ij_dev && d->brislr_ab_dev, RID_ERR_INVALID_ARG,
                "null long-range ris tensor (or no ris tensor)");
    for (int i = 0; i < d->no; ++i) RID_CHECK(std::isfinite(d->eps_occ_host[i]), RID_ERR_INVALID_ARG, "eps not finite");
    for (int a = 0; a < d->nv; ++a) RID_CHECK(std::isfinite(d->eps_vir_host[a]), RID_ERR_INVALID_ARG, "eps not finite");
    for (int i = 1; i < d->no; ++i)
      RID_CHECK(d->eps_occ_host[i] >= d->eps_occ_host[i - 1], RID_ERR_INVALID_ARG, "eps_occ not ascending");
    for (int a = 1; a < d->nv; ++a)
      RID_CHECK(d->eps_vir_host[a] >= d->eps_vir_host[a - 1], RID_ERR_INVALID_ARG, "eps_vir not ascending");
    use_device(ctx);
    rid_problem* P = new rid_problem(ctx);
    try {
      P->no = d->no;
      P->nv = d->nv;
      P->naux = d->naux;
      P->naux_ris = d->naux_ris;
      P->naux_ris_k = d->naux_ris_k;
      P->a_x = d->a_x;
      P->t_cut = d->t_cut_ha;
      P->eps_occ.assign(d->eps_occ_host, d->eps_occ_host + d->no);
      P->eps_vir.assign(d->eps_vir_host, d->eps_vir_host + d->nv);
      P->b_dt = d->b_dtype;
      if (d->b_dtype == RID_F64) {
        P->b_ia = static_cast<const double*>(d->b_ia_dev);
        P->b_ij = static_cast<const double*>(d->b_ij_dev);
        P->b_ab = static_cast<const double*>(d->b_ab_dev);
      } else {
        P->b_ia_f = static_cast<const float*>(d->b_ia_dev);
        P->b_ij_f = static_cast<const float*>(d->b_ij_dev);
        P->b_ab_f = static_cast<const float*>(d->b_ab_dev);
      }
      if (d->naux_ris > 0) {
        P->bris_dt = d->bris_dtype;
        if (d->bris_dtype == RID_F64) {
          P->bris_ia = static_cast<const double*>(d->bris_ia_dev);
          P->bris_ij = static_cast<const double*>(d->bris_ij_dev);
          P->bris_ab = static_cast<const double*>(d->bris_ab_dev);
        } else {
          P->bris_ia_f = static_cast<const float*>(d->bris_ia_dev);
          P->bris_ij_f = static_cast<const float*>(d->bris_ij_dev);
          P->bris_ab_f = static_cast<const float*>(d->bris_ab_dev);
        }
      }
      P->b_x = d->b_x;
      auto lend = [](rid::LrSet& L, int rows, int dt, const void* ia, const void* ij, const void* ab) {
        L.rows = rows;
        L.dt = dt;
        if (rows <= 0) return;
        if (dt == RID_F64) {
          L.ia = static_cast<const double*>(ia);
          L.ij = static_cast<const double*>(ij);
          L.ab = static_cast<const double*>(ab);
        } else {
          L.ia_f = static_cast<const float*>(ia);
          L.ij_f = static_cast<const float*>(ij);
          L.ab_f = static_cast<const float*>(ab);
        }
      };
      lend(P->lr, d->naux_lr, d->b_dtype, d->blr_ia_dev, d->blr_ij_dev, d->blr_ab_dev);
      lend(P->rislr, d->naux_ris_lr, d->bris_dtype, d->brislr_ia_dev, d->brislr_ij_dev, d->brislr_ab_dev);
      // exchange window of the ris model (energies sorted)
      const double homo = P->eps_occ.back(), lumo = P->eps_vir.front();
      if (!(d->t_cut_ha > 0.0) || !std::isfinite(d->t_cut_ha)) {
        P->i0 = 0;
        P->nv_act = P->nv;
      } else {
        P->nv_act = (int)std::count_if(P->eps_vir.begin(), P->eps_vir.end(),
                                       [&](double e) { return e <= homo + d->t_cut_ha; });
        P->i0 = (int)std::count_if(P->eps_occ.begin(), P->eps_occ.end(),
                                   [&](double e) { return e < lumo - d->t_cut_ha; });
      }
      const long n = P->n();
      std::vector<double> de(n);
      double dmin = INFINITY;
      for (int i = 0; i < P->no; ++i)
        for (int a = 0; a < P->nv; ++a) {
          de[(long)i * P->nv + a] = P->eps_vir[a] - P->eps_occ[i];
          dmin = std::min(dmin, de[(long)i * P->nv + a]);
        }
      RID_CHECK(dmin > 0.0, RID_ERR_INVALID_ARG, "orbital energy differences must be positive");
      P->de_min = dmin;
      P->de.ensure(sizeof(double) * n);
      RID_HIP(hipMemcpyAsync(P->de.p, de.data(), sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
      RID_HIP(hipStreamSynchronize(ctx->stream));
    } catch (...) {
      delete P;
      throw;
    }
    *out = P;
    return RID_OK;
  });
}

rid_status rid_problem_destroy(rid_problem* prob) {
  if (!prob) return RID_ERR_INVALID_ARG;
  (void)hipSetDevice(prob->ctx->device);
  delete prob;
  return RID_OK;
}

rid_status rid_problem_footprint(const rid_problem* prob, uint64_t* bytes) {
  if (!prob || !bytes) return RID_ERR_INVALID_ARG;
  *bytes = prob->footprint();
  return RID_OK;
}

rid_status rid_problem_window(const rid_problem* prob, int32_t* i0, int32_t* nv_act) {
  if (!prob || !i0 || !nv_act) return RID_ERR_INVALID_ARG;
  *i0 = prob->i0;
  *nv_act = prob->nv_act;
  return RID_OK;
}

rid_status rid_apply_operator(rid_problem* prob, int32_t op, int32_t precision, int32_t nvec, const double* x_dev,
                              double* y_dev, double* y2_dev) {
  if (!prob) return RID_ERR_INVALID_ARG;
  rid_context* ctx = prob->ctx;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(op >= RID_OP_A && op <= RID_OP_TPM, RID_ERR_INVALID_ARG, "unknown operator");
    RID_CHECK(precision >= RID_F64 && precision <= RID_BF16, RID_ERR_INVALID_ARG, "unknown precision");
    RID_CHECK(nvec >= 0, RID_ERR_SHAPE, "nvec must be >= 0");
    if (nvec == 0) return RID_OK;
    RID_CHECK(x_dev && y_dev, RID_ERR_INVALID_ARG, "null vector pointer");
    const bool pair = op == RID_OP_APB_AMB || op == RID_OP_TPM;
    RID_CHECK(!pair || y2_dev, RID_ERR_INVALID_ARG, "pair operators need y2");
    const int kind = op == RID_OP_A ? rid::OPK_A : op == RID_OP_APB_AMB ? rid::OPK_PAIR
                   : op == RID_OP_T ? rid::OPK_T : rid::OPK_TPAIR;
    const int prec = precision == RID_F64 ? rid::PREC_F64 : precision == RID_F32 ? rid::PREC_F32 : rid::PREC_BF16;
    use_device(ctx);
    rid::apply_operator(prob, kind, prec, nvec, x_dev, y_dev, y2_dev);
    RID_HIP(hipStreamSynchronize(ctx->stream));
    return RID_OK;
  });
}

rid_status rid_apply_operator_noalloc(rid_problem* prob, int32_t op, int32_t precision, int32_t nvec,
                                      const double* x_dev, double* y_dev, double* y2_dev) {
  if (!prob) return RID_ERR_INVALID_ARG;
  rid_context* ctx = prob->ctx;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(op >= RID_OP_A && op <= RID_OP_TPM, RID_ERR_INVALID_ARG, "unknown operator");
    RID_CHECK(precision >= RID_F64 && precision <= RID_BF16, RID_ERR_INVALID_ARG, "unknown precision");
    RID_CHECK(nvec >= 0, RID_ERR_SHAPE, "nvec must be >= 0");
    if (nvec == 0) return RID_OK;
    RID_CHECK(x_dev && y_dev, RID_ERR_INVALID_ARG, "null vector pointer");
    const bool pair = op == RID_OP_APB_AMB || op == RID_OP_TPM;
    RID_CHECK(!pair || y2_dev, RID_ERR_INVALID_ARG, "pair operators need y2");
    RID_CHECK(ctx->scratch != nullptr, RID_ERR_INTERNAL, "fixed scratch not set up");
    const int kind = op == RID_OP_A ? rid::OPK_A : op == RID_OP_APB_AMB ? rid::OPK_PAIR
                   : op == RID_OP_T ? rid::OPK_T : rid::OPK_TPAIR;
    const int prec = precision == RID_F64 ? rid::PREC_F64 : precision == RID_F32 ? rid::PREC_F32 : rid::PREC_BF16;
    use_device(ctx);
    rid::Arena arena;
    arena.base = static_cast<char*>(ctx->scratch);
    arena.cap = RID_NOALLOC_SCRATCH_BYTES;
    // an eighth of the region per exchange chunk, at most 16 partial sums
    const rid::OpLimits lim{(long)(RID_NOALLOC_SCRATCH_BYTES / 8), 16};
    rid::apply_operator_fixed(prob, kind, prec, nvec, x_dev, y_dev, y2_dev, arena, lim);
    RID_HIP(hipGetLastError());
    return RID_OK;
  });
}

rid_status rid_aux_basis_size(const rid_aux_basis_desc* desc, int32_t* naux, int32_t* naux_s) {
  return guarded(nullptr, [&]() -> rid_status {
    RID_CHECK(desc && naux && naux_s, RID_ERR_INVALID_ARG, "null argument");
    int n = 0, ns = 0;
    rid::aux_basis_size(*desc, &n, &ns);
    *naux = n;
    *naux_s = ns;
    return RID_OK;
  });
}

rid_status rid_aux_tensor_build(rid_context* ctx, const rid_aux_basis_desc* desc, double* b_ia_dev, double* b_ij_dev,
                                double* b_ab_dev) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(desc, RID_ERR_INVALID_ARG, "desc is NULL");
    use_device(ctx);
    rid::aux_tensor_build(ctx, *desc, b_ia_dev, b_ij_dev, b_ab_dev);
    return RID_OK;
  });
}

rid_status rid_eigen_solve(rid_problem* prob, const rid_solve_opts* opts, int32_t k, int32_t mode,
                           double* omega_host, double* x_dev, double* y_dev, double* resid_host, rid_stats* stats) {
  if (!prob) return RID_ERR_INVALID_ARG;
  rid_context* ctx = prob->ctx;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(opts && omega_host, RID_ERR_INVALID_ARG, "opts or omega_host is NULL");
    use_device(ctx);
    rid::SolveStats st;
    rid_status s = rid::eigen_solve(prob, *opts, k, mode, omega_host, x_dev, y_dev, resid_host, st);
    fill_stats(stats, st);
    if (s == RID_WARN_NOT_CONVERGED) set_error(ctx, "maximum number of iterations reached");
    return s;
  });
}

rid_status rid_response_solve(rid_problem* prob, const rid_solve_opts* opts, int32_t nrhs, const double* p_dev,
                              int32_t nfreq, const double* omega_host, double* alpha_host, double* u_dev,
                              double* resid_host, rid_stats* stats) {
  if (!prob) return RID_ERR_INVALID_ARG;
  rid_context* ctx = prob->ctx;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(opts, RID_ERR_INVALID_ARG, "opts is NULL");
    use_device(ctx);
    rid::SolveStats st;
    rid_status s = rid::response_solve(prob, *opts, nrhs, p_dev, nfreq, omega_host, alpha_host, u_dev, resid_host, st);
    fill_stats(stats, st);
    if (s == RID_WARN_NOT_CONVERGED) set_error(ctx, "maximum number of iterations reached");
    return s;
  });
}

rid_status rid_profile_enable(rid_context* ctx, int32_t on) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    use_device(ctx);
    RID_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    ctx->prof.on = on != 0;
    return RID_OK;
  });
}

rid_status rid_tune_save(rid_context* ctx, const char* path, int32_t* count) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(path, RID_ERR_INVALID_ARG, "path is NULL");
    const int n = rid::tune_save(ctx, path);
    if (count) *count = n;
    return RID_OK;
  });
}

rid_status rid_tune_load(rid_context* ctx, const char* path, int32_t* count) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(path, RID_ERR_INVALID_ARG, "path is NULL");
    const int n = rid::tune_load(ctx, path);
    if (count) *count = n;
    return RID_OK;
  });
}

rid_status rid_profile_only(rid_context* ctx, const char* family) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(!family || std::strlen(family) < 32, RID_ERR_INVALID_ARG, "family name too long");
    std::lock_guard<std::mutex> g(ctx->prof.mu);
    ctx->prof.only = family ? family : "";
    return RID_OK;
  });
}

rid_status rid_profile_read(rid_context* ctx, rid_kernel_stat* out, int32_t cap, int32_t* n) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(n && (out || cap == 0) && cap >= 0, RID_ERR_INVALID_ARG, "bad output arguments");
    use_device(ctx);
    RID_HIP(hipStreamSynchronize(ctx->stream));
    const auto fams = ctx->prof.take();
    int cnt = 0;
    for (const auto& f : fams) {
      if (cnt < cap) {
        rid_kernel_stat& s = out[cnt];
        std::memset(&s, 0, sizeof(s));
        std::strncpy(s.name, f.first.c_str(), sizeof(s.name) - 1);
        s.launches = f.second.launches;
        s.total_ms = f.second.ms;
        s.flops = f.second.flops;
        s.bytes = f.second.bytes;
      }
      ++cnt;
    }
    *n = cnt;
    return RID_OK;
  });
}

rid_status rid_batch_solve(rid_context* ctx, int32_t n, rid_problem* const* probs, const rid_request* reqs,
                           rid_result* results) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(n >= 0, RID_ERR_SHAPE, "n must be >= 0");
    if (n == 0) return RID_OK;
    RID_CHECK(probs && reqs && results, RID_ERR_INVALID_ARG, "null array");
    for (int i = 0; i < n; ++i) {
      RID_CHECK(probs[i] && probs[i]->ctx == ctx, RID_ERR_INVALID_ARG, "problem from another context");
      RID_CHECK(reqs[i].kind == 0 || reqs[i].kind == 1, RID_ERR_INVALID_ARG, "bad request kind");
    }
    use_device(ctx);
    return rid::batch_run(ctx, n, probs, reqs, results);
  });
}

rid_status rid_request_footprint(const rid_problem* prob, const rid_request* req, uint64_t* bytes) {
  if (!prob || !req || !bytes) return RID_ERR_INVALID_ARG;
  if (req->kind != 0 && req->kind != 1) return RID_ERR_INVALID_ARG;
  *bytes = rid::request_footprint(prob, *req);
  return RID_OK;
}

rid_status rid_server_create(rid_context* ctx, const rid_server_opts* opts, rid_server** out) {
  if (!ctx) return RID_ERR_INVALID_ARG;
  return guarded(ctx, [&]() -> rid_status {
    RID_CHECK(opts && out, RID_ERR_INVALID_ARG, "opts or out is NULL");
    RID_CHECK(opts->max_slots >= 1, RID_ERR_INVALID_ARG, "max_slots must be >= 1");
    *out = rid::server_create(ctx, *opts);
    return RID_OK;
  });
}

rid_status rid_server_submit(rid_server* srv, rid_problem* prob, const rid_request* req, rid_result* result,
                             uint64_t* ticket) {
  if (!srv) return RID_ERR_INVALID_ARG;
  return rid::server_submit(srv, prob, req, result, ticket);
}

rid_status rid_server_poll(rid_server* srv, uint64_t ticket) {
  if (!srv) return RID_ERR_INVALID_ARG;
  return rid::server_poll(srv, ticket);
}

rid_status rid_server_wait(rid_server* srv, uint64_t ticket, int32_t timeout_ms) {
  if (!srv) return RID_ERR_INVALID_ARG;
  return rid::server_wait(srv, ticket, timeout_ms);
}

rid_status rid_server_cancel(rid_server* srv, uint64_t ticket) {
  if (!srv) return RID_ERR_INVALID_ARG;
  return rid::server_cancel(srv, ticket);
}

rid_status rid_server_destroy(rid_server* srv) {
  if (!srv) return RID_ERR_INVALID_ARG;
  rid::server_destroy(srv);
  return RID_OK;
}

}  // extern "C"
