// C-ABI entry points (include/bhx.h): argument validation on the host, then
// the batched solver.  Nothing is thrown across this boundary.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "bhx_runtime.h"

using bhx::Resolved;

extern "C" {

void bhx_default_opts(bhx_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = BHX_PREC_FP64;
  o->maxit = 0;
  o->precond = 1;
  o->accurate = 0;
  o->tol_inner = 0.0;
  o->flexible = -1;
  o->chunk = 0;
}

const char* bhx_version(void) { return "bhx 0.1 (gfx950)"; }

const char* bhx_last_error(void) { return bhx::last_error(); }

const char* bhx_status_string(int s) {
  switch (s) {
    case BHX_OK: return "ok";
    case BHX_NOT_CONVERGED: return "not converged";
    case BHX_ERR_ARG: return "invalid argument";
    case BHX_ERR_SINGULAR: return "singular: no known node and no Dirichlet axis";
    case BHX_ERR_NONFINITE: return "non-finite known value within stencil reach";
    case BHX_ERR_NOMEM: return "out of memory";
    case BHX_ERR_HIP: return "HIP runtime error";
    case BHX_BUSY: return "busy: request does not fit now";
    case BHX_ERR_BREAKDOWN: return "breakdown: non-finite or non-positive curvature";
    default: return "unknown status";
  }
}

int bhx_create(bhx_handle** out, int device) {
  if (!out) return BHX_ERR_ARG;
  *out = nullptr;
  bhx_handle* h = new (std::nothrow) bhx_handle();
  if (!h) return BHX_ERR_NOMEM;
  int s = bhx::init_handle(h, device);
  if (s != BHX_OK) {
    bhx::free_handle(h);
    delete h;
    return s;
  }
  *out = h;
  return BHX_OK;
}

void bhx_destroy(bhx_handle* h) {
  if (!h) return;
  bhx::free_handle(h);
  delete h;
}

static std::mutex g_default_mu;
static bhx_handle* g_default = nullptr;

int bhx_extend(const double* phi, double* F, int nx, int ny, double h, int bc, double tol) {
  bhx_opts o;
  bhx_default_opts(&o);
  const Resolved R = bhx::resolve_opts(&o);
  int v = bhx::validate(phi, F, nx, ny, h, bc, tol, R);
  if (v != BHX_OK) return v;
  std::lock_guard<std::mutex> lk(g_default_mu);
  if (!g_default) {
    int s = bhx_create(&g_default, 0);
    if (s != BHX_OK) return s;
  }
  return bhx_extend_ex(g_default, phi, F, nx, ny, h, bc, tol, &o, nullptr, nullptr);
}

int bhx_extend_ex(bhx_handle* hd, const double* phi, double* F, int nx, int ny, double h, int bc,
                  double tol, const bhx_opts* o, void* stream, bhx_stats* out) {
  if (!hd) return BHX_ERR_ARG;
  const Resolved R = bhx::resolve_opts(o);
  int v = bhx::validate(phi, F, nx, ny, h, bc, tol, R);
  if (v != BHX_OK) return v;
  bhx::InstSpec s{phi, F, nx, ny, bc & 15, (bc >> 4) & 15, tol};
  std::lock_guard<std::mutex> lk(hd->mu);
  return bhx::solve_batch(hd, 1, &s, R, (hipStream_t)stream, out);
}

int bhx_extend_noalloc(bhx_handle* hd, const double* phi, double* F, int nx, int ny, double h,
                       int bc, double tol, const bhx_opts* o, void* stream, bhx_stats* out) {
  if (!hd) return BHX_ERR_ARG;
  const Resolved R = bhx::resolve_opts(o);
  int v = bhx::validate(phi, F, nx, ny, h, bc, tol, R);
  if (v != BHX_OK) return v;
  bhx::InstSpec s{phi, F, nx, ny, bc & 15, (bc >> 4) & 15, tol};
  std::lock_guard<std::mutex> lk(hd->mu);
  return bhx::solve_noalloc(hd, s, R, (hipStream_t)stream, out);
}

int bhx_extend_batched(bhx_handle* hd, int count, const double* const* phi, double* const* F,
                       const int* nx, const int* ny, const double* h, const int* bc,
                       const double* tol, const bhx_opts* o, void* stream, bhx_stats* out) {
  if (!hd || count < 1 || count > (1 << (31 - bhx::kItemShift)) || !phi || !F || !nx || !ny ||
      !h || !bc || !tol)
    return BHX_ERR_ARG;
  const Resolved R = bhx::resolve_opts(o);
  std::vector<bhx::InstSpec> specs(count);
  for (int i = 0; i < count; ++i) {
    int v = bhx::validate(phi[i], F[i], nx[i], ny[i], h[i], bc[i], tol[i], R);
    if (v != BHX_OK) return v;
    specs[i] = bhx::InstSpec{phi[i], F[i], nx[i], ny[i], bc[i] & 15, (bc[i] >> 4) & 15, tol[i]};
  }
  std::lock_guard<std::mutex> lk(hd->mu);
  return bhx::solve_batch(hd, count, specs.data(), R, (hipStream_t)stream, out);
}

int bhx_extend_fields(bhx_handle* hd, int nfields, const double* phi, double* const* F, int nx,
                      int ny, double h, int bc, double tol, const bhx_opts* o, void* stream,
                      bhx_stats* out) {
  if (!hd || nfields < 1 || nfields > (1 << (31 - bhx::kItemShift)) || !F) return BHX_ERR_ARG;
  const Resolved R = bhx::resolve_opts(o);
  std::vector<bhx::InstSpec> specs(nfields);
  for (int i = 0; i < nfields; ++i) {
    int v = bhx::validate(phi, F[i], nx, ny, h, bc, tol, R);
    if (v != BHX_OK) return v;
    for (int j = 0; j < i; ++j)
      if (F[j] == F[i]) return BHX_ERR_ARG;     // two solves writing one array
    specs[i] = bhx::InstSpec{phi, F[i], nx, ny, bc & 15, (bc >> 4) & 15, tol};
  }
  std::lock_guard<std::mutex> lk(hd->mu);
  return bhx::solve_batch(hd, nfields, specs.data(), R, (hipStream_t)stream, out);
}

int bhx_extend3d(bhx_handle* hd, const double* phi, double* F, int nx, int ny, int nz, double h,
                 int bc, double tol, const bhx_opts* o, void* stream, bhx_stats* out) {
  if (!hd) return BHX_ERR_ARG;
  const Resolved R = bhx::resolve_opts(o);
  int v = bhx::validate3(phi, F, nx, ny, nz, h, bc, tol, R);
  if (v != BHX_OK) return v;
  bhx::InstSpec s{phi, F, nx, ny, bc & 15, (bc >> 4) & 15, tol};
  s.nz = nz;
  s.bcz = (bc >> 8) & 15;
  s.dim = 3;
  std::lock_guard<std::mutex> lk(hd->mu);
  return bhx::solve_batch(hd, 1, &s, R, (hipStream_t)stream, out);
}

size_t bhx_workspace_bytes3d(int nx, int ny, int nz, int bc, const bhx_opts* o) {
  const Resolved R = bhx::resolve_opts(o);
  static const double dummy = 0;
  if (bhx::validate3(&dummy, (double*)&dummy, nx, ny, nz, 1.0, bc, 0.5, R) != BHX_OK) return 0;
  return bhx::instance_bytes3(nx, ny, nz, bc & 15, (bc >> 4) & 15, (bc >> 8) & 15,
                              R.precision) +
         sizeof(bhx::Inst) + 64;
}

int bhx_debug_apply3d(bhx_handle* hd, int op, const double* phi, const double* in, double* out,
                      int nx, int ny, int nz, int bc, int precision, void* stream) {
  if (!hd || !in || (op != 0 && op != 1)) return BHX_ERR_ARG;
  bhx_opts o;
  bhx_default_opts(&o);
  o.precision = precision & 15;           // bits 4-7: the transform form (three
  o.transform = (precision >> 4) & 15;    // dimensions always use the FFT family)
  if (precision < 0 || (precision >> 8) != 0) return BHX_ERR_ARG;
  const Resolved R = bhx::resolve_opts(&o);
  int v = bhx::validate3(phi, out, nx, ny, nz, 1.0, bc, 0.5, R);
  if (v != BHX_OK) return v;
  std::lock_guard<std::mutex> lk(hd->mu);
  return bhx::debug_apply(hd, op, phi, in, out, nx, ny, nz, bc & 15, (bc >> 4) & 15,
                          (bc >> 8) & 15, precision, (hipStream_t)stream);
}

size_t bhx_workspace_bytes(int nx, int ny, int bc, const bhx_opts* o) {
  const Resolved R = bhx::resolve_opts(o);
  static const double dummy = 0;
  if (bhx::validate(&dummy, (double*)&dummy, nx, ny, 1.0, bc, 0.5, R) != BHX_OK) return 0;
  return bhx::instance_bytes(nx, ny, bc & 15, (bc >> 4) & 15, R.precision) + sizeof(bhx::Inst) +
         64;
}

int bhx_debug_apply(bhx_handle* hd, int op, const double* phi, const double* in, double* out,
                    int nx, int ny, int bc, int precision, void* stream) {
  if (!hd || !in || (op != 0 && op != 1)) return BHX_ERR_ARG;
  bhx_opts o;
  bhx_default_opts(&o);
  o.precision = precision & 15;           // bits 4-7: the transform form
  o.transform = (precision >> 4) & 15;
  if (precision < 0 || (precision >> 8) != 0) return BHX_ERR_ARG;
  const Resolved R = bhx::resolve_opts(&o);
  int v = bhx::validate(phi, out, nx, ny, 1.0, bc, 0.5, R);
  if (v != BHX_OK) return v;
  std::lock_guard<std::mutex> lk(hd->mu);
  return bhx::debug_apply(hd, op, phi, in, out, nx, ny, 1, bc & 15, (bc >> 4) & 15, 0, precision,
                          (hipStream_t)stream);
}

}  // extern "C"
