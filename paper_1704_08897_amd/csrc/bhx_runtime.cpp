// Host runtime: transform plans, workspace layout, batch construction and the
// driver loop of the preconditioned conjugate-gradient solve.
#include "bhx_runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <type_traits>

namespace bhx {

namespace {

constexpr long double kPi = 3.141592653589793238462643383279502884L;

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2(int m) {
  int l = 0;
  while ((1 << l) < m) ++l;
  return l;
}
size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Iterative radix-2 FFT in long double (host), sign -1, in place.
void host_fft(std::vector<std::complex<long double>>& a) {
  const int m = (int)a.size();
  const int lg = ilog2(m);
  for (int i = 0; i < m; ++i) {
    int r = 0;
    for (int b = 0; b < lg; ++b) r |= ((i >> b) & 1) << (lg - 1 - b);
    if (r > i) std::swap(a[i], a[r]);
  }
  for (int len = 2; len <= m; len <<= 1) {
    for (int i = 0; i < m; i += len) {
      for (int k = 0; k < len / 2; ++k) {
        const long double ang = -2 * kPi * k / len;
        const std::complex<long double> w(cosl(ang), sinl(ang));
        const auto u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
    }
  }
}

template <typename T>
hipError_t grow(T** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return hipSuccess;
  if (*p) {
    hipError_t e = hipFree(*p);
    if (e != hipSuccess) return e;
    *p = nullptr;
  }
  size_t c = std::max(need, *cap * 2);
  hipError_t e = hipMalloc((void**)p, c * sizeof(T));
  if (e != hipSuccess) {
    *cap = 0;
    return e;
  }
  *cap = c;
  return hipSuccess;
}

void free_graph(Graph& G) {
  if (G.exec) (void)hipGraphExecDestroy(G.exec);
  for (auto& x : G.ev)
    if (x) (void)hipEventDestroy(x);
  G.exec = nullptr;
  G.ev.clear();
}

}  // namespace

size_t vec_stride(int nx, int ny) { return align_up((size_t)nx * ny, 32); }

int core_length(int n) {
  if (is_pow2(n)) return n;
  int m = 1;
  while (m < 2 * n - 1) m <<= 1;
  return m;
}

// Complex slots of one packed FFT row in LDS, pad slots included (the
// kernels' rpos(m, shift)).
int row_slots(int m) { return rpos_code(m, rpos_shift(ilog2(m))); }


// Length of the DFT behind the 1-D transform of an axis of n nodes.
// A Dirichlet axis of 1024 to 2046 nodes, whose odd extension of 2(n + 1)
// points would need an 8192-point Bluestein core (no room in LDS in FP64),
// takes its DST-I as a chirp-z transform of n + 1 points instead: the DFT of
// length 2(n + 1) of x placed at 1..n, evaluated at 0..n (dst_chirp).
bool dst_chirp(int n, int bc) { return bc == kDirichlet && n >= 1024 && n <= 2046; }
int fft_length(int n, int bc) {
  if (bc != kDirichlet) return n;
  return dst_chirp(n, bc) ? n + 1 : 2 * (n + 1);
}

bool length_supported(int n, int bc, int prec) {
  if (n < 4) return false;
  const int csize = prec == 0 ? 16 : 8;
  const int m = core_length(fft_length(n, bc));
  if ((long)row_slots(m) * csize > kLdsBytes) return false;        // one packed row must fit
  if ((long)(row_slots(m) + table_slots(n, m, bc, true)) * csize > kLdsDynMax) return false;
  if ((n / 2 + 1) > kThreads * kMaxPairs) return false;
  return true;
}

bool make_layout(int nx, int ny, int nz, int prec, int mx, int my, int mz, int rows_user,
                 Layout* L, bool dense) {
  const bool d3 = mz > 0;
  const int csize = prec == 0 ? 16 : 8;
  const int rows_cap = prec == 0 ? 4 : 8;
  // packed rows per item: the most that fit LDS and the register pair pass
  // (rows_user < 0: the fullest items, for launches shared with other
  // instances), reduced until the instance supplies kTargetItems items (two
  // per CU) when it is to fill the GPU alone (rows_user = 0)
  auto rows_for = [&](int n, int m, long lines, int cap) {
    int r = std::min(cap, kLdsBytes / (row_slots(m) * csize));
    r = std::min(r, (kThreads * kMaxPairs) / (n / 2 + 1));
    if (rows_user > 0) return std::min(r, rows_user);
    if (rows_user < 0) return r;
    while (r > 1 && (lines + 2 * r - 1) / (2 * r) < kTargetItems) --r;
    return r;
  };
  const long nrows = (long)ny * nz;                      // x rows
  const int rx = rows_for(nx, mx, nrows, rows_cap);
  const int ry = rows_for(ny, my, (long)nx * nz, rows_cap);
  // z pencils are strided: wider groups give longer contiguous runs
  const int rz = d3 ? rows_for(nz, mz, (long)nx * ny, kMaxGc / 2) : 1;
  if (rx < 1 || ry < 1 || rz < 1) return false;
  L->G = dense ? kDenseG : 2 * rx;
  L->Gc = dense ? kDenseG : 2 * ry;
  L->Gz = d3 ? 2 * rz : 0;
  if (L->Gc > kMaxGc || L->Gz > kMaxGc) return false;
  const int tx = d3 ? kTileX3 : kTileX, ty = d3 ? kTileY3 : kTileY, tz = d3 ? kTileZ3 : 1;
  L->tiles_x = (nx + tx - 1) / tx;
  L->tiles_y = (ny + ty - 1) / ty;
  L->tiles_z = (nz + tz - 1) / tz;
  const long items[kNumPass] = {(long)L->tiles_x * L->tiles_y * L->tiles_z,
                                (nrows + L->G - 1) / L->G,
                                ((long)nx * nz + L->Gc - 1) / L->Gc,
                                d3 ? (long)nx * ((ny + L->Gz - 1) / L->Gz) : 0, 0, 0};
  for (int p = 0; p < kNumPass; ++p) {
    if (items[p] > kItemMask) return false;
    L->n_items[p] = (int)items[p];
  }
  const size_t N = (size_t)nx * ny * nz;
  const size_t Np = vec_stride(nx, ny * nz);
  const PartLayout PL(L->n_items[kPassS], L->n_items[kPassR]);
  size_t o = 0;
  L->off_mask = o; o = align_up(o + N);
  L->off_vec = o;  o = align_up(o + 5 * Np * sizeof(double));
  L->off_t = o;    o = align_up(o + N * (prec == 0 ? sizeof(double) : sizeof(float)));
  L->off_part = o; o = align_up(o + (size_t)PL.total() * sizeof(double));
  L->off_ctl = o;  o = align_up(o + sizeof(Ctl));
  L->bytes = o;
  return true;
}

size_t instance_bytes(int nx, int ny, int bcx, int bcy, int prec, int rows_user) {
  Layout L;
  if (!length_supported(nx, bcx, prec) || !length_supported(ny, bcy, prec)) return 0;
  if (!make_layout(nx, ny, prec, core_length(fft_length(nx, bcx)),
                   core_length(fft_length(ny, bcy)), rows_user, &L))
    return 0;
  return L.bytes;
}

size_t instance_bytes3(int nx, int ny, int nz, int bcx, int bcy, int bcz, int prec) {
  Layout L;
  if (!length_supported(nx, bcx, prec) || !length_supported(ny, bcy, prec) ||
      !length_supported(nz, bcz, prec))
    return 0;
  // the three-dimensional column passes have no chirp-z DST-I
  if (dst_chirp(ny, bcy) || dst_chirp(nz, bcz)) return 0;
  if (!make_layout(nx, ny, nz, prec, core_length(fft_length(nx, bcx)),
                   core_length(fft_length(ny, bcy)), core_length(fft_length(nz, bcz)), 0, &L))
    return 0;
  return L.bytes;
}

Resolved resolve_opts(const bhx_opts* o) {
  bhx_opts d;
  bhx_default_opts(&d);
  if (!o) o = &d;
  Resolved R;
  R.precision = o->precision;
  R.maxit_user = o->maxit;
  R.precond = o->precond;
  R.accurate = o->accurate;
  R.tol_inner = o->tol_inner > 0 ? o->tol_inner : 1e-8;
  // standard PCG by default, also with the FP32 preconditioner (it needed fewer
  // iterations than the flexible form on every case measured)
  R.flexible = o->flexible < 0 ? 0 : o->flexible;
  R.chunk = o->chunk > 0 ? o->chunk : 32;
  R.chunk += R.chunk & 1;     // even: the buffer parity restarts at 0 every chunk
  R.profile = o->profile;
  R.autotune = o->autotune;
  R.warm = o->warm_start;
  R.solver = o->solver;
  R.rows_opt = o->rows;
  R.occ_opt = o->occupancy;
  R.transform = o->transform;
  if (o->rows != 0) R.sched.rows_cap = o->rows;   // -1: fullest work items
  if (o->occupancy > 0) R.sched.occ_r = R.sched.occ_c = o->occupancy;
  return R;
}

// ---------------------------------------------------------------------------
// PlanCache
// ---------------------------------------------------------------------------

PlanCache::~PlanCache() { release(); }

void PlanCache::release() {
  if (plans_d_) (void)hipFree(plans_d_);
  if (ctab_d_) (void)hipFree(ctab_d_);
  if (ctab_f_) (void)hipFree(ctab_f_);
  if (rtab_d_) (void)hipFree(rtab_d_);
  if (rtab_f_) (void)hipFree(rtab_f_);
  plans_d_ = nullptr; ctab_d_ = nullptr; ctab_f_ = nullptr; rtab_d_ = nullptr; rtab_f_ = nullptr;
  cap_plans_ = cap_c_ = cap_r_ = 0;
  dirty_ = !plans_.empty();
}

int PlanCache::get(int n, int bc) {
  auto key = std::make_pair(n, bc);
  auto it = index_.find(key);
  if (it != index_.end()) return it->second;
  AxisPlan P;
  std::memset(&P, 0, sizeof(P));
  P.n = n;
  P.bc = bc;
  P.nf = fft_length(n, bc);
  const int nf = P.nf;
  P.cz = dst_chirp(n, bc);
  P.m = core_length(nf);
  P.logm = ilog2(P.m);
  P.bluestein = P.m != nf;
  // the chirp's period: the DFT length (2 nf for the chirp-z DST-I)
  const long long L = P.cz ? 2LL * nf : nf;
  using cl = std::complex<long double>;
  auto expi = [](long double a) { return cl(cosl(a), sinl(a)); };
  P.off_tw = (int)ctab_.size();
  for (int k = 0; k < P.m / 2; ++k) ctab_.push_back(expi(-2 * kPi * k / P.m));
  P.off_chirp = (int)ctab_.size();
  P.off_bhat = P.off_chirp;
  if (P.bluestein) {
    std::vector<cl> w(nf);
    for (int k = 0; k < nf; ++k) {
      const long long kk = ((long long)k * k) % (2LL * L);   // exact argument reduction
      w[k] = expi(-kPi * (long double)kk / L);
    }
    for (int k = 0; k < nf; ++k) ctab_.push_back(w[k]);
    std::vector<cl> b(P.m, cl(0, 0));
    for (int l = 0; l < nf; ++l) b[l] = std::conj(w[l]);
    for (int l = 1; l < nf; ++l) b[P.m - l] = std::conj(w[l]);
    host_fft(b);
    P.off_bhat = (int)ctab_.size();
    for (int k = 0; k < P.m; ++k) ctab_.push_back(b[k] / (long double)P.m);
  }
  P.off_post = (int)ctab_.size();
  for (int k = 0; k < n; ++k) ctab_.push_back(expi(-kPi * k / (2.0L * n)));
  P.s0 = (double)sqrtl(1.0L / n);
  P.s1 = (double)sqrtl(2.0L / n);
  P.g0 = (double)(1.0L / sqrtl((long double)n));
  P.g1 = (double)(1.0L / sqrtl(2.0L * n));
  P.hs = bc == kDirichlet ? (double)(0.5L * sqrtl(2.0L / (n + 1)))
                          : (double)(0.5L / sqrtl((long double)n));
  P.off_lam = (int)rtab_.size();
  for (int k = 0; k < n; ++k) {
    // eigenvalues of the 1-D second difference, 4 sin^2(theta/2):
    // Neumann theta = pi k / n, periodic 2 pi k / n, Dirichlet pi (k+1) / (n+1)
    const long double th = bc == kNeumann    ? kPi * k / n
                           : bc == kPeriodic ? 2 * kPi * k / n
                                             : kPi * (k + 1) / (n + 1);
    const long double s = sinl(th / 2);
    rtab_.push_back(4 * s * s);
  }
  if (n <= kDenseMax) {
    // basis of the dense form (see AxisPlan): DCT-II cos(pi a / 2n) over
    // a <= 2n (folded), Hartley cas(2 pi a / n), DST-I sin(pi a / (n + 1))
    P.dense_P = bc == kNeumann ? 4 * n : (bc == kPeriodic ? n : 2 * (n + 1));
    P.dense_fold = bc == kNeumann;
    P.dense_len = P.dense_fold ? P.dense_P / 2 + 1 : P.dense_P;
    P.off_dtab = (int)rtab_.size();
    for (int a = 0; a < P.dense_len; ++a) {
      long double v;
      if (bc == kNeumann) v = cosl(kPi * a / (2.0L * n));
      else if (bc == kPeriodic) v = cosl(2 * kPi * a / n) + sinl(2 * kPi * a / n);
      else v = sinl(kPi * a / (n + 1.0L));
      rtab_.push_back(v);
    }
  }
  const int idx = (int)plans_.size();
  plans_.push_back(P);
  index_[key] = idx;
  dirty_ = true;
  return idx;
}

hipError_t PlanCache::sync_device(hipStream_t st) {
  if (!dirty_) return hipSuccess;
  hipError_t e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;   // before tables move
  if ((e = grow(&plans_d_, &cap_plans_, plans_.size())) != hipSuccess) return e;
  size_t cc = cap_c_;
  if ((e = grow(&ctab_d_, &cap_c_, ctab_.size())) != hipSuccess) return e;
  cap_c_ = cc;
  if ((e = grow(&ctab_f_, &cap_c_, ctab_.size())) != hipSuccess) return e;
  size_t rc = cap_r_;
  if ((e = grow(&rtab_d_, &cap_r_, rtab_.size())) != hipSuccess) return e;
  cap_r_ = rc;
  if ((e = grow(&rtab_f_, &cap_r_, rtab_.size())) != hipSuccess) return e;
  std::vector<double2> cd;
  std::vector<float2> cf;
  std::vector<double> rd;
  std::vector<float> rf;
  tables_host(&cd, &cf, &rd, &rf);
  // stream-ordered: launches on st must not read tables still in transit
  const Upload u[5] = {{plans_d_, plans_.data(), plans_.size() * sizeof(AxisPlan)},
                       {ctab_d_, cd.data(), cd.size() * sizeof(double2)},
                       {ctab_f_, cf.data(), cf.size() * sizeof(float2)},
                       {rtab_d_, rd.data(), rd.size() * sizeof(double)},
                       {rtab_f_, rf.data(), rf.size() * sizeof(float)}};
  for (const Upload& x : u)
    if ((e = hipMemcpyAsync(x.dst, x.src, x.bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
      return e;
  // the host vectors above are temporaries: finish the copies here
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  dirty_ = false;
  return hipSuccess;
}

void PlanCache::tables_host(std::vector<double2>* cd, std::vector<float2>* cf,
                            std::vector<double>* rd, std::vector<float>* rf) const {
  cd->resize(ctab_.size());
  cf->resize(ctab_.size());
  for (size_t i = 0; i < ctab_.size(); ++i) {
    (*cd)[i] = make_double2((double)ctab_[i].real(), (double)ctab_[i].imag());
    (*cf)[i] = make_float2((float)ctab_[i].real(), (float)ctab_[i].imag());
  }
  rd->resize(rtab_.size());
  rf->resize(rtab_.size());
  for (size_t i = 0; i < rtab_.size(); ++i) {
    (*rd)[i] = (double)rtab_[i];
    (*rf)[i] = (float)rtab_[i];
  }
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------

int validate(const double* phi, const double* F, int nx, int ny, double h, int bc, double tol,
             const Resolved& R) {
  if (!phi || !F) return BHX_ERR_ARG;
  if (nx < 4 || ny < 4) return BHX_ERR_ARG;
  if (!std::isfinite(h) || !(h > 0)) return BHX_ERR_ARG;
  if (!std::isfinite(tol) || !(tol > 0) || !(tol < 1)) return BHX_ERR_ARG;
  if (bc < 0 || (bc >> 8) != 0) return BHX_ERR_ARG;
  const int bx = bc & 15, by = (bc >> 4) & 15;
  if (bx > BHX_DIRICHLET || by > BHX_DIRICHLET) return BHX_ERR_ARG;
  if (R.precision != BHX_PREC_FP64 && R.precision != BHX_PREC_FP32) return BHX_ERR_ARG;
  if (R.precond != 0 && R.precond != 1) return BHX_ERR_ARG;
  if (R.accurate != 0 && R.accurate != 1) return BHX_ERR_ARG;
  if (R.maxit_user < 0 || R.chunk > 100000) return BHX_ERR_ARG;
  if (!(R.tol_inner > 0 && R.tol_inner < 1)) return BHX_ERR_ARG;
  if (R.flexible != 0 && R.flexible != 1) return BHX_ERR_ARG;
  if (R.profile < 0 || R.profile > 15) return BHX_ERR_ARG;
  if (R.autotune != 0 && R.autotune != 1) return BHX_ERR_ARG;
  if (R.warm != 0 && R.warm != 1) return BHX_ERR_ARG;
  if (R.solver != 0 && R.solver != 1) return BHX_ERR_ARG;
  if (R.solver == 1 && (R.precision != BHX_PREC_FP64 || !direct_supported(bx, by))) return BHX_ERR_ARG;
  if (R.rows_opt < -1 || R.rows_opt > 8 || R.occ_opt < 0 || R.occ_opt > 8) return BHX_ERR_ARG;
  if (R.transform < 0 || R.transform > 2) return BHX_ERR_ARG;
  if (!length_supported(nx, bx, R.precision) || !length_supported(ny, by, R.precision))
    return BHX_ERR_ARG;
  if ((long long)nx * ny > (1LL << 31)) return BHX_ERR_ARG;
  return BHX_OK;
}

int validate3(const double* phi, const double* F, int nx, int ny, int nz, double h, int bc,
              double tol, const Resolved& R) {
  if (bc < 0 || (bc >> 12) != 0) return BHX_ERR_ARG;
  const int bz = (bc >> 8) & 15;
  if (bz > BHX_DIRICHLET || nz < 4 || R.solver != 0) return BHX_ERR_ARG;
  const int v = validate(phi, F, nx, ny, h, bc & 0xff, tol, R);
  if (v != BHX_OK) return v;
  if (!length_supported(nz, bz, R.precision)) return BHX_ERR_ARG;
  // the three-dimensional column passes (along y and z) have no chirp-z DST-I
  if (dst_chirp(ny, (bc >> 4) & 15) || dst_chirp(nz, bz)) return BHX_ERR_ARG;
  if ((long long)nx * ny * nz >= (1LL << 31)) return BHX_ERR_ARG;
  return BHX_OK;
}

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------

int init_handle(bhx_handle* hd, int device) {
  if (device < 0) return BHX_ERR_ARG;
  int ndev = 0;
  const hipError_t ec = hipGetDeviceCount(&ndev);
  if (ec != hipSuccess) {
    set_last_error("hipGetDeviceCount", __LINE__, ec);
    return BHX_ERR_HIP;
  }
  if (device >= ndev) return BHX_ERR_ARG;
  hd->device = device;
  if (hipSetDevice(device) != hipSuccess) return BHX_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return BHX_ERR_HIP;
  hd->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  if (set_kernel_attributes() != hipSuccess) return BHX_ERR_HIP;
  {
    // the allocation-free entry point's scratch: its device address, looked
    // up once per device with that device current (a failure here shows
    // again, with its reason, on that entry point's first call)
    void* p = nullptr;
    size_t b = 0;
    (void)noalloc_scratch(device, &p, &b);
  }
  if (hipMalloc((void**)&hd->batch_d, sizeof(Batch)) != hipSuccess) return BHX_ERR_NOMEM;
  if (hipStreamCreate(&hd->own_stream) != hipSuccess) return BHX_ERR_HIP;
  return BHX_OK;
}

hipError_t upload_ordered(bhx_handle* hd, hipStream_t st, const Upload* u, int n) {
  size_t total = 0;
  for (int i = 0; i < n; ++i) total += align_up(u[i].bytes);
  if (total > hd->stage_cap) {
    if (hd->stage_h) (void)hipHostFree(hd->stage_h);
    hd->stage_h = nullptr;
    hd->stage_cap = 0;
    const size_t cap = std::max(total, 2 * hd->stage_cap);
    hipError_t e = hipHostMalloc((void**)&hd->stage_h, cap);
    if (e != hipSuccess) return e;
    hd->stage_cap = cap;
  }
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    if (u[i].bytes == 0) continue;
    std::memcpy(hd->stage_h + off, u[i].src, u[i].bytes);
    hipError_t e = hipMemcpyAsync(u[i].dst, hd->stage_h + off, u[i].bytes,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    off += align_up(u[i].bytes);
  }
  return hipSuccess;
}

void free_handle(bhx_handle* hd) {
  if (!hd) return;
  (void)hipSetDevice(hd->device);
  if (hd->own_stream) (void)hipStreamSynchronize(hd->own_stream);
  for (auto& g : hd->graphs) free_graph(g);
  hd->graphs.clear();
  hd->plans.release();
  if (hd->ws) (void)hipFree(hd->ws);
  if (hd->batch_d) (void)hipFree(hd->batch_d);
  if (hd->inst_d) (void)hipFree(hd->inst_d);
  for (int p = 0; p < kNumPass; ++p)
    if (hd->items_d[p]) (void)hipFree(hd->items_d[p]);
  if (hd->flag_d) (void)hipFree(hd->flag_d);
  if (hd->ctl_h) (void)hipHostFree(hd->ctl_h);
  if (hd->stage_h) (void)hipHostFree(hd->stage_h);
  if (hd->dws) (void)hipFree(hd->dws);
  if (hd->band) (void)hipFree(hd->band);
  if (hd->own_stream) (void)hipStreamDestroy(hd->own_stream);
}

// ---------------------------------------------------------------------------
// Solve
// ---------------------------------------------------------------------------

namespace {

}  // namespace

// The column-transform launches of one preconditioner application: one in
// two dimensions; y forward, z (with the scale) and y inverse in three.
// Given events, they time the whole group (in three dimensions, recorded on
// the stream around the three launches).
hipError_t launch_columns(const Batch* B, const Resolved& R, const Grids& g, int count_iter,
                          hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (g.dim == 2)
    return launch_col(B, R.precision, g.shape_c, kCol2D, count_iter, g.c, g.lds_c, g.tw_c, st,
                      e0, e1);
  hipError_t e;
  if (e0 && (e = hipEventRecord(e0, st)) != hipSuccess) return e;
  if ((e = launch_col(B, R.precision, g.shape_c, kColYFwd, 0, g.c, g.lds_c, g.tw_c, st)) !=
      hipSuccess)
    return e;
  if ((e = launch_col(B, R.precision, g.shape_z, kColZ, count_iter, g.z, g.lds_z, g.tw_z, st)) !=
      hipSuccess)
    return e;
  if ((e = launch_col(B, R.precision, g.shape_c, kColYInv, 0, g.c, g.lds_c, g.tw_c, st)) !=
      hipSuccess)
    return e;
  if (e1) return hipEventRecord(e1, st);
  return hipSuccess;
}

// k_reduce after a pass, when some instance of the batch reduces its scalars once.
static hipError_t maybe_reduce(const Batch* B, const Grids& g, int which, int lpar,
                               hipStream_t st) {
  return g.reduce ? launch_reduce(B, g.count, which, lpar, st) : hipSuccess;
}

// The three transform passes over both families: the FFT kernels for the
// instances in the kPassR / kPassC lists, the dense ones for the kPassRD /
// kPassCD lists.  Given events, the first launch of a pass records e0 at its
// start and the last e1 at its end.
static hipError_t launch_rowpass_fwd(const Batch* B, const Resolved& R, const Grids& g,
                                     int update, int lpar, hipStream_t st, hipEvent_t e0,
                                     hipEvent_t e1) {
  hipError_t e;
  if (g.fft && (e = launch_rowfwd(B, R.precision, g.shape_r, update, g.stream_t, g.r, g.lds_r,
                                  g.tw_r, lpar, st, e0, g.dense ? nullptr : e1)) != hipSuccess)
    return e;
  if (g.dense && (e = launch_rowfwd_dense(B, R.precision, update, g.rd, g.lds_rd, g.tab_rd, lpar,
                                          st, g.fft ? nullptr : e0, e1)) != hipSuccess)
    return e;
  return hipSuccess;
}
static hipError_t launch_colpass(const Batch* B, const Resolved& R, const Grids& g,
                                 int count_iter, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  hipError_t e;
  if (g.fft && (e = launch_columns(B, R, g, count_iter, st, e0, g.dense ? nullptr : e1)) !=
                   hipSuccess)
    return e;
  if (g.dense && (e = launch_col_dense(B, R.precision, count_iter, g.cd, g.lds_cd, g.tab_cd, st,
                                       g.fft ? nullptr : e0, e1)) != hipSuccess)
    return e;
  return hipSuccess;
}
static hipError_t launch_rowpass_inv(const Batch* B, const Resolved& R, const Grids& g,
                                     int lpar, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  hipError_t e;
  if (g.fft && (e = launch_rowinv(B, R.precision, g.shape_r, g.r, g.lds_r, g.tw_r, lpar, st, e0,
                                  g.dense ? nullptr : e1)) != hipSuccess)
    return e;
  if (g.dense && (e = launch_rowinv_dense(B, R.precision, g.rd, g.lds_rd, g.tab_rd, lpar, st,
                                          g.fft ? nullptr : e0, e1)) != hipSuccess)
    return e;
  return hipSuccess;
}

hipError_t launch_precond(const Batch* B, const Resolved& R, const Grids& g, hipStream_t st) {
  hipError_t e;
  // parity 1: the r.z partials it writes are the ones the first iteration
  // (parity 0) reads
  if (!R.precond) {
    if ((e = launch_identity(B, g.r, 1, st)) != hipSuccess) return e;
    return maybe_reduce(B, g, kRedRZ, 1, st);
  }
  if ((e = launch_rowpass_fwd(B, R, g, 0, 1, st, nullptr, nullptr)) != hipSuccess) return e;
  if ((e = launch_colpass(B, R, g, 0, st, nullptr, nullptr)) != hipSuccess) return e;
  if ((e = launch_rowpass_inv(B, R, g, 1, st, nullptr, nullptr)) != hipSuccess) return e;
  return maybe_reduce(B, g, kRedRZ, 1, st);
}

// Event of pass p, iteration c, edge e (0 start, 1 end) in a Graph's array.
static inline hipEvent_t ev_at(const std::vector<hipEvent_t>* ev, int chunk, int p, int c,
                                int e) {
  return (*ev)[((size_t)p * chunk + c) * 2 + e];
}

hipError_t launch_iterations(const Batch* B, int n_inst, const Resolved& R, const Grids& g,
                             int count, hipStream_t st, const std::vector<hipEvent_t>* ev) {
  hipError_t e;
  // events of pass p, iteration c (null unless the pass is profiled)
  auto e0 = [&](int p, int c) -> hipEvent_t {
    return ev && (R.profile & (1 << p)) ? ev_at(ev, count, p, c, 0) : nullptr;
  };
  auto e1 = [&](int p, int c) -> hipEvent_t {
    return ev && (R.profile & (1 << p)) ? ev_at(ev, count, p, c, 1) : nullptr;
  };
#define BHX_TRY(x) do { if ((e = (x)) != hipSuccess) return e; } while (0)
  for (int c = 0; c < count; ++c) {
    const int par = c & 1;               // count is even: every chunk starts at 0
    BHX_TRY(launch_stencil(B, g.dim, kModeIter, g.s, par, st, e0(0, c), e1(0, c)));
    BHX_TRY(maybe_reduce(B, g, kRedPQ, par, st));
    if (R.precond) {
      BHX_TRY(launch_rowpass_fwd(B, R, g, 1, par, st, e0(1, c), e1(1, c)));
      BHX_TRY(maybe_reduce(B, g, kRedRR, par, st));
      BHX_TRY(launch_colpass(B, R, g, 1, st, e0(2, c), e1(2, c)));
      BHX_TRY(launch_rowpass_inv(B, R, g, par, st, e0(3, c), e1(3, c)));
    } else {
      // plain CG: update-only row pass, iteration count, z = r
      BHX_TRY(launch_rowfwd(B, R.precision, g.shape_r, 2, g.stream_t, g.r, g.lds_r, g.tw_r, par, st,
                            e0(1, c), e1(1, c)));
      BHX_TRY(maybe_reduce(B, g, kRedRR, par, st));
      BHX_TRY(launch_bump(B, n_inst, st));
      BHX_TRY(launch_identity(B, g.r, par, st, e0(3, c), e1(3, c)));
    }
    BHX_TRY(maybe_reduce(B, g, kRedRZ, par, st));
  }
#undef BHX_TRY
  return hipSuccess;
}

namespace {

bool use_graphs() {
  const char* v = getenv("BHX_NO_GRAPH");
  return !(v && v[0] == '1');
}

hipError_t make_events(std::vector<hipEvent_t>* ev, int chunk) {
  ev->assign((size_t)4 * chunk * 2, nullptr);
  for (auto& x : *ev) {
    hipError_t e = hipEventCreate(&x);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// Launch one chunk of iterations over batch B (device header) of n_inst
// instances; returns the Graph used (for its events).
hipError_t run_chunk(bhx_handle* hd, const Batch* B, int n_inst, const Resolved& R,
                     const Grids& g, hipStream_t st, Graph** used) {
  *used = nullptr;
  // HIP cannot time events recorded as graph nodes, so a profiled chunk is
  // launched directly with events around the selected passes.
  const bool graph = use_graphs() && R.profile == 0;
  for (auto& gr : hd->graphs) {
    if (gr.stream == st && gr.batch == B &&
        gr.count == ((R.precond && !g.reduce) ? 0 : n_inst) && gr.reduce == g.reduce &&
        gr.prec == R.precision && gr.chunk == R.chunk &&
        gr.precond == R.precond && gr.gs == g.s && gr.gr == g.r && gr.gc == g.c &&
        gr.lds_r == g.lds_r && gr.tw_r == g.tw_r && gr.lds_c == g.lds_c && gr.tw_c == g.tw_c &&
        gr.dim == g.dim && gr.gz == g.z && gr.lds_z == g.lds_z && gr.tw_z == g.tw_z &&
        gr.shape_r == g.shape_r && gr.shape_c == g.shape_c && gr.shape_z == g.shape_z &&
        gr.stream_t == g.stream_t && gr.fft == g.fft && gr.dense == g.dense &&
        gr.rd == g.rd && gr.cd == g.cd && gr.lds_rd == g.lds_rd && gr.tab_rd == g.tab_rd &&
        gr.lds_cd == g.lds_cd && gr.tab_cd == g.tab_cd &&
        gr.profile == R.profile && (gr.exec != nullptr) == graph) {
      *used = &gr;
      if (gr.exec) return hipGraphLaunch(gr.exec, st);
      return launch_iterations(B, n_inst, R, g, R.chunk, st, &gr.ev);
    }
  }
  Graph G;
  G.stream = st; G.prec = R.precision; G.chunk = R.chunk; G.precond = R.precond;
  G.batch = B; G.count = (R.precond && !g.reduce) ? 0 : n_inst;
  G.reduce = g.reduce;
  G.gs = g.s; G.gr = g.r; G.gc = g.c; G.profile = R.profile;
  G.lds_r = g.lds_r; G.tw_r = g.tw_r; G.lds_c = g.lds_c; G.tw_c = g.tw_c;
  G.dim = g.dim; G.gz = g.z; G.lds_z = g.lds_z; G.tw_z = g.tw_z;
  G.shape_r = g.shape_r; G.shape_c = g.shape_c; G.shape_z = g.shape_z;
  G.stream_t = g.stream_t;
  G.fft = g.fft; G.dense = g.dense; G.rd = g.rd; G.cd = g.cd;
  G.lds_rd = g.lds_rd; G.tab_rd = g.tab_rd; G.lds_cd = g.lds_cd; G.tab_cd = g.tab_cd;
  hipError_t e;
  if (R.profile && (e = make_events(&G.ev, R.chunk)) != hipSuccess) {
    free_graph(G);
    return e;
  }
  if (graph) {
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { free_graph(G); return e; }
    hipError_t el = launch_iterations(B, n_inst, R, g, R.chunk, st, nullptr);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (el != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      free_graph(G);
      return el != hipSuccess ? el : e;
    }
    e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { free_graph(G); return e; }
  }
  if (hd->graphs.size() >= 16) {
    free_graph(hd->graphs.front());
    hd->graphs.erase(hd->graphs.begin());
  }
  hd->graphs.push_back(G);
  Graph* gp = &hd->graphs.back();
  *used = gp;
  if (gp->exec) return hipGraphLaunch(gp->exec, st);
  return launch_iterations(B, n_inst, R, g, R.chunk, st, R.profile ? &gp->ev : nullptr);
}

namespace {

}  // namespace

thread_local char g_last_error[512] = "";

void set_last_error(const char* what, int line, hipError_t e) {
  snprintf(g_last_error, sizeof(g_last_error), "%s (bhx_runtime.cpp:%d): %s", what, line,
           hipGetErrorString(e));
}

void set_last_message(const char* what) { snprintf(g_last_error, sizeof(g_last_error), "%s", what); }

const char* last_error() { return g_last_error; }

#define BHX_CHECK(x)                                                      \
  do {                                                                    \
    hipError_t _e = (x);                                                  \
    if (_e != hipSuccess) {                                               \
      set_last_error(#x, __LINE__, _e);                                   \
      return _e == hipErrorOutOfMemory ? BHX_ERR_NOMEM : BHX_ERR_HIP;     \
    }                                                                     \
  } while (0)

bool dense_eligible(const AxisPlan& X, const AxisPlan& Y) {
  return X.dense_P > 0 && Y.dense_P > 0;
}

// Built-in choice of the dense form for an eligible instance (transform 0):
// none.  Measured on one MI355X (FP64, 64^2 to 512^2, single instances and
// the 256-instance batch), the FFT family was faster at every size, also
// where Bluestein doubles its length: the dense products cost 2 n flops per
// node and transform against the FFT's O(log n), and run at about a fifth of
// the FP64 matrix rate.  The autotuner still times the dense form.
static bool dense_policy(const AxisPlan&, const AxisPlan&) { return false; }

bool use_dense(const Resolved& R, const AxisPlan& X, const AxisPlan& Y) {
  if (!R.precond || !dense_eligible(X, Y)) return false;
  const int t = R.sched.transform >= 0 ? R.sched.transform : R.transform;
  if (t == 2) return true;
  if (t == 1) return false;
  return dense_policy(X, Y);
}

int plan_layouts(PlanCache& plans, int n, const InstSpec* specs, const Resolved& R,
                 BatchDesc* D) {
  const int dim = specs[0].dim;
  D->dim = dim;
  D->px.assign(n, 0);
  D->py.assign(n, 0);
  D->pz.assign(n, 0);
  D->lay.assign(n, Layout());
  D->dense.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    const InstSpec& S = specs[i];
    if (S.dim != dim) return BHX_ERR_ARG;
    D->px[i] = plans.get(S.nx, S.bcx);
    D->py[i] = plans.get(S.ny, S.bcy);
    if (dim == 3) D->pz[i] = plans.get(S.nz, S.bcz);
    const int mz = dim == 3 ? plans.plan(D->pz[i]).m : 0;
    D->dense[i] = dim == 2 && use_dense(R, plans.plan(D->px[i]), plans.plan(D->py[i]));
    if (!make_layout(S.nx, S.ny, dim == 3 ? S.nz : 1, R.precision, plans.plan(D->px[i]).m,
                     plans.plan(D->py[i]).m, mz, R.sched.rows_cap, &D->lay[i], D->dense[i]))
      return BHX_ERR_ARG;
  }
  return BHX_OK;
}

size_t ctl_region_bytes(int n) { return align_up((size_t)n * sizeof(Ctl)); }

void describe_batch(const PlanCache& plans, int n, const InstSpec* specs, const Resolved& R,
                    char* ws, Ctl* ctl_d, BatchDesc* D) {
  const int dim = D->dim;
  D->inst.assign(n, Inst());
  D->ctl.assign(n, Ctl());
  for (int p = 0; p < kNumPass; ++p) D->items[p].clear();
  // workspace: the control blocks, then one region per instance
  size_t total = ctl_region_bytes(n);
  std::vector<size_t> base(n);
  for (int i = 0; i < n; ++i) {
    base[i] = total;
    total += D->lay[i].bytes;
  }
  D->ws_bytes = total;
  for (int i = 0; i < n; ++i) {
    const InstSpec& S = specs[i];
    const Layout& L = D->lay[i];
    Inst& I = D->inst[i];
    std::memset(&I, 0, sizeof(I));
    const int nz = dim == 3 ? S.nz : 1;
    I.nx = S.nx; I.ny = S.ny; I.nz = nz; I.nrows = S.ny * nz;
    I.bcx = S.bcx; I.bcy = S.bcy; I.bcz = dim == 3 ? S.bcz : 0;
    I.planx = D->px[i]; I.plany = D->py[i]; I.planz = D->pz[i];
    I.G = L.G; I.Gc = L.Gc; I.Gz = L.Gz;
    I.tiles_x = L.tiles_x; I.tiles_y = L.tiles_y; I.tiles_z = L.tiles_z;
    for (int p = 0; p < kNumPass; ++p) I.n_items[p] = L.n_items[p];
    I.maxit = R.maxit_user > 0 ? R.maxit_user : 50 * std::max(std::max(S.nx, S.ny), nz);
    I.flexible = R.flexible;
    I.warm = R.warm;
    I.reduce = L.n_items[kPassS] + 3 * L.n_items[kPassR] > kReduceMin;
    I.dense = D->dense[i];
    I.phi = (decltype(I.phi))S.phi;
    I.F = (decltype(I.F))S.F;
    const size_t Np = vec_stride(S.nx, S.ny * nz);
    char* b = ws ? ws + base[i] : nullptr;
    if (b) {
      I.mask = (decltype(I.mask))(b + L.off_mask);
      double* v = (double*)(b + L.off_vec);
      I.r = (decltype(I.r))v;
      I.p[0] = (decltype(I.r))(v + Np);
      I.p[1] = (decltype(I.r))(v + 2 * Np);
      I.q = (decltype(I.r))(v + 3 * Np);
      I.z = (decltype(I.r))(v + 4 * Np);
      I.t = (decltype(I.t))(b + L.off_t);
      I.part = (decltype(I.part))(b + L.off_part);
      I.ctl = (decltype(I.ctl))(ctl_d + i);
    }
    for (int p = 0; p < kNumPass; ++p)
      for (int k = 0; k < list_items(I, p); ++k) D->items[p].push_back((i << kItemShift) | k);
    Ctl& C = D->ctl[i];
    std::memset(&C, 0, sizeof(C));
    C.tol2 = S.tol * S.tol;
    C.tol_inner2 = R.tol_inner * R.tol_inner;
    C.accurate = R.accurate;
    C.max_restarts = R.accurate ? 12 : 8;
  }
}

void fill_header(Batch* Bh, const BatchDesc& D, const Inst* inst_d, int* const items_d[kNumPass],
                 const AxisPlan* plans_d, const void* const ctab[2], const void* const rtab[2]) {
  std::memset(Bh, 0, sizeof(*Bh));
  Bh->count = (int)D.inst.size();
  for (int p = 0; p < kNumPass; ++p) {
    Bh->n_items[p] = (int)D.items[p].size();
    Bh->items[p] = (std::remove_reference_t<decltype(Bh->items[p])>)items_d[p];
  }
  Bh->inst = (decltype(Bh->inst))inst_d;
  Bh->plans = (decltype(Bh->plans))plans_d;
  for (int p = 0; p < 2; ++p) {
    Bh->ctab[p] = (std::remove_reference_t<decltype(Bh->ctab[p])>)ctab[p];
    Bh->rtab[p] = (std::remove_reference_t<decltype(Bh->rtab[p])>)rtab[p];
  }
}

void dense_grids(int prec, int nx_max, int ny_max, int n_rd, int n_cd, int num_cu, int occ,
                 Grids* g) {
  g->rd = std::max(1, std::min(n_rd, num_cu * occ));
  g->cd = std::max(1, std::min(n_cd, num_cu * occ));
  g->lds_rd = dense_lds_bytes(kPassRD, prec, nx_max);
  g->tab_rd = dense_tab_off(nx_max);
  g->lds_cd = dense_lds_bytes(kPassCD, prec, ny_max);
  g->tab_cd = dense_tab_off(ny_max);
}

int batch_grids(const PlanCache& plans, const BatchDesc& D, const Resolved& R, int num_cu,
                Grids* gout) {
  const int n = (int)D.inst.size();
  const int dim = D.dim;
  Grids g;
  g.dim = dim;
  g.count = n;
  for (int i = 0; i < n; ++i) g.reduce |= D.inst[i].reduce;
  const int ni[kNumPass] = {(int)D.items[kPassS].size(), (int)D.items[kPassR].size(),
                            (int)D.items[kPassC].size(), (int)D.items[kPassZ].size()};
  g.s = std::max(1, std::min(ni[kPassS], num_cu * R.sched.occ_s));
  g.r = std::max(1, std::min(ni[kPassR], num_cu * R.sched.occ_r));
  g.c = std::max(1, std::min(ni[kPassC], num_cu * R.sched.occ_c));
  g.z = dim == 3 ? std::max(1, std::min(ni[kPassZ], num_cu * R.sched.occ_c)) : 0;
  {
    // dynamic LDS: packed rows followed by the staged plan tables
    const int csize = R.precision == 0 ? 16 : 8;
    int buf_r = 0, tab_r = 0, buf_c = 0, tab_c = 0, buf_z = 0, tab_z = 0;
    for (int i = 0; i < n; ++i) {
      if (D.dense[i]) continue;                 // no FFT pass works on it
      const AxisPlan& PX = plans.plan(D.px[i]);
      const AxisPlan& PY = plans.plan(D.py[i]);
      buf_r = std::max(buf_r, (D.lay[i].G / 2) * row_slots(PX.m));
      tab_r = std::max(tab_r, table_slots(PX.n, PX.m, PX.bc, false));
      buf_c = std::max(buf_c, (D.lay[i].Gc / 2) * row_slots(PY.m));
      tab_c = std::max(tab_c, table_slots(PY.n, PY.m, PY.bc, dim == 2));
      if (dim == 3) {
        const AxisPlan& PZ = plans.plan(D.pz[i]);
        buf_z = std::max(buf_z, (D.lay[i].Gz / 2) * row_slots(PZ.m));
        tab_z = std::max(tab_z, table_slots(PZ.n, PZ.m, PZ.bc, true));
      }
    }
    g.tw_r = buf_r;
    g.lds_r = (buf_r + tab_r) * csize;
    g.tw_c = buf_c;
    g.lds_c = (buf_c + tab_c) * csize;
    g.tw_z = buf_z;
    g.lds_z = (buf_z + tab_z) * csize;
    if (g.lds_r > kLdsDynMax || g.lds_c > kLdsDynMax || g.lds_z > kLdsDynMax) return BHX_ERR_ARG;
  }
  int f0 = -1;                                  // first FFT-family instance
  for (int i = 0; i < n && f0 < 0; ++i)
    if (!D.dense[i]) f0 = i;
  g.fft = f0 >= 0;
  if (f0 >= 0) {
    // compile-time-shape kernels when every FFT-family instance shares the
    // axis plan and the line grouping of the first one
    auto key = [&](int pass, const AxisPlan& P, int group) {
      return shape_key(pass, R.precision, P.n, P.m, P.logm, P.bluestein, P.bc, group);
    };
    g.shape_r = key(kShapeRow, plans.plan(D.px[f0]), D.lay[f0].G);
    g.shape_c = key(dim == 3 ? kShapeColY : kShapeCol2D, plans.plan(D.py[f0]), D.lay[f0].Gc);
    g.shape_z = dim == 3 ? key(kShapeColZ, plans.plan(D.pz[f0]), D.lay[f0].Gz) : 0;
    for (int i = f0 + 1; i < n; ++i) {
      if (D.dense[i]) continue;
      if (D.px[i] != D.px[f0] || D.lay[i].G != D.lay[f0].G) g.shape_r = 0;
      if (D.pz[i] != D.pz[f0] || D.lay[i].Gz != D.lay[f0].Gz) g.shape_z = 0;
      if (D.py[i] != D.py[f0] || D.lay[i].Gc != D.lay[f0].Gc) g.shape_c = 0;
    }
    // plan-table launches: the kernel family from the longest work item
    // and the chirp-z axes
    plan_families(plans, D, &g);
  }
  {
    // plan-table launches read their tables from global memory: their LDS
    // is the packed rows alone
    const int csize = R.precision == 0 ? 16 : 8;
    if (plan_table_shape(g.shape_r)) g.lds_r = g.tw_r * csize;
    if (plan_table_shape(g.shape_c)) g.lds_c = g.tw_c * csize;
    if (dim == 3 && plan_table_shape(g.shape_z)) g.lds_z = g.tw_z * csize;
  }
  {
    int nxm = 0, nym = 0;
    for (int i = 0; i < n; ++i)
      if (D.dense[i]) {
        nxm = std::max(nxm, plans.plan(D.px[i]).n);
        nym = std::max(nym, plans.plan(D.py[i]).n);
      }
    g.dense = nxm > 0;
    if (g.dense)
      dense_grids(R.precision, nxm, nym, (int)D.items[kPassRD].size(),
                  (int)D.items[kPassCD].size(), num_cu, R.sched.occ_d, &g);
  }
  {
    // non-temporal stores of t in the row-forward pass while the launch's t
    // arrays are small (1024^2 FP64: 12.5 -> 11.8 us per launch; 2048^2:
    // 46 -> 91 us, so never for large t)
    size_t tb = 0;
    for (int i = 0; i < n; ++i) tb += D.lay[i].off_part - D.lay[i].off_t;
    g.stream_t = tb <= kStreamTMax;
  }
  *gout = g;
  return BHX_OK;
}

void plan_family(const AxisPlan& P, int rows, int* shape) {
  if (*shape != kShapeNarrowKey && *shape != kShapeWideKey) return;   // compile-time shape or cz
  if (P.cz)
    *shape = kShapeCzKey;
  else if ((long)rows * P.m >= kFftWideLaunch)
    *shape = kShapeWideKey;
}

void plan_families(const PlanCache& plans, const BatchDesc& D, Grids* g) {
  const bool sr = g->shape_r == 0, sc = g->shape_c == 0, sz = g->shape_z == 0;
  for (size_t i = 0; i < D.inst.size(); ++i) {
    if (D.dense[i]) continue;
    if (sr) plan_family(plans.plan(D.px[i]), D.lay[i].G / 2, &g->shape_r);
    if (sc) plan_family(plans.plan(D.py[i]), D.lay[i].Gc / 2, &g->shape_c);
    if (sz && D.dim == 3) plan_family(plans.plan(D.pz[i]), D.lay[i].Gz / 2, &g->shape_z);
  }
}

int prepare_batch(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R,
                  hipStream_t st, Grids* gout) {
  BHX_CHECK(hipSetDevice(hd->device));
  // earlier launches on st may still read the descriptors, tables and
  // staging buffer replaced below
  BHX_CHECK(hipStreamSynchronize(st));
  BatchDesc D;
  {
    const int rc = plan_layouts(hd->plans, n, specs, R, &D);
    if (rc != BHX_OK) return rc;
  }
  BHX_CHECK(hd->plans.sync_device(st));
  describe_batch(hd->plans, n, specs, R, nullptr, nullptr, &D);   // sizes only
  if (D.ws_bytes > hd->ws_cap) {
    if (hd->ws) BHX_CHECK(hipFree(hd->ws));
    hd->ws = nullptr;
    hd->ws_cap = 0;
    BHX_CHECK(hipMalloc(&hd->ws, D.ws_bytes));
    hd->ws_cap = D.ws_bytes;
  }
  char* ws = (char*)hd->ws;
  Ctl* ctl_d = (Ctl*)ws;
  describe_batch(hd->plans, n, specs, R, ws, ctl_d, &D);
  // device descriptors
  if (n > hd->inst_cap) {
    if (hd->inst_d) BHX_CHECK(hipFree(hd->inst_d));
    hd->inst_d = nullptr;
    BHX_CHECK(hipMalloc((void**)&hd->inst_d, std::max(n, 2 * hd->inst_cap) * sizeof(Inst)));
    hd->inst_cap = std::max(n, 2 * hd->inst_cap);
  }
  for (int p = 0; p < kNumPass; ++p) {
    const int need = std::max<int>(1, (int)D.items[p].size());
    if (need > hd->items_cap[p]) {
      if (hd->items_d[p]) BHX_CHECK(hipFree(hd->items_d[p]));
      hd->items_d[p] = nullptr;
      const int cap = std::max(need, 2 * hd->items_cap[p]);
      BHX_CHECK(hipMalloc((void**)&hd->items_d[p], cap * sizeof(int)));
      hd->items_cap[p] = cap;
    }
  }
  if (n > hd->flag_cap) {
    if (hd->flag_d) BHX_CHECK(hipFree(hd->flag_d));
    hd->flag_d = nullptr;
    BHX_CHECK(hipMalloc((void**)&hd->flag_d, std::max(n, 2 * hd->flag_cap) * sizeof(int)));
    hd->flag_cap = std::max(n, 2 * hd->flag_cap);
  }
  if (n > hd->ctl_h_cap) {
    if (hd->ctl_h) BHX_CHECK(hipHostFree(hd->ctl_h));
    hd->ctl_h = nullptr;
    BHX_CHECK(hipHostMalloc((void**)&hd->ctl_h, std::max(n, 2 * hd->ctl_h_cap) * sizeof(Ctl)));
    hd->ctl_h_cap = std::max(n, 2 * hd->ctl_h_cap);
  }
  Batch Bh;
  const void* ctab[2] = {hd->plans.ctab(0), hd->plans.ctab(1)};
  const void* rtab[2] = {hd->plans.rtab(0), hd->plans.rtab(1)};
  fill_header(&Bh, D, hd->inst_d, hd->items_d, hd->plans.plans_d(), ctab, rtab);
  hd->batch_count = n;
  // stream-ordered: the setup launches that follow on st read all of these
  {
    Upload u[3 + kNumPass] = {{hd->inst_d, D.inst.data(), n * sizeof(Inst)},
                              {ctl_d, D.ctl.data(), n * sizeof(Ctl)},
                              {hd->batch_d, &Bh, sizeof(Batch)}};
    for (int p = 0; p < kNumPass; ++p)
      u[3 + p] = {hd->items_d[p], D.items[p].data(), D.items[p].size() * sizeof(int)};
    BHX_CHECK(upload_ordered(hd, st, u, 3 + kNumPass));
  }
  hd->batch_h = Bh;
  for (int p = 0; p < kNumPass; ++p) hd->items_h[p] = D.items[p];
  return batch_grids(hd->plans, D, R, hd->num_cu, gout);
}

// Upload the work lists of the handle's current batch with only the items of
// instances still running (all = false), or in full (all = true), together
// with the header that carries their lengths.  The kernels read both at run
// time, so captured chunks stay valid; an item's work does not depend on
// which block takes it, so results are unchanged.  The stream must be idle
// (the staging buffer is reused).
static hipError_t upload_work_lists(bhx_handle* hd, hipStream_t st, const Ctl* ch, bool all) {
  std::vector<int> lists[kNumPass];
  Batch Bh = hd->batch_h;
  Upload u[1 + kNumPass];
  int nu = 0;
  for (int p = 0; p < kNumPass; ++p) {
    const std::vector<int>& full = hd->items_h[p];
    if (all) {
      lists[p] = full;
    } else {
      lists[p].reserve(full.size());
      for (int c : full)
        if (ch[c >> kItemShift].done == kRunning) lists[p].push_back(c);
    }
    Bh.n_items[p] = (int)lists[p].size();
    if (!lists[p].empty())
      u[nu++] = {hd->items_d[p], lists[p].data(), lists[p].size() * sizeof(int)};
  }
  u[nu++] = {hd->batch_d, &Bh, sizeof(Batch)};
  return upload_ordered(hd, st, u, nu);
}

static bool compaction_enabled() {
  const char* v = getenv("BHX_COMPACT");
  return !(v && v[0] == '0');
}

int drive_batch(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R, const Grids& g,
                hipStream_t st, const DriveCtx& X, bhx_stats* stats,
                std::chrono::steady_clock::time_point t0) {
  Ctl* ctl_d = X.ctl_d;
  // setup: mask, right-hand side, counts
  BHX_CHECK(launch_setup(X.B, g.dim, g.s, st));
  BHX_CHECK(launch_setup_rows(X.B, std::max(g.r, g.rd), st));
  BHX_CHECK(launch_stencil(X.B, g.dim, kModeRhs, g.s, 0, st));
  BHX_CHECK(launch_finalize(X.B, n, kFinSetupH, st));
  Ctl* ch = X.ch;
  BHX_CHECK(hipMemcpyAsync(ch, ctl_d, n * sizeof(Ctl), hipMemcpyDeviceToHost, st));
  BHX_CHECK(hipStreamSynchronize(st));
  std::vector<int> status(n, BHX_OK), preset(n, 0), zero_flag(n, 0);
  int active = 0, any_zero = 0;
  for (int i = 0; i < n; ++i) {
    const InstSpec& S = specs[i];
    const double N = (double)S.nx * S.ny * (S.dim == 3 ? S.nz : 1);
    const bool dirichlet = S.bcx == kDirichlet || S.bcy == kDirichlet ||
                           (S.dim == 3 && S.bcz == kDirichlet);
    const double nu = ch[i].n_unknown;
    if (nu == 0) {
      preset[i] = 1;
    } else if (nu == N && !dirichlet) {
      // nothing known and only Neumann/periodic axes: u is fixed up to a
      // constant (with a Dirichlet axis, b = 0 and the extension is 0)
      preset[i] = 1;
      status[i] = BHX_ERR_SINGULAR;
    } else if (!std::isfinite(ch[i].bb)) {
      preset[i] = 1;
      status[i] = BHX_ERR_NONFINITE;
    } else if (ch[i].bb == 0.0) {
      preset[i] = 1;
      zero_flag[i] = 1;
      any_zero = 1;
    }
    if (preset[i]) ch[i].done = kSkip;
    else ++active;
  }
  if (active < n) {
    BHX_CHECK(hipMemcpyAsync(ctl_d, ch, n * sizeof(Ctl), hipMemcpyHostToDevice, st));
    if (any_zero) {
      if (X.graphs) {
        const Upload u{X.flag_d, zero_flag.data(), n * sizeof(int)};
        BHX_CHECK(upload_ordered(hd, st, &u, 1));
      } else {
        // from pageable memory; zero_flag outlives the synchronisation below
        BHX_CHECK(hipMemcpyAsync(X.flag_d, zero_flag.data(), n * sizeof(int),
                                 hipMemcpyHostToDevice, st));
      }
      BHX_CHECK(launch_zero_unknown(X.B, g.dim, X.flag_d, g.s, st));
    }
    BHX_CHECK(hipStreamSynchronize(st));
  }
  // warm start: r0 = b - A x0 for the instances still active; those whose
  // start already meets the tolerance, or whose residual is not finite, end
  // here with F untouched
  std::vector<int> warm_done(n, 0);
  if (R.warm && active > 0) {
    BHX_CHECK(launch_stencil(X.B, g.dim, kModeWarm, g.s, 0, st));
    BHX_CHECK(launch_finalize(X.B, n, kFinWarmH, st));
    BHX_CHECK(hipMemcpyAsync(ch, ctl_d, n * sizeof(Ctl), hipMemcpyDeviceToHost, st));
    BHX_CHECK(hipStreamSynchronize(st));
    int ended = 0;
    for (int i = 0; i < n; ++i) {
      if (preset[i]) continue;
      const int w = warm_start_outcome(ch[i]);
      if (w == 0) continue;
      preset[i] = 1;
      warm_done[i] = 1;
      status[i] = w == 1 ? BHX_OK : BHX_ERR_NONFINITE;
      ch[i].done = kSkip;
      --active;
      ++ended;
    }
    if (ended) {
      BHX_CHECK(hipMemcpyAsync(ctl_d, ch, n * sizeof(Ctl), hipMemcpyHostToDevice, st));
      BHX_CHECK(hipStreamSynchronize(st));
    }
  }
  double pass_ms[4] = {0, 0, 0, 0};
  int pass_cnt[4] = {0, 0, 0, 0};
  std::vector<int> iter_before(n);
  int listed = n;                     // instances whose items the work lists hold
  if (active > 0) {
    BHX_CHECK(launch_precond(X.B, R, g, st));
    for (;;) {
      for (int i = 0; i < n; ++i) iter_before[i] = ch[i].iter;
      Graph* used = nullptr;
      if (X.graphs) BHX_CHECK(run_chunk(hd, X.B, n, R, g, st, &used));
      else BHX_CHECK(launch_iterations(X.B, n, R, g, R.chunk, st, nullptr));
      BHX_CHECK(hipMemcpyAsync(ch, ctl_d, n * sizeof(Ctl), hipMemcpyDeviceToHost, st));
      BHX_CHECK(hipStreamSynchronize(st));
      if (R.profile && used && !used->ev.empty()) {
        int worked = 0;
        for (int i = 0; i < n; ++i) worked = std::max(worked, ch[i].iter - iter_before[i]);
        for (int p = 0; p < 4; ++p) {
          if (!(R.profile & (1 << p))) continue;
          for (int c = 0; c < worked && c < R.chunk; ++c) {
            float ms = 0;
            BHX_CHECK(hipEventElapsedTime(&ms, ev_at(&used->ev, R.chunk, p, c, 0),
                                          ev_at(&used->ev, R.chunk, p, c, 1)));
            pass_ms[p] += ms;
            pass_cnt[p] += 1;
          }
        }
      }
      int running = 0;
      for (int i = 0; i < n; ++i) running += ch[i].done == kRunning;
      if (running > 0) {
        // once a quarter of the listed instances have finished, list only the
        // running ones: a finished instance's items would still cost each
        // block that meets one a round trip of loads before it is skipped
        if (X.compact && 4 * running <= 3 * listed) {
          BHX_CHECK(upload_work_lists(hd, st, ch, false));
          listed = running;
        }
        continue;
      }
      // the residual, finalisation, restart and preconditioner launches below
      // go over every instance: full lists again
      if (listed < n) {
        BHX_CHECK(upload_work_lists(hd, st, ch, true));
        listed = n;
      }
      // true residual of finished instances; restart those that miss the target
      BHX_CHECK(launch_resid(X.B, g.dim, g.s, st));
      BHX_CHECK(launch_finalize(X.B, n, kFinResidH, st));
      BHX_CHECK(launch_restart(X.B, n, st));
      BHX_CHECK(hipMemcpyAsync(ch, ctl_d, n * sizeof(Ctl), hipMemcpyDeviceToHost, st));
      BHX_CHECK(hipStreamSynchronize(st));
      bool restarted = false;
      for (int i = 0; i < n; ++i)
        if (ch[i].done == kRunning) restarted = true;
      if (!restarted) break;
      BHX_CHECK(launch_precond(X.B, R, g, st));
    }
  }
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int ret = BHX_OK;
  for (int i = 0; i < n; ++i) {
    int s = status[i];
    if (!preset[i]) {
      switch (ch[i].done) {
        case kConverged:
          s = ch[i].true_rr <= ch[i].accept ? BHX_OK : BHX_NOT_CONVERGED;
          break;
        case kMaxIt: s = BHX_NOT_CONVERGED; break;
        default: s = BHX_ERR_BREAKDOWN; break;
      }
    }
    if (s < 0 && ret >= 0) ret = s;
    else if (s > 0 && ret == BHX_OK) ret = s;
    if (stats) {
      bhx_stats& o = stats[i];
      o.status = s;
      o.iterations = preset[i] ? 0 : ch[i].iter;
      o.restarts = preset[i] ? 0 : ch[i].restarts;
      o.n_unknown = (int)ch[i].n_unknown;
      const double bb0 = ch[i].bb0;
      const bool rep = (!preset[i] || warm_done[i]) && bb0 > 0;   // residuals to report
      o.rel_residual = rep ? std::sqrt(ch[i].rr / bb0) : 0.0;
      o.true_rel_residual = rep ? std::sqrt(ch[i].true_rr / bb0) : 0.0;
      o.seconds = secs;
      for (int p = 0; p < 4; ++p) {
        o.pass_ms[p] = pass_ms[p];
        o.pass_launches[p] = pass_cnt[p];
      }
    }
  }
  return ret;
}

static int solve_batch_once(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R,
                            hipStream_t stream, bhx_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = stream ? stream : hd->own_stream;
  Grids g;
  {
    const int s = prepare_batch(hd, n, specs, R, st, &g);
    if (s != BHX_OK) return s;
  }
  DriveCtx X;
  X.B = hd->batch_d;
  X.ctl_d = (Ctl*)hd->ws;
  X.ch = hd->ctl_h;
  X.flag_d = hd->flag_d;
  X.graphs = true;
  // one instance runs without work lists (its item index is its item)
  X.compact = n > 1 && compaction_enabled();
  return drive_batch(hd, n, specs, R, g, st, X, stats, t0);
}

int warm_start_outcome(const Ctl& c) {
  if (!std::isfinite(c.rr)) return 2;
  return c.rr <= c.accept ? 1 : 0;
}

int debug_apply(bhx_handle* hd, int op, const double* phi, const double* in, double* out, int nx,
                int ny, int nz, int bcx, int bcy, int bcz, int precision, hipStream_t stream) {
  bhx_opts o;
  bhx_default_opts(&o);
  o.precision = precision & 15;          // bits 4-7: the transform choice (bhx_opts.transform)
  o.transform = (precision >> 4) & 15;
  const Resolved R = resolve_opts(&o);
  if (R.transform > 2) return BHX_ERR_ARG;
  hipStream_t st = stream ? stream : hd->own_stream;
  InstSpec s{phi, out, nx, ny, bcx, bcy, 0.5};
  const bool d3 = nz > 1;
  if (d3) {
    s.nz = nz;
    s.bcz = bcz;
    s.dim = 3;
  }
  Grids g;
  int rc = prepare_batch(hd, 1, &s, R, st, &g);
  if (rc != BHX_OK) return rc;
  Layout L;
  {
    const AxisPlan PX = hd->plans.plan(hd->plans.get(nx, bcx));
    const AxisPlan PY = hd->plans.plan(hd->plans.get(ny, bcy));
    make_layout(nx, ny, nz, R.precision, PX.m, PY.m, d3 ? core_length(fft_length(nz, bcz)) : 0,
                R.sched.rows_cap, &L, !d3 && use_dense(R, PX, PY));
  }
  const size_t N = (size_t)nx * ny * nz;
  const size_t Np = vec_stride(nx, ny * nz);
  double* v = (double*)((char*)hd->ws + align_up(sizeof(Ctl)) + L.off_vec);
  double* r = v;
  double* q = v + 3 * Np;
  double* z = v + 4 * Np;
  BHX_CHECK(launch_setup(hd->batch_d, g.dim, g.s, st));
  BHX_CHECK(launch_setup_rows(hd->batch_d, std::max(g.r, g.rd), st));
  if (op == 0) {
    BHX_CHECK(hipMemcpyAsync(z, in, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    BHX_CHECK(launch_stencil(hd->batch_d, g.dim, kModeApply, g.s, 0, st));
    BHX_CHECK(hipMemcpyAsync(out, q, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    BHX_CHECK(hipMemcpyAsync(r, in, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    BHX_CHECK(launch_precond(hd->batch_d, R, g, st));
    BHX_CHECK(hipMemcpyAsync(out, z, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  BHX_CHECK(hipStreamSynchronize(st));
  return BHX_OK;
}

// Shape signature of a batch for the autotuner cache.
static unsigned long long batch_signature(int n, const InstSpec* specs, const Resolved& R) {
  unsigned long long h = 1469598103934665603ULL;
  auto mix = [&](unsigned long long v) {
    h ^= v;
    h *= 1099511628211ULL;
  };
  mix((unsigned long long)n);
  mix((unsigned long long)(R.precision * 4 + R.precond * 2 + R.flexible + 16 * R.transform));
  for (int i = 0; i < n; ++i) {
    mix((unsigned long long)specs[i].nx);
    mix((unsigned long long)specs[i].ny);
    mix((unsigned long long)(specs[i].dim == 3 ? specs[i].nz : 1));
    mix((unsigned long long)(specs[i].bcx * 16 + specs[i].bcy + 256 * specs[i].bcz));
  }
  return h;
}

// Project autotuner: time short trial solves (a fixed number of iterations
// in one graph) of this batch's shape under candidate schedules and keep the
// fastest.  A trial writes F only at unknown nodes, which a cold solve
// ignores on input and overwrites; a warm start is saved before the trials
// and put back after them (solve_batch).
static int autotune_schedule(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R,
                             hipStream_t stream, Schedule* best) {
  const int trial_iters = 24;
  std::vector<Schedule> cands;
  // the FFT family under every grouping and occupancy (the option's
  // transform choice when it fixes one)
  const int t_opt = R.transform;
  for (int rows : {1, 2, 4})
    for (int occ : {1, 2, 4}) {
      Schedule s;
      s.rows_cap = rows;
      s.occ_r = occ;
      s.occ_c = occ;
      s.occ_s = 8;
      s.chunk = trial_iters;
      s.transform = t_opt == 0 ? 1 : t_opt;
      cands.push_back(s);
    }
  // with the transform left to the library: the built-in choice and dense
  // wherever the axes allow, at one or two dense blocks per CU
  bool eligible = false;
  for (int i = 0; i < n; ++i)
    eligible |= specs[i].dim == 2 && specs[i].nx <= kDenseMax && specs[i].ny <= kDenseMax;
  if (t_opt == 0 && eligible && R.precond)
    for (int t : {0, 2})
      for (int occ_d : {1, 2}) {
        Schedule s;
        s.rows_cap = 2;
        s.occ_r = s.occ_c = 2;
        s.occ_s = 8;
        s.chunk = trial_iters;
        s.transform = t;
        s.occ_d = occ_d;
        cands.push_back(s);
      }
  double best_t = 1e30;
  std::vector<bhx_stats> st(n);
  for (const Schedule& s : cands) {
    Resolved T = R;
    T.sched = s;
    T.maxit_user = trial_iters;
    T.chunk = trial_iters;
    T.profile = 0;
    T.accurate = 0;
    T.warm = 0;                               // timed from x0 = 0, whatever F holds
    double t = 0;
    for (int rep = 0; rep < 2; ++rep) {       // first run captures the graph
      const auto a = std::chrono::steady_clock::now();
      int rc = solve_batch_once(hd, n, specs, T, stream, st.data());
      if (rc < 0 && rc != BHX_ERR_SINGULAR && rc != BHX_ERR_NONFINITE) return rc;
      t = std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
    }
    if (t < best_t) {
      best_t = t;
      *best = s;
    }
  }
  best->chunk = 0;
  return BHX_OK;
}

static size_t field_bytes(const InstSpec& S) {
  return (size_t)S.nx * S.ny * (S.dim == 3 ? S.nz : 1) * sizeof(double);
}

// The autotuner with the fields' contents kept: F (the warm start) is copied
// to a temporary device buffer before the trial solves and back after them.
static int autotune_keeping_fields(bhx_handle* hd, int n, const InstSpec* specs,
                                   const Resolved& R, hipStream_t stream, Schedule* best) {
  hipStream_t st = stream ? stream : hd->own_stream;
  BHX_CHECK(hipSetDevice(hd->device));
  size_t total = 0;
  std::vector<size_t> off(n);
  for (int i = 0; i < n; ++i) {
    off[i] = total;
    total += align_up(field_bytes(specs[i]));
  }
  char* keep = nullptr;
  BHX_CHECK(hipMalloc((void**)&keep, total));
  int rc = BHX_OK;
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i)
    e = hipMemcpyAsync(keep + off[i], specs[i].F, field_bytes(specs[i]),
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) rc = autotune_schedule(hd, n, specs, R, stream, best);
  for (int i = 0; i < n && e == hipSuccess; ++i)
    e = hipMemcpyAsync(specs[i].F, keep + off[i], field_bytes(specs[i]),
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const hipError_t ef = hipFree(keep);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) {
    set_last_error("autotune_keeping_fields", __LINE__, e);
    return BHX_ERR_HIP;
  }
  return rc;
}

int solve_batch(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R0,
                hipStream_t stream, bhx_stats* stats) {
  if (R0.solver == 1) {
    // banded Cholesky: consecutive instances sharing phi, size and rules
    // (the fields of one level set) share one factorisation
    int ret = BHX_OK;
    for (int i = 0; i < n;) {
      int j = i + 1;
      while (j < n && specs[j].phi == specs[i].phi && specs[j].nx == specs[i].nx &&
             specs[j].ny == specs[i].ny && specs[j].bcx == specs[i].bcx &&
             specs[j].bcy == specs[i].bcy && specs[j].dim == specs[i].dim)
        ++j;
      const int s = solve_direct(hd, j - i, specs + i, R0, stream, stats ? stats + i : nullptr);
      if (s < 0 && ret >= 0) ret = s;
      else if (s > 0 && ret == BHX_OK) ret = s;
      if (s == BHX_ERR_HIP || s == BHX_ERR_NOMEM || s == BHX_ERR_ARG) return s;
      i = j;
    }
    return ret;
  }
  Resolved R = R0;
  if (R.autotune && R.rows_opt == 0 && R.occ_opt == 0) {
    const unsigned long long sig = batch_signature(n, specs, R);
    auto it = hd->tuned.find(sig);
    if (it == hd->tuned.end()) {
      Schedule s;
      int rc = R.warm ? autotune_keeping_fields(hd, n, specs, R, stream, &s)
                      : autotune_schedule(hd, n, specs, R, stream, &s);
      if (rc != BHX_OK) return rc;
      it = hd->tuned.emplace(sig, s).first;
    }
    R.sched = it->second;
  }
  return solve_batch_once(hd, n, specs, R, stream, stats);
}

int tuned_schedule(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R, int* out4) {
  auto it = hd->tuned.find(batch_signature(n, specs, R));
  if (it == hd->tuned.end()) return 0;
  out4[0] = it->second.rows_cap;
  out4[1] = it->second.occ_s;
  out4[2] = it->second.occ_r;
  out4[3] = it->second.occ_c;
  return 1;
}

}  // namespace bhx
