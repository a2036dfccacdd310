// Host runtime of the biharmonic-extension library: transform plans, device
// workspace, batch construction and the PCG driver loop.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <complex>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bhx.h"
#include "bhx_internal.h"

namespace bhx {

// Transform tables for every (n, bc) seen by a handle.  Host master copies
// are long double; device copies are double and float with one layout.
class PlanCache {
 public:
  ~PlanCache();
  int get(int n, int bc);                // plan index, created on first use
  // Upload the tables if new plans were added: stream-ordered on `st`, and
  // complete on return.
  hipError_t sync_device(hipStream_t st);
  const AxisPlan& plan(int i) const { return plans_[i]; }
  const AxisPlan* plans_d() const { return plans_d_; }
  const void* ctab(int p) const { return p == 0 ? (const void*)ctab_d_ : (const void*)ctab_f_; }
  const void* rtab(int p) const { return p == 0 ? (const void*)rtab_d_ : (const void*)rtab_f_; }
  void release();
  // Host copies of every plan and table, rounded as the device copies are
  // (for callers that place them in memory of their own).
  const std::vector<AxisPlan>& plans_host() const { return plans_; }
  void tables_host(std::vector<double2>* cd, std::vector<float2>* cf, std::vector<double>* rd,
                   std::vector<float>* rf) const;

 private:
  std::vector<AxisPlan> plans_;
  std::vector<std::complex<long double>> ctab_;
  std::vector<long double> rtab_;
  std::map<std::pair<int, int>, int> index_;
  bool dirty_ = false;
  AxisPlan* plans_d_ = nullptr;
  double2* ctab_d_ = nullptr;
  float2* ctab_f_ = nullptr;
  double* rtab_d_ = nullptr;
  float* rtab_f_ = nullptr;
  size_t cap_plans_ = 0, cap_c_ = 0, cap_r_ = 0;
};

// Static description of one instance before device pointers are assigned.
struct InstSpec {
  const double* phi;
  double* F;
  int nx, ny, bcx, bcy;
  double tol;
  int nz = 1, bcz = 0;       // three dimensions: nz >= 4 and dim = 3
  int dim = 2;
};

// Per-instance layout decisions.
struct Layout {
  int G, Gc, Gz, tiles_x, tiles_y, tiles_z;
  int n_items[kNumPass];
  size_t off_mask, off_vec, off_t, off_part, off_ctl, bytes;
};

// Choose row-group sizes and item counts; false if the size is unsupported.
// mz = 0: two dimensions (nz = 1); otherwise the z core length.
// dense: the instance's preconditioner runs the dense-transform passes
// (row and column groups of kDenseG lines).
// rows_cap: packed rows per transform work item; 0 = the built-in policy
// (as many as fit, reduced until the instance alone supplies kTargetItems
// items), -1 = as many as fit.
bool make_layout(int nx, int ny, int nz, int prec, int mx, int my, int mz, int rows_cap,
                 Layout* L, bool dense = false);
inline bool make_layout(int nx, int ny, int prec, int mx, int my, int rows_cap, Layout* L,
                        bool dense = false) {
  return make_layout(nx, ny, 1, prec, mx, my, 0, rows_cap, L, dense);
}
// Core FFT length of a transform of length n (power of two, or Bluestein).
int core_length(int n);
// Spacing of the float64 workspace vectors (elements), 256-byte aligned.
size_t vec_stride(int nx, int ny);
// Largest supported transform length for a precision (0 fp64, 1 fp32).
bool length_supported(int n, int prec);

// Launch schedule: packed rows per transform item (0 = policy), persistent
// blocks per CU of the stencil / row / column passes.
struct Schedule {
  int rows_cap = 0;
  int occ_s = 8, occ_r = 2, occ_c = 2;
  int chunk = 0;             // 0 = option's chunk
  int transform = -1;        // -1: the option's; else 0 policy, 1 FFT, 2 dense where possible
  int occ_d = 2;             // persistent blocks per CU of the dense-transform passes
};

struct Resolved {           // options after defaults
  int precision, maxit_user, precond, accurate, flexible, chunk, profile, autotune, warm;
  int solver;               // 0 PCG, 1 banded Cholesky (two dimensions)
  int rows_opt = 0, occ_opt = 0;
  int transform = 0;        // 0 built-in choice, 1 FFT only, 2 dense where the axes allow
  double tol_inner;
  Schedule sched;
};
Resolved resolve_opts(const bhx_opts* o);

struct Grids {
  int s, r, c;             // persistent grid sizes of the stencil, row and column passes
  int lds_r, tw_r;         // row passes: dynamic LDS bytes, twiddle offset (complex elements)
  int lds_c, tw_c;         // column (y) passes
  int dim = 2;             // 3: column passes along y, z, y
  int z = 0, lds_z = 0, tw_z = 0;   // z pass (three dimensions)
  int count = 0;           // instances of the batch
  int reduce = 0;          // 1: some instance has Inst::reduce (k_reduce launches)
  int shape_r = 0, shape_c = 0, shape_z = 0;   // compile-time shapes of the passes (shape_key)
  int stream_t = 0;        // 1: the row-forward pass stores t non-temporally
  int fft = 1, dense = 0;  // launch the FFT-family / dense-transform passes
  int rd = 0, cd = 0;      // persistent grids of the dense row and column passes
  int lds_rd = 0, tab_rd = 0, lds_cd = 0, tab_cd = 0;   // their LDS and table offsets
};

// Host description of a batch: plans, layouts, descriptors, work lists,
// control blocks and workspace size.
struct BatchDesc {
  int dim = 2;
  std::vector<int> px, py, pz;
  std::vector<Layout> lay;
  std::vector<int> dense;   // per instance: dense-transform passes
  std::vector<Inst> inst;
  std::vector<int> items[kNumPass];
  std::vector<Ctl> ctl;
  size_t ws_bytes = 0;      // control blocks + instance regions
};

// Plan-table kernel family of a pass (shape kShapeNarrowKey, kShapeWideKey or
// kShapeCzKey): raised to what an axis plan with `rows` packed rows per work
// item needs; compile-time shapes are left alone.
void plan_family(const AxisPlan& P, int rows, int* shape);
// The same over every FFT-family instance of a batch, for the three passes.
void plan_families(const PlanCache& plans, const BatchDesc& D, Grids* g);

// Where the driver loop finds a prepared batch's device state.
struct DriveCtx {
  const Batch* B = nullptr;   // device batch header
  Ctl* ctl_d = nullptr;       // device control blocks [n]
  Ctl* ch = nullptr;          // host copy [n]
  int* flag_d = nullptr;      // device flags [n]
  bool graphs = true;         // captured chunks and pinned uploads; false: direct
                              // launches and pageable copies (no allocation)
  bool compact = false;       // between chunks, drop finished instances' items from
                              // the work lists (needs the handle's host copies)
};

// Largest total of a launch's t arrays (bytes) whose row-forward stores go
// non-temporal: one 1024 x 1024 FP64 instance.
constexpr size_t kStreamTMax = (size_t)8 << 20;

struct Graph {
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  const Batch* batch = nullptr;
  int count = 0;
  int prec = -1, chunk = 0, precond = -1, gs = 0, gr = 0, gc = 0, profile = 0;
  int lds_r = 0, tw_r = 0, lds_c = 0, tw_c = 0;
  int dim = 2, gz = 0, lds_z = 0, tw_z = 0, reduce = 0, shape_r = 0, shape_c = 0, shape_z = 0;
  int stream_t = 0;
  int fft = 1, dense = 0, rd = 0, cd = 0, lds_rd = 0, tab_rd = 0, lds_cd = 0, tab_cd = 0;
  std::vector<hipEvent_t> ev;   // [pass][iteration][start, end] when profiling
};

}  // namespace bhx

struct bhx_handle {
  int device = 0;
  int num_cu = 256;
  bhx::PlanCache plans;
  void* ws = nullptr;          // device workspace (grow-only)
  size_t ws_cap = 0;
  bhx::Batch* batch_d = nullptr;   // device batch header
  bhx::Inst* inst_d = nullptr;
  int inst_cap = 0;
  int* items_d[bhx::kNumPass] = {nullptr, nullptr, nullptr};
  int items_cap[bhx::kNumPass] = {0, 0, 0};
  int batch_count = 0;         // instances of the current batch
  // host copies of the current batch's full work lists and of its header, for
  // compacting the lists while instances finish (drive_batch)
  std::vector<int> items_h[bhx::kNumPass];
  bhx::Batch batch_h{};
  int* flag_d = nullptr;
  int flag_cap = 0;
  bhx::Ctl* ctl_h = nullptr;   // pinned copy of the control blocks
  int ctl_h_cap = 0;
  hipStream_t own_stream = nullptr;
  unsigned char* stage_h = nullptr;   // pinned staging of host->device uploads
  size_t stage_cap = 0;
  std::vector<bhx::Graph> graphs;
  std::map<unsigned long long, bhx::Schedule> tuned;   // autotuner results per batch shape
  void* dws = nullptr;         // direct solver: ordering (grow-only)
  size_t dws_cap = 0;
  void* band = nullptr;        // direct solver: band panels and solve vector (grow-only)
  size_t band_cap = 0;
  std::mutex mu;
};

namespace bhx {
// Validate one instance's arguments (host only).  Returns BHX_OK or BHX_ERR_ARG.
int validate(const double* phi, const double* F, int nx, int ny, double h, int bc, double tol,
             const Resolved& R);
// Three dimensions: bc packs three rules (x, y, z nibbles).
int validate3(const double* phi, const double* F, int nx, int ny, int nz, double h, int bc,
              double tol, const Resolved& R);
// Solve `n` instances on `hd`; stats[n] filled (may be null).
// With R.warm the values of F at the unknown nodes are the first iterate.
int solve_batch(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R,
                hipStream_t stream, bhx_stats* stats);
size_t instance_bytes(int nx, int ny, int bcx, int bcy, int prec, int rows_cap = 0);
size_t instance_bytes3(int nx, int ny, int nz, int bcx, int bcy, int bcz, int prec);
const char* last_error();
void set_last_error(const char* what, int line, hipError_t e);
void set_last_message(const char* what);
int row_slots(int m);
hipError_t launch_precond(const Batch* B, const Resolved& R, const Grids& g, hipStream_t st);
hipError_t run_chunk(bhx_handle* hd, const Batch* B, int n_inst, const Resolved& R,
                     const Grids& g, hipStream_t st, Graph** used);
// One application of the masked operator (op 0) or the preconditioner (op 1)
// to `in`; nz = 1 in two dimensions.
int debug_apply(bhx_handle* hd, int op, const double* phi, const double* in, double* out, int nx,
                int ny, int nz, int bcx, int bcy, int bcz, int precision, hipStream_t stream);
int init_handle(bhx_handle* hd, int device);
// Descriptors, layouts, plans and launch grids of a batch (the solve's first step).
int prepare_batch(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R,
                  hipStream_t st, Grids* gout);
int fft_length(int n, int bc);
// A Dirichlet axis whose DST-I runs as a chirp-z transform of n + 1 points
// (1024 to 2046 nodes; AxisPlan::cz).
bool dst_chirp(int n, int bc);
// Both axes have a dense form (at most kDenseMax nodes).
bool dense_eligible(const AxisPlan& X, const AxisPlan& Y);
// Whether an instance with these axes runs the dense-transform passes under
// the options (transform choice, schedule) R.
bool use_dense(const Resolved& R, const AxisPlan& X, const AxisPlan& Y);
// Launch geometry of the dense-transform passes for axes of at most nx_max,
// ny_max nodes, with `occ` blocks per CU (fills g.rd, g.cd, g.lds_*, g.tab_*).
void dense_grids(int prec, int nx_max, int ny_max, int n_rd, int n_cd, int num_cu, int occ,
                 Grids* g);
// Plan indices and layouts of a batch (host only).
int plan_layouts(PlanCache& plans, int n, const InstSpec* specs, const Resolved& R,
                 BatchDesc* D);
// Bytes of the control-block region at the start of a batch workspace.
size_t ctl_region_bytes(int n);
// Descriptors, work lists and control blocks of a batch whose workspace
// starts at `ws` (control blocks at ctl_d); ws = nullptr computes sizes only.
void describe_batch(const PlanCache& plans, int n, const InstSpec* specs, const Resolved& R,
                    char* ws, Ctl* ctl_d, BatchDesc* D);
// The batch header of a description, given the device copies' addresses.
void fill_header(Batch* Bh, const BatchDesc& D, const Inst* inst_d, int* const items_d[kNumPass],
                 const AxisPlan* plans_d, const void* const ctab[2], const void* const rtab[2]);
// Launch geometry of a described batch.
int batch_grids(const PlanCache& plans, const BatchDesc& D, const Resolved& R, int num_cu,
                Grids* g);
// The solve after a batch is prepared: setup, iterations, exit checks, stats.
int drive_batch(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R, const Grids& g,
                hipStream_t st, const DriveCtx& X, bhx_stats* stats,
                std::chrono::steady_clock::time_point t0);
// `count` iterations launched directly (events of the profiled passes from ev).
hipError_t launch_iterations(const Batch* B, int n_inst, const Resolved& R, const Grids& g,
                             int count, hipStream_t st, const std::vector<hipEvent_t>* ev);
// Allocation-free single solve: every device buffer in the library's static
// scratch array (bhx_noalloc.hip).
int solve_noalloc(bhx_handle* hd, const InstSpec& spec, const Resolved& R, hipStream_t stream,
                  bhx_stats* stats);
// Device address of the scratch array on `device` (looked up once per device
// with that device current) and its size; BHX_OK or BHX_ERR_HIP.
int noalloc_scratch(int device, void** ptr, size_t* bytes);
// Banded Cholesky solve of fields sharing one phi (all specs: same phi, size
// and rules; two dimensions, at most one periodic axis).
int solve_direct(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R,
                 hipStream_t stream, bhx_stats* stats);
bool direct_supported(int bcx, int bcy);
// One host array to copy to device memory.
struct Upload {
  void* dst;
  const void* src;
  size_t bytes;
};
// Copy `n` host arrays to the device in stream order on `st`, through the
// handle's pinned staging buffer, so every later launch on `st` sees them.
// The caller has synchronised `st` since the previous upload (the staging
// buffer is then free); the host sources may be reused on return.
hipError_t upload_ordered(bhx_handle* hd, hipStream_t st, const Upload* u, int n);
// Outcome of the residual of a given first iterate (warm start), decided on
// the host from the control block after the kFinWarm finalisation:
// 0 = iterate from it, 1 = it already meets the tolerance (0 iterations),
// 2 = its residual is not finite.
int warm_start_outcome(const Ctl& c);
void free_handle(bhx_handle* hd);
}  // namespace bhx
