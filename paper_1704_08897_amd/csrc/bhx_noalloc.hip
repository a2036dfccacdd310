// Allocation-free single solve.  Every device buffer the solve needs - the
// batch header, the instance descriptor, the work lists, the transform plans
// and tables, the control block, the flags and the workspace vectors - is
// carved from one static device array of the library, `scratch`, so the call
// itself allocates no device or pinned memory.  The kernels are the ones of
// the handle path; only where their buffers live differs, and the iteration
// chunks are launched directly instead of from captured graphs.
#include <cstdio>
#include <cstring>
#include <mutex>

#include "bhx_runtime.h"

namespace bhx {

namespace {

constexpr size_t kScratchBytes = (size_t)BHX_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per device; its device address is looked up once per device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lookup_mu;
void* g_scratch_ptr[kMaxDevices] = {};
// Calls on one device share its array: they are serialised in this process.
std::mutex g_call_mu[kMaxDevices];

size_t up256(size_t x) { return (x + 255) / 256 * 256; }


}  // namespace

int noalloc_scratch(int device, void** ptr, size_t* bytes) {
  if (device < 0 || device >= kMaxDevices) return BHX_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_lookup_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) {
      hipError_t e = hipSetDevice(device);
      if (e != hipSuccess) {
        set_last_error("hipSetDevice (scratch lookup)", __LINE__, e);
        return BHX_ERR_HIP;
      }
    }
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_last_error("hipGetSymbolAddress(scratch)", __LINE__, e);
      return BHX_ERR_HIP;
    }
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  *bytes = kScratchBytes;
  return BHX_OK;
}

int solve_noalloc(bhx_handle* hd, const InstSpec& spec, const Resolved& R, hipStream_t stream,
                  bhx_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (R.autotune || R.profile || R.solver != 0) {
    set_last_message("bhx_extend_noalloc: autotune, profile and solver = 1 are not available here");
    return BHX_ERR_ARG;
  }
  if (hd->device < 0 || hd->device >= kMaxDevices) return BHX_ERR_ARG;
  std::lock_guard<std::mutex> call(g_call_mu[hd->device]);
  hipError_t e = hipSetDevice(hd->device);
  if (e != hipSuccess) {
    set_last_error("hipSetDevice", __LINE__, e);
    return BHX_ERR_HIP;
  }
  void* base_v = nullptr;
  size_t cap = 0;
  {
    const int rc = noalloc_scratch(hd->device, &base_v, &cap);
    if (rc != BHX_OK) return rc;
  }
  char* base = (char*)base_v;           // device address of this device's scratch
  hipStream_t st = stream ? stream : hd->own_stream;

  // host side: plans of the two axes in a cache of their own (never uploaded
  // by it), layout, descriptors
  PlanCache plans;
  BatchDesc D;
  {
    const int rc = plan_layouts(plans, 1, &spec, R, &D);
    if (rc != BHX_OK) return rc;
  }
  describe_batch(plans, 1, &spec, R, nullptr, nullptr, &D);     // sizes only
  std::vector<double2> cd;
  std::vector<float2> cf;
  std::vector<double> rd;
  std::vector<float> rf;
  plans.tables_host(&cd, &cf, &rd, &rf);
  const std::vector<AxisPlan>& ph = plans.plans_host();

  // scratch layout (256-byte aligned pieces)
  size_t o = 0;
  const size_t o_hdr = o;   o = up256(o + sizeof(Batch));
  const size_t o_inst = o;  o = up256(o + sizeof(Inst));
  size_t o_items[kNumPass];
  for (int p = 0; p < kNumPass; ++p) {
    o_items[p] = o;
    o = up256(o + std::max<size_t>(1, D.items[p].size()) * sizeof(int));
  }
  const size_t o_plans = o; o = up256(o + ph.size() * sizeof(AxisPlan));
  const size_t o_cd = o;    o = up256(o + cd.size() * sizeof(double2));
  const size_t o_cf = o;    o = up256(o + cf.size() * sizeof(float2));
  const size_t o_rd = o;    o = up256(o + rd.size() * sizeof(double));
  const size_t o_rf = o;    o = up256(o + rf.size() * sizeof(float));
  const size_t o_flag = o;  o = up256(o + sizeof(int));
  const size_t o_ws = o;    o = up256(o + D.ws_bytes);
  if (o > cap) {
    char msg[200];
    snprintf(msg, sizeof(msg),
             "bhx_extend_noalloc: %dx%d needs %zu bytes of scratch, the limit is %zu", spec.nx,
             spec.ny, o, cap);
    set_last_message(msg);
    return BHX_ERR_ARG;
  }
  describe_batch(plans, 1, &spec, R, base + o_ws, (Ctl*)(base + o_ws), &D);
  int* items_d[kNumPass];
  for (int p = 0; p < kNumPass; ++p) items_d[p] = (int*)(base + o_items[p]);
  const void* ctab[2] = {base + o_cd, base + o_cf};
  const void* rtab[2] = {base + o_rd, base + o_rf};
  Batch Bh;
  fill_header(&Bh, D, (const Inst*)(base + o_inst), items_d, (const AxisPlan*)(base + o_plans),
              ctab, rtab);
  Grids g;
  {
    const int rc = batch_grids(plans, D, R, hd->num_cu, &g);
    if (rc != BHX_OK) return rc;
  }

  // device side: earlier work on st may still read the scratch of a previous
  // call; then stream-ordered copies from pageable host memory, complete
  // before the host buffers above go out of scope (the driver synchronises
  // st before it reads its first control block)
#define NA_CHECK(x)                                                     \
  do {                                                                  \
    hipError_t _e = (x);                                                \
    if (_e != hipSuccess) {                                             \
      set_last_error(#x, __LINE__, _e);                                 \
      return BHX_ERR_HIP;                                               \
    }                                                                   \
  } while (0)
  NA_CHECK(hipStreamSynchronize(st));
  struct Piece {
    size_t off;
    const void* src;
    size_t bytes;
  };
  const Piece pieces[] = {
      {o_hdr, &Bh, sizeof(Batch)},
      {o_inst, D.inst.data(), sizeof(Inst)},
      {o_items[kPassS], D.items[kPassS].data(), D.items[kPassS].size() * sizeof(int)},
      {o_items[kPassR], D.items[kPassR].data(), D.items[kPassR].size() * sizeof(int)},
      {o_items[kPassC], D.items[kPassC].data(), D.items[kPassC].size() * sizeof(int)},
      {o_items[kPassZ], D.items[kPassZ].data(), D.items[kPassZ].size() * sizeof(int)},
      {o_plans, ph.data(), ph.size() * sizeof(AxisPlan)},
      {o_cd, cd.data(), cd.size() * sizeof(double2)},
      {o_cf, cf.data(), cf.size() * sizeof(float2)},
      {o_rd, rd.data(), rd.size() * sizeof(double)},
      {o_rf, rf.data(), rf.size() * sizeof(float)},
      {o_ws, D.ctl.data(), sizeof(Ctl)},
  };
  for (const Piece& pc : pieces)
    if (pc.bytes) NA_CHECK(hipMemcpyAsync(base + pc.off, pc.src, pc.bytes,
                                          hipMemcpyHostToDevice, st));
  NA_CHECK(hipStreamSynchronize(st));
#undef NA_CHECK
  Ctl ch;
  DriveCtx X;
  X.B = (const Batch*)(base + o_hdr);
  X.ctl_d = (Ctl*)(base + o_ws);
  X.ch = &ch;
  X.flag_d = (int*)(base + o_flag);
  X.graphs = false;
  return drive_batch(hd, 1, &spec, R, g, st, X, stats, t0);
}

}  // namespace bhx
