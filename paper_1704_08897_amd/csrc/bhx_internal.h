// Internal layout shared by the HIP kernels and the host driver.
//
// Every solve is a batch of instances.  Each instance has a descriptor in
// device memory (Inst) and a control block (Ctl).  Each pass of the
// conjugate-gradient iteration is one launch over a flat list of work items
// (instance, local item) covering all instances of the batch; a persistent
// grid loops over the list, and items of finished instances return at once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Device pointers inside descriptors carry the global address space in
// device code, so loads through them are global (not flat) accesses.
// Read-only descriptors (batch header, instances, work lists, plans) use the
// constant address space, so kernels fetch them with scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define BHX_GLOBAL __attribute__((address_space(1)))
#define BHX_CONST __attribute__((address_space(4)))
#else
#define BHX_GLOBAL
#define BHX_CONST
#endif

namespace bhx {

constexpr int kThreads = 256;          // threads per workgroup, every kernel
constexpr int kTileX = 64;             // stencil tile (nodes), two dimensions
constexpr int kTileY = 32;
constexpr int kTileX3 = 16;            // stencil tile (nodes), three dimensions
constexpr int kTileY3 = 8;
constexpr int kTileZ3 = 4;
constexpr int kLdsBytes = 80 * 1024;   // LDS for the packed rows of one transform item
constexpr int kLdsMax = 160 * 1024;    // LDS of a CU (gfx950)
constexpr int kLdsDynMax = 152 * 1024; // dynamic LDS cap of a transform launch
constexpr int kMaxPairs = 8;           // (k, n-k) pairs held in registers per thread
constexpr int kMaxGc = 16;             // columns per column-pass item (2 x rows cap)
constexpr int kTargetItems = 512;      // row/column items one instance should supply
// Partial-sum arrays longer than this (tiles + 3 x row groups) are reduced
// once per pass by a one-block launch instead of in every consumer block.
constexpr int kReduceMin = 8192;

enum Bc { kNeumann = 0, kPeriodic = 1, kDirichlet = 2 };

// Pad code of an FFT row of 2^logm complex points in LDS: one pad slot after
// every 2^a elements and one more after every 2^b (b = 31: none), packed as
// (a << 8) | b (see rpos in the kernels).  Chosen per length so that the
// register passes the length runs, the bit-reversed scatter of the inputs and
// natural-order reads spread over the LDS banks (16-byte elements, eight lanes
// per bank cycle): 4096 points (the wide schedule only) pad every 16 and every
// 512, 512 points every 8 and every 64, other lengths every 8 and (from 256
// points) every 2^(logm-4).
__host__ __device__ constexpr int rpos_shift(int logm) {
  return logm == 12 ? (4 << 8) | 9
       : logm == 9  ? (3 << 8) | 6
                    : (3 << 8) | (logm >= 8 ? logm - 4 : 31);
}
// Position of element i of a row with pad code `code`.
__host__ __device__ constexpr int rpos_code(int i, int code) {
  return i + (i >> (code >> 8)) + (i >> (code & 255));
}
// Complex slots of the per-stage twiddle tables of a length-2^logm FFT: h
// for each radix-4 stage of span h (h = 1, 4, 16, ... or 2, 8, 32, ...).
__host__ __device__ inline int stage_twiddles(int logm) {
  int t = 0;
  for (int h = (logm & 1) ? 2 : 1; h < (1 << logm); h <<= 2) t += h;
  return t;
}
// Work lists: stencil tiles, row groups (x rows), column groups (y pencils of
// the transposed buffer) and, in three dimensions, z-pencil groups.
// Spectral pairs (k, partner k) of a transform of n nodes: (k, n-k) mod n
// for k <= n/2; DST-I (k, n-1-k) for k < (n+1)/2.
__host__ __device__ inline int plan_pairs(int n, int bc) {
  return bc == 2 ? (n + 1) >> 1 : (n >> 1) + 1;
}
// Complex LDS slots of a plan's staged tables: the per-stage twiddles, the
// DCT post-twiddles of the pairs' first members (Neumann only: the partner's
// follows by symmetry) and, for passes that scale by the eigenvalues, those
// of the first members (two reals per slot).  m: the core length.
__host__ __device__ inline int table_slots(int n, int m, int bc, bool lam) {
  const int np = plan_pairs(n, bc);
  return stage_twiddles(31 - __builtin_clz(m)) + (bc == 0 ? np : 0) + (lam ? (np + 1) / 2 : 0);
}
// Ghost-node rule of one axis: global index g in [-2, n+1] -> stored index,
// with sign s (Dirichlet odd reflection of Algorithm 1: g[-1] = 0,
// g[-2] = -f[0]); Neumann half-sample even reflection; periodic wrap.
__device__ __forceinline__ int map_axis(int g, int n, int bc, double& s) {
  s = 1.0;
  if (g >= 0 && g < n) return g;
  if (bc == kNeumann) return g < 0 ? -g - 1 : 2 * n - 1 - g;
  if (bc == kPeriodic) return g < 0 ? g + n : g - n;
  if (g == -1 || g == n) { s = 0.0; return 0; }
  s = -1.0;
  return g < 0 ? 0 : n - 1;
}

// Work lists: stencil tiles, row groups, column groups, z-pencil groups, and
// the row and column groups of instances whose preconditioner runs as dense
// matrix products (kPassRD, kPassCD; those instances are absent from the
// kPassR and kPassC lists).
enum Pass { kPassS = 0, kPassR = 1, kPassC = 2, kPassZ = 3, kPassRD = 4, kPassCD = 5,
            kNumPass = 6 };

// Dense transforms: lines per work item (one 16-wide matrix-core tile) and
// the longest axis they take.
constexpr int kDenseG = 16;
constexpr int kDenseMax = 512;

// Kinds of column-transform launch.  Two dimensions: one launch transforms
// along y, scales by 1/(lambda_x + lambda_y)^2 and transforms back.  Three
// dimensions: forward along y, then along z with the scale by
// 1/(lambda_x + lambda_y + lambda_z)^2 and the inverse along z, then the
// inverse along y.
enum ColKind { kCol2D = 0, kColYFwd = 1, kColZ = 2, kColYInv = 3 };

// Stencil kernel modes.
enum SMode {
  kModeRhs = 0,     // r = -(A f_K) at U, f_K = F at K and 0 at U; partial ||r||^2
  kModeIter = 1,    // p = z + beta p; q = A p at U; partial p.q; convergence test
  kModeResid = 2,   // r = -(A F) at U in double-double (true residual); partial ||r||^2
  kModeApply = 3,   // q = A (z at U, 0 at K) at U (diagnostic operator application)
  kModeWarm = 4,    // r = -(A F) at U with F's values at U as the start x0 (b - A_UU x0);
                    // partial ||r||^2
};

// Done codes in Ctl::done.
enum Done { kRunning = 0, kConverged = 1, kMaxIt = 2, kBreakdown = 3, kSkip = 4 };

// One 1-D transform: length n, boundary rule, FFT core of length m.
struct AxisPlan {
  int n;
  int bc;          // Bc
  int m;           // power-of-two core length (== nf, or >= 2nf-1 for Bluestein)
  int logm;
  int bluestein;   // 0: direct radix-4/2 core; 1: chirp-z through length m
  int off_tw;      // W_m^k = exp(-2 pi i k / m), k < m/2        (complex table)
  int off_chirp;   // exp(-i pi k^2 / nf), k < nf                (complex table)
  int off_bhat;    // FFT_m(conj chirp, wrapped) / m, length m   (complex table)
  int off_post;    // DCT: exp(-i pi k / (2n)), k < n; Dirichlet: unused
  int off_lam;     // eigenvalues lambda_k of T, k < n           (real table)
  int nf;          // length of the DFT computed: n (DCT-II via Makhoul, Hartley);
                   // 2(n+1) for DST-I (odd extension 0, x, 0, -reversed x); n + 1
                   // points for the chirp-z DST-I (cz)
  int cz;          // 1: DST-I as a chirp-z transform: x at 1..n of a DFT of length
                   // 2(n+1) (chirp exp(-i pi k^2 / (2 nf))), outputs 0..n, one real
                   // line per complex row (Dirichlet axes of 1024-2046 nodes)
  // Dense form of the 1-D transform (n <= kDenseMax, else dense_P = 0): the
  // unnormalised basis T(k, i) = dtab[f(((k + ck) (di i + ci)) mod P)] with
  // (ck, di, ci, P) = (0, 2, 1, 4n) and dtab[a] = cos(pi a / 2n) (DCT-II),
  // (0, 1, 0, n) and cos(2 pi a / n) + sin(2 pi a / n) (Hartley), (1, 1, 1,
  // 2(n+1)) and sin(pi a / (n+1)) (DST-I); f(a) = min(a, P - a) for the
  // cosine (dense_fold = 1, P/2 + 1 entries), f(a) = a otherwise.  The
  // orthonormal transform is nk(k) T(k, i) with nk = s_0, s_1 (DCT) or 2 hs.
  int dense_P;
  int dense_fold;
  int off_dtab;    // dense basis table (real table), dense_len entries
  int dense_len;
  // normalisations: DCT-II s_0 = sqrt(1/n), s_k = sqrt(2/n); its inverse's
  // pre-scale g_0 = 1/sqrt(n), g_k = 1/sqrt(2n); hs: Hartley 1/(2 sqrt(n)),
  // DST-I sqrt(2/(n+1)) / 2
  double s0, s1, g0, g1, hs;
};

struct Ctl {
  int iter;           // completed iterations (matrix-vector products)
  int done;           // Done
  int restart_iter;   // iteration at which beta restarts from 0
  int restarts;
  double bb;          // ||b||^2 (of the current restart's right-hand side)
  double bb0;         // ||b||^2 of the original system
  double rr;          // last recursive ||r||^2 (written when done)
  double true_rr;     // compensated true ||r||^2 (finalize)
  double thresh;      // stop when the recursive ||r||^2 <= thresh
  double accept;      // accept when the true ||r||^2 <= accept (= tol^2 bb0)
  double tol_inner2;  // accurate mode: thresh = tol_inner^2 * (restart ||r||^2)
  double tol2;        // tol^2
  double n_unknown;
  int accurate;
  int max_restarts;
  // scalars of an instance with Inst::reduce, summed by k_reduce from the
  // partials of the pass before: p.q, ||r||^2, r.z and r.z_old by parity
  double red_pq, red_rr, red_rz[2], red_rzo[2];
  double pad[2];
};

struct Inst {
  int nx, ny, nz;       // nz = 1 in two dimensions
  int nrows;            // x rows: ny * nz
  int bcx, bcy, bcz;
  int planx, plany, planz;   // AxisPlan indices (planz unused in two dimensions)
  int G;                // rows per item in the row passes (even)
  int Gc;               // columns per item in the column pass (even)
  int Gz;               // z pencils per item in the z pass (even; three dimensions)
  int tiles_x, tiles_y, tiles_z; // stencil tiles
  int n_items[kNumPass];
  int maxit;
  int flexible;
  int warm;             // 1: F's values at U on input are the first iterate x0
  int reduce;           // 1: scalars come from Ctl::red_* (k_reduce), not the partials
  int dense;            // 1: the preconditioner's transforms are dense matrix
                        //    products on the matrix cores (k_rowfwd_dense, k_col_dense,
                        //    k_rowinv_dense; G = Gc = kDenseG)
  BHX_GLOBAL const double* phi;
  BHX_GLOBAL double* F;
  BHX_GLOBAL uint8_t* mask;   // 1 = unknown, 0 = known
  BHX_GLOBAL double* r;
  BHX_GLOBAL double* p[2];    // search direction, double-buffered by iteration parity
  BHX_GLOBAL double* q;
  BHX_GLOBAL double* z;
  BHX_GLOBAL void* t;         // transform buffer, [nx][nz][ny] (y fastest), double or float
  BHX_GLOBAL double* part;    // partial sums, see PartLayout
  BHX_GLOBAL Ctl* ctl;
};

// Offsets (in doubles) of the partial-sum arrays inside Inst::part.
struct PartLayout {
  int nS, nR;
  __host__ __device__ PartLayout(int s, int r) : nS(s), nR(r) {}
  __host__ __device__ int pq() const { return 0; }                  // [nS]
  __host__ __device__ int aux() const { return nS; }                // [nS]  counts U / ||r||^2
  __host__ __device__ int aux2() const { return 2 * nS; }           // [nS]  counts K
  __host__ __device__ int rr() const { return 3 * nS; }             // [nR]
  __host__ __device__ int rz(int par) const { return 3 * nS + nR + par * nR; }    // 2 x [nR]
  __host__ __device__ int rzo(int par) const { return 3 * nS + 3 * nR + par * nR; } // 2 x [nR]
  __host__ __device__ int rowcnt() const { return 3 * nS + 5 * nR; }   // [nR] unknowns per row group
  __host__ __device__ int total() const { return 3 * nS + 6 * nR; }
};

// Items instance I contributes to the work list of pass p: a dense
// instance's row and column groups go to the dense lists instead of the FFT
// ones; I.n_items holds the group counts either way (the partial sums are
// laid out by them).
__host__ __device__ inline int list_items(const Inst& I, int p) {
  if (p == kPassR || p == kPassC) return I.dense ? 0 : I.n_items[p];
  if (p == kPassRD) return I.dense ? I.n_items[kPassR] : 0;
  if (p == kPassCD) return I.dense ? I.n_items[kPassC] : 0;
  return I.n_items[p];
}

// Flat work list of one pass: items[i] = (instance << 20) | local item.
constexpr int kItemShift = 20;
constexpr int kItemMask = (1 << kItemShift) - 1;

// Batch header, resident in device memory; kernels read it at run time so a
// captured graph stays valid while the batch's contents change.
struct Batch {
  int count;                 // instances
  int n_items[kNumPass];     // total items per pass
  BHX_CONST const Inst* inst;           // [count]
  BHX_CONST const int* items[kNumPass];
  BHX_CONST const AxisPlan* plans;
  BHX_GLOBAL const void* ctab[2];       // complex tables: [0] double2, [1] float2
  BHX_GLOBAL const void* rtab[2];       // real tables (eigenvalues): [0] double, [1] float
};

}  // namespace bhx

// Launch wrappers (defined with the kernels).
namespace bhx {
enum FinModeHost { kFinSetupH = 0, kFinResidH = 1, kFinWarmH = 2 };
// The pass launches take an optional pair of events that the dispatch itself
// records at kernel start and end (hipExtLaunchKernelGGL), so their elapsed
// time is the kernel's execution time.
// The stencil-family launches (setup, stencil, residual, zeroing) take the
// batch's dimension `dim` (2 or 3; a batch holds one dimension).
hipError_t launch_setup(const Batch* B, int dim, int grid, hipStream_t st);
// `lpar` is the buffer parity of an iteration's launches: consecutive
// iterations alternate it; the preconditioner applied after setup or a
// restart runs with parity 1, so the first iteration runs with parity 0.
hipError_t launch_stencil(const Batch* B, int dim, int mode, int grid, int lpar, hipStream_t st,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_resid(const Batch* B, int dim, int grid, hipStream_t st);
// Transform launches: `lds` dynamic LDS bytes, `twoff` complex-element offset
// of the twiddle table staged in LDS (after the largest packed-row buffer).
// `shape`: 0 = kernels that read every shape from the plan table; otherwise
// (G << 8) | (L << 2) | bc of the pass's axis and line group (2^L nodes,
// Neumann or periodic, FP64, G lines per work item), whose compile-time
// instance runs instead.  shape_key() gives it for one instance's axis of
// pass family `pass` (ShapePass), or 0 when that shape is not instantiated; a
// batch uses it when every instance has that axis plan and grouping.
enum ShapePass { kShapeRow = 0, kShapeCol2D = 1, kShapeColY = 2, kShapeColZ = 3 };
// Plan-table kernel families (`shape` values below 2^8, which no compile-time
// shape takes): kShapeNarrowKey (0) has only the one-stage FFT passes, which
// keeps its register use low; kShapeWideKey also has the 16-point passes,
// for launches with a work item of at least kFftWideLaunch points
// (rows x FFT length); kShapeCzKey in addition the chirp-z Dirichlet path,
// for launches with such an axis.  All three give bit-identical results.
constexpr int kShapeNarrowKey = 0;
constexpr int kShapeCzKey = 1;
constexpr int kShapeWideKey = 2;
enum PlanFamily { kFamNarrow = 0, kFamWide = 1, kFamCz = 2 };
constexpr int kFftWideLaunch = 4096;
// Plan-table families take the shape values below 2^8; compile-time shapes
// have G >= 2 in bits 8 and up.
inline bool plan_table_shape(int shape) { return shape < 256; }
int shape_key(int pass, int prec, int n, int m, int logm, int bluestein, int bc, int group);
// `stream_t` != 0: the row-forward pass writes t with non-temporal stores.
// Its transposed store writes G-element pieces of many lines.  While the
// launch's whole t is small the pass is latency-bound, and streaming those
// pieces past the L2 shortens the write-back at the kernel's end; on a large
// t the unmerged pieces cost HBM bandwidth instead.  The runtime sets it when
// the launch's t arrays total at most kStreamTMax bytes.
hipError_t launch_rowfwd(const Batch* B, int prec, int shape, int update, int stream_t, int grid,
                         int lds, int twoff, int lpar, hipStream_t st, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
hipError_t launch_col(const Batch* B, int prec, int shape, int kind, int count_iter, int grid,
                      int lds, int twoff, hipStream_t st, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
hipError_t launch_rowinv(const Batch* B, int prec, int shape, int grid, int lds, int twoff,
                         int lpar, hipStream_t st, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
// Unknown counts per row group, over the FFT and the dense row-group lists.
hipError_t launch_setup_rows(const Batch* B, int grid, hipStream_t st);
// Dense-transform passes (instances with Inst::dense): `lds` dynamic LDS
// bytes (dense_lds_bytes of the pass and the longest axis of the launch),
// `tab_off` the element offset of the basis table in it (dense_tab_off).
hipError_t launch_rowfwd_dense(const Batch* B, int prec, int update, int grid, int lds,
                               int tab_off, int lpar, hipStream_t st, hipEvent_t e0 = nullptr,
                               hipEvent_t e1 = nullptr);
hipError_t launch_col_dense(const Batch* B, int prec, int count_iter, int grid, int lds,
                            int tab_off, hipStream_t st, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);
hipError_t launch_rowinv_dense(const Batch* B, int prec, int grid, int lds, int tab_off,
                               int lpar, hipStream_t st, hipEvent_t e0 = nullptr,
                               hipEvent_t e1 = nullptr);
int dense_lds_bytes(int pass, int prec, int n_max);
int dense_tab_off(int n_max);
hipError_t launch_identity(const Batch* B, int grid, int lpar, hipStream_t st,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_finalize(const Batch* B, int count, int mode, hipStream_t st);
// k_reduce after the pass that wrote the partials: p.q (stencil), ||r||^2
// (row forward) or r.z (row inverse / identity, launched with parity lpar).
enum RedWhich { kRedPQ = 0, kRedRR = 1, kRedRZ = 2 };
hipError_t launch_reduce(const Batch* B, int count, int which, int lpar, hipStream_t st);
hipError_t launch_restart(const Batch* B, int count, hipStream_t st);
hipError_t launch_bump(const Batch* B, int count, hipStream_t st);
hipError_t launch_zero_unknown(const Batch* B, int dim, const int* flag, int grid,
                               hipStream_t st);
hipError_t set_kernel_attributes();
}  // namespace bhx
