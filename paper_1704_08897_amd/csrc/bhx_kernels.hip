// HIP kernels of the biharmonic-extension PCG (gfx950).
//
// One PCG iteration is four launches, each over the work items of every
// unfinished instance of a batch:
//   S  (k_stencil, mode iter): p = z + beta p; q = A p at unknown nodes; p.q
//   R  (k_rowfwd, update):     alpha = r.z / p.q; x += alpha p; r -= alpha q;
//                              ||r||^2; forward transform of r along x,
//                              written transposed ([nx][ny], y fastest)
//   C  (k_col):                forward transform along y, divide by
//                              (lambda_x + lambda_y)^2, inverse along y
//   RI (k_rowinv):             inverse transform along x, restrict to the
//                              unknown nodes -> z; r.z (and r.z_old)
// The method is Sec. 2.2 and Algorithm 1 of the paper: the 13-point stencil
// of eq. (12) evaluated on demand as the 5-point Laplacian applied twice over
// two ghost layers, and the fast Poisson preconditioner (embed, transform,
// scale by the inverse squared eigenvalues, transform back, restrict).
//
// Transforms: Neumann axes use the orthonormal DCT-II (inverse DCT-III)
// through a complex FFT of the same length (Makhoul's even/odd reordering);
// periodic axes use the orthonormal discrete Hartley transform, a real
// eigenbasis of the symmetric circulant second difference.  Two real rows are
// packed into one complex row.  The complex FFT runs in LDS: radix-4/2
// decimation in time on bit-reversed input for power-of-two lengths, and
// Bluestein's chirp-z (through a power-of-two length m >= 2n-1) otherwise.
//
// Scalars never cross blocks inside a kernel: a producer writes one partial
// sum per work item; every consumer item reduces the partial array itself in
// a fixed order, so each block computes bit-identical alpha/beta and the
// result does not depend on scheduling or on the batch composition (within
// one kernel family: the compile-time-shape instances run only when every
// instance of a launch shares the shape, and agree with the plan-table ones
// to rounding).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <hsa/hsa.h>
#include <stdint.h>
#include <cstdlib>

#include "bhx_internal.h"

namespace bhx {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

template <typename C> __device__ __forceinline__ C mk(decltype(C::x) a, decltype(C::x) b) {
  C c; c.x = a; c.y = b; return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return mk<C>(a.x, -a.y); }
// a * (-i)
template <typename C> __device__ __forceinline__ C cmul_mi(C a) { return mk<C>(a.y, -a.x); }
// a * (+i)
template <typename C> __device__ __forceinline__ C cmul_pi(C a) { return mk<C>(-a.y, a.x); }

// 1 / x by the hardware reciprocal estimate refined with Newton-Raphson
// steps r <- r + r (1 - x r) (quadratic convergence from the estimate).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
// Spectral weight 1 / s^2 for s = lambda_x + lambda_y, 0 when s = 0.
template <typename R> __device__ __forceinline__ R inv_sq(R s) {
  return s > (R)0 ? recip(s * s) : (R)0;
}

// LDS position of element i of a packed FFT row: a pad slot after every 2^a
// elements and another after every 2^b, sh = rpos_shift(logm) = (a << 8) | b.
// The first spreads the small-stride pass loads over the banks, the second
// the bit-reversed scatter of the inputs, whose consecutive indices differ in
// the top bits.
__device__ __forceinline__ int rpos(int i, int sh) { return rpos_code(i, sh); }


__device__ __forceinline__ int bitrev(int k, int logm) {
  return (int)(__brev((unsigned)k) >> (32 - logm));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of a[0..n) by the whole block in a fixed order; every thread gets it.
__device__ double block_sum_array(BHX_GLOBAL const double* __restrict__ a, int n, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) s += a[i];
  s = wave_sum(s);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = s;
  __syncthreads();
  double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// Sum of a long array a[0..n) by one block (the scalars of instances with
// tens of thousands of partials): 16 loads in flight per thread, thread t
// accumulating entries t + kThreads (16 r + u) in acc[u]; the accumulators,
// lanes and waves are then combined in a fixed order.  n is uniform over the
// block.
__device__ double block_sum_long(BHX_GLOBAL const double* __restrict__ a, int n, double* red) {
  constexpr int kU = 16;
  if (n <= 0) return 0.0;
  double acc[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) acc[u] = 0.0;
  for (int i0 = 0; i0 < n; i0 += kU * kThreads) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = a[min(i0 + u * kThreads + (int)threadIdx.x, n - 1)];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      acc[u] += (i0 + u * kThreads + (int)threadIdx.x < n) ? v[u] : 0.0;
  }
#pragma unroll
  for (int h = kU / 2; h > 0; h >>= 1)
#pragma unroll
    for (int u = 0; u < h; ++u) acc[u] += acc[u + h];
  const double s = wave_sum(acc[0]);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = s;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// Sums of K partial arrays a[k][0..n[k]) in one pass (all loads in flight
// together); the order of every sum is fixed, so each block of a launch
// obtains bit-identical values.  red must hold 4*K doubles.
template <int K>
__device__ __forceinline__ void block_sums(BHX_GLOBAL const double* const (&a)[K],
                                           const int (&n)[K], double (&out)[K], double* red) {
  double s[K];
  int nmax = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s[k] = 0.0;
    nmax = max(nmax, n[k]);
  }
  // Straight-line loads from clamped in-bounds indices; out-of-range and
  // empty arrays contribute 0 through a select, so no load sits behind a
  // branch and all of them are in flight together.
  for (int i0 = 0; i0 < nmax; i0 += 4 * kThreads) {
    double v[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * kThreads + threadIdx.x;
        const int ic = min(i, max(n[k] - 1, 0));
        v[k][u] = n[k] > 0 ? a[k][ic] : 0.0;
      }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * kThreads + threadIdx.x;
        s[k] += (i < n[k]) ? v[k][u] : 0.0;
      }
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = wave_sum(s[k]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[w * K + k] = s[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k)
    out[k] = (red[k] + red[K + k]) + (red[2 * K + k] + red[3 * K + k]);
  __syncthreads();
}

// The same sums in two steps, so the loads can be issued early and overlap
// other loads: sums_issue() loads the first 4*kThreads entries of each array
// into registers; sums_finish() adds any remainder and reduces.
template <int K>
struct Partials {
  double v[K][4];
};
// sums_issue() takes the arrays' lengths (>= 1), sums_finish() the counts of
// entries to add (<= length, 0 to skip an array), so the loads need nothing
// decided at run time.  The loads are unconditional, from clamped indices: a
// load behind a branch is followed by a wait for it, which would serialise
// the round trips.
template <int K>
__device__ __forceinline__ void sums_issue(BHX_GLOBAL const double* const (&a)[K],
                                           const int (&len)[K], Partials<K>& P) {
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = u * kThreads + threadIdx.x;
      P.v[k][u] = a[k][min(i, len[k] - 1)];
    }
}
template <int K>
__device__ __forceinline__ void sums_finish(BHX_GLOBAL const double* const (&a)[K],
                                            const int (&n)[K], const Partials<K>& P,
                                            double (&out)[K], double* red) {
  double s[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s[k] = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) s[k] += (u * kThreads + (int)threadIdx.x < n[k]) ? P.v[k][u] : 0.0;
    for (int i = 4 * kThreads + threadIdx.x; i < n[k]; i += kThreads) s[k] += a[k][i];
  }
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = wave_sum(s[k]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[w * K + k] = s[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k)
    out[k] = (red[k] + red[K + k]) + (red[2 * K + k] + red[3 * K + k]);
  __syncthreads();
}

// Block reduction of one value per thread; result valid in every thread.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}


// Branch-free form of map_axis for g in [-2, n+1] (selects only); any other
// g maps to index 0 with sign 0.
__device__ __forceinline__ int map_axis_sel(int g, int n, int bc, double& s) {
  const bool lo = g < 0, hi = g >= n;
  const bool inside = !lo && !hi;
  const bool valid = g >= -2 && g <= n + 1;
  const int refl = lo ? -g - 1 : 2 * n - 1 - g;                // Neumann
  const int wrap = lo ? g + n : g - n;                         // periodic
  const int dir = lo ? 0 : n - 1;                              // Dirichlet, g = -2 or n+1
  const double sdir = (g == -1 || g == n) ? 0.0 : -1.0;
  const int ghost = bc == kNeumann ? refl : (bc == kPeriodic ? wrap : dir);
  const double sghost = bc == kDirichlet ? sdir : 1.0;
  s = inside ? 1.0 : (valid ? sghost : 0.0);
  return inside ? g : (valid ? ghost : 0);
}

// Debug build (BHX_DEBUG_LDS_NAN=1): every transform kernel starts by
// filling its dynamic LDS with NaN, so a read of LDS that no thread of the
// block wrote shows up as NaN in the results instead of as stale values.  The
// dispatch packet gives the block's whole group segment; the dynamic part
// starts at smem.  A no-op in the normal build.
#ifndef BHX_DEBUG_LDS_NAN
#define BHX_DEBUG_LDS_NAN 0
#endif
__device__ __forceinline__ void debug_fill_lds(unsigned char* dyn) {
#if BHX_DEBUG_LDS_NAN
  const hsa_kernel_dispatch_packet_t* pkt =
      (const hsa_kernel_dispatch_packet_t*)__builtin_amdgcn_dispatch_ptr();
  const unsigned total = pkt->group_segment_size;
  const unsigned start =
      (unsigned)(size_t)(__attribute__((address_space(3))) unsigned char*)dyn;
  double* d = (double*)dyn;
  for (unsigned i = threadIdx.x; start + 8 * (i + 1) <= total; i += blockDim.x)
    d[i] = __builtin_nan("");
  __syncthreads();
#else
  (void)dyn;
#endif
}

// Work item `it` of pass `p`: (instance << kItemShift) | local item.  A
// single-instance batch needs no table.
__device__ __forceinline__ int item_code(const Batch& B, int p, int it) {
  return B.count == 1 ? it : B.items[p][it];
}

// Persistent-grid item loop with an XCD-aware block order: consecutive
// logical blocks (neighbouring tiles / row groups) land on the same XCD,
// whose L2 then serves their shared halo rows.
__device__ __forceinline__ int logical_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  if (nb % 8 != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// Transform plan access
// ---------------------------------------------------------------------------

// Logical FFT input index of spatial sample i for the forward transform:
// DCT-II reorders evens ascending then odds descending (Makhoul); the
// Hartley transform takes the samples in order.
__device__ __forceinline__ int fwd_index(int i, int n, int bc) {
  if (bc != kNeumann) return i;
  return (i & 1) ? n - 1 - (i >> 1) : (i >> 1);
}
// Position in the inverse DCT's FFT output holding spatial sample j.
__device__ __forceinline__ int inv_index(int j, int n) {
  return (j & 1) ? n - 1 - (j >> 1) : (j >> 1);
}

constexpr int kStageRound = 4;    // plan-table entries per thread per staging round

// Nodes of an axis of compile-time shape SP: 2^L for the Neumann and periodic
// rules; 2^(L-1) - 1 for the Dirichlet rule, whose DST-I runs through the
// 2(n + 1) = 2^L point odd extension.
__host__ __device__ constexpr int sp_nodes(int sp) {
  return (sp & 3) == kDirichlet ? (1 << (((sp >> 2) & 63) - 1)) - 1 : 1 << ((sp >> 2) & 63);
}

// A transform plan as the kernels use it.  SP = 0 reads the shape from the
// plan table; SP = (G << 8) | (L << 2) | bc fixes it at compile time (an axis
// whose core FFT has 2^L points without Bluestein: sp_nodes(SP) nodes, G
// lines per work item), so that the index arithmetic of every stage folds to
// constants.
template <typename R, int SP = 0>
struct XPlan {
  using C = typename V2<R>::T;
  int n, nf, m, logm, blue, bc, sh;
  int cz;                     // chirp-z DST-I: one real line per FFT row, the two
                              // lines of a pair in turn (plan-table family only)
  R s0, s1, g0, g1, hs;
  BHX_GLOBAL const C* twg;    // W_m^k, k < m/2, in device memory
  const C* tw;                // per-stage twiddle tables in LDS once staged
  BHX_GLOBAL const C* chirp;
  BHX_GLOBAL const C* bhat;
  BHX_GLOBAL const C* post;
  BHX_GLOBAL const R* lam;
  const C* postl;             // post-twiddles of the pairs' first members, in LDS
  const R* laml;              // eigenvalues of the pairs' first members, in LDS
  // Copy the plan's twiddles, the DCT post-twiddles and (with `with_lam`,
  // for passes that scale) the eigenvalues of the pairs' first members into
  // LDS at `lds` (table_slots(n, m, bc, with_lam) complex slots) unless plan
  // `idx` is staged there already; every thread of the block must call this
  // at the same point.  The twiddles are laid out per radix-4 stage of span
  // h: W_4h^k for k < h (stage_twiddles), so each stage reads them at unit
  // stride; the stage squares them for W_2h^k.  The tables are copied as one
  // flat index space in rounds of kStageRound entries per thread, all loads of
  // a round issued before its LDS writes: one or two memory round trips per
  // launch instead of one per table.
  __device__ void stage(C* lds, int idx, int& staged, bool with_lam) {
    if constexpr (SP == 0) {
      // plan-table instances read every table from global memory (L2): the
      // LDS holds the packed rows alone, so two work items fit on a CU even
      // for 4096-point FP64 rows
      return;
    }
    const int np = pairs();
    const int ntw = stage_twiddles(logm);
    C* tw_l = lds;
    C* post_l = lds + ntw;
    R* lam_l = (R*)(post_l + (bc == kNeumann ? np : 0));
    if (idx != staged) {
      const int nc = ntw + (bc == kNeumann ? np : 0);   // complex entries
      const int nl = with_lam ? np : 0;                  // real entries
      const int h0 = (logm & 1) ? 2 : 1;
      for (int base = 0; base < max(nc, nl); base += kStageRound * kThreads) {
        R vr[kStageRound], vi[kStageRound], vl[kStageRound];   // real arrays stay in VGPRs
#pragma unroll
        for (int u = 0; u < kStageRound; ++u) {
          const int e = base + (int)threadIdx.x + u * kThreads;
          C v = mk<C>(0, 0);
          if (e < ntw) {
            // the table of span h = h0 4^j starts at (h - h0) / 3: entry e
            // lies in table j where h0 4^j <= 3e + h0 < h0 4^(j+1)
            const int j = ((31 - __clz(3 * e + h0)) - (h0 - 1)) >> 1;
            const int h = h0 << (2 * j);
            const int ls = logm - 2 - (31 - __clz(h));   // W_4h^k = twg[k << ls]
            v = twg[(e - (h - h0) / 3) << ls];
          } else if (e < nc) {
            v = post[e - ntw];
          }
          vr[u] = v.x;
          vi[u] = v.y;
          vl[u] = e < nl ? lam[e] : (R)0;
        }
#pragma unroll
        for (int u = 0; u < kStageRound; ++u) {
          const int e = base + (int)threadIdx.x + u * kThreads;
          if (e < nc) tw_l[e] = mk<C>(vr[u], vi[u]);
          if (e < nl) lam_l[e] = vl[u];
        }
      }
      __syncthreads();
      staged = idx;
    }
    tw = tw_l;
    postl = post_l;
    laml = lam_l;
  }
  __device__ XPlan(const Batch& B, int idx) {
    const AxisPlan P = B.plans[idx];
    if constexpr (SP != 0) {
      logm = (SP >> 2) & 63;
      nf = m = 1 << logm;
      n = sp_nodes(SP);
      blue = 0;
      bc = SP & 3;
      cz = 0;
    } else {
      n = P.n; nf = P.nf; m = P.m; logm = P.logm; blue = P.bluestein; bc = P.bc;
      cz = P.cz;
    }
    sh = rpos_shift(logm);
    s0 = (R)P.s0; s1 = (R)P.s1; g0 = (R)P.g0; g1 = (R)P.g1; hs = (R)P.hs;
    const int pi = sizeof(R) == 8 ? 0 : 1;
    BHX_GLOBAL const C* ct = (BHX_GLOBAL const C*)B.ctab[pi];
    twg = ct + P.off_tw;
    tw = nullptr;
    postl = nullptr;
    laml = nullptr;
    chirp = ct + P.off_chirp;
    bhat = ct + P.off_bhat;
    post = ct + P.off_post;
    lam = (BHX_GLOBAL const R*)B.rtab[pi] + P.off_lam;
  }
  // LDS position of logical FFT input k (bit-reversed)
  __device__ __forceinline__ int pos(int k) const { return rpos(bitrev(k, logm), sh); }
  // row stride of the packed rows
  __device__ __forceinline__ int stride() const { return rpos(m, sh); }
  // logical FFT output k of a row (after core())
  __device__ __forceinline__ C out(const C* row, int k) const {
    if (!blue) return row[rpos(k, sh)];
    return cmul(chirp[k], row[rpos(bitrev(k, logm), sh)]);
  }
  // Spectral indices are handled in pairs (k, partner(k)): k < pairs().
  // DCT / Hartley: (k, n - k) mod n, k <= n/2; DST-I: (k, n - 1 - k).
  __device__ __forceinline__ int pairs() const { return plan_pairs(n, bc); }
  // DCT-II post-twiddles of the pair: t[k] = exp(-i pi k / 2n) staged, and
  // t[n-k] = -i conj(t[k])
  __device__ __forceinline__ void post_pair(int k, int kk, C& tk, C& tkk) const {
    if constexpr (SP == 0)
      tk = post[k];
    else
      tk = postl[k];
    tkk = kk == k ? tk : mk<C>(-tk.y, -tk.x);
  }
  // eigenvalues of the pair: lambda[partner] = lambda[k] for the periodic
  // axis, 4 - lambda[k] for the DCT and DST-I ones (4 sin^2 -> 4 cos^2)
  __device__ __forceinline__ void lam_pair(int k, int kk, R& lk, R& lkk) const {
    if constexpr (SP == 0)
      lk = lam[k];
    else
      lk = laml[k];
    lkk = kk == k ? lk : (bc == kPeriodic ? lk : (R)4 - lk);
  }
  __device__ __forceinline__ int partner(int k) const {
    return bc == kDirichlet ? n - 1 - k : (k == 0 ? 0 : n - k);
  }
  // FFT bin holding spectral index k (DST-I: bin k+1 of the odd extension)
  __device__ __forceinline__ int bin(int k) const { return bc == kDirichlet ? k + 1 : k; }
  // Forward-transform input: sample i of half h (one of two real rows) of a
  // packed row.  DCT-II: Makhoul order; Hartley: in order; DST-I: +x at
  // i+1 and -x at nf-1-i (odd extension), see zero_ends().
  __device__ __forceinline__ void put(C* row, int i, int h, R v) const {
    if (bc == kDirichlet) {
      ((R*)(row + pos(i + 1)))[h] = v;
      ((R*)(row + pos(nf - 1 - i)))[h] = -v;
    } else {
      ((R*)(row + pos(fwd_index(i, n, bc))))[h] = v;
    }
  }
  // Inputs of the second transform of a pass (values a at k, b at partner
  // kk), placed like put() but for both halves at once.
  __device__ __forceinline__ void put_pair(C* row, int k, int kk, C a, C b) const {
    if (bc == kDirichlet) {
      row[pos(k + 1)] = a;
      row[pos(nf - 1 - k)] = mk<C>(-a.x, -a.y);
      if (kk != k) {
        row[pos(kk + 1)] = b;
        row[pos(nf - 1 - kk)] = mk<C>(-b.x, -b.y);
      }
    } else {
      row[pos(k)] = a;
      if (kk != k) row[pos(kk)] = b;
    }
  }
  // DST-I: the odd extension is zero at 0 and n+1 (no other rule writes them);
  // the chirp-z form has input 0 at 0 (the points past n are zeroed by the
  // Bluestein step)
  __device__ __forceinline__ void zero_ends(C* buf, int rows, int st) const {
    if (bc != kDirichlet) return;
    for (int r = threadIdx.x; r < rows; r += kThreads) {
      buf[r * st + pos(0)] = mk<C>(0, 0);
      if (!cz) buf[r * st + pos(n + 1)] = mk<C>(0, 0);
    }
  }
  // Chirp-z DST-I: sample i of the row's one real line at point i + 1.
  __device__ __forceinline__ void put_cz(C* row, int i, R v) const {
    row[pos(i + 1)] = mk<C>(v, (R)0);
  }
  // Chirp-z DST-I: orthonormal coefficient k of the row's line.  The row
  // holds sum_{j=1..n} x_j W^(jk), W = exp(-2 pi i / (2(n+1))), whose
  // imaginary part is -sum_j x_j sin(pi j k / (n+1)); hs is half of
  // sqrt(2/(n+1)).
  __device__ __forceinline__ R coef_cz(const C* row, int k) const {
    return -out(row, k + 1).y * ((R)2 * hs);
  }
};

// ---------------------------------------------------------------------------
// LDS FFT in register passes
//
// The complex DFT of length m = 2^L is the in-place radix-4 decimation-in-time
// FFT on bit-reversed input (with one radix-2 stage first when L is odd).  Its
// stages are grouped into passes of one or two radix-4 stages (4 or 16
// points; the radix-2 stage joins the first radix-4 one as an 8-point pass):
// each thread loads the RAD points a pass combines into registers, runs the
// pass's stages there and stores them back, so a row goes through LDS once
// per pass instead of once per stage.  A pass of smallest span h combines
// the points base + j h, j < RAD, with base = g RAD h + k and k < h; that set
// is closed under each of its stages.  The inverse transform used inside
// Bluestein's method is decimation in frequency over the same passes in the
// reverse order, so the last forward pass and the first inverse pass combine
// the same points: the pointwise product with the kernel spectrum between the
// two convolution transforms happens in registers, as does the chirp on the
// inputs in the first pass's loads.
// ---------------------------------------------------------------------------

// Passes of a length-2^L FFT in forward order: count, radix, log2 of the
// span.  Wide schedule: 16-point passes (two radix-4 stages each), for blocks
// whose rows hold enough points that every thread gets a 16-point group
// (rows 2^L >= kFftWideMin); narrow schedule otherwise: one radix-4 stage per
// pass, so that more threads share the short rows.
constexpr int kFftWideMin = 2048;
__host__ __device__ constexpr int fft_npass(int L, bool wide) {
  return !wide ? (L & 1) ? 1 + (L - 3) / 2 : L / 2
       : L <= 4 ? 1 : (L & 1) ? 1 + ((L - 3) / 2 + 1) / 2 : (L / 2 + 1) / 2;
}
__host__ __device__ constexpr int fft_pass_rad(int L, int p, bool wide) {
  return !wide ? ((L & 1) && p == 0 ? 8 : 4)
       : L <= 4 ? (1 << L)
       : (L & 1) ? (p == 0 ? 8 : ((((L - 3) / 2) & 1) && p == 1) ? 4 : 16)
                 : (((L / 2) & 1) && p == 0) ? 4 : 16;
}
__host__ __device__ constexpr int fft_pass_lspan(int L, int p, bool wide) {
  // narrow: the 8-point pass (odd L) then radix-4 passes of span 8, 32, ...
  // or (even L) of span 1, 4, ...; wide, odd L: the 8-point pass, an
  // optional radix-4 pass of span 8, then 16-point passes from span 8 or 32;
  // wide, even L: an optional radix-4 pass of span 1, then 16-point passes
  // from span 1 or 4
  return !wide ? ((L & 1) ? (p == 0 ? 0 : 3 + 2 * (p - 1)) : 2 * p)
       : L <= 4 ? 0
       : (L & 1) ? (p == 0 ? 0
                    : (((L - 3) / 2) & 1) ? (p == 1 ? 3 : 5 + 4 * (p - 2)) : 3 + 4 * (p - 1))
                 : (((L / 2) & 1) ? (p == 0 ? 0 : 2 + 4 * (p - 1)) : 4 * p);
}

// Radix-4 butterflies of one stage with twiddle w2 = W_4h^k (forward, the
// stage's W_2h^k = w2^2) and its inverse with conj(w2).
template <typename C>
__device__ __forceinline__ void dit4(C& a0, C& a1, C& a2, C& a3, C w2) {
  const C w1 = cmul(w2, w2);
  C t = cmul(w1, a1);
  const C t0 = cadd(a0, t), tt1 = csub(a0, t);
  t = cmul(w1, a3);
  const C tt2 = cadd(a2, t), tt3 = csub(a2, t);
  t = cmul(w2, tt2);
  a0 = cadd(t0, t);
  a2 = csub(t0, t);
  t = cmul_mi(cmul(w2, tt3));           // W_4h^(k+h) = W_4h^k (-i)
  a1 = cadd(tt1, t);
  a3 = csub(tt1, t);
}
template <typename C>
__device__ __forceinline__ void dif4(C& a0, C& a1, C& a2, C& a3, C tw) {
  const C w2 = cconj(tw);
  const C w1 = cmul(w2, w2);
  const C t0 = cadd(a0, a2), t2v = cmul(csub(a0, a2), w2);
  const C t1v = cadd(a1, a3), t3 = cmul_pi(cmul(csub(a1, a3), w2));
  a0 = cadd(t0, t1v);
  a1 = cmul(csub(t0, t1v), w1);
  a2 = cadd(t2v, t3);
  a3 = cmul(csub(t2v, t3), w1);
}
template <typename C> __device__ __forceinline__ void bfly2(C& a0, C& a1) {
  const C u = a0, v = a1;
  a0 = cadd(u, v);
  a1 = csub(u, v);
}

enum { kFftChirp = 1, kFftDit = 2, kFftBhat = 4, kFftDif = 8 };

// One pass of RAD points (4, 8 or 16) and span 2^lh over `rows` rows of
// length 2^logm (stride st, pad shift sh).  `fl` selects, in this order: the
// chirp on the inputs (Bluestein; inputs at logical index >= nf are zero),
// the forward stages, the product with the kernel spectrum bhat, the inverse
// stages.  Stage twiddles: the table of span h starts at (h - h0) / 3.
template <typename R, int RAD, bool TG>
__device__ __forceinline__ void fft_pass(typename V2<R>::T* buf, int rows, int st, int logm,
                                         int sh, int lh, int fl,
                                         const typename V2<R>::T* __restrict__ tw,
                                         BHX_GLOBAL const typename V2<R>::T* twg,
                                         BHX_GLOBAL const typename V2<R>::T* chirp, int nf,
                                         BHX_GLOBAL const typename V2<R>::T* bhat) {
  using C = typename V2<R>::T;
  constexpr int LR = RAD == 4 ? 2 : RAD == 8 ? 3 : 4;
  const int h = 1 << lh;
  const int h0 = (logm & 1) ? 2 : 1;
  const int lnb = logm - LR;                  // log2 of the point groups per row
  // stage twiddles W_4h^k: from the LDS tables (TG = false) or the global
  // table W_m^j (TG), the same values
  const C* __restrict__ ta = tw + ((h - h0) / 3);            // span h (RAD 4, 16)
  const C* __restrict__ tb = tw + ((4 * h - h0) / 3);        // span 4h (RAD 16)
  auto wa = [&](int k) { return TG ? twg[k << (logm - 2 - lh)] : ta[k]; };
  auto wb = [&](int k) { return TG ? twg[k << (logm - 4 - lh)] : tb[k]; };
  auto w8 = [&](int q) { return TG ? twg[q << (logm - 3)] : tw[q]; };
  for (int u = threadIdx.x; u < (rows << lnb); u += kThreads) {
    const int r = u >> lnb, rem = u & ((1 << lnb) - 1);
    const int k = rem & (h - 1);
    const int base = ((rem >> lh) << (LR + lh)) + k;
    C* a = buf + r * st;
    C v[RAD];
#pragma unroll
    for (int j = 0; j < RAD; ++j) v[j] = a[rpos(base + (j << lh), sh)];
    if (fl & kFftChirp) {
#pragma unroll
      for (int j = 0; j < RAD; ++j) {
        const int q = bitrev(base + (j << lh), logm);
        const C c = chirp[min(q, nf - 1)];
        v[j] = q < nf ? cmul(v[j], c) : mk<C>(0, 0);
      }
    }
    if (fl & kFftDit) {
      if constexpr (RAD == 4) {
        dit4(v[0], v[1], v[2], v[3], wa(k));
      } else if constexpr (RAD == 8) {
        // radix-2 (span 1), then radix-4 of span 2 (its table starts at 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) bfly2(v[2 * q], v[2 * q + 1]);
#pragma unroll
        for (int q = 0; q < 2; ++q) dit4(v[q], v[q + 2], v[q + 4], v[q + 6], w8(q));
      } else {
        const C w = wa(k);
#pragma unroll
        for (int q = 0; q < 4; ++q) dit4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3], w);
#pragma unroll
        for (int q = 0; q < 4; ++q) dit4(v[q], v[q + 4], v[q + 8], v[q + 12], wb(k + q * h));
      }
    }
    if (fl & kFftBhat) {
#pragma unroll
      for (int j = 0; j < RAD; ++j) v[j] = cmul(v[j], bhat[base + (j << lh)]);
    }
    if (fl & kFftDif) {
      if constexpr (RAD == 4) {
        dif4(v[0], v[1], v[2], v[3], wa(k));
      } else if constexpr (RAD == 8) {
#pragma unroll
        for (int q = 0; q < 2; ++q) dif4(v[q], v[q + 2], v[q + 4], v[q + 6], w8(q));
#pragma unroll
        for (int q = 0; q < 4; ++q) bfly2(v[2 * q], v[2 * q + 1]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) dif4(v[q], v[q + 4], v[q + 8], v[q + 12], wb(k + q * h));
        const C w = wa(k);
#pragma unroll
        for (int q = 0; q < 4; ++q) dif4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3], w);
      }
    }
#pragma unroll
    for (int j = 0; j < RAD; ++j) a[rpos(base + (j << lh), sh)] = v[j];
  }
}

// The forward passes of a length-2^L FFT known at compile time.
template <typename R, int L, bool W, int P>
__device__ __forceinline__ void fft_fixed(typename V2<R>::T* buf, int rows, int st,
                                          const typename V2<R>::T* __restrict__ tw) {
  if constexpr (P < fft_npass(L, W)) {
    fft_pass<R, fft_pass_rad(L, P, W), false>(buf, rows, st, L, rpos_shift(L),
                                              fft_pass_lspan(L, P, W), kFftDit, tw, nullptr,
                                              nullptr, 0, nullptr);
    __syncthreads();
    fft_fixed<R, L, W, P + 1>(buf, rows, st, tw);
  }
}

// After inputs are placed at pos(k) (k < nf): the forward DFT of length nf of
// every row.  Power-of-two nf: the FFT passes, natural-order output.
// Otherwise Bluestein: chirp (zero past nf), FFT, product with the kernel
// spectrum, inverse FFT (bit-reversed output; out() applies the final chirp).
template <bool W, typename R, int SP>
__device__ void dft_core(const XPlan<R, SP>& X, typename V2<R>::T* buf, int rows) {
  if constexpr (SP != 0) {
    constexpr int L = (SP >> 2) & 63;
    // rows is a constant of the instance here
    if ((rows << L) >= kFftWideMin)
      fft_fixed<R, L, true, 0>(buf, rows, X.stride(), X.tw);
    else
      fft_fixed<R, L, false, 0>(buf, rows, X.stride(), X.tw);
  } else {
    const int st = X.stride();
    const int logm = X.logm;
    // W = false: instances compiled without the 16-point pass body (lower
    // register use); every row takes the narrow schedule, same arithmetic
    const bool wide = W && (rows << logm) >= kFftWideMin;
    const int np = fft_npass(logm, wide);
    const bool blue = X.blue;
    // steps 0..np-1: forward passes; then (Bluestein) passes np-2..0 inverse
    const int nstep = blue ? 2 * np - 1 : np;
#pragma unroll 1
    for (int s = 0; s < nstep; ++s) {
      const int p = s < np ? s : 2 * np - 2 - s;
      int fl = s < np ? kFftDit : kFftDif;
      if (blue && s == 0) fl |= kFftChirp;
      if (blue && s == np - 1) fl |= kFftBhat | kFftDif;
      const int rad = fft_pass_rad(logm, p, wide), lh = fft_pass_lspan(logm, p, wide);
      // twiddles from the global table (no LDS tables in these instances)
      if (W && rad == 16)
        fft_pass<R, W ? 16 : 4, true>(buf, rows, st, logm, X.sh, lh, fl, nullptr, X.twg,
                                      X.chirp, X.nf, X.bhat);
      else if (rad == 8)
        fft_pass<R, 8, true>(buf, rows, st, logm, X.sh, lh, fl, nullptr, X.twg, X.chirp, X.nf,
                             X.bhat);
      else
        fft_pass<R, 4, true>(buf, rows, st, logm, X.sh, lh, fl, nullptr, X.twg, X.chirp, X.nf,
                             X.bhat);
      __syncthreads();
    }
  }
}

// Forward real spectra of the two rows packed in one complex FFT output, at
// the pair (k, kk = (n - k) mod n).  C = out(k), D = out(kk).
//   DCT-II (orthonormal): V_a = (C + conj D)/2, V_b = (C - conj D)/(2i),
//     X[k] = s_k Re(exp(-i pi k/2n) V[k]), s_0 = sqrt(1/n), s_k = sqrt(2/n).
//   Hartley (orthonormal): H_a = (Cr + Dr - Ci + Di) / (2 sqrt n),
//                          H_b = (Ci + Di + Cr - Dr) / (2 sqrt n).
//   DST-I (orthonormal; C = out(k+1), D = out(kk+1)): the odd extensions'
//     spectra are imaginary, so X_a[k] = -Im(C) hs, X_b[k] = Re(C) hs with
//     hs = sqrt(2/(n+1)) / 2.
template <typename R, int SP>
__device__ __forceinline__ void fwd_post_pair(const XPlan<R, SP>& X, typename V2<R>::T Ck,
                                              typename V2<R>::T Dk, int k, int kk, R& xa_k,
                                              R& xb_k, R& xa_kk, R& xb_kk) {
  using C = typename V2<R>::T;
  if (X.bc == kNeumann) {
    const C va = mk<C>((Ck.x + Dk.x) * (R)0.5, (Ck.y - Dk.y) * (R)0.5);
    // (C - conj D)/(2i) = ((Ci + Di) - i (Cr - Dr)) / 2
    const C vb = mk<C>((Ck.y + Dk.y) * (R)0.5, -(Ck.x - Dk.x) * (R)0.5);
    C tk, tkk;
    X.post_pair(k, kk, tk, tkk);
    xa_k = (k == 0 ? X.s0 : X.s1) * (tk.x * va.x - tk.y * va.y);
    xb_k = (k == 0 ? X.s0 : X.s1) * (tk.x * vb.x - tk.y * vb.y);
    // V[kk] = conj(V[k])
    xa_kk = (kk == 0 ? X.s0 : X.s1) * (tkk.x * va.x + tkk.y * va.y);
    xb_kk = (kk == 0 ? X.s0 : X.s1) * (tkk.x * vb.x + tkk.y * vb.y);
  } else if (X.bc == kDirichlet) {
    xa_k = -Ck.y * X.hs;
    xb_k = Ck.x * X.hs;
    xa_kk = -Dk.y * X.hs;
    xb_kk = Dk.x * X.hs;
  } else {
    const R sc = X.hs;
    xa_k = (Ck.x + Dk.x - Ck.y + Dk.y) * sc;
    xb_k = (Ck.y + Dk.y + Ck.x - Dk.x) * sc;
    xa_kk = (Dk.x + Ck.x - Dk.y + Ck.y) * sc;
    xb_kk = (Dk.y + Ck.y + Dk.x - Ck.x) * sc;
  }
}

// Inverse-transform FFT inputs for the pair (k, kk) from the two rows' real
// spectra.  DCT: W[k] = exp(i pi k/2n) (P[k] - i P[n-k]) with
// P = g (Y_a + i Y_b), g_0 = 1/sqrt n, g_k = 1/sqrt(2n), P[n] = 0; the
// unnormalised inverse DFT is taken as conj(DFT(conj W)), so conj(W) is
// returned.  Hartley and DST-I: the forward transform again (both are their
// own inverses), inputs Y_a + i Y_b.
template <typename R, int SP>
__device__ __forceinline__ void inv_pre_pair(const XPlan<R, SP>& X, R ya_k, R yb_k, R ya_kk,
                                             R yb_kk, int k, int kk, typename V2<R>::T& in_k,
                                             typename V2<R>::T& in_kk) {
  using C = typename V2<R>::T;
  if (X.bc == kNeumann) {
    const R gk = k == 0 ? X.g0 : X.g1, gkk = kk == 0 ? X.g0 : X.g1;
    C Pk = mk<C>(gk * ya_k, gk * yb_k);
    C Pkk = mk<C>(gkk * ya_kk, gkk * yb_kk);
    if (k == 0) {
      in_k = cconj(Pk);                    // W[0] = P[0]
      in_kk = in_k;
      return;
    }
    C tk, tkk;
    X.post_pair(k, kk, tk, tkk);
    tk = cconj(tk);                        // exp(+i pi k / 2n)
    tkk = cconj(tkk);
    const C Wk = cmul(tk, csub(Pk, cmul_pi(Pkk)));    // P[k] - i P[n-k]
    const C Wkk = cmul(tkk, csub(Pkk, cmul_pi(Pk)));
    in_k = cconj(Wk);
    in_kk = cconj(Wkk);
  } else {
    in_k = mk<C>(ya_k, yb_k);
    in_kk = mk<C>(ya_kk, yb_kk);
  }
}

// ---------------------------------------------------------------------------
// Stencil tile geometry.  An item of the stencil-family passes is a tile of
// TX x TY (x TZ) nodes; the operand is staged with a two-node halo (PX x PY x
// PZ) and L f computed on the one-node ring (LX x LY x LZ).  Two dimensions:
// L is the 5-point negative Laplacian; three dimensions (Sec. 3, Example 2):
// the 7-point one.  LDS arrays are [z][y][x]; HZ is the z offset of a halo
// layer (0 in two dimensions, where z has no halo).
// ---------------------------------------------------------------------------

template <int DIM> struct Geo;

template <> struct Geo<2> {
  static constexpr int TX = kTileX, TY = kTileY, TZ = 1;
  static constexpr int PX = TX + 4, PY = TY + 4, PZ = 1;
  static constexpr int LX = TX + 2, LY = TY + 2, LZ = 1;
  static constexpr int HZ = 0;
  __device__ static void origin(const Inst& I, int tile, int& i0, int& j0, int& k0) {
    const int tx = tile % I.tiles_x, ty = tile / I.tiles_x;
    i0 = tx * TX;
    j0 = ty * TY;
    k0 = 0;
  }
  // element e of an X x Y box -> (i, j, k)
  template <int X, int Y> __device__ static void coords(int e, int& i, int& j, int& k) {
    j = e / X;
    i = e - j * X;
    k = 0;
  }
  template <typename A> __device__ static double lap(const A& a, int k, int j, int i) {
    return 4.0 * a[k][j][i] - a[k][j - 1][i] - a[k][j + 1][i] - a[k][j][i - 1] - a[k][j][i + 1];
  }
};

template <> struct Geo<3> {
  static constexpr int TX = kTileX3, TY = kTileY3, TZ = kTileZ3;
  static constexpr int PX = TX + 4, PY = TY + 4, PZ = TZ + 4;
  static constexpr int LX = TX + 2, LY = TY + 2, LZ = TZ + 2;
  static constexpr int HZ = 1;
  __device__ static void origin(const Inst& I, int tile, int& i0, int& j0, int& k0) {
    const int tx = tile % I.tiles_x, r = tile / I.tiles_x;
    const int ty = r % I.tiles_y, tz = r / I.tiles_y;
    i0 = tx * TX;
    j0 = ty * TY;
    k0 = tz * TZ;
  }
  template <int X, int Y> __device__ static void coords(int e, int& i, int& j, int& k) {
    const int r = e / X;
    i = e - r * X;
    k = r / Y;
    j = r - k * Y;
  }
  template <typename A> __device__ static double lap(const A& a, int k, int j, int i) {
    return 6.0 * a[k][j][i] - a[k - 1][j][i] - a[k + 1][j][i] - a[k][j - 1][i] -
           a[k][j + 1][i] - a[k][j][i - 1] - a[k][j][i + 1];
  }
};

// ---------------------------------------------------------------------------
// Setup: mask from the sign of phi; zero the workspace vectors; count |U|.
// ---------------------------------------------------------------------------

template <int DIM>
__global__ void __launch_bounds__(kThreads) k_setup(const Batch* __restrict__ Bp) {
  using G = Geo<DIM>;
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  __shared__ double red[4];
  for (int it = logical_block(); it < B.n_items[kPassS]; it += gridDim.x) {
    const int code = item_code(B, kPassS, it);
    const Inst I = B.inst[code >> kItemShift];
    const int tile = code & kItemMask;
    if (I.ctl->done) continue;
    int i0, j0, k0;
    G::origin(I, tile, i0, j0, k0);
    double cnt = 0;
    for (int e = threadIdx.x; e < G::TX * G::TY * G::TZ; e += kThreads) {
      int ii, jj, kk;
      G::template coords<G::TX, G::TY>(e, ii, jj, kk);
      const int i = i0 + ii, j = j0 + jj, k = k0 + kk;
      if (i < I.nx && j < I.ny && k < I.nz) {
        const size_t o = ((size_t)k * I.ny + j) * I.nx + i;
        const uint8_t u = !(I.phi[o] < 0.0);
        I.mask[o] = u;
        cnt += u;
        I.r[o] = 0.0;
        I.p[0][o] = 0.0;
        I.p[1][o] = 0.0;
        I.q[o] = 0.0;
        I.z[o] = 0.0;
      }
    }
    cnt = block_sum(cnt, red);
    if (threadIdx.x == 0) {
      PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
      I.part[PL.aux2() + tile] = cnt;
    }
  }
}

// Unknown nodes per row group (row passes skip groups without any).
// `pass`: the row-group list, kPassR (FFT instances) or kPassRD (dense ones).
__global__ void __launch_bounds__(kThreads) k_setup_rows(const Batch* __restrict__ Bp, int pass) {
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  __shared__ double red[4];
  for (int it = logical_block(); it < B.n_items[pass]; it += gridDim.x) {
    const int code = item_code(B, pass, it);
    const Inst I = B.inst[code >> kItemShift];
    const int g = code & kItemMask;
    if (I.ctl->done) continue;
    const int j0 = g * I.G;
    const int E = min(I.G, I.nrows - j0) * I.nx;
    BHX_GLOBAL const uint8_t* mk = I.mask + (size_t)j0 * I.nx;
    double cnt = 0;
    for (int e = threadIdx.x; e < E; e += kThreads) cnt += mk[e];
    cnt = block_sum(cnt, red);
    if (threadIdx.x == 0) {
      PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
      I.part[PL.rowcnt() + g] = cnt;
    }
  }
}

// ---------------------------------------------------------------------------
// Stencil pass: the 13-point (two dimensions) or 25-point (three) operator
// as L(L f) on an LDS tile with a two-node halo whose ghost values follow
// each axis' rule.
// ---------------------------------------------------------------------------

constexpr int kUnroll = 4;                          // loads in flight per thread
constexpr int kPre = 8;                             // elements per thread loaded up front

// `lpar` is the buffer parity of this launch: p_old = p[lpar], p_new =
// p[lpar ^ 1], and the current / previous r.z partials are rz(lpar) /
// rz(lpar ^ 1).  Launches alternate it, so addresses never wait for the
// control block.
// Three dimensions: at most 168 VGPRs, three waves per SIMD (more tiles in
// flight per CU; measured faster than two with more registers).
template <int MODE, int DIM>
__global__ void __launch_bounds__(kThreads, DIM == 3 ? 3 : 2)
    k_stencil(const Batch* __restrict__ Bp, int lpar) {
  using G = Geo<DIM>;
  constexpr int kPN = G::PX * G::PY * G::PZ;               // halo tile nodes
  constexpr int kPL = (kPN + kThreads - 1) / kThreads;     // halo loads per thread
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  __shared__ double P[G::PZ][G::PY][G::PX + 1];
  __shared__ double L[G::LZ][G::LY][G::LX + 1];
  __shared__ double red[16];
  // `done` is the one control field this pass writes (the block owning tile 0
  // of an instance sets it when the instance stops) while other blocks of the
  // same launch read it.  Waves of one block that read it at different times
  // could disagree and take different barrier sequences, so one thread reads
  // it for the block; two slots alternate between items, so a slow wave still
  // finds its item's value (the writer cannot pass the next item's barrier
  // before that wave arrives there).
  __shared__ int s_done[2];
  int slot = 0;
  constexpr int kOut = G::TX * G::TY * G::TZ / kThreads;
  for (int it = logical_block(); it < B.n_items[kPassS]; it += gridDim.x) {
    const int code = item_code(B, kPassS, it);
    const Inst I = B.inst[code >> kItemShift];
    const int tile = code & kItemMask;
    BHX_GLOBAL Ctl* ctl = I.ctl;
    const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
    // 1. loads that need nothing from the control block go out with it: the
    //    control fields, the tile's unknown count and the partial sums behind
    //    alpha/beta; none but `done` changes during the pass
    const int par = lpar;
    BHX_GLOBAL const double* pold = par ? I.p[1] : I.p[0];
    BHX_GLOBAL double* pnew = par ? I.p[0] : I.p[1];
    BHX_GLOBAL const double* arrs[4] = {I.part + PL.rz(par), I.part + PL.rr(),
                                        I.part + PL.rz(par ^ 1), I.part + PL.rzo(par)};
    // an instance with reduced scalars reads them from the control block;
    // its partial loads shrink to one element (no branch before the loads)
    const int nRs = I.reduce ? 1 : PL.nR;
    const int lens[4] = {nRs, nRs, nRs, nRs};
    Partials<4> PS;
    if (MODE == kModeIter) sums_issue<4>(arrs, lens, PS);
    double rsc[4] = {0.0, 0.0, 0.0, 0.0};
    if (MODE == kModeIter) {
      rsc[0] = ctl->red_rz[par];
      rsc[1] = ctl->red_rr;
      rsc[2] = ctl->red_rz[par ^ 1];
      rsc[3] = ctl->red_rzo[par];
    }
    const int ld_done = ctl->done;
    const int c_iter = ctl->iter, c_rit = ctl->restart_iter;
    const double c_thresh = ctl->thresh;
    const bool has_u = I.part[PL.aux2() + tile] != 0.0;     // unknown nodes in this tile
    if (threadIdx.x == 0) s_done[slot] = ld_done;
    __syncthreads();
    const int c_done = s_done[slot];
    slot ^= 1;
    if (c_done) continue;
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const int out_slot = (MODE == kModeIter ? PL.pq() : PL.aux()) + tile;
    if (!has_u && tile != 0) {             // nothing to compute or store here
      if (threadIdx.x == 0) I.part[out_slot] = 0.0;
      continue;
    }
    // 2. the halo tile (z and p_old, or F, and the mask) and the output masks
    const int k = c_iter;
    const bool first = (k == c_rit);       // beta = 0: p = z
    const int nRn = I.reduce ? 0 : PL.nR;
    const int ns[4] = {MODE == kModeIter ? nRn : 0, (MODE == kModeIter && !first) ? nRn : 0,
                       (MODE == kModeIter && !first) ? nRn : 0,
                       (MODE == kModeIter && !first && I.flexible) ? nRn : 0};
    int i0, j0, k0;
    G::origin(I, tile, i0, j0, k0);
    int oo[kPL];
    double sg[kPL], va[kPL], vb[kPL];
    uint8_t vm[kPL], mo[kOut];
    // a tile whose halo lies inside the grid on every axis needs no ghost
    // rule: the offsets are affine in the box coordinates (most tiles of a
    // large grid; the same values as the general path)
    const bool interior = i0 >= 2 && i0 + G::PX - 2 <= nx && j0 >= 2 && j0 + G::PY - 2 <= ny &&
                          (DIM == 2 || (k0 >= 2 && k0 + G::PZ - 2 <= nz));
    const int base = DIM == 2 ? (j0 - 2) * nx + (i0 - 2)
                              : ((k0 - 2) * ny + (j0 - 2)) * nx + (i0 - 2);
#pragma unroll
    for (int s = 0; s < kPL; ++s) {
      const int e = min((int)threadIdx.x + s * kThreads, kPN - 1);
      int ii, jj, kk;
      G::template coords<G::PX, G::PY>(e, ii, jj, kk);
      if (interior) {
        sg[s] = 1.0;
        oo[s] = base + (kk * ny + jj) * nx + ii;
        continue;
      }
      double sx, sy;
      const int mi = map_axis_sel(i0 + ii - 2, nx, I.bcx, sx);
      const int mj = map_axis_sel(j0 + jj - 2, ny, I.bcy, sy);
      if constexpr (DIM == 2) {
        sg[s] = sx * sy;
        oo[s] = mj * nx + mi;
      } else {
        double sz;
        const int mk = map_axis_sel(k0 + kk - 2, nz, I.bcz, sz);
        sg[s] = sx * sy * sz;
        oo[s] = (mk * ny + mj) * nx + mi;
      }
    }
#pragma unroll
    for (int s = 0; s < kPL; ++s) {
      const int o = oo[s];
      if (MODE == kModeIter) {
        va[s] = I.z[o];
        vb[s] = pold[o];
      } else if (MODE == kModeRhs || MODE == kModeWarm) {
        va[s] = I.F[o];
        vm[s] = I.mask[o];
      } else {
        va[s] = I.z[o];
        vm[s] = I.mask[o];
      }
    }
#pragma unroll
    for (int s = 0; s < kOut; ++s) {
      const int e = threadIdx.x + s * kThreads;
      int ii, jj, kk;
      G::template coords<G::TX, G::TY>(e, ii, jj, kk);
      const int gi = min(i0 + ii, nx - 1), gj = min(j0 + jj, ny - 1);
      const int gk = min(k0 + kk, nz - 1);
      mo[s] = I.mask[(gk * ny + gj) * nx + gi];
    }
    // every load of the item is issued above; keep the arithmetic on any of
    // them from being scheduled before the last one is issued
    __builtin_amdgcn_sched_barrier(0);
    // 3. scalars: convergence test and beta (the data loads stay in flight)
    double beta = 0.0;
    if (MODE == kModeIter) {
      double sums[4];
      sums_finish<4>(arrs, ns, PS, sums, red);
      if (I.reduce) {
#pragma unroll
        for (int k = 0; k < 4; ++k) sums[k] = rsc[k];
      }
      const double rz = sums[0];
      if (!first) {
        const double rr = sums[1];
        int d = kRunning;
        if (!(rr <= c_thresh)) {
          if (k >= I.maxit) d = kMaxIt;
          else if (!(rr == rr) || rr > 1e300) d = kBreakdown;
        } else {
          d = kConverged;
        }
        if (d != kRunning) {
          if (tile == 0 && threadIdx.x == 0) {
            ctl->rr = rr;
            ctl->done = d;
          }
          continue;
        }
        beta = I.flexible ? (rz - sums[3]) / sums[2] : rz / sums[2];
      }
      if (!(rz > 0.0) || !(beta == beta)) {
        if (tile == 0 && threadIdx.x == 0) ctl->done = kBreakdown;
        continue;
      }
    }
    if (!has_u) {
      if (threadIdx.x == 0) I.part[out_slot] = 0.0;
      continue;
    }
    // 4. tile of the operand in LDS, L f on the one-node ring, then L L f
#pragma unroll
    for (int s = 0; s < kPL; ++s) {
      const int e = threadIdx.x + s * kThreads;
      double v;
      if (MODE == kModeIter) v = first ? va[s] : va[s] + beta * vb[s];
      else if (MODE == kModeRhs) v = vm[s] ? 0.0 : va[s];
      else if (MODE == kModeWarm) v = va[s];
      else v = vm[s] ? va[s] : 0.0;
      if (e < kPN) {
        int ii, jj, kk;
        G::template coords<G::PX, G::PY>(e, ii, jj, kk);
        P[kk][jj][ii] = sg[s] * v;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < G::LX * G::LY * G::LZ; e += kThreads) {
      int ii, jj, kk;
      G::template coords<G::LX, G::LY>(e, ii, jj, kk);
      L[kk][jj][ii] = G::lap(P, kk + G::HZ, jj + 1, ii + 1);
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < kOut; ++s) {
      const int e = threadIdx.x + s * kThreads;
      int ii, jj, kk;
      G::template coords<G::TX, G::TY>(e, ii, jj, kk);
      const int gi = i0 + ii, gj = j0 + jj, gk = k0 + kk;
      const double qv = G::lap(L, kk + G::HZ, jj + 1, ii + 1);
      const bool st = gi < nx && gj < ny && gk < nz && mo[s];
      const int o = (gk * ny + gj) * nx + gi;
      if (MODE == kModeIter) {
        const double pv = P[kk + 2 * G::HZ][jj + 2][ii + 2];
        if (st) {
          pnew[o] = pv;
          I.q[o] = qv;
        }
        acc += st ? pv * qv : 0.0;
      } else if (MODE == kModeApply) {
        if (st) I.q[o] = qv;
      } else {
        if (st) I.r[o] = -qv;
        acc += st ? qv * qv : 0.0;
      }
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) I.part[out_slot] = acc;
  }
}

// ---------------------------------------------------------------------------
// True residual r = -(A F) at U with F = known values at K and the current
// iterate at U, in double-double arithmetic (error-free transformations).
// ---------------------------------------------------------------------------

struct dd { double hi, lo; };
__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_x4(dd a) { return {4.0 * a.hi, 4.0 * a.lo}; }

__device__ __forceinline__ dd dd_x2(dd a) { return {2.0 * a.hi, 2.0 * a.lo}; }

__device__ __forceinline__ dd five_point_dd(dd c, dd n, dd s, dd w, dd e) {
  dd t = dd_add(dd_neg(n), dd_neg(s));
  t = dd_add(t, dd_add(dd_neg(w), dd_neg(e)));
  return dd_add(dd_x4(c), t);
}

// 6 c - (six neighbours); 6 c as 4 c + 2 c keeps the scaling exact
__device__ __forceinline__ dd seven_point_dd(dd c, dd zm, dd zp, dd ym, dd yp, dd xm, dd xp) {
  dd t = dd_add(dd_neg(zm), dd_neg(zp));
  t = dd_add(t, dd_add(dd_neg(ym), dd_neg(yp)));
  t = dd_add(t, dd_add(dd_neg(xm), dd_neg(xp)));
  return dd_add(dd_add(dd_x4(c), dd_x2(c)), t);
}

// L at (k, j, i) of the double-double values at(k, j, i).
template <int DIM, typename F>
__device__ __forceinline__ dd lap_dd(const F& at, int k, int j, int i) {
  if constexpr (DIM == 2)
    return five_point_dd(at(k, j, i), at(k, j - 1, i), at(k, j + 1, i), at(k, j, i - 1),
                         at(k, j, i + 1));
  else
    return seven_point_dd(at(k, j, i), at(k - 1, j, i), at(k + 1, j, i), at(k, j - 1, i),
                          at(k, j + 1, i), at(k, j, i - 1), at(k, j, i + 1));
}

template <int DIM>
__global__ void __launch_bounds__(kThreads) k_resid(const Batch* __restrict__ Bp) {
  using G = Geo<DIM>;
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  __shared__ double P[G::PZ][G::PY][G::PX + 1];
  __shared__ double Lh[G::LZ][G::LY][G::LX + 1];
  __shared__ double Ll[G::LZ][G::LY][G::LX + 1];
  __shared__ double red[4];
  for (int it = logical_block(); it < B.n_items[kPassS]; it += gridDim.x) {
    const int code = item_code(B, kPassS, it);
    const Inst I = B.inst[code >> kItemShift];
    const int tile = code & kItemMask;
    const int dn = I.ctl->done;
    if (dn != kConverged && dn != kMaxIt) continue;
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
    if (I.part[PL.aux2() + tile] == 0.0) {
      if (threadIdx.x == 0) I.part[PL.aux() + tile] = 0.0;
      continue;
    }
    int i0, j0, k0;
    G::origin(I, tile, i0, j0, k0);
    for (int e = threadIdx.x; e < G::PX * G::PY * G::PZ; e += kThreads) {
      int ii, jj, kk;
      G::template coords<G::PX, G::PY>(e, ii, jj, kk);
      const int gi = i0 + ii - 2, gj = j0 + jj - 2;
      const int gk = DIM == 2 ? 0 : k0 + kk - 2;
      double v = 0.0;
      if (gi >= -2 && gi <= nx + 1 && gj >= -2 && gj <= ny + 1 && gk >= -2 && gk <= nz + 1) {
        double sx, sy, sz = 1.0;
        const int mi = map_axis(gi, nx, I.bcx, sx);
        const int mj = map_axis(gj, ny, I.bcy, sy);
        const int mk = DIM == 2 ? 0 : map_axis(gk, nz, I.bcz, sz);
        const double s = sx * sy * sz;
        if (s != 0.0) v = s * I.F[((size_t)mk * ny + mj) * nx + mi];
      }
      P[kk][jj][ii] = v;
    }
    __syncthreads();
    auto atP = [&](int k, int j, int i) { return dd{P[k][j][i], 0.0}; };
    auto atL = [&](int k, int j, int i) { return dd{Lh[k][j][i], Ll[k][j][i]}; };
    for (int e = threadIdx.x; e < G::LX * G::LY * G::LZ; e += kThreads) {
      int ii, jj, kk;
      G::template coords<G::LX, G::LY>(e, ii, jj, kk);
      const dd l = lap_dd<DIM>(atP, kk + G::HZ, jj + 1, ii + 1);
      Lh[kk][jj][ii] = l.hi;
      Ll[kk][jj][ii] = l.lo;
    }
    __syncthreads();
    double acc = 0.0;
    for (int e = threadIdx.x; e < G::TX * G::TY * G::TZ; e += kThreads) {
      int ii, jj, kk;
      G::template coords<G::TX, G::TY>(e, ii, jj, kk);
      const int gi = i0 + ii, gj = j0 + jj, gk = k0 + kk;
      if (gi < nx && gj < ny && gk < nz) {
        const size_t o = ((size_t)gk * ny + gj) * nx + gi;
        if (I.mask[o]) {
          const dd q = lap_dd<DIM>(atL, kk + G::HZ, jj + 1, ii + 1);
          const double rv = -(q.hi + q.lo);
          I.r[o] = rv;
          acc += rv * rv;
        }
      }
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) I.part[PL.aux() + tile] = acc;
  }
}

// ---------------------------------------------------------------------------
// Row pass, forward: optional CG update, then forward transform of r along x
// for G rows, written transposed to t[k * nrows + j].  Rows are the x lines:
// j = y in two dimensions, j = z * ny + y in three (nrows = ny * nz).
// ---------------------------------------------------------------------------

// `mode`: bits 0-1 the update (0 none, 1 PCG update then transform, 2 plain
// CG update only), bit 2 set: store t with non-temporal stores.  `lpar`:
// buffer parity of the iteration (as in k_stencil): p_new = p[lpar ^ 1],
// current r.z partials rz(lpar).  SP: compile-time shape of the x axis and
// row group (see XPlan), 0 for any shape.
template <typename R, int SP, int FAM = 0>
__global__ void __launch_bounds__(kThreads) k_rowfwd(const Batch* __restrict__ Bp, int mode,
                                                     int twoff, int lpar) {
  using C = typename V2<R>::T;
  constexpr bool CZ = FAM == kFamCz;
  constexpr bool kWide = FAM != kFamNarrow;
  const int update = mode & 3;
  const bool stream_t = (mode & 4) != 0;
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  extern __shared__ __align__(16) unsigned char smem[];
  debug_fill_lds(smem);
  C* buf = (C*)smem;
  R* stg = (R*)smem;
  C* twl = buf + twoff;
  int staged = -1;
  __shared__ double red[8];
  for (int itm = logical_block(); itm < B.n_items[kPassR]; itm += gridDim.x) {
    const int code = item_code(B, kPassR, itm);
    const Inst I = B.inst[code >> kItemShift];
    const int g = code & kItemMask;
    BHX_GLOBAL Ctl* ctl = I.ctl;
    const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
    // ny: rows of the pass
    const int nx = SP ? sp_nodes(SP) : I.nx, ny = I.nrows, G = SP ? SP >> 8 : I.G,
              j0 = g * G;
    const int E = min(G, ny - j0) * nx;          // valid elements of this row group
    const size_t base = (size_t)j0 * nx;
    BHX_GLOBAL const uint8_t* __restrict__ mk = I.mask + base;
    BHX_GLOBAL double* __restrict__ Fb = I.F + base;
    BHX_GLOBAL double* __restrict__ rb = I.r + base;
    BHX_GLOBAL const double* __restrict__ pb = (lpar ? I.p[0] : I.p[1]) + base;
    BHX_GLOBAL const double* __restrict__ qb = I.q + base;
    // 1. issue together: control fields, the row group's unknown count, the
    //    partial sums behind alpha and the masks of the first kPre elements
    //    per thread (rows j0 .. j0+G-1 are contiguous); `done` and the counts
    //    do not change during the pass
    BHX_GLOBAL const double* arrs[2] = {I.part + PL.rz(lpar), I.part + PL.pq()};
    const int lens[2] = {I.reduce ? 1 : PL.nR, I.reduce ? 1 : PL.nS};
    const int ns[2] = {update && !I.reduce ? PL.nR : 0, update && !I.reduce ? PL.nS : 0};
    Partials<2> PS;
    sums_issue<2>(arrs, lens, PS);             // unconditional: no branch before the loads
    const double rsc[2] = {ctl->red_rz[lpar], ctl->red_pq};
    int m0[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = threadIdx.x + u * kThreads;
      m0[u] = mk[min(e, E - 1)] && e < E;
    }
    const int c_done = ctl->done, k_it = ctl->iter;
    const double rowcnt = I.part[PL.rowcnt() + g];
    if (c_done) continue;
    if (rowcnt == 0.0) {
      // no unknown node in these rows: r = 0 there, so is its transform
      BHX_GLOBAL R* t = (BHX_GLOBAL R*)I.t;
      for (int e = threadIdx.x; e < nx * G; e += kThreads) {
        const int kx = e / G, j = j0 + (e - kx * G);
        if (j < ny) t[(size_t)kx * ny + j] = (R)0;
      }
      if (update && threadIdx.x == 0) I.part[PL.rr() + g] = 0.0;
      continue;
    }
    // 2. values at unknown nodes (lanes of known nodes read element 0: one
    //    cached line per wave), in flight while tables and scalars settle
    double rv0[kPre], pv0[kPre], qv0[kPre], xv0[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int ea = m0[u] ? threadIdx.x + u * kThreads : 0;
      rv0[u] = rb[ea];
      pv0[u] = update ? pb[ea] : 0.0;
      qv0[u] = update ? qb[ea] : 0.0;
      xv0[u] = update ? Fb[ea] : 0.0;
    }
    XPlan<R, SP> X(B, I.planx);
    if constexpr (!CZ) X.cz = 0;   // chirp-z axes run on the CZ instances only
    if (update != 2) X.stage(twl, I.planx, staged, false);
    double alpha = 0.0;
    if (update) {
      double sums[2];
      sums_finish<2>(arrs, ns, PS, sums, red);
      alpha = I.reduce ? rsc[0] / rsc[1] : sums[0] / sums[1];
    }
    const int rows = G >> 1;
    const int st = X.stride();
    const bool first = k_it == 0;
    double acc = 0.0;
    // 3. update and place r into the packed rows
    auto consume = [&](int e, int m, double rv, double pv, double qv, double xv) {
      if (e >= G * nx) return;
      double v = m ? rv : 0.0;
      if (update && m) {
        Fb[e] = (first && !I.warm ? 0.0 : xv) + alpha * pv;
        v -= alpha * qv;
        rb[e] = v;
        acc += v * v;
      }
      if (update != 2) {
        const int jr = e / nx, i = e - jr * nx;
        if (!X.cz) X.put(buf + (jr >> 1) * st, i, jr & 1, (R)v);
        else if (!(jr & 1)) X.put_cz(buf + (jr >> 1) * st, i, (R)v);   // first lines now
      }
    };
#pragma unroll
    for (int u = 0; u < kPre; ++u)
      consume(threadIdx.x + u * kThreads, m0[u], rv0[u], pv0[u], qv0[u], xv0[u]);
    for (int e0 = threadIdx.x + kPre * kThreads; e0 < G * nx; e0 += kUnroll * kThreads) {
      int m[kUnroll];
      double rv[kUnroll], pv[kUnroll], qv[kUnroll], xv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = e0 + u * kThreads;
        m[u] = mk[min(e, E - 1)] && e < E;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int ea = m[u] ? e0 + u * kThreads : 0;
        rv[u] = rb[ea];
        pv[u] = update ? pb[ea] : 0.0;
        qv[u] = update ? qb[ea] : 0.0;
        xv[u] = update ? Fb[ea] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        consume(e0 + u * kThreads, m[u], rv[u], pv[u], qv[u], xv[u]);
    }
    if (update != 2) X.zero_ends(buf, rows, st);
    __syncthreads();
    if (update) {
      acc = block_sum(acc, red);
      if (threadIdx.x == 0) I.part[PL.rr() + g] = acc;
      if (update == 2) continue;       // plain CG: update only
    }
    // 2. FFT
    dft_core<kWide>(X, buf, rows);
    // 3. real spectra of the pairs (k, n-k) into registers
    const int np = X.pairs();
    R va[kMaxPairs][4];
    if (X.cz) {
      // chirp-z DST-I: the first line of each pair is in its row now; then
      // the second, whose updated r this block wrote to rb above
#pragma unroll
      for (int s = 0; s < kMaxPairs; ++s) {
        const int pidx = threadIdx.x + s * kThreads;
        if (pidx < rows * np) {
          const int rr = pidx / np, k = pidx - rr * np;
          const C* row = buf + rr * st;
          va[s][0] = X.coef_cz(row, k);
          va[s][2] = X.coef_cz(row, X.partner(k));
        }
      }
      __syncthreads();
      for (int e = threadIdx.x; e < G * nx; e += kThreads) {
        const int jr = e / nx, i = e - jr * nx;
        if (jr & 1) X.put_cz(buf + (jr >> 1) * st, i, (e < E && mk[e]) ? (R)rb[e] : (R)0);
      }
      X.zero_ends(buf, rows, st);
      __syncthreads();
      dft_core<kWide>(X, buf, rows);
#pragma unroll
      for (int s = 0; s < kMaxPairs; ++s) {
        const int pidx = threadIdx.x + s * kThreads;
        if (pidx < rows * np) {
          const int rr = pidx / np, k = pidx - rr * np;
          const C* row = buf + rr * st;
          va[s][1] = X.coef_cz(row, k);
          va[s][3] = X.coef_cz(row, X.partner(k));
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < kMaxPairs; ++s) {
        const int pidx = threadIdx.x + s * kThreads;
        if (pidx < rows * np) {
          const int rr = pidx / np, k = pidx - rr * np;
          const int kk = X.partner(k);
          const C* row = buf + rr * st;
          fwd_post_pair<R>(X, X.out(row, X.bin(k)), X.out(row, X.bin(kk)), k, kk, va[s][0],
                           va[s][1], va[s][2], va[s][3]);
        }
      }
    }
    __syncthreads();
    // 4. stage transposed in LDS: stg[k * G + jr]
#pragma unroll
    for (int s = 0; s < kMaxPairs; ++s) {
      const int pidx = threadIdx.x + s * kThreads;
      if (pidx < rows * np) {
        const int rr = pidx / np, k = pidx - rr * np;
        const int kk = X.partner(k);
        stg[k * G + 2 * rr] = va[s][0];
        stg[k * G + 2 * rr + 1] = va[s][1];
        if (kk != k) {
          stg[kk * G + 2 * rr] = va[s][2];
          stg[kk * G + 2 * rr + 1] = va[s][3];
        }
      }
    }
    __syncthreads();
    // 5. coalesced transposed store (one loop per store kind: a store kind
    //    chosen inside the loop body is merged away by the compiler)
    BHX_GLOBAL R* t = (BHX_GLOBAL R*)I.t;
    if (stream_t) {
      for (int e = threadIdx.x; e < nx * G; e += kThreads) {
        const int k = e / G, j = j0 + e - k * G;
        if (j < ny) __builtin_nontemporal_store(stg[e], &t[(size_t)k * ny + j]);
      }
    } else {
      for (int e = threadIdx.x; e < nx * G; e += kThreads) {
        const int k = e / G, j = j0 + e - k * G;
        if (j < ny) t[(size_t)k * ny + j] = stg[e];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Column passes on the transposed buffer t ([nx][nz][ny], y fastest).  A
// pencil is a line of t along y (contiguous) or, in three dimensions, along z
// (stride ny); the pencils of one item are transformed two to a complex FFT.
//   kCol2D    forward along y, scale by 1/(lambda_x + lambda_y)^2, inverse;
//   kColYFwd  forward along y (three dimensions);
//   kColZ     forward along z, scale by 1/(lambda_x + lambda_y + lambda_z)^2,
//             inverse along z;
//   kColYInv  inverse along y.
// All in place on t.  SP: compile-time shape of the pass's axis and pencil
// group (see XPlan), 0 for any shape.
// ---------------------------------------------------------------------------

template <typename R, int KIND, int SP, int FAM = 0>
__global__ void __launch_bounds__(kThreads) k_col(const Batch* __restrict__ Bp, int count_iter,
                                                  int twoff) {
  using C = typename V2<R>::T;
  constexpr bool CZ = FAM == kFamCz;
  constexpr bool kWide = FAM != kFamNarrow;
  constexpr int kPass = KIND == kColZ ? kPassZ : kPassC;
  constexpr bool kStrided = KIND == kColZ;       // z pencils: stride ny
  constexpr bool kScale = KIND == kCol2D || KIND == kColZ;
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  extern __shared__ __align__(16) unsigned char smem[];
  debug_fill_lds(smem);
  C* buf = (C*)smem;
  R* stg = (R*)smem;
  C* twl = buf + twoff;
  __shared__ R s_lam[kMaxGc];      // per pencil: eigenvalue sum of the other axes
  int staged = -1;
  for (int itm = logical_block(); itm < B.n_items[kPass]; itm += gridDim.x) {
    const int code = item_code(B, kPass, itm);
    const Inst I = B.inst[code >> kItemShift];
    const int c = code & kItemMask;
    BHX_GLOBAL Ctl* ctl = I.ctl;
    BHX_GLOBAL R* t = (BHX_GLOBAL R*)I.t;
    // 1. the item's pencils: cnt <= Gp of length n; element j of pencil cr at
    //    t[pb + cr * ps + j * js]
    int n, Gp, cnt, ps, js, plan, c0 = 0, kx = 0, ky0 = 0;
    size_t pb;
    if constexpr (kStrided) {
      n = SP ? sp_nodes(SP) : I.nz;
      Gp = SP ? SP >> 8 : I.Gz;
      plan = I.planz;
      const int ngy = (I.ny + Gp - 1) / Gp;
      kx = c / ngy;
      ky0 = (c - kx * ngy) * Gp;
      cnt = min(Gp, I.ny - ky0);
      pb = (size_t)kx * I.nz * I.ny + ky0;
      ps = 1;
      js = I.ny;
    } else {
      n = SP ? sp_nodes(SP) : I.ny;
      Gp = SP ? SP >> 8 : I.Gc;
      plan = I.plany;
      c0 = c * Gp;
      cnt = min(Gp, I.nx * I.nz - c0);    // pencils (kx, z); nz = 1 in two dimensions
      pb = (size_t)c0 * n;
      ps = n;
      js = 1;
    }
    // element e of the load/store order -> (pencil, index): y pencils
    // pencil-major; z pencils index-major, so neighbouring lanes touch
    // neighbouring pencils, adjacent in memory
    auto split = [&](int e, int& cr, int& j) {
      if constexpr (kStrided) {
        j = e / Gp;
        cr = e - j * Gp;
      } else {
        cr = e / n;
        j = e - cr * n;
      }
    };
    auto at = [&](int cr, int j) { return pb + (size_t)cr * ps + (size_t)j * js; };
    const int Et = Gp * n;
    //    issue together: the first kPre loads of the item, the eigenvalues of
    //    its pencils and `done` (unchanged during the pass); then stage the
    //    plan tables
    R tv[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      int cr, j;
      split(min((int)threadIdx.x + u * kThreads, Et - 1), cr, j);
      tv[u] = t[cr < cnt ? at(cr, j) : pb];
    }
    R lam = (R)0;
    if constexpr (KIND == kCol2D) {
      const XPlan<R> Xx(B, I.planx);
      lam = Xx.lam[min(c0 + min((int)threadIdx.x, kMaxGc - 1), I.nx - 1)];
    } else if constexpr (KIND == kColZ) {
      const XPlan<R> Xx(B, I.planx);
      const XPlan<R> Xy(B, I.plany);
      lam = Xx.lam[kx] + Xy.lam[min(ky0 + min((int)threadIdx.x, kMaxGc - 1), I.ny - 1)];
    }
    if (ctl->done) continue;
    XPlan<R, SP> X(B, plan);
    if constexpr (!CZ) X.cz = 0;   // chirp-z axes run on the CZ instances only
    X.stage(twl, plan, staged, kScale);
    const int rows = Gp >> 1;
    const int st = X.stride();
    const int np = X.pairs();
    if constexpr (KIND == kCol2D && SP == 0) {
      if (X.cz) {
        // chirp-z DST-I along y: the first pencil of each pair, then the
        // second, each through forward, scale and inverse (the DST-I is its
        // own inverse) in the pair's row
        if (threadIdx.x < kMaxGc) s_lam[threadIdx.x] = lam;
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
          for (int e = threadIdx.x; e < Et; e += kThreads) {
            int cr, j;
            split(e, cr, j);
            if ((cr & 1) == h) X.put_cz(buf + (cr >> 1) * st, j, cr < cnt ? t[at(cr, j)] : (R)0);
          }
          X.zero_ends(buf, rows, st);
          __syncthreads();
          dft_core<kWide>(X, buf, rows);
          R ys[kMaxPairs][2];
#pragma unroll
          for (int s = 0; s < kMaxPairs; ++s) {
            const int pidx = threadIdx.x + s * kThreads;
            if (pidx < rows * np) {
              const int rr = pidx / np, k = pidx - rr * np;
              const int kk = X.partner(k);
              const C* row = buf + rr * st;
              const R la = s_lam[2 * rr + h];
              R lk, lkk;
              X.lam_pair(k, kk, lk, lkk);
              ys[s][0] = X.coef_cz(row, k) * inv_sq<R>(la + lk);
              ys[s][1] = X.coef_cz(row, kk) * inv_sq<R>(la + lkk);
            }
          }
          __syncthreads();
#pragma unroll
          for (int s = 0; s < kMaxPairs; ++s) {
            const int pidx = threadIdx.x + s * kThreads;
            if (pidx < rows * np) {
              const int rr = pidx / np, k = pidx - rr * np;
              const int kk = X.partner(k);
              X.put_cz(buf + rr * st, k, ys[s][0]);
              if (kk != k) X.put_cz(buf + rr * st, kk, ys[s][1]);
            }
          }
          X.zero_ends(buf, rows, st);
          __syncthreads();
          dft_core<kWide>(X, buf, rows);
#pragma unroll
          for (int s = 0; s < kMaxPairs; ++s) {
            const int pidx = threadIdx.x + s * kThreads;
            if (pidx < rows * np) {
              const int rr = pidx / np, k = pidx - rr * np;
              const int kk = X.partner(k);
              const int cr = 2 * rr + h;
              const C* row = buf + rr * st;
              if (cr < cnt) {
                t[at(cr, k)] = X.coef_cz(row, k);
                if (kk != k) t[at(cr, kk)] = X.coef_cz(row, kk);
              }
            }
          }
          __syncthreads();
        }
        if (count_iter && c == 0 && threadIdx.x == 0) ctl->iter = ctl->iter + 1;
        continue;
      }
    }
    C vin[kMaxPairs][2];
    if constexpr (KIND != kColYInv) {
      // 2. forward: place the pencils into the packed rows, FFT, spectra
      auto place = [&](int e, R v) {
        if (e >= Et) return;
        int cr, j;
        split(e, cr, j);
        X.put(buf + (cr >> 1) * st, j, cr & 1, cr < cnt ? v : (R)0);
      };
#pragma unroll
      for (int u = 0; u < kPre; ++u) place(threadIdx.x + u * kThreads, tv[u]);
      for (int e = threadIdx.x + kPre * kThreads; e < Et; e += kThreads) {
        int cr, j;
        split(e, cr, j);
        place(e, t[cr < cnt ? at(cr, j) : pb]);
      }
      if (kScale && threadIdx.x < kMaxGc) s_lam[threadIdx.x] = lam;
      X.zero_ends(buf, rows, st);
      __syncthreads();
      dft_core<kWide>(X, buf, rows);
#pragma unroll
      for (int s = 0; s < kMaxPairs; ++s) {
        const int pidx = threadIdx.x + s * kThreads;
        if (pidx < rows * np) {
          const int rr = pidx / np, k = pidx - rr * np;
          const int kk = X.partner(k);
          const C* row = buf + rr * st;
          R xa, xb, xak, xbk;
          fwd_post_pair<R>(X, X.out(row, X.bin(k)), X.out(row, X.bin(kk)), k, kk, xa, xb, xak,
                           xbk);
          if constexpr (KIND == kColYFwd) {
            const int ca = 2 * rr, cb = ca + 1;
            if (ca < cnt) {
              t[at(ca, k)] = xa;
              if (kk != k) t[at(ca, kk)] = xak;
            }
            if (cb < cnt) {
              t[at(cb, k)] = xb;
              if (kk != k) t[at(cb, kk)] = xbk;
            }
          } else {
            // 3. scale by the inverse squared eigenvalue sums, inverse inputs
            const R la = s_lam[2 * rr];
            const R lb = s_lam[2 * rr + 1];
            R lk, lkk;
            X.lam_pair(k, kk, lk, lkk);
            xa *= inv_sq<R>(la + lk);
            xb *= inv_sq<R>(lb + lk);
            xak *= inv_sq<R>(la + lkk);
            xbk *= inv_sq<R>(lb + lkk);
            inv_pre_pair<R>(X, xa, xb, xak, xbk, k, kk, vin[s][0], vin[s][1]);
          }
        }
      }
      if constexpr (KIND == kColYFwd) {
        __syncthreads();
        continue;
      }
    } else {
      // 2. inverse only: the spectra staged as stg[cr * n + k], inverse inputs
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int e = threadIdx.x + u * kThreads;
        if (e < Et) stg[e] = (e / n) < cnt ? tv[u] : (R)0;
      }
      for (int e = threadIdx.x + kPre * kThreads; e < Et; e += kThreads) {
        int cr, j;
        split(e, cr, j);
        stg[e] = cr < cnt ? t[at(cr, j)] : (R)0;
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < kMaxPairs; ++s) {
        const int pidx = threadIdx.x + s * kThreads;
        if (pidx < rows * np) {
          const int rr = pidx / np, k = pidx - rr * np;
          const int kk = X.partner(k);
          const R* ra = stg + 2 * rr * n;
          inv_pre_pair<R>(X, ra[k], ra[n + k], ra[kk], ra[n + kk], k, kk, vin[s][0], vin[s][1]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kMaxPairs; ++s) {
      const int pidx = threadIdx.x + s * kThreads;
      if (pidx < rows * np) {
        const int rr = pidx / np, k = pidx - rr * np;
        X.put_pair(buf + rr * st, k, X.partner(k), vin[s][0], vin[s][1]);
      }
    }
    X.zero_ends(buf, rows, st);
    __syncthreads();
    dft_core<kWide>(X, buf, rows);
    // 4. inverse outputs back into t
    if (X.bc == kNeumann) {
      for (int e = threadIdx.x; e < Et; e += kThreads) {
        int cr, j;
        split(e, cr, j);
        if (cr < cnt) {
          const C v = X.out(buf + (cr >> 1) * st, inv_index(j, n));
          t[at(cr, j)] = (cr & 1) ? -v.y : v.x;
        }
      }
    } else {
      // Hartley, DST-I: the inverse is the forward transform; reuse vin's registers
#pragma unroll
      for (int s = 0; s < kMaxPairs; ++s) {
        const int pidx = threadIdx.x + s * kThreads;
        if (pidx < rows * np) {
          const int rr = pidx / np, k = pidx - rr * np;
          const int kk = X.partner(k);
          const C* row = buf + rr * st;
          R a, b, ak, bk;
          fwd_post_pair<R>(X, X.out(row, X.bin(k)), X.out(row, X.bin(kk)), k, kk, a, b, ak, bk);
          vin[s][0] = mk<C>(a, b);
          vin[s][1] = mk<C>(ak, bk);
        }
      }
      if constexpr (kStrided) {
        // through LDS, index-major (stg[k * Gp + cr]), for coalesced stores
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kMaxPairs; ++s) {
          const int pidx = threadIdx.x + s * kThreads;
          if (pidx < rows * np) {
            const int rr = pidx / np, k = pidx - rr * np;
            const int kk = X.partner(k);
            stg[k * Gp + 2 * rr] = vin[s][0].x;
            stg[k * Gp + 2 * rr + 1] = vin[s][0].y;
            if (kk != k) {
              stg[kk * Gp + 2 * rr] = vin[s][1].x;
              stg[kk * Gp + 2 * rr + 1] = vin[s][1].y;
            }
          }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < Et; e += kThreads) {
          int cr, j;
          split(e, cr, j);
          if (cr < cnt) t[at(cr, j)] = stg[e];
        }
      } else {
#pragma unroll
        for (int s = 0; s < kMaxPairs; ++s) {
          const int pidx = threadIdx.x + s * kThreads;
          if (pidx < rows * np) {
            const int rr = pidx / np, k = pidx - rr * np;
            const int kk = X.partner(k);
            const int ca = 2 * rr, cb = ca + 1;
            if (ca < cnt) {
              t[at(ca, k)] = vin[s][0].x;
              if (kk != k) t[at(ca, kk)] = vin[s][1].x;
            }
            if (cb < cnt) {
              t[at(cb, k)] = vin[s][0].y;
              if (kk != k) t[at(cb, kk)] = vin[s][1].y;
            }
          }
        }
      }
    }
    if (count_iter && c == 0 && threadIdx.x == 0) ctl->iter = ctl->iter + 1;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Row pass, inverse: read G rows of spectra transposed from t, inverse
// transform along x, restrict to U -> z; partial r.z and r.z_old.
// ---------------------------------------------------------------------------

// `lpar`: buffer parity of the iteration; the r.z partials written here are
// the next iteration's current ones, rz(lpar ^ 1) (and rzo(lpar ^ 1)).  SP as
// in k_rowfwd.
template <typename R, int SP, int FAM = 0>
__global__ void __launch_bounds__(kThreads, FAM == kFamCz ? 1 : 2)
    k_rowinv(const Batch* __restrict__ Bp, int twoff, int lpar) {
  using C = typename V2<R>::T;
  constexpr bool CZ = FAM == kFamCz;
  constexpr bool kWide = FAM != kFamNarrow;
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  extern __shared__ __align__(16) unsigned char smem[];
  debug_fill_lds(smem);
  C* buf = (C*)smem;
  R* stg = (R*)smem;
  C* twl = buf + twoff;
  int staged = -1;
  __shared__ double red[4];
  for (int itm = logical_block(); itm < B.n_items[kPassR]; itm += gridDim.x) {
    const int code = item_code(B, kPassR, itm);
    const Inst I = B.inst[code >> kItemShift];
    const int g = code & kItemMask;
    BHX_GLOBAL Ctl* ctl = I.ctl;
    const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
    const int par = lpar ^ 1;
    // ny: rows of the pass
    const int nx = SP ? sp_nodes(SP) : I.nx, ny = I.nrows, G = SP ? SP >> 8 : I.G,
              j0 = g * G;
    BHX_GLOBAL const R* t = (BHX_GLOBAL const R*)I.t;
    // 1. issue together: `done` and the row group's unknown count (both
    //    unchanged during the pass), the first kPre transposed loads of the
    //    spectra (stg[k * G + jr] = t[k * ny + j0 + jr]) and the masks of
    //    the output elements; then the output r (and z_old) values
    const int jn = min(G, ny - j0);
    R tv[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = min((int)threadIdx.x + u * kThreads, nx * G - 1);
      const int k = e / G, jr = e - k * G;
      tv[u] = t[(size_t)k * ny + j0 + min(jr, jn - 1)];
    }
    const int E = jn * nx;
    const size_t base = (size_t)j0 * nx;
    BHX_GLOBAL const uint8_t* __restrict__ mk = I.mask + base;
    BHX_GLOBAL const double* __restrict__ rb = I.r + base;
    BHX_GLOBAL double* __restrict__ zb = I.z + base;
    const bool flex = I.flexible != 0;
    // outputs prefetched across the transform (compile-time shapes only, and
    // fewer for rows of 2048 points or more: the registers go to the
    // transform passes)
    constexpr int kPreO = SP == 0 ? 0 : ((SP >> 2) & 63) >= 11 ? kPre / 2 : kPre;
    int m0[kPreO + 1];
#pragma unroll
    for (int u = 0; u < kPreO; ++u) {
      const int e = threadIdx.x + u * kThreads;
      m0[u] = mk[min(e, E - 1)] && e < E;
    }
    const int c_done = ctl->done;
    const double rowcnt = I.part[PL.rowcnt() + g];
    if (c_done) continue;
    if (rowcnt == 0.0) {      // z stays 0 on rows without unknowns
      if (threadIdx.x == 0) {
        I.part[PL.rz(par) + g] = 0.0;
        if (I.flexible) I.part[PL.rzo(par) + g] = 0.0;
      }
      continue;
    }
    double rv0[kPreO + 1], zo0[kPreO + 1];
#pragma unroll
    for (int u = 0; u < kPreO; ++u) {
      const int ea = m0[u] ? threadIdx.x + u * kThreads : 0;
      rv0[u] = rb[ea];
      zo0[u] = flex ? zb[ea] : 0.0;
    }
    XPlan<R, SP> X(B, I.planx);
    if constexpr (!CZ) X.cz = 0;   // chirp-z axes run on the CZ instances only
    X.stage(twl, I.planx, staged, false);
    const int rows = G >> 1;
    const int st = X.stride();
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int e = threadIdx.x + u * kThreads;
      if (e < nx * G) stg[e] = (e % G) < jn ? tv[u] : (R)0;
    }
    for (int e = threadIdx.x + kPre * kThreads; e < nx * G; e += kThreads) {
      const int k = e / G, jr = e - k * G;
      stg[e] = jr < jn ? t[(size_t)k * ny + j0 + jr] : (R)0;
    }
    __syncthreads();
    const int np = X.pairs();
    double acc = 0.0, acco = 0.0;
    if (X.cz) {
      // chirp-z DST-I (its own inverse): the first line of each pair, then
      // the second, in the pair's row; outputs, z and dots per line.  The
      // spectra share LDS with the rows: the first lines' ones go through
      // registers before the rows are written, the second lines' are read
      // again from t.
#pragma unroll 1
      for (int h = 0; h < 2; ++h) {
        R sv[kMaxPairs][2];
#pragma unroll
        for (int s = 0; s < kMaxPairs; ++s) {
          const int pidx = threadIdx.x + s * kThreads;
          if (pidx < rows * np) {
            const int rr = pidx / np, k = pidx - rr * np;
            const int kk = X.partner(k);
            const int jr = 2 * rr + h;
            if (h == 0) {
              sv[s][0] = stg[k * G + jr];
              sv[s][1] = stg[kk * G + jr];
            } else {
              sv[s][0] = jr < jn ? t[(size_t)k * ny + j0 + jr] : (R)0;
              sv[s][1] = jr < jn ? t[(size_t)kk * ny + j0 + jr] : (R)0;
            }
          }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kMaxPairs; ++s) {
          const int pidx = threadIdx.x + s * kThreads;
          if (pidx < rows * np) {
            const int rr = pidx / np, k = pidx - rr * np;
            const int kk = X.partner(k);
            X.put_cz(buf + rr * st, k, sv[s][0]);
            if (kk != k) X.put_cz(buf + rr * st, kk, sv[s][1]);
          }
        }
        X.zero_ends(buf, rows, st);
        __syncthreads();
        dft_core<kWide>(X, buf, rows);
        for (int e = threadIdx.x; e < E; e += kThreads) {
          const int jr = e / nx, i = e - jr * nx;
          if ((jr & 1) != h || !mk[e]) continue;
          const double zo = flex ? zb[e] : 0.0;
          const double zv = (double)X.coef_cz(buf + (jr >> 1) * st, i);
          const double rv = rb[e];
          zb[e] = zv;
          acc += rv * zv;
          acco += rv * zo;
        }
        __syncthreads();
      }
    } else {
    // 2. inverse inputs of the pairs, through registers
    C vin[kMaxPairs][2];
#pragma unroll
    for (int s = 0; s < kMaxPairs; ++s) {
      const int pidx = threadIdx.x + s * kThreads;
      if (pidx < rows * np) {
        const int rr = pidx / np, k = pidx - rr * np;
        const int kk = X.partner(k);
        inv_pre_pair<R>(X, stg[k * G + 2 * rr], stg[k * G + 2 * rr + 1], stg[kk * G + 2 * rr],
                        stg[kk * G + 2 * rr + 1], k, kk, vin[s][0], vin[s][1]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kMaxPairs; ++s) {
      const int pidx = threadIdx.x + s * kThreads;
      if (pidx < rows * np) {
        const int rr = pidx / np, k = pidx - rr * np;
        X.put_pair(buf + rr * st, k, X.partner(k), vin[s][0], vin[s][1]);
      }
    }
    X.zero_ends(buf, rows, st);
    __syncthreads();
    dft_core<kWide>(X, buf, rows);
    // 3. outputs: restrict, store z, dots
    auto emit = [&](int e, int m, double rv, double zo) {
      if (!m) return;
      const int jr = e / nx, i = e - jr * nx;
      const C* row = buf + (jr >> 1) * st;
      R v;
      if (X.bc == kNeumann) {
        const C c = X.out(row, inv_index(i, nx));
        v = (jr & 1) ? -c.y : c.x;
      } else if (X.bc == kDirichlet) {
        const C c = X.out(row, i + 1);
        v = (jr & 1) ? c.x * X.hs : -c.y * X.hs;
      } else {
        const int ii = i == 0 ? 0 : nx - i;
        R xa, xb, xak, xbk;
        fwd_post_pair<R>(X, X.out(row, i), X.out(row, ii), i, ii, xa, xb, xak, xbk);
        v = (jr & 1) ? xb : xa;
      }
      const double zv = (double)v;
      zb[e] = zv;
      acc += rv * zv;
      acco += rv * zo;
    };
#pragma unroll
    for (int u = 0; u < kPreO; ++u) emit(threadIdx.x + u * kThreads, m0[u], rv0[u], zo0[u]);
    for (int e0 = threadIdx.x + kPreO * kThreads; e0 < E; e0 += kUnroll * kThreads) {
      int m[kUnroll];
      double rv[kUnroll], zo[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = e0 + u * kThreads;
        m[u] = mk[min(e, E - 1)] && e < E;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int ea = m[u] ? e0 + u * kThreads : 0;
        rv[u] = rb[ea];
        zo[u] = flex ? zb[ea] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) emit(e0 + u * kThreads, m[u], rv[u], zo[u]);
    }
    }
    acc = block_sum(acc, red);
    if (flex) acco = block_sum(acco, red);
    if (threadIdx.x == 0) {
      I.part[PL.rz(par) + g] = acc;
      if (flex) I.part[PL.rzo(par) + g] = acco;
    }
  }
}

// Plain CG (no preconditioner): z = r at U; partial r.z (and r.z_old).
__global__ void __launch_bounds__(kThreads) k_identity(const Batch* __restrict__ Bp, int lpar) {
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  __shared__ double red[4];
  for (int itm = logical_block(); itm < B.n_items[kPassR]; itm += gridDim.x) {
    const int code = item_code(B, kPassR, itm);
    const Inst I = B.inst[code >> kItemShift];
    const int g = code & kItemMask;
    BHX_GLOBAL Ctl* ctl = I.ctl;
    if (ctl->done) continue;
    const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
    const int par = lpar ^ 1;          // as in k_rowinv
    const int nx = I.nx, ny = I.nrows, j0 = g * I.G;
    const int jn = min(I.G, ny - j0);
    const bool flex = I.flexible != 0;
    double acc = 0.0, acco = 0.0;
    for (int e = threadIdx.x; e < jn * nx; e += kThreads) {
      const size_t o = (size_t)j0 * nx + e;
      if (!I.mask[o]) continue;
      const double rv = I.r[o];
      if (flex) acco += rv * I.z[o];
      I.z[o] = rv;
      acc += rv * rv;
    }
    acc = block_sum(acc, red);
    if (flex) acco = block_sum(acco, red);
    if (threadIdx.x == 0) {
      I.part[PL.rz(par) + g] = acc;
      if (flex) I.part[PL.rzo(par) + g] = acco;
    }
  }
}

// ---------------------------------------------------------------------------
// Dense transforms on the matrix cores.  For an axis of at most kDenseMax
// nodes the 1-D transform is applied as a product with its basis matrix
// T(k, i), whose entries come from a table in LDS through the index rule of
// AxisPlan (dense_P, dense_fold): v_mfma_f64_16x16x4 for the FP64
// preconditioner, v_mfma_f32_16x16x4 for the FP32 one.  A work item is 16
// lines, one matrix tile wide.  The passes and their results are those of
// the FFT family (the orthonormal coefficients in t, laid out [kx][y]):
//   k_rowfwd_dense   CG update of 16 rows, then t[k][j] = nk(k) sum_i T(k, i) r[j][i]
//   k_col_dense      16 columns of t: forward along y, scale by
//                    nk(ky)^2 / (lambda_x + lambda_y)^2, inverse along y
//   k_rowinv_dense   z[j][i] = sum_k T(k, i) nk(k) t[k][j] at unknown nodes; r.z
// ---------------------------------------------------------------------------

typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

template <typename R> struct Mfma;
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of a 16 x 4 by
// 4 x 16 product; accumulator element v of lane l is D[row(v, l)][l % 16].
template <> struct Mfma<double> {
  using Acc = v4d_t;
  static __device__ __forceinline__ Acc mac(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return 4 * v + (l >> 4); }
};
template <> struct Mfma<float> {
  using Acc = v4f_t;
  static __device__ __forceinline__ Acc mac(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return 4 * (l >> 4) + v; }
};

// Matrix tiles one wave owns at most (tiles w, w + 4, ... of an axis).
constexpr int kDenseTiles = (kDenseMax / 16 + 3) / 4;

// LDS stride of one line of an item buffer holding K entries: K rounded up
// to the matrix step (4) plus one, odd, so the 16 lines of a tile fall on
// different banks.
__host__ __device__ inline int dense_stride(int K) { return ((K + 3) & ~3) + 1; }

// The dense form of one axis' transform, with its basis table staged in LDS.
template <typename R>
struct DPlan {
  int n, P, fold, ck, di, ci;
  R nk0, nk1;          // orthonormal factor of coefficient 0 and of the others
  const R* tab;        // LDS
  BHX_GLOBAL const R* gtab;
  BHX_GLOBAL const R* glam;
  __device__ DPlan(const Batch& B, int idx) {
    const AxisPlan A = B.plans[idx];
    n = A.n;
    P = A.dense_P;
    fold = A.dense_fold;
    ck = A.bc == kDirichlet ? 1 : 0;
    di = A.bc == kNeumann ? 2 : 1;
    ci = A.bc == kPeriodic ? 0 : 1;
    nk0 = A.bc == kNeumann ? (R)A.s0 : (R)(2 * A.hs);
    nk1 = A.bc == kNeumann ? (R)A.s1 : (R)(2 * A.hs);
    const int pi = sizeof(R) == 8 ? 0 : 1;
    gtab = (BHX_GLOBAL const R*)B.rtab[pi] + A.off_dtab;
    glam = (BHX_GLOBAL const R*)B.rtab[pi] + A.off_lam;
    tab = nullptr;
  }
  __device__ __forceinline__ R nk(int k) const { return k == 0 ? nk0 : nk1; }
  __device__ __forceinline__ int len() const { return fold ? P / 2 + 1 : P; }
  __device__ __forceinline__ R at(int idx) const { return tab[fold ? min(idx, P - idx) : idx]; }
  // Copy the basis table (and, given `lam`, the eigenvalues) of plan `idx`
  // into LDS unless it is there already; every thread calls this at the
  // same point.
  __device__ void stage(R* lds, R* lam, int idx, int& staged) {
    if (idx != staged) {
      const int L = len();
      for (int e = threadIdx.x; e < L; e += kThreads) lds[e] = gtab[e];
      if (lam)
        for (int e = threadIdx.x; e < n; e += kThreads) lam[e] = glam[e];
      __syncthreads();
      staged = idx;
    }
    tab = lds;
  }
};

// acc[t] = the wave's matrix tile t (axis tile w + 4t) of a product with the
// basis over K = n entries, from the item buffer dat (16 lines, stride S,
// zero past K up to a multiple of 4):
//   TAB_A: D[k][c] = sum_i T(k, i) dat[c][i]   (tiles along k)
//   TAB_B: D[c][i] = sum_k dat[c][k] T(k, i)   (tiles along i)
// Each lane walks its basis row or column by the index rule, one modular
// addition per step.
template <typename R, bool TAB_A>
__device__ __forceinline__ void dense_product(const DPlan<R>& X, const R* dat, int S, int K,
                                              typename Mfma<R>::Acc (&acc)[kDenseTiles]) {
  using M = Mfma<R>;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lo = l & 15, hi = l >> 4;
  const int ntiles = (X.n + 15) >> 4;
  const int nt = (ntiles - w + 3) >> 2;          // this wave's tiles (wave-uniform)
  int idx[kDenseTiles], inc[kDenseTiles];
#pragma unroll
  for (int t = 0; t < kDenseTiles; ++t) {
    acc[t] = (typename M::Acc){0, 0, 0, 0};
    const int u = ((w + 4 * t) << 4) + lo;       // the tile's fixed coordinate (k or i)
    // T(k, i) index ((k + ck)(di i + ci)) mod P; the moving coordinate is
    // hi, hi + 4, ...
    const int F = TAB_A ? u + X.ck : X.di * u + X.ci;
    const int G0 = TAB_A ? X.di * hi + X.ci : hi + X.ck;
    const int step = TAB_A ? 4 * X.di : 4;
    idx[t] = (F * G0) % X.P;
    inc[t] = (F * step) % X.P;
  }
  const R* line = dat + lo * S + hi;
#pragma unroll 2
  for (int k0 = 0; k0 < K; k0 += 4) {
    const R s = line[k0];
#pragma unroll
    for (int t = 0; t < kDenseTiles; ++t) {
      if (t < nt) {
        const R tv = X.at(idx[t]);
        acc[t] = TAB_A ? M::mac(tv, s, acc[t]) : M::mac(s, tv, acc[t]);
        idx[t] += inc[t];
        idx[t] -= idx[t] >= X.P ? X.P : 0;
      }
    }
  }
}

// Row pass, forward, dense: the CG update of 16 rows (as k_rowfwd), the rows
// staged in LDS, then the x transform as a product with the basis, written
// transposed to t[k * nrows + j].  `mode` bits 0-1: 0 transform only, 1 PCG
// update then transform.  `tab_off`: element offset of the basis table in
// the dynamic LDS (after the largest item buffer of the launch).
template <typename R>
__global__ void __launch_bounds__(kThreads) k_rowfwd_dense(const Batch* __restrict__ Bp,
                                                           int mode, int tab_off, int lpar) {
  using M = Mfma<R>;
  const int update = mode & 3;
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  extern __shared__ __align__(16) unsigned char smem[];
  debug_fill_lds(smem);
  R* dat = (R*)smem;
  R* tabl = dat + tab_off;
  __shared__ double red[8];
  int staged = -1;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int itm = logical_block(); itm < B.n_items[kPassRD]; itm += gridDim.x) {
    const int code = item_code(B, kPassRD, itm);
    const Inst I = B.inst[code >> kItemShift];
    const int g = code & kItemMask;
    BHX_GLOBAL Ctl* ctl = I.ctl;
    const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
    const int nx = I.nx, ny = I.nrows, j0 = g * kDenseG;
    const int jn = min(kDenseG, ny - j0);
    const int E = jn * nx;
    const size_t base = (size_t)j0 * nx;
    BHX_GLOBAL const uint8_t* __restrict__ mk = I.mask + base;
    BHX_GLOBAL double* __restrict__ Fb = I.F + base;
    BHX_GLOBAL double* __restrict__ rb = I.r + base;
    BHX_GLOBAL const double* __restrict__ pb = (lpar ? I.p[0] : I.p[1]) + base;
    BHX_GLOBAL const double* __restrict__ qb = I.q + base;
    BHX_GLOBAL const double* arrs[2] = {I.part + PL.rz(lpar), I.part + PL.pq()};
    const int lens[2] = {I.reduce ? 1 : PL.nR, I.reduce ? 1 : PL.nS};
    const int ns[2] = {update && !I.reduce ? PL.nR : 0, update && !I.reduce ? PL.nS : 0};
    Partials<2> PS;
    sums_issue<2>(arrs, lens, PS);
    const double rsc[2] = {ctl->red_rz[lpar], ctl->red_pq};
    const int c_done = ctl->done, k_it = ctl->iter;
    const double rowcnt = I.part[PL.rowcnt() + g];
    if (c_done) continue;
    BHX_GLOBAL R* t = (BHX_GLOBAL R*)I.t;
    if (rowcnt == 0.0) {
      // no unknown node in these rows: r = 0 there, so is its transform
      for (int e = threadIdx.x; e < nx * kDenseG; e += kThreads) {
        const int kx = e / kDenseG, j = j0 + (e - kx * kDenseG);
        if (j < ny) t[(size_t)kx * ny + j] = (R)0;
      }
      if (update && threadIdx.x == 0) I.part[PL.rr() + g] = 0.0;
      continue;
    }
    double alpha = 0.0;
    if (update) {
      double sums[2];
      sums_finish<2>(arrs, ns, PS, sums, red);
      alpha = I.reduce ? rsc[0] / rsc[1] : sums[0] / sums[1];
    }
    const bool first = k_it == 0;
    const int S = dense_stride(nx);
    double acc_rr = 0.0;
    for (int e0 = threadIdx.x; e0 < kDenseG * nx; e0 += kUnroll * kThreads) {
      int m[kUnroll];
      double rv[kUnroll], pv[kUnroll], qv[kUnroll], xv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = e0 + u * kThreads;
        m[u] = e < E ? mk[min(e, E - 1)] : 0;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int ea = m[u] ? e0 + u * kThreads : 0;
        rv[u] = rb[ea];
        pv[u] = update ? pb[ea] : 0.0;
        qv[u] = update ? qb[ea] : 0.0;
        xv[u] = update ? Fb[ea] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = e0 + u * kThreads;
        if (e >= kDenseG * nx) break;
        double v = m[u] ? rv[u] : 0.0;
        if (update && m[u]) {
          Fb[e] = (first && !I.warm ? 0.0 : xv[u]) + alpha * pv[u];
          v -= alpha * qv[u];
          rb[e] = v;
          acc_rr += v * v;
        }
        const int jr = e / nx, i = e - jr * nx;
        dat[jr * S + i] = (R)v;
      }
    }
    for (int e = threadIdx.x; e < kDenseG * (S - nx); e += kThreads) {
      const int jr = e / (S - nx);
      dat[jr * S + nx + (e - jr * (S - nx))] = (R)0;
    }
    DPlan<R> X(B, I.planx);
    X.stage(tabl, nullptr, I.planx, staged);       // synchronises the block
    __syncthreads();
    if (update) {
      acc_rr = block_sum(acc_rr, red);
      if (threadIdx.x == 0) I.part[PL.rr() + g] = acc_rr;
    }
    typename M::Acc acc[kDenseTiles];
    dense_product<R, true>(X, dat, S, nx, acc);
    const int nt = (((nx + 15) >> 4) - w + 3) >> 2;
#pragma unroll
    for (int tt = 0; tt < kDenseTiles; ++tt) {
      if (tt < nt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = ((w + 4 * tt) << 4) + M::row(v, l), c = l & 15;
          if (k < nx && c < jn) t[(size_t)k * ny + j0 + c] = acc[tt][v] * X.nk(k);
        }
      }
    }
    __syncthreads();          // dat is reused by the block's next item
  }
}

// Column pass, dense: 16 columns (kx lines of t, y contiguous) per item:
// U = T_y t (forward), scaled by nk(ky)^2 / (lambda_x + lambda_y)^2 (0 for a
// zero sum) - both orthonormal factors of the pair of transforms at once -
// then t = T_y^T U (inverse), in place.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_col_dense(const Batch* __restrict__ Bp,
                                                        int count_iter, int tab_off) {
  using M = Mfma<R>;
  const Batch B = *(BHX_CONST const Batch*)Bp;
  extern __shared__ __align__(16) unsigned char smem[];
  debug_fill_lds(smem);
  R* dat = (R*)smem;
  R* tabl = dat + tab_off;
  R* laml = tabl + 2 * kDenseMax + 2;       // after the longest table (DST-I: 2(n+1))
  __shared__ R s_lamx[kDenseG];
  int staged = -1;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int itm = logical_block(); itm < B.n_items[kPassCD]; itm += gridDim.x) {
    const int code = item_code(B, kPassCD, itm);
    const Inst I = B.inst[code >> kItemShift];
    const int c = code & kItemMask;
    BHX_GLOBAL Ctl* ctl = I.ctl;
    if (ctl->done) continue;
    const int nx = I.nx, ny = I.ny, c0 = c * kDenseG;
    const int cnt = min(kDenseG, nx - c0);
    const int S = dense_stride(ny);
    BHX_GLOBAL R* t = (BHX_GLOBAL R*)I.t;
    for (int e = threadIdx.x; e < kDenseG * S; e += kThreads) {
      const int cr = e / S, j = e - cr * S;
      dat[e] = (cr < cnt && j < ny) ? t[(size_t)(c0 + cr) * ny + j] : (R)0;
    }
    if (threadIdx.x < kDenseG) {
      const DPlan<R> Xx(B, I.planx);
      s_lamx[threadIdx.x] = Xx.glam[min(c0 + (int)threadIdx.x, nx - 1)];
    }
    DPlan<R> X(B, I.plany);
    X.stage(tabl, laml, I.plany, staged);
    __syncthreads();
    typename M::Acc acc[kDenseTiles];
    dense_product<R, true>(X, dat, S, ny, acc);     // U[ky][cr]
    const int nt = (((ny + 15) >> 4) - w + 3) >> 2;
    __syncthreads();                                 // every wave is done reading dat
#pragma unroll
    for (int tt = 0; tt < kDenseTiles; ++tt) {
      if (tt < nt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ky = ((w + 4 * tt) << 4) + M::row(v, l), cr = l & 15;
          if (ky < ny) {
            const R f = X.nk(ky);
            dat[cr * S + ky] = acc[tt][v] * (f * f) * inv_sq<R>(laml[ky] + s_lamx[cr]);
          }
        }
      }
    }
    __syncthreads();
    dense_product<R, false>(X, dat, S, ny, acc);    // t[cr][j]
#pragma unroll
    for (int tt = 0; tt < kDenseTiles; ++tt) {
      if (tt < nt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cr = M::row(v, l), j = ((w + 4 * tt) << 4) + (l & 15);
          if (cr < cnt && j < ny) t[(size_t)(c0 + cr) * ny + j] = acc[tt][v];
        }
      }
    }
    if (count_iter && c == 0 && threadIdx.x == 0) ctl->iter = ctl->iter + 1;
    __syncthreads();
  }
}

// Row pass, inverse, dense: 16 rows of spectra read transposed from t,
// pre-scaled by nk(k), multiplied by the basis; z at the unknown nodes;
// partial r.z (and r.z_old), as k_rowinv.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_rowinv_dense(const Batch* __restrict__ Bp,
                                                           int tab_off, int lpar) {
  using M = Mfma<R>;
  const Batch B = *(BHX_CONST const Batch*)Bp;
  extern __shared__ __align__(16) unsigned char smem[];
  debug_fill_lds(smem);
  R* dat = (R*)smem;
  R* tabl = dat + tab_off;
  __shared__ double red[4];
  int staged = -1;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int itm = logical_block(); itm < B.n_items[kPassRD]; itm += gridDim.x) {
    const int code = item_code(B, kPassRD, itm);
    const Inst I = B.inst[code >> kItemShift];
    const int g = code & kItemMask;
    BHX_GLOBAL Ctl* ctl = I.ctl;
    const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
    const int par = lpar ^ 1;
    const int nx = I.nx, ny = I.nrows, j0 = g * kDenseG;
    const int jn = min(kDenseG, ny - j0);
    const int c_done = ctl->done;
    const double rowcnt = I.part[PL.rowcnt() + g];
    if (c_done) continue;
    const bool flex = I.flexible != 0;
    if (rowcnt == 0.0) {      // z stays 0 on rows without unknowns
      if (threadIdx.x == 0) {
        I.part[PL.rz(par) + g] = 0.0;
        if (flex) I.part[PL.rzo(par) + g] = 0.0;
      }
      continue;
    }
    DPlan<R> X(B, I.planx);
    const int S = dense_stride(nx);
    BHX_GLOBAL const R* t = (BHX_GLOBAL const R*)I.t;
    // dat[jr][k] = nk(k) t[k][j0 + jr]: 16 consecutive j per k in memory
    for (int e = threadIdx.x; e < kDenseG * S; e += kThreads) {
      const int k = e / kDenseG, jr = e - k * kDenseG;
      if (k < S) dat[jr * S + k] = (jr < jn && k < nx) ? t[(size_t)k * ny + j0 + jr] * X.nk(k)
                                                        : (R)0;
    }
    X.stage(tabl, nullptr, I.planx, staged);
    __syncthreads();
    typename M::Acc acc[kDenseTiles];
    dense_product<R, false>(X, dat, S, nx, acc);
    const size_t base = (size_t)j0 * nx;
    BHX_GLOBAL const uint8_t* __restrict__ mk = I.mask + base;
    BHX_GLOBAL const double* __restrict__ rb = I.r + base;
    BHX_GLOBAL double* __restrict__ zb = I.z + base;
    const int nt = (((nx + 15) >> 4) - w + 3) >> 2;
    double a_rz = 0.0, a_rzo = 0.0;
#pragma unroll
    for (int tt = 0; tt < kDenseTiles; ++tt) {
      if (tt < nt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int jr = M::row(v, l), i = ((w + 4 * tt) << 4) + (l & 15);
          if (jr < jn && i < nx) {
            const size_t o = (size_t)jr * nx + i;
            if (mk[o]) {
              const double zv = (double)acc[tt][v];
              const double rv = rb[o];
              if (flex) a_rzo += rv * zb[o];
              zb[o] = zv;
              a_rz += rv * zv;
            }
          }
        }
      }
    }
    a_rz = block_sum(a_rz, red);
    if (flex) a_rzo = block_sum(a_rzo, red);
    if (threadIdx.x == 0) {
      I.part[PL.rz(par) + g] = a_rz;
      if (flex) I.part[PL.rzo(par) + g] = a_rzo;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-instance finalisation (one block per instance) and helpers.
// ---------------------------------------------------------------------------

enum FinMode { kFinSetup = 0, kFinResid = 1, kFinWarm = 2 };

__global__ void __launch_bounds__(kThreads) k_finalize(const Batch* __restrict__ Bp, int mode) {
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  __shared__ double red[4];
  const int inst = blockIdx.x;
  if (inst >= B.count) return;
  const Inst I = B.inst[inst];
  BHX_GLOBAL Ctl* ctl = I.ctl;
  const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
  if (mode == kFinSetup) {
    if (ctl->done) return;
    const double nu = block_sum_array(I.part + PL.aux2(), PL.nS, red);
    const double bb = block_sum_array(I.part + PL.aux(), PL.nS, red);
    if (threadIdx.x == 0) {
      ctl->n_unknown = nu;
      ctl->bb = bb;
      ctl->bb0 = bb;
      ctl->accept = ctl->tol2 * bb;
      ctl->thresh = (ctl->accurate ? ctl->tol_inner2 : ctl->tol2) * bb;
    }
  } else if (mode == kFinWarm) {
    // residual of the given start x0 (the host compares it with the target)
    if (ctl->done) return;
    const double rr = block_sum_array(I.part + PL.aux(), PL.nS, red);
    if (threadIdx.x == 0) {
      ctl->true_rr = rr;
      ctl->rr = rr;
      if (ctl->accurate) {           // the first inner solve reduces this residual
        ctl->bb = rr;
        ctl->thresh = ctl->tol_inner2 * rr;
      }
    }
  } else {
    if (ctl->done != kConverged && ctl->done != kMaxIt) return;
    const double rr = block_sum_array(I.part + PL.aux(), PL.nS, red);
    if (threadIdx.x == 0) ctl->true_rr = rr;
  }
}

// Plain CG counts its iterations here (the preconditioned path counts in k_col).
__global__ void k_bump(const Batch* __restrict__ Bp) {
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= B.count) return;
  BHX_GLOBAL Ctl* ctl = B.inst[inst].ctl;
  if (ctl->done) return;
  ctl->iter = ctl->iter + 1;
}

// Instances whose true residual misses the target restart from it.
// Scalars of instances with long partial-sum arrays (Inst::reduce): one
// block per instance sums the partials of the pass just run in a fixed order
// into the control block, which the next pass reads instead of reducing the
// partials again in each of its blocks.
__global__ void __launch_bounds__(kThreads) k_reduce(const Batch* __restrict__ Bp, int which,
                                                     int lpar) {
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  __shared__ double red[4];
  const Inst I = B.inst[blockIdx.x];
  if (!I.reduce) return;
  BHX_GLOBAL Ctl* ctl = I.ctl;
  if (ctl->done) return;             // no writer of `done` runs during this launch
  const PartLayout PL(I.n_items[kPassS], I.n_items[kPassR]);
  if (which == kRedPQ) {
    const double v = block_sum_long(I.part + PL.pq(), PL.nS, red);
    if (threadIdx.x == 0) ctl->red_pq = v;
  } else if (which == kRedRR) {
    const double v = block_sum_long(I.part + PL.rr(), PL.nR, red);
    if (threadIdx.x == 0) ctl->red_rr = v;
  } else {
    const int par = lpar ^ 1;        // the parity the row-inverse pass wrote
    const double v = block_sum_long(I.part + PL.rz(par), PL.nR, red);
    const double w = I.flexible ? block_sum_long(I.part + PL.rzo(par), PL.nR, red) : 0.0;
    if (threadIdx.x == 0) {
      ctl->red_rz[par] = v;
      ctl->red_rzo[par] = w;
    }
  }
}

__global__ void k_restart(const Batch* __restrict__ Bp) {
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= B.count) return;
  BHX_GLOBAL Ctl* ctl = B.inst[inst].ctl;
  if (ctl->done != kConverged) return;
  if (ctl->true_rr <= ctl->accept) return;
  if (ctl->restarts >= ctl->max_restarts || ctl->iter >= B.inst[inst].maxit) return;
  ctl->restarts = ctl->restarts + 1;
  ctl->restart_iter = ctl->iter;
  ctl->bb = ctl->true_rr;
  if (ctl->accurate) {
    ctl->thresh = ctl->tol_inner2 * ctl->true_rr;
  } else {
    // the recursive residual met tol but the true one did not: tighten the
    // recursive target by 2 per restart so the true residual must follow
    ctl->thresh = ctl->thresh * 0.25;
  }
  ctl->done = kRunning;
}

// F = 0 at the unknown nodes of instances flagged by `flag` (zero right-hand side).
template <int DIM>
__global__ void __launch_bounds__(kThreads) k_zero_unknown(const Batch* __restrict__ Bp,
                                                           const int* __restrict__ flag) {
  using G = Geo<DIM>;
  const Batch B = *(BHX_CONST const Batch*)Bp;   // scalar loads, kept in registers
  for (int it = logical_block(); it < B.n_items[kPassS]; it += gridDim.x) {
    const int code = item_code(B, kPassS, it);
    const int ins = code >> kItemShift;
    if (!flag[ins]) continue;
    const Inst I = B.inst[ins];
    const int tile = code & kItemMask;
    int i0, j0, k0;
    G::origin(I, tile, i0, j0, k0);
    for (int e = threadIdx.x; e < G::TX * G::TY * G::TZ; e += kThreads) {
      int ii, jj, kk;
      G::template coords<G::TX, G::TY>(e, ii, jj, kk);
      const int i = i0 + ii, j = j0 + jj, k = k0 + kk;
      if (i < I.nx && j < I.ny && k < I.nz) {
        const size_t o = ((size_t)k * I.ny + j) * I.nx + i;
        if (I.mask[o]) I.F[o] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers (host side)
// ---------------------------------------------------------------------------

hipError_t launch_setup(const Batch* B, int dim, int grid, hipStream_t st) {
  if (dim == 3)
    hipLaunchKernelGGL(k_setup<3>, dim3(grid), dim3(kThreads), 0, st, B);
  else
    hipLaunchKernelGGL(k_setup<2>, dim3(grid), dim3(kThreads), 0, st, B);
  return hipGetLastError();
}
// Launch on `st`; given events, through hipExtLaunchKernelGGL, whose dispatch
// records them at kernel start and end.
#define BHX_LAUNCH(kernel, grid, lds, st, e0, e1, ...)                                  \
  do {                                                                                \
    if ((e0) || (e1))                                                                 \
      hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), lds, st, e0, e1, 0,   \
                            __VA_ARGS__);                                             \
    else                                                                              \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), lds, st, __VA_ARGS__);   \
  } while (0)

template <int DIM>
static hipError_t launch_stencil_dim(const Batch* B, int mode, int grid, int lpar,
                                     hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  switch (mode) {
    case kModeIter: BHX_LAUNCH((k_stencil<kModeIter, DIM>), grid, 0, st, e0, e1, B, lpar); break;
    case kModeRhs: BHX_LAUNCH((k_stencil<kModeRhs, DIM>), grid, 0, st, e0, e1, B, lpar); break;
    case kModeApply: BHX_LAUNCH((k_stencil<kModeApply, DIM>), grid, 0, st, e0, e1, B, lpar); break;
    case kModeWarm: BHX_LAUNCH((k_stencil<kModeWarm, DIM>), grid, 0, st, e0, e1, B, lpar); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_stencil(const Batch* B, int dim, int mode, int grid, int lpar, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1) {
  return dim == 3 ? launch_stencil_dim<3>(B, mode, grid, lpar, st, e0, e1)
                  : launch_stencil_dim<2>(B, mode, grid, lpar, st, e0, e1);
}
hipError_t launch_resid(const Batch* B, int dim, int grid, hipStream_t st) {
  if (dim == 3)
    hipLaunchKernelGGL(k_resid<3>, dim3(grid), dim3(kThreads), 0, st, B);
  else
    hipLaunchKernelGGL(k_resid<2>, dim3(grid), dim3(kThreads), 0, st, B);
  return hipGetLastError();
}
// Compile-time shapes instantiated per pass family, as (G, L, bc): G lines
// per work item, a 2^L-point core, Neumann (0), periodic (1) or Dirichlet (2).
// Two dimensions: 64-2048 nodes (Neumann, periodic) and 63-2047 nodes with
// n + 1 a power of two (Dirichlet), one packed row per item, FP64 and FP32
// transforms; three dimensions (FP64): 128 and 256 nodes with the groups the
// layout gives 128^3 and 256^3 (rows and y pencils 8, z pencils 16).
#define BHX_COL2D_SHAPES(X)                                                             \
  X(2, 6, 0) X(2, 6, 1) X(2, 7, 0) X(2, 7, 1) X(2, 8, 0) X(2, 8, 1) X(2, 9, 0) X(2, 9, 1) \
  X(2, 10, 0) X(2, 10, 1) X(2, 11, 0) X(2, 11, 1) X(2, 7, 2) X(2, 8, 2) X(2, 9, 2)         \
  X(2, 10, 2) X(2, 11, 2) X(2, 12, 2)
#define BHX_ROW_SHAPES(X) BHX_COL2D_SHAPES(X) X(8, 7, 0) X(8, 7, 1) X(8, 8, 0) X(8, 8, 1)
#define BHX_COLY_SHAPES(X) X(8, 7, 0) X(8, 7, 1) X(8, 8, 0) X(8, 8, 1)
#define BHX_COLZ_SHAPES(X) X(16, 7, 0) X(16, 7, 1) X(16, 8, 0) X(16, 8, 1)
#define BHX_KEY(G, L, bc) (((G) << 8) | ((L) << 2) | (bc))

// The environment variable BHX_SHAPE_KERNELS=0 keeps every launch on the
// plan-table kernels (for comparing the two).
int shape_key(int pass, int prec, int n, int m, int logm, int bluestein, int bc, int group) {
  if (bluestein || m != (bc == kDirichlet ? 2 * (n + 1) : n)) return 0;
  if (prec != 0 && (group != 2 || (pass != kShapeRow && pass != kShapeCol2D))) return 0;
  if (logm < 1 || logm > 15 || group < 2 || group > 64) return 0;
  const int key = BHX_KEY(group, logm, bc);
  bool listed = false;
#define BHX_IS(G, L, b) listed = listed || key == BHX_KEY(G, L, b);
  switch (pass) {
    case kShapeRow: BHX_ROW_SHAPES(BHX_IS) break;
    case kShapeCol2D: BHX_COL2D_SHAPES(BHX_IS) break;
    case kShapeColY: BHX_COLY_SHAPES(BHX_IS) break;
    case kShapeColZ: BHX_COLZ_SHAPES(BHX_IS) break;
    default: break;
  }
#undef BHX_IS
  if (!listed) return 0;
  const char* v = std::getenv("BHX_SHAPE_KERNELS");
  if (v && v[0] == '0') return 0;
  return key;
}

hipError_t launch_rowfwd(const Batch* B, int prec, int shape, int update, int stream_t, int grid,
                         int lds, int twoff, int lpar, hipStream_t st, hipEvent_t e0,
                         hipEvent_t e1) {
  update |= stream_t ? 4 : 0;
  if (prec != 0) {
    switch (shape) {
#define BHX_CASE(G, L, bc)                                                             \
  case BHX_KEY(G, L, bc):                                                              \
    BHX_LAUNCH((k_rowfwd<float, BHX_KEY(G, L, bc)>), grid, lds, st, e0, e1, B, update, \
               twoff, lpar);                                                           \
    break;
      BHX_COL2D_SHAPES(BHX_CASE)
#undef BHX_CASE
      case 0: BHX_LAUNCH((k_rowfwd<float, 0>), grid, lds, st, e0, e1, B, update, twoff, lpar); break;
      case kShapeWideKey:
        BHX_LAUNCH((k_rowfwd<float, 0, kFamWide>), grid, lds, st, e0, e1, B, update, twoff, lpar);
        break;
      case kShapeCzKey:
        BHX_LAUNCH((k_rowfwd<float, 0, kFamCz>), grid, lds, st, e0, e1, B, update, twoff, lpar);
        break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (shape) {
#define BHX_CASE(G, L, bc)                                                              \
  case BHX_KEY(G, L, bc):                                                               \
    BHX_LAUNCH((k_rowfwd<double, BHX_KEY(G, L, bc)>), grid, lds, st, e0, e1, B, update, \
               twoff, lpar);                                                            \
    break;
    BHX_ROW_SHAPES(BHX_CASE)
#undef BHX_CASE
    case 0: BHX_LAUNCH((k_rowfwd<double, 0>), grid, lds, st, e0, e1, B, update, twoff, lpar); break;
    case kShapeWideKey:
      BHX_LAUNCH((k_rowfwd<double, 0, kFamWide>), grid, lds, st, e0, e1, B, update, twoff, lpar);
      break;
    case kShapeCzKey:
      BHX_LAUNCH((k_rowfwd<double, 0, kFamCz>), grid, lds, st, e0, e1, B, update, twoff, lpar);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <typename R, int FAM>
static hipError_t launch_col_fam(const Batch* B, int kind, int count_iter, int grid, int lds,
                                 int twoff, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  switch (kind) {
    case kCol2D: BHX_LAUNCH((k_col<R, kCol2D, 0, FAM>), grid, lds, st, e0, e1, B, count_iter, twoff); break;
    case kColYFwd: BHX_LAUNCH((k_col<R, kColYFwd, 0, FAM>), grid, lds, st, e0, e1, B, count_iter, twoff); break;
    case kColZ: BHX_LAUNCH((k_col<R, kColZ, 0, FAM>), grid, lds, st, e0, e1, B, count_iter, twoff); break;
    case kColYInv: BHX_LAUNCH((k_col<R, kColYInv, 0, FAM>), grid, lds, st, e0, e1, B, count_iter, twoff); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <typename R>
static hipError_t launch_col_prec(const Batch* B, int kind, int shape, int count_iter, int grid,
                                  int lds, int twoff, hipStream_t st, hipEvent_t e0,
                                  hipEvent_t e1) {
  if (shape == kShapeCzKey) {
    // chirp-z Dirichlet axes exist in two dimensions only
    if (kind != kCol2D) return hipErrorInvalidValue;
    BHX_LAUNCH((k_col<R, kCol2D, 0, kFamCz>), grid, lds, st, e0, e1, B, count_iter, twoff);
    return hipGetLastError();
  }
  return shape == kShapeWideKey
             ? launch_col_fam<R, kFamWide>(B, kind, count_iter, grid, lds, twoff, st, e0, e1)
             : launch_col_fam<R, kFamNarrow>(B, kind, count_iter, grid, lds, twoff, st, e0, e1);
}
hipError_t launch_col(const Batch* B, int prec, int shape, int kind, int count_iter, int grid,
                      int lds, int twoff, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (shape == kShapeCzKey || shape == kShapeWideKey) {
    return prec == 0
               ? launch_col_prec<double>(B, kind, shape, count_iter, grid, lds, twoff, st, e0, e1)
               : launch_col_prec<float>(B, kind, shape, count_iter, grid, lds, twoff, st, e0, e1);
  }
  if (shape != 0 && prec != 0) {
    if (kind != kCol2D) return hipErrorInvalidValue;
    switch (shape) {
#define BHX_CASE_F(G, L, bc)                                                               \
  case BHX_KEY(G, L, bc):                                                                  \
    BHX_LAUNCH((k_col<float, kCol2D, BHX_KEY(G, L, bc)>), grid, lds, st, e0, e1, B,        \
               count_iter, twoff);                                                         \
    break;
      BHX_COL2D_SHAPES(BHX_CASE_F)
#undef BHX_CASE_F
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (shape != 0) {
#define BHX_CASE_K(K, G, L, bc)                                                          \
  case BHX_KEY(G, L, bc):                                                                \
    BHX_LAUNCH((k_col<double, K, BHX_KEY(G, L, bc)>), grid, lds, st, e0, e1, B, count_iter, \
               twoff);                                                                   \
    break;
#define BHX_CASE_2D(G, L, bc) BHX_CASE_K(kCol2D, G, L, bc)
#define BHX_CASE_YF(G, L, bc) BHX_CASE_K(kColYFwd, G, L, bc)
#define BHX_CASE_YI(G, L, bc) BHX_CASE_K(kColYInv, G, L, bc)
#define BHX_CASE_Z(G, L, bc) BHX_CASE_K(kColZ, G, L, bc)
    switch (kind) {
      case kCol2D:
        switch (shape) { BHX_COL2D_SHAPES(BHX_CASE_2D) default: return hipErrorInvalidValue; }
        break;
      case kColYFwd:
        switch (shape) { BHX_COLY_SHAPES(BHX_CASE_YF) default: return hipErrorInvalidValue; }
        break;
      case kColYInv:
        switch (shape) { BHX_COLY_SHAPES(BHX_CASE_YI) default: return hipErrorInvalidValue; }
        break;
      case kColZ:
        switch (shape) { BHX_COLZ_SHAPES(BHX_CASE_Z) default: return hipErrorInvalidValue; }
        break;
      default: return hipErrorInvalidValue;
    }
#undef BHX_CASE_2D
#undef BHX_CASE_YF
#undef BHX_CASE_YI
#undef BHX_CASE_Z
#undef BHX_CASE_K
    return hipGetLastError();
  }
  return prec == 0
             ? launch_col_prec<double>(B, kind, 0, count_iter, grid, lds, twoff, st, e0, e1)
             : launch_col_prec<float>(B, kind, 0, count_iter, grid, lds, twoff, st, e0, e1);
}
hipError_t launch_rowinv(const Batch* B, int prec, int shape, int grid, int lds, int twoff,
                         int lpar, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (prec != 0) {
    switch (shape) {
#define BHX_CASE(G, L, bc)                                                                \
  case BHX_KEY(G, L, bc):                                                                 \
    BHX_LAUNCH((k_rowinv<float, BHX_KEY(G, L, bc)>), grid, lds, st, e0, e1, B, twoff, lpar); \
    break;
      BHX_COL2D_SHAPES(BHX_CASE)
#undef BHX_CASE
      case 0: BHX_LAUNCH((k_rowinv<float, 0>), grid, lds, st, e0, e1, B, twoff, lpar); break;
      case kShapeWideKey:
        BHX_LAUNCH((k_rowinv<float, 0, kFamWide>), grid, lds, st, e0, e1, B, twoff, lpar);
        break;
      case kShapeCzKey:
        BHX_LAUNCH((k_rowinv<float, 0, kFamCz>), grid, lds, st, e0, e1, B, twoff, lpar);
        break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (shape) {
#define BHX_CASE(G, L, bc)                                                                 \
  case BHX_KEY(G, L, bc):                                                                  \
    BHX_LAUNCH((k_rowinv<double, BHX_KEY(G, L, bc)>), grid, lds, st, e0, e1, B, twoff, lpar); \
    break;
    BHX_ROW_SHAPES(BHX_CASE)
#undef BHX_CASE
    case 0: BHX_LAUNCH((k_rowinv<double, 0>), grid, lds, st, e0, e1, B, twoff, lpar); break;
    case kShapeWideKey:
      BHX_LAUNCH((k_rowinv<double, 0, kFamWide>), grid, lds, st, e0, e1, B, twoff, lpar);
      break;
    case kShapeCzKey:
      BHX_LAUNCH((k_rowinv<double, 0, kFamCz>), grid, lds, st, e0, e1, B, twoff, lpar);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_setup_rows(const Batch* B, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_setup_rows, dim3(grid), dim3(kThreads), 0, st, B, (int)kPassR);
  hipLaunchKernelGGL(k_setup_rows, dim3(grid), dim3(kThreads), 0, st, B, (int)kPassRD);
  return hipGetLastError();
}
hipError_t launch_rowfwd_dense(const Batch* B, int prec, int update, int grid, int lds,
                               int tab_off, int lpar, hipStream_t st, hipEvent_t e0,
                               hipEvent_t e1) {
  if (prec != 0)
    BHX_LAUNCH((k_rowfwd_dense<float>), grid, lds, st, e0, e1, B, update, tab_off, lpar);
  else
    BHX_LAUNCH((k_rowfwd_dense<double>), grid, lds, st, e0, e1, B, update, tab_off, lpar);
  return hipGetLastError();
}
hipError_t launch_col_dense(const Batch* B, int prec, int count_iter, int grid, int lds,
                            int tab_off, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (prec != 0)
    BHX_LAUNCH((k_col_dense<float>), grid, lds, st, e0, e1, B, count_iter, tab_off);
  else
    BHX_LAUNCH((k_col_dense<double>), grid, lds, st, e0, e1, B, count_iter, tab_off);
  return hipGetLastError();
}
hipError_t launch_rowinv_dense(const Batch* B, int prec, int grid, int lds, int tab_off,
                               int lpar, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (prec != 0)
    BHX_LAUNCH((k_rowinv_dense<float>), grid, lds, st, e0, e1, B, tab_off, lpar);
  else
    BHX_LAUNCH((k_rowinv_dense<double>), grid, lds, st, e0, e1, B, tab_off, lpar);
  return hipGetLastError();
}
int dense_lds_bytes(int pass, int prec, int n_max) {
  const int sz = prec == 0 ? 8 : 4;
  const int tab = 2 * kDenseMax + 2;                     // longest basis table
  return (kDenseG * dense_stride(n_max) + tab + (pass == kPassCD ? n_max : 0)) * sz;
}
int dense_tab_off(int n_max) { return kDenseG * dense_stride(n_max); }
hipError_t launch_identity(const Batch* B, int grid, int lpar, hipStream_t st, hipEvent_t e0,
                           hipEvent_t e1) {
  BHX_LAUNCH(k_identity, grid, 0, st, e0, e1, B, lpar);
  return hipGetLastError();
}
hipError_t launch_finalize(const Batch* B, int count, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(count), dim3(kThreads), 0, st, B, mode);
  return hipGetLastError();
}
hipError_t launch_reduce(const Batch* B, int count, int which, int lpar, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(count), dim3(kThreads), 0, st, B, which, lpar);
  return hipGetLastError();
}
hipError_t launch_restart(const Batch* B, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_restart, dim3((count + 255) / 256), dim3(256), 0, st, B);
  return hipGetLastError();
}
hipError_t launch_bump(const Batch* B, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_bump, dim3((count + 255) / 256), dim3(256), 0, st, B);
  return hipGetLastError();
}
hipError_t launch_zero_unknown(const Batch* B, int dim, const int* flag, int grid,
                               hipStream_t st) {
  if (dim == 3)
    hipLaunchKernelGGL(k_zero_unknown<3>, dim3(grid), dim3(kThreads), 0, st, B, flag);
  else
    hipLaunchKernelGGL(k_zero_unknown<2>, dim3(grid), dim3(kThreads), 0, st, B, flag);
  return hipGetLastError();
}

hipError_t set_kernel_attributes() {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f) {
    hipError_t x = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kLdsDynMax);
    if (x != hipSuccess) e = x;
  };
  set((const void*)k_rowfwd<double, 0>);
  set((const void*)k_rowfwd<float, 0>);
  set((const void*)k_col<double, kCol2D, 0>);
  set((const void*)k_col<float, kCol2D, 0>);
  set((const void*)k_col<double, kColYFwd, 0>);
  set((const void*)k_col<float, kColYFwd, 0>);
  set((const void*)k_col<double, kColZ, 0>);
  set((const void*)k_col<float, kColZ, 0>);
  set((const void*)k_col<double, kColYInv, 0>);
  set((const void*)k_col<float, kColYInv, 0>);
  set((const void*)k_rowinv<double, 0>);
  set((const void*)k_rowinv<float, 0>);
  set((const void*)k_rowfwd<double, 0, kFamCz>);
  set((const void*)k_rowfwd<float, 0, kFamCz>);
  set((const void*)k_col<double, kCol2D, 0, kFamCz>);
  set((const void*)k_col<float, kCol2D, 0, kFamCz>);
  set((const void*)k_rowinv<double, 0, kFamCz>);
  set((const void*)k_rowinv<float, 0, kFamCz>);
  set((const void*)k_rowfwd<double, 0, kFamWide>);
  set((const void*)k_rowfwd<float, 0, kFamWide>);
  set((const void*)k_col<double, kCol2D, 0, kFamWide>);
  set((const void*)k_col<float, kCol2D, 0, kFamWide>);
  set((const void*)k_col<double, kColYFwd, 0, kFamWide>);
  set((const void*)k_col<float, kColYFwd, 0, kFamWide>);
  set((const void*)k_col<double, kColZ, 0, kFamWide>);
  set((const void*)k_col<float, kColZ, 0, kFamWide>);
  set((const void*)k_col<double, kColYInv, 0, kFamWide>);
  set((const void*)k_col<float, kColYInv, 0, kFamWide>);
  set((const void*)k_rowinv<double, 0, kFamWide>);
  set((const void*)k_rowinv<float, 0, kFamWide>);
  set((const void*)k_rowfwd_dense<double>);
  set((const void*)k_rowfwd_dense<float>);
  set((const void*)k_col_dense<double>);
  set((const void*)k_col_dense<float>);
  set((const void*)k_rowinv_dense<double>);
  set((const void*)k_rowinv_dense<float>);
#define BHX_SET_ROW(G, L, bc)                                        \
  set((const void*)k_rowfwd<double, BHX_KEY(G, L, bc)>);             \
  set((const void*)k_rowinv<double, BHX_KEY(G, L, bc)>);
#define BHX_SET_2D(G, L, bc)                                         \
  set((const void*)k_col<double, kCol2D, BHX_KEY(G, L, bc)>);        \
  set((const void*)k_col<float, kCol2D, BHX_KEY(G, L, bc)>);         \
  set((const void*)k_rowfwd<float, BHX_KEY(G, L, bc)>);              \
  set((const void*)k_rowinv<float, BHX_KEY(G, L, bc)>);
#define BHX_SET_Y(G, L, bc)                                          \
  set((const void*)k_col<double, kColYFwd, BHX_KEY(G, L, bc)>);      \
  set((const void*)k_col<double, kColYInv, BHX_KEY(G, L, bc)>);
#define BHX_SET_Z(G, L, bc) set((const void*)k_col<double, kColZ, BHX_KEY(G, L, bc)>);
  BHX_ROW_SHAPES(BHX_SET_ROW)
  BHX_COL2D_SHAPES(BHX_SET_2D)
  BHX_COLY_SHAPES(BHX_SET_Y)
  BHX_COLZ_SHAPES(BHX_SET_Z)
#undef BHX_SET_ROW
#undef BHX_SET_2D
#undef BHX_SET_Y
#undef BHX_SET_Z
  return e;
}

}  // namespace bhx
