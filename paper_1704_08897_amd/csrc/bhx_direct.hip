// Direct solve of the masked biharmonic system on the GPU (two dimensions):
// banded Cholesky factorisation of A_UU, the direct route of Sec. 2.2.
//
// The unknowns are numbered line by line, along grid rows (x fastest) or
// along grid columns (y fastest), so a 13-point row of A_UU reaches back at
// most about two lines of unknowns: the lower band width w is the largest
// distance, in that numbering, from an unknown to the first unknown its
// stencil couples to (computed exactly from the stencil and the ghost rules).
// A periodic axis across the lines would couple the first and last lines and
// make the band span the whole grid, so a periodic y axis takes the column
// numbering, and otherwise the lines run along the shorter axis (the band, and
// the factorisation's work, shrink with the line length).  Both axes periodic
// is rejected.
//
// Storage: panels of kNb columns.  Panel k holds columns [k*kNb, (k+1)*kNb)
// of the lower band, rows [k*kNb, k*kNb + H) with H = kNb + W (W = w rounded
// up to kNb), column-major: P[(k*kNb + c)*H + r] = A[k*kNb + r][k*kNb + c].
// Rows beyond the last unknown are an identity pad.
//
// Factorisation (right-looking, one step per panel): the diagonal block is
// factored in LDS in steps of 16 columns (each 16 x 16 diagonal in one wave's
// registers, pivots exchanged by readlane), the panel below it solved against
// it (TRSM, L read from LDS), and the trailing band updated by tile products
// of the panel with itself.
// Solves: forward and backward substitution, two panels per launch, each
// block updating the right-hand side block it owns (no cross-block sums).
// Every sum runs in a fixed order, so results are deterministic.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "bhx_runtime.h"

namespace bhx {
namespace {

constexpr int kNb = 64;          // panel width (block size)

struct Band {
  double* p;     // panels
  double* d;     // factored diagonal blocks L_kk, two 64 x 64 copies per panel:
                 // column-major (forward substitution), row-major (backward)
  int n;         // unknowns
  int npad;      // n rounded up to kNb
  int nblk;      // panels
  int H;         // panel height kNb + W
  int Q;         // W / kNb: tiles below the diagonal block
};

__device__ __forceinline__ size_t band_at(const Band& B, int k, int r, int c) {
  return ((size_t)k * kNb + c) * B.H + r;
}
// L_kk[r][c] in the column-major and the row-major copy
__device__ __forceinline__ size_t diag_col(int k, int r, int c) {
  return ((size_t)k * 2 * kNb + c) * kNb + r;
}
__device__ __forceinline__ size_t diag_row(int k, int r, int c) {
  return ((size_t)k * 2 * kNb + kNb + r) * kNb + c;
}

__device__ double block_sum_d(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// Unknown nodes per line (one block per line): line l holds the nodes
// l * sl + j * sj, j < len.
__global__ void __launch_bounds__(kThreads) k_dir_linecount(const uint8_t* __restrict__ mask,
                                                            int len, int sl, int sj,
                                                            int* __restrict__ cnt) {
  __shared__ double red[4];
  const int l = blockIdx.x;
  double c = 0;
  for (int j = threadIdx.x; j < len; j += kThreads) c += mask[(size_t)l * sl + (size_t)j * sj];
  c = block_sum_d(c, red);
  if (threadIdx.x == 0) cnt[l] = (int)c;
}

// Position of each unknown in the line-by-line numbering (-1 at known
// nodes): line offset plus the exclusive prefix count within the line (block
// scan).
__global__ void __launch_bounds__(kThreads) k_dir_index(const uint8_t* __restrict__ mask, int len,
                                                        int sl, int sj,
                                                        const int* __restrict__ line_off,
                                                        int* __restrict__ uidx) {
  __shared__ int wsum[4];
  __shared__ int carry;
  const int l = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = line_off[l];
  __syncthreads();
  for (int j0 = 0; j0 < len; j0 += kThreads) {
    const int j = j0 + threadIdx.x;
    const size_t node = (size_t)l * sl + (size_t)j * sj;
    const int u = j < len ? mask[node] : 0;
    // inclusive scan within the wave
    int v = u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(v, o, 64);
      if (lane >= o) v += t;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    int before = carry;
    for (int i = 0; i < w; ++i) before += wsum[i];
    if (j < len) uidx[node] = u ? before + v - 1 : -1;
    __syncthreads();
    if (threadIdx.x == kThreads - 1) carry = before + v;
    __syncthreads();
  }
}

// The row of A_UU of unknown node (x, y): A = L L with L the 5-point
// negative Laplacian applied to the ghost-padded field, so each of the 25
// (first, second) stencil pairs contributes cL(d1) cL(d2) s to the node the
// padded position maps to (s: the ghost sign).  Calls f(target node, coef).
template <typename Fn>
__device__ __forceinline__ void row_of_a(int x, int y, int nx, int ny, int bcx, int bcy, Fn f) {
  const int dx[5] = {0, -1, 1, 0, 0}, dy[5] = {0, 0, 0, -1, 1};
  const double cl[5] = {4.0, -1.0, -1.0, -1.0, -1.0};
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      double sx, sy;
      const int mx = map_axis(x + dx[a] + dx[b], nx, bcx, sx);
      const int my = map_axis(y + dy[a] + dy[b], ny, bcy, sy);
      const double s = sx * sy;
      if (s != 0.0) f(my * nx + mx, cl[a] * cl[b] * s);
    }
}

// Lower band width: max over unknowns of (own index - smallest coupled index).
__global__ void __launch_bounds__(kThreads) k_dir_width(const uint8_t* __restrict__ mask,
                                                        const int* __restrict__ uidx, int nx,
                                                        int ny, int bcx, int bcy,
                                                        int* __restrict__ wmax) {
  const int node = blockIdx.x * kThreads + threadIdx.x;
  if (node >= nx * ny || !mask[node]) return;
  const int gi = uidx[node];
  int w = 0;
  row_of_a(node % nx, node / nx, nx, ny, bcx, bcy, [&](int t, double) {
    if (mask[t]) w = max(w, gi - uidx[t]);
  });
  atomicMax(wmax, w);
}

// Assemble the lower band: each unknown adds its row's entries at columns
// not after it (the band is zeroed first; a row is written by its own
// thread only).
__global__ void __launch_bounds__(kThreads) k_dir_assemble(const uint8_t* __restrict__ mask,
                                                           const int* __restrict__ uidx, int nx,
                                                           int ny, int bcx, int bcy, Band B) {
  const int node = blockIdx.x * kThreads + threadIdx.x;
  if (node >= nx * ny || !mask[node]) return;
  const int gi = uidx[node];
  row_of_a(node % nx, node / nx, nx, ny, bcx, bcy, [&](int t, double c) {
    if (!mask[t]) return;
    const int gt = uidx[t];
    if (gt > gi) return;
    const int k = gt / kNb;
    B.p[band_at(B, k, gi - k * kNb, gt - k * kNb)] += c;
  });
}

// Identity on the padded diagonal entries (indices n .. npad-1).
__global__ void k_dir_pad(Band B) {
  const int g = B.n + blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= B.npad) return;
  const int k = g / kNb;
  B.p[band_at(B, k, g - k * kNb, g - k * kNb)] = 1.0;
}

// Value of v in lane `lane` of the wave (uniform result, no memory access).
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row `lane` of L_kk (zeros above the diagonal), from the column-major copy.
__device__ __forceinline__ void load_diag_row(const Band& B, int k, int lane, double (&a)[kNb]) {
#pragma unroll
  for (int c = 0; c < kNb; ++c) a[c] = B.d[diag_col(k, lane, c)];
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Step k, part 1: every block factors panel k's diagonal block in LDS (held
// column-major, M[c][r] = A[r][c], lower part), right-looking in four steps of
// 16 columns: wave 0 factors the 16 x 16 diagonal in its registers (one row
// per lane, pivots exchanged by readlane), threads solve the rows below it,
// and all threads update the trailing block.  Block 0 then stores L; block
// t >= 1 solves tile t of the panel (rows 64 t..) against L on the matrix
// cores, with L read from LDS, 16 rows per wave.
__global__ void __launch_bounds__(kThreads) k_dir_potrf_trsm(Band B, int k, int tiles) {
  __shared__ __align__(16) double M[kNb][kNb + 2];
  __shared__ double rinv[kNb];                 // 1 / L[j][j]
  constexpr int kStep = 16;
  __shared__ double Li[kNb / kStep][kStep][kStep + 1];   // Li[d][i][j] = (L_dd^-1)[i][j]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  {
    // all of a thread's loads issued before its first LDS write (rows r < c
    // of the block lie inside the band's storage too: H >= 64)
    constexpr int kPer = kNb * kNb / kThreads;
    double mv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * kThreads, c = e >> 6, r = e & 63;
      mv[u] = B.p[band_at(B, k, r, c)];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * kThreads, c = e >> 6, r = e & 63;
      M[c][r] = r >= c ? mv[u] : 0.0;
    }
  }
  __syncthreads();
  // Only the lower part of M is read from here on: the products below also
  // write the strictly upper half of diagonal 16 x 16 tiles, which no step
  // reads.
  for (int c0 = 0, d = 0; c0 < kNb; c0 += kStep, ++d) {
    if (w == 0) {
      // diagonal kStep x kStep block: lane l < kStep holds row c0 + l
      // one reciprocal square root per pivot p on the serial chain:
      // L_jj = p / sqrt(p), the column below it a / sqrt(p)
      double a[kStep];
      double rl = 1.0;                           // 1 / L[c0 + lane][c0 + lane]
#pragma unroll
      for (int dd = 0; dd < kStep; ++dd) a[dd] = lane < kStep ? M[c0 + dd][c0 + lane] : 0.0;
#pragma unroll
      for (int j = 0; j < kStep; ++j) {
        const double pj = lane_value(a[j], j);
        const double rj = rsqrt(pj);
        const double l = lane > j ? a[j] * rj : (lane == j ? pj * rj : 0.0);
        rl = lane == j ? rj : rl;
        a[j] = l;
#pragma unroll
        for (int m = j + 1; m < kStep; ++m) a[m] -= l * lane_value(l, m);
      }
      if (lane < kStep) {
#pragma unroll
        for (int dd = 0; dd < kStep; ++dd)
          if (dd <= lane) M[c0 + dd][c0 + lane] = a[dd];
        rinv[c0 + lane] = rl;
      }
    }
    __syncthreads();
    if (tid < kStep) {
      // column tid of L_dd^-1: solve L_dd y = e_tid, column-oriented so that
      // each step's updates are independent (every entry still subtracts
      // its terms in ascending order)
      const int jc = tid;
      double y[kStep];
#pragma unroll
      for (int i = 0; i < kStep; ++i) y[i] = i == jc ? 1.0 : 0.0;
      // step i's column of L and 1 / L_ii are read one step ahead, so the
      // chain does not wait for LDS
      double lc[kStep], ln[kStep];
      double rc = rinv[c0], rn = 0.0;
#pragma unroll
      for (int m = 1; m < kStep; ++m) lc[m] = M[c0][c0 + m];
#pragma unroll
      for (int i = 0; i < kStep; ++i) {
        if (i + 1 < kStep) {
#pragma unroll
          for (int m = i + 2; m < kStep; ++m) ln[m] = M[c0 + i + 1][c0 + m];
          rn = rinv[c0 + i + 1];
        }
        const double yi = i >= jc ? y[i] * rc : 0.0;
        y[i] = yi;
#pragma unroll
        for (int m = i + 1; m < kStep; ++m) y[m] -= lc[m] * yi;
#pragma unroll
        for (int m = i + 2; m < kStep; ++m) lc[m] = ln[m];
        rc = rn;
      }
#pragma unroll
      for (int i = 0; i < kStep; ++i) Li[d][i][jc] = y[i];
    }
    __syncthreads();
    const int rb = c0 + kStep, nt = (kNb - rb) / kStep;   // 16-row tiles below
    // rows below: X = A_below L_dd^-T on the matrix cores, wave w takes tile w
    // (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of each k-step
    // and holds D[4 v + l / 16][l % 16] in accumulator element v)
    if (w < nt) {
      const int rw = rb + kStep * w;
      v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const double aop = M[c0 + 4 * s4 + lk][rw + li];   // A[rw + i][c0 + kk]
        const double bop = Li[d][li][4 * s4 + lk];          // L_dd^-T[kk][j] = Linv[j][kk]
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) M[c0 + li][rw + 4 * v + lk] = acc[v];   // L[rw+i][c0+j]
    }
    __syncthreads();
    // trailing block: C -= X X^T over the lower 16 x 16 tiles (ti >= tj)
    const int ntl = nt * (nt + 1) / 2;
    for (int tt = w; tt < ntl; tt += 4) {
      int ti = 0;
      while ((ti + 1) * (ti + 2) / 2 <= tt) ++ti;
      const int tj = tt - ti * (ti + 1) / 2;
      const int ri = rb + kStep * ti, rj = rb + kStep * tj;
      v4d acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = M[rj + li][ri + 4 * v + lk];   // C[ri + 4v + kk][rj + j]
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const double aop = -M[c0 + 4 * s4 + lk][ri + li];   // -X[ri + i][kk]
        const double bop = M[c0 + 4 * s4 + lk][rj + li];    // X^T[kk][rj + j]
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) M[rj + li][ri + 4 * v + lk] = acc[v];
    }
    __syncthreads();
  }
  // Block 0 stores L_kk outside the band: the other blocks of this launch
  // read the band's diagonal block (A_kk) when they start, at any time.
  if (blockIdx.x == 0) {
    for (int e = tid; e < kNb * kNb; e += kThreads) {
      const int c = e >> 6, r = e & 63;
      B.d[diag_col(k, r, c)] = r >= c ? M[c][r] : 0.0;
      const int r2 = e >> 6, c2 = e & 63;
      B.d[diag_row(k, r2, c2)] = r2 >= c2 ? M[c2][r2] : 0.0;
    }
  }
  const int t = blockIdx.x;
  if (t == 0 || t >= tiles) return;      // no barrier below
  // Tile t solves X L^T = T (rows 64 t.. of the panel), as L Z = T^T with
  // Z = X^T, by 16-row blocks on the matrix cores:
  //   Z_d = L_dd^-1 (W_d - sum_{a<d} L_da Z_a),  W = T^T.
  // Wave w takes the tile's rows 16 w.. (one 16-column strip of Z, which no
  // other strip's products touch).  Z_d is held as a 16 x 16 tile in the
  // v_mfma_f64_16x16x4 output layout (lane l, element v: row 4 v + l / 16,
  // column l % 16), in which element s is exactly the B operand of k-step s,
  // so the products chain without leaving registers.
  const int r0 = t * kNb + kStep * w;
  v4d Z[4];
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      Z[d][v] = B.p[band_at(B, k, r0 + li, kStep * d + 4 * v + lk)];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
#pragma unroll
    for (int a2 = 0; a2 < d; ++a2)
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        // A operand -L[16 d + i][16 a2 + 4 s4 + kk], i = l % 16, kk = l / 16
        const double aop = -M[kStep * a2 + 4 * s4 + lk][kStep * d + li];
        Z[d] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, Z[a2][s4], Z[d], 0, 0, 0);
      }
    v4d T = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const double aop = Li[d][li][4 * s4 + lk];
      T = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, Z[d][s4], T, 0, 0, 0);
    }
    Z[d] = T;
  }
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      B.p[band_at(B, k, r0 + li, kStep * d + 4 * v + lk)] = Z[d][v];
}

// Step k, part 2: trailing update of the band by panel k.  Tile (q, rt):
// rows rt*kNb.. of panel k+q -= (panel k rows (rt+q)*kNb..) (panel k rows
// q*kNb..)^T, a 64 x 64 x 64 FP64 product on the matrix cores: the operands
// are staged in LDS and each of the block's 16 waves computes one 16 x 16
// output tile with v_mfma_f64_16x16x4 over k in steps of 4.  Lane layout of
// that instruction: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[4 v + l / 16][l % 16] in accumulator element v.
constexpr int kUpdThreads = 1024;
__global__ void __launch_bounds__(kUpdThreads) k_dir_update(Band B, int k) {
  __shared__ double sA[kNb][kNb];   // [t][r]
  __shared__ double sB[kNb][kNb];   // [t][c]
  const int q = 1 + blockIdx.x / (B.Q + 1), rt = blockIdx.x % (B.Q + 1);
  const int j = k + q;
  if (rt > B.Q - q || j + rt >= B.nblk) return;       // no such tile, or past the pad
  const int ra = (rt + q) * kNb, rb = q * kNb;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tr = (w >> 2) * 16, tc = (w & 3) * 16;      // the wave's output tile
  const int li = lane & 15, lk = lane >> 4;
  // every load of the block is issued before the first wait: the thread's
  // part of the output tile (which only this block reads or writes), then
  // the two operand tiles
  double cv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) cv[v] = B.p[band_at(B, j, rt * kNb + tr + 4 * v + lk, tc + li)];
  {
    constexpr int kPer = kNb * kNb / kUpdThreads;
    double va[kPer], vb[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + u * kUpdThreads, t = e / kNb, r = e - t * kNb;
      va[u] = B.p[band_at(B, k, ra + r, t)];
      vb[u] = B.p[band_at(B, k, rb + r, t)];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + u * kUpdThreads, t = e / kNb, r = e - t * kNb;
      sA[t][r] = va[u];
      sB[t][r] = vb[u];
    }
  }
  __syncthreads();
  v4d acc = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int t0 = 0; t0 < kNb; t0 += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[t0 + lk][tr + li], sB[t0 + lk][tc + li], acc,
                                               0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = tr + 4 * v + lk, c = tc + li;
    B.p[band_at(B, j, rt * kNb + r, c)] = cv[v] - acc[v];
  }
}

// Column `lane` of L_kk (zeros below the diagonal of L^T), from the
// row-major copy: col[j] = L[j][lane].
__device__ __forceinline__ void load_diag_col(const Band& B, int k, int lane, double (&col)[kNb]) {
#pragma unroll
  for (int j = 0; j < kNb; ++j) col[j] = B.d[diag_row(k, j, lane)];
}

// One wave solves L_kk u = v (lane t: v_t in, u_t out; a = row t of L_kk);
// 1 / L_tt is formed once, so the serial chain multiplies.
__device__ __forceinline__ double tri_lower(const double (&a)[kNb], double v, int lane) {
  double dg = 1.0;
#pragma unroll
  for (int j = 0; j < kNb; ++j) dg = lane == j ? a[j] : dg;
  const double rd = 1.0 / dg;
#pragma unroll
  for (int j = 0; j < kNb; ++j) {
    const double yj = lane_value(v, j) * lane_value(rd, j);
    if (lane == j) v = yj;
    else if (lane > j) v -= a[j] * yj;
  }
  return v;
}

// One wave solves L_kk^T u = v (lane t: v_t in, u_t out; col = column t of
// L_kk).
__device__ __forceinline__ double tri_upper(const double (&col)[kNb], double v, int lane) {
  double dg = 1.0;
#pragma unroll
  for (int j = 0; j < kNb; ++j) dg = lane == j ? col[j] : dg;
  const double rd = 1.0 / dg;
#pragma unroll
  for (int j = kNb - 1; j >= 0; --j) {
    const double xj = lane_value(v, j) * lane_value(rd, j);
    if (lane == j) v = xj;
    else if (lane < j) v -= col[j] * xj;
  }
  return v;
}

// Forward substitution step k: wave 0 of every block solves L_kk z_k = y_k
// (lane t: y_t and row t of L_kk in registers, and 1 / L_tt, so that the
// serial chain multiplies instead of dividing); block 0 stores z_k, block
// b >= 1 updates y_(k+b) -= L_(k+b,k) z_k.  z_k goes to its own vector: the
// other blocks read y_k when they start, at any time.
__global__ void __launch_bounds__(kThreads) k_dir_fwd(Band B, int k, double* __restrict__ y,
                                                      double* __restrict__ z) {
  __shared__ double yk[kNb];
  __shared__ double part[4][kNb];
  // the update's part of L_(k+b,k) (row r, columns 16 cs..), loaded before
  // the triangular solve so that its latency overlaps the serial chain
  const int b = blockIdx.x;
  const int r = threadIdx.x & 63, cs = threadIdx.x >> 6;
  double lv[16];
  if (b > 0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) lv[u] = B.p[band_at(B, k, b * kNb + r, cs * 16 + u)];
  }
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double a[kNb];
    load_diag_row(B, k, lane, a);
    yk[lane] = tri_lower(a, y[k * kNb + lane], lane);
  }
  __syncthreads();
  if (b == 0) {
    if (threadIdx.x < kNb) z[k * kNb + threadIdx.x] = yk[threadIdx.x];
    return;
  }
  // rows b*kNb.. of panel k: r = tid % 64, columns in four strips of 16
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s += lv[u] * yk[cs * 16 + u];
  part[cs][r] = s;
  __syncthreads();
  if (threadIdx.x < kNb)
    y[(k + b) * kNb + threadIdx.x] -=
        (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
}

// Backward substitution step k (k descending): wave 0 of every block solves
// L_kk^T x_k = z_k (lane t: z_t, column t of L_kk and 1 / L_tt in
// registers); block 0 stores x_k into x (its own vector, as in the forward
// step), block b >= 1 updates z_(k-b) -= L_(k,k-b)^T x_k (rows b*kNb.. of
// panel k-b).
__global__ void __launch_bounds__(kThreads) k_dir_bwd(Band B, int k, double* __restrict__ z,
                                                      double* __restrict__ x) {
  __shared__ double xk[kNb];
  __shared__ double part[4][kNb];
  // the update's part of panel k-b (column c, rows b*kNb + 16 rs..), loaded
  // before the triangular solve so that its latency overlaps the serial chain
  const int b = blockIdx.x, kb = k - b;
  const int c = threadIdx.x & 63, rs = threadIdx.x >> 6;
  double lv[16];
  if (b > 0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) lv[u] = B.p[band_at(B, kb, b * kNb + rs * 16 + u, c)];
  }
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double col[kNb];                     // col[j] = L[j][lane]
    load_diag_col(B, k, lane, col);
    xk[lane] = tri_upper(col, z[k * kNb + lane], lane);
  }
  __syncthreads();
  if (b == 0) {
    if (threadIdx.x < kNb) x[k * kNb + threadIdx.x] = xk[threadIdx.x];
    return;
  }
  // z_(k-b)[c] -= sum_r P_(k-b)[c][b*kNb + r] x_k[r]: c = tid % 64, r strips
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s += lv[u] * xk[rs * 16 + u];
  part[rs][c] = s;
  __syncthreads();
  if (threadIdx.x < kNb)
    z[kb * kNb + threadIdx.x] -=
        (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
}

// Two forward steps in one launch, k and k + 1 (k + 1 < nblk): wave 0
// solves z_k, every thread then takes its part of L_(k+1,k) z_k, wave 1
// solves z_(k+1) from y_(k+1) less that product, and block b >= 1 updates
// y_(k+1+b) by both steps' terms in the order two single steps would apply
// them (so the results equal the one-step kernel's bit for bit).  Block 0
// stores z_k and z_(k+1).
__global__ void __launch_bounds__(kThreads) k_dir_fwd2(Band B, int k, double* __restrict__ y,
                                                       double* __restrict__ z) {
  __shared__ double yk[2][kNb];
  __shared__ double part[2][4][kNb];
  const int b = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int r = tid & 63, cs = tid >> 6;
  const bool mid = B.Q >= 1;                 // L_(k+1,k) is inside the band
  const bool has0 = b > 0 && b + 1 <= B.Q;   // L_(k+1+b,k)
  const bool has1 = b > 0;                   // L_(k+1+b,k+1)
  double lm[16], l0[16], l1[16];
  if (mid) {
#pragma unroll
    for (int u = 0; u < 16; ++u) lm[u] = B.p[band_at(B, k, kNb + r, cs * 16 + u)];
  }
  if (has0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) l0[u] = B.p[band_at(B, k, (b + 1) * kNb + r, cs * 16 + u)];
  }
  if (has1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) l1[u] = B.p[band_at(B, k + 1, b * kNb + r, cs * 16 + u)];
  }
  double a[kNb];
  double v1 = 0.0;
  if (w == 0) load_diag_row(B, k, lane, a);
  else if (w == 1) {
    load_diag_row(B, k + 1, lane, a);
    v1 = y[(k + 1) * kNb + lane];
  }
  if (w == 0) yk[0][lane] = tri_lower(a, y[k * kNb + lane], lane);
  __syncthreads();
  if (mid) {
    double sm = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) sm += lm[u] * yk[0][cs * 16 + u];
    part[0][cs][r] = sm;
  }
  __syncthreads();
  if (w == 1) {
    if (mid)
      v1 -= (part[0][0][lane] + part[0][1][lane]) + (part[0][2][lane] + part[0][3][lane]);
    yk[1][lane] = tri_lower(a, v1, lane);
  }
  __syncthreads();
  if (b == 0) {
    if (tid < kNb) {
      z[k * kNb + tid] = yk[0][tid];
      z[(k + 1) * kNb + tid] = yk[1][tid];
    }
    return;
  }
  double s0 = 0.0, s1 = 0.0;
  if (has0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) s0 += l0[u] * yk[0][cs * 16 + u];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) s1 += l1[u] * yk[1][cs * 16 + u];
  part[0][cs][r] = s0;
  part[1][cs][r] = s1;
  __syncthreads();
  if (tid < kNb) {
    double v = y[(k + 1 + b) * kNb + tid];
    if (has0)
      v -= (part[0][0][tid] + part[0][1][tid]) + (part[0][2][tid] + part[0][3][tid]);
    v -= (part[1][0][tid] + part[1][1][tid]) + (part[1][2][tid] + part[1][3][tid]);
    y[(k + 1 + b) * kNb + tid] = v;
  }
}

// Two backward steps in one launch, k and k - 1 (k >= 1), as k_dir_fwd2
// for L^T: wave 0 solves x_k, every thread takes its part of
// L_(k,k-1)^T x_k, wave 1 solves x_(k-1), block b >= 1 updates
// z_(k-1-b) by both steps' terms in single-step order; block 0 stores
// x_k and x_(k-1).
__global__ void __launch_bounds__(kThreads) k_dir_bwd2(Band B, int k, double* __restrict__ z,
                                                       double* __restrict__ x) {
  __shared__ double xk[2][kNb];
  __shared__ double part[2][4][kNb];
  const int b = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int c = tid & 63, rs = tid >> 6;
  const int kb = k - 1 - b;                  // row block this block updates (b >= 1)
  const bool mid = B.Q >= 1;                 // L_(k,k-1): panel k-1, rows kNb..
  const bool has0 = b > 0 && b + 1 <= B.Q;   // L_(k,kb): panel kb, rows (b+1) kNb..
  const bool has1 = b > 0;                   // L_(k-1,kb): panel kb, rows b kNb..
  double lm[16], l0[16], l1[16];
  if (mid) {
#pragma unroll
    for (int u = 0; u < 16; ++u) lm[u] = B.p[band_at(B, k - 1, kNb + rs * 16 + u, c)];
  }
  if (has0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) l0[u] = B.p[band_at(B, kb, (b + 1) * kNb + rs * 16 + u, c)];
  }
  if (has1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) l1[u] = B.p[band_at(B, kb, b * kNb + rs * 16 + u, c)];
  }
  double col[kNb];
  double v1 = 0.0;
  if (w == 0) load_diag_col(B, k, lane, col);
  else if (w == 1) {
    load_diag_col(B, k - 1, lane, col);
    v1 = z[(k - 1) * kNb + lane];
  }
  if (w == 0) xk[0][lane] = tri_upper(col, z[k * kNb + lane], lane);
  __syncthreads();
  if (mid) {
    double sm = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) sm += lm[u] * xk[0][rs * 16 + u];
    part[0][rs][c] = sm;
  }
  __syncthreads();
  if (w == 1) {
    if (mid)
      v1 -= (part[0][0][lane] + part[0][1][lane]) + (part[0][2][lane] + part[0][3][lane]);
    xk[1][lane] = tri_upper(col, v1, lane);
  }
  __syncthreads();
  if (b == 0) {
    if (tid < kNb) {
      x[k * kNb + tid] = xk[0][tid];
      x[(k - 1) * kNb + tid] = xk[1][tid];
    }
    return;
  }
  double s0 = 0.0, s1 = 0.0;
  if (has0) {
#pragma unroll
    for (int u = 0; u < 16; ++u) s0 += l0[u] * xk[0][rs * 16 + u];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) s1 += l1[u] * xk[1][rs * 16 + u];
  part[0][rs][c] = s0;
  part[1][rs][c] = s1;
  __syncthreads();
  if (tid < kNb) {
    double v = z[kb * kNb + tid];
    if (has0)
      v -= (part[0][0][tid] + part[0][1][tid]) + (part[0][2][tid] + part[0][3][tid]);
    v -= (part[1][0][tid] + part[1][1][tid]) + (part[1][2][tid] + part[1][3][tid]);
    z[kb * kNb + tid] = v;
  }
}

// y[uidx] = r at unknown nodes; the pad is zeroed.
__global__ void k_dir_gather(const uint8_t* __restrict__ mask, const int* __restrict__ uidx,
                             const double* __restrict__ r, int N, int n, int npad,
                             double* __restrict__ y) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node < N && mask[node]) y[uidx[node]] = r[node];
  const int g = n + node;
  if (g < npad) y[g] = 0.0;
}

// F = y (first solve) or F += y (refinement) at unknown nodes.
__global__ void k_dir_scatter(const uint8_t* __restrict__ mask, const int* __restrict__ uidx,
                              const double* __restrict__ y, int N, int add,
                              double* __restrict__ F) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N || !mask[node]) return;
  const double v = y[uidx[node]];
  F[node] = add ? F[node] + v : v;
}

#define DIR_CHECK(x)                                                      \
  do {                                                                    \
    hipError_t _e = (x);                                                  \
    if (_e != hipSuccess) {                                               \
      set_last_error(#x, __LINE__, _e);                                   \
      return _e == hipErrorOutOfMemory ? BHX_ERR_NOMEM : BHX_ERR_HIP;     \
    }                                                                     \
  } while (0)

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Device addresses of instance 0 of the handle's current batch.
struct InstPtrs {
  uint8_t* mask;
  double* r;
  Ctl* ctl;
};
InstPtrs instance0(bhx_handle* hd, const InstSpec& S, const Resolved& R) {
  Layout L;
  make_layout(S.nx, S.ny, R.precision, core_length(fft_length(S.nx, S.bcx)),
              core_length(fft_length(S.ny, S.bcy)), R.sched.rows_cap, &L);
  char* base = (char*)hd->ws + align256(sizeof(Ctl));
  return {(uint8_t*)(base + L.off_mask), (double*)(base + L.off_vec), (Ctl*)hd->ws};
}

}  // namespace

bool direct_supported(int bcx, int bcy) { return !(bcx == kPeriodic && bcy == kPeriodic); }

// Banded Cholesky solve of a group of fields sharing phi (specs[0..n) have
// the same phi, sizes and rules): factor once, then per field: right-hand
// side, solve, and refinement with the compensated residual until
// ||b - A u|| <= tol ||b|| (at most 4 refinement solves).
int solve_direct(bhx_handle* hd, int n, const InstSpec* specs, const Resolved& R0,
                 hipStream_t stream, bhx_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = stream ? stream : hd->own_stream;
  Resolved R = R0;
  R.warm = 0;
  R.transform = 1;              // the layout instance0() recomputes (FFT row groups)
  R.sched.transform = -1;
  const InstSpec& S0 = specs[0];
  const int nx = S0.nx, ny = S0.ny, N = nx * ny;
  if (S0.dim != 2 || !direct_supported(S0.bcx, S0.bcy)) return BHX_ERR_ARG;
  int ret = BHX_OK;
  bool factored = false;
  Band B{};
  int* uidx = nullptr;
  double* y = nullptr;   // right-hand side, then the solution
  double* z = nullptr;   // forward substitution's result
  for (int f = 0; f < n; ++f) {
    const InstSpec& S = specs[f];
    Grids g;
    int rc = prepare_batch(hd, 1, &S, R, st, &g);
    if (rc != BHX_OK) return rc;
    const InstPtrs P = instance0(hd, S, R);
    DIR_CHECK(launch_setup(hd->batch_d, 2, g.s, st));
    DIR_CHECK(launch_setup_rows(hd->batch_d, g.r, st));
    DIR_CHECK(launch_stencil(hd->batch_d, 2, kModeRhs, g.s, 0, st));
    DIR_CHECK(launch_finalize(hd->batch_d, 1, kFinSetupH, st));
    Ctl* ch = hd->ctl_h;
    DIR_CHECK(hipMemcpyAsync(ch, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    DIR_CHECK(hipStreamSynchronize(st));
    int s = BHX_OK, refines = 0;
    bool preset = true;
    if (ch->n_unknown == 0) {
    } else if (ch->n_unknown == N && S.bcx != kDirichlet && S.bcy != kDirichlet) {
      s = BHX_ERR_SINGULAR;
    } else if (!std::isfinite(ch->bb)) {
      s = BHX_ERR_NONFINITE;
    } else {
      preset = false;
    }
    if (!preset && !factored) {
      // ordering, band width, storage: lines along y (columns) when y is
      // periodic or x the longer non-periodic axis, else along x (rows)
      const bool cols = S.bcy == kPeriodic || (S.bcx != kPeriodic && nx > ny);
      const int nl = cols ? nx : ny, len = cols ? ny : nx;
      const int sl = cols ? 1 : nx, sj = cols ? nx : 1;
      std::vector<int> cnt(nl), off(nl + 1, 0);
      const size_t need = align256((size_t)N * sizeof(int)) + align256((nl + 2) * sizeof(int));
      if (need > hd->dws_cap) {
        if (hd->dws) DIR_CHECK(hipFree(hd->dws));
        hd->dws = nullptr;
        hd->dws_cap = 0;
        DIR_CHECK(hipMalloc(&hd->dws, need));
        hd->dws_cap = need;
      }
      uidx = (int*)hd->dws;
      int* cnt_d = (int*)((char*)hd->dws + align256((size_t)N * sizeof(int)));
      hipLaunchKernelGGL(k_dir_linecount, dim3(nl), dim3(kThreads), 0, st, P.mask, len, sl, sj,
                         cnt_d);
      DIR_CHECK(hipGetLastError());
      DIR_CHECK(hipMemcpyAsync(cnt.data(), cnt_d, nl * sizeof(int), hipMemcpyDeviceToHost, st));
      DIR_CHECK(hipStreamSynchronize(st));
      for (int j = 0; j < nl; ++j) off[j + 1] = off[j] + cnt[j];
      const int nu = off[nl];
      {
        const Upload u{cnt_d, off.data(), (nl + 1) * sizeof(int)};
        DIR_CHECK(upload_ordered(hd, st, &u, 1));
      }
      hipLaunchKernelGGL(k_dir_index, dim3(nl), dim3(kThreads), 0, st, P.mask, len, sl, sj, cnt_d,
                         uidx);
      DIR_CHECK(hipGetLastError());
      int* w_d = cnt_d + nl + 1;
      DIR_CHECK(hipMemsetAsync(w_d, 0, sizeof(int), st));
      hipLaunchKernelGGL(k_dir_width, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                         P.mask, uidx, nx, ny, S.bcx, S.bcy, w_d);
      DIR_CHECK(hipGetLastError());
      int w = 0;
      DIR_CHECK(hipMemcpyAsync(&w, w_d, sizeof(int), hipMemcpyDeviceToHost, st));
      DIR_CHECK(hipStreamSynchronize(st));
      B.n = nu;
      B.nblk = (nu + kNb - 1) / kNb;
      B.npad = B.nblk * kNb;
      B.Q = (w + kNb - 1) / kNb;
      B.H = kNb + B.Q * kNb;
      const size_t pbytes = (size_t)B.nblk * kNb * B.H * sizeof(double);
      const size_t dbytes = (size_t)B.nblk * 2 * kNb * kNb * sizeof(double);
      const size_t ybytes = (size_t)B.npad * sizeof(double);
      const size_t bytes = pbytes + dbytes + 2 * ybytes;
      if (pbytes > ((size_t)200 << 30)) return BHX_ERR_NOMEM;
      if (bytes > hd->band_cap) {
        if (hd->band) DIR_CHECK(hipFree(hd->band));
        hd->band = nullptr;
        hd->band_cap = 0;
        DIR_CHECK(hipMalloc(&hd->band, bytes));
        hd->band_cap = bytes;
      }
      B.p = (double*)hd->band;
      B.d = (double*)((char*)hd->band + pbytes);
      y = (double*)((char*)hd->band + pbytes + dbytes);
      z = y + B.npad;
      // assemble and factor
      DIR_CHECK(hipMemsetAsync(B.p, 0, pbytes, st));
      hipLaunchKernelGGL(k_dir_assemble, dim3((N + kThreads - 1) / kThreads), dim3(kThreads), 0,
                         st, P.mask, uidx, nx, ny, S.bcx, S.bcy, B);
      DIR_CHECK(hipGetLastError());
      if (B.npad > B.n) {
        hipLaunchKernelGGL(k_dir_pad, dim3(1), dim3(kNb), 0, st, B);
        DIR_CHECK(hipGetLastError());
      }
      for (int k = 0; k < B.nblk; ++k) {
        const int below = std::min(B.Q, B.nblk - 1 - k);
        hipLaunchKernelGGL(k_dir_potrf_trsm, dim3(1 + below), dim3(kThreads), 0, st, B,
                           k, 1 + below);
        if (below > 0)
          hipLaunchKernelGGL(k_dir_update, dim3(below * (B.Q + 1)), dim3(kUpdThreads), 0, st, B,
                             k);
      }
      DIR_CHECK(hipGetLastError());
      factored = true;
    }
    if (!preset) {
      const int grid = (std::max(N, B.npad) + 255) / 256;
      for (int it = 0; it < 5; ++it) {
        // y = residual at U (the right-hand side on the first pass)
        hipLaunchKernelGGL(k_dir_gather, dim3(grid), dim3(256), 0, st, P.mask, uidx, P.r, N, B.n,
                           B.npad, y);
        // two panels per launch, one for an odd last panel
        for (int k = 0; k < B.nblk; k += 2) {
          if (k + 1 < B.nblk)
            hipLaunchKernelGGL(k_dir_fwd2, dim3(1 + std::min(B.Q, B.nblk - 2 - k)),
                               dim3(kThreads), 0, st, B, k, y, z);
          else
            hipLaunchKernelGGL(k_dir_fwd, dim3(1 + std::min(B.Q, B.nblk - 1 - k)),
                               dim3(kThreads), 0, st, B, k, y, z);
        }
        for (int k = B.nblk - 1; k >= 0; k -= 2) {
          if (k >= 1)
            hipLaunchKernelGGL(k_dir_bwd2, dim3(1 + std::min(B.Q, k - 1)), dim3(kThreads), 0,
                               st, B, k, z, y);
          else
            hipLaunchKernelGGL(k_dir_bwd, dim3(1 + std::min(B.Q, k)), dim3(kThreads), 0, st, B,
                               k, z, y);
        }
        hipLaunchKernelGGL(k_dir_scatter, dim3((N + 255) / 256), dim3(256), 0, st, P.mask, uidx,
                           y, N, it > 0 ? 1 : 0, S.F);
        DIR_CHECK(hipGetLastError());
        refines = it + 1;
        // compensated true residual of F (k_resid runs on converged instances)
        ch->done = kConverged;
        DIR_CHECK(hipMemcpyAsync(P.ctl, ch, sizeof(Ctl), hipMemcpyHostToDevice, st));
        DIR_CHECK(launch_resid(hd->batch_d, 2, g.s, st));
        DIR_CHECK(launch_finalize(hd->batch_d, 1, kFinResidH, st));
        DIR_CHECK(hipMemcpyAsync(ch, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        DIR_CHECK(hipStreamSynchronize(st));
        if (!std::isfinite(ch->true_rr)) {
          s = BHX_ERR_BREAKDOWN;
          break;
        }
        if (ch->true_rr <= ch->accept) break;
      }
      if (s == BHX_OK && !(ch->true_rr <= ch->accept)) s = BHX_NOT_CONVERGED;
    }
    if (s < 0 && ret >= 0) ret = s;
    else if (s > 0 && ret == BHX_OK) ret = s;
    if (stats) {
      bhx_stats& o = stats[f];
      std::memset(&o, 0, sizeof(o));
      o.status = s;
      o.iterations = refines;
      o.n_unknown = (int)ch->n_unknown;
      const double bb0 = ch->bb0;
      o.rel_residual = (!preset && bb0 > 0) ? std::sqrt(ch->true_rr / bb0) : 0.0;
      o.true_rel_residual = o.rel_residual;
      o.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  }
  return ret;
}

}  // namespace bhx
