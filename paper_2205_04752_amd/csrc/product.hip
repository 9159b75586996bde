// K3, the H-matrix-vector product y = sum_far U_b (V_b^T x_s) + sum_near D_b x_s
// (Sec. 2): gather into cluster order, phase A (V^T x items and dense-block
// chunks, k_mv1), phase B (U z chunks, k_mv2), the tile reduction (k_reduce);
// vector-ALU kernels for one right-hand side, matrix-core kernels for 2..16.
// Stored entries are FP64 or their FP32 copies; arithmetic is FP64. Also the
// layout kernels of the product-order stream and the FP32 conversion.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "hmat_internal.hpp"

namespace hm {

// ---------------------------------------------------------------------------
// K3: H-matrix-vector product.

// xp[r*ldxp + 3p+a] = x[r*ldx + 3 order[p] + a]
__global__ void k_gather(int nr, const double* __restrict__ x, int64_t ldx,
                         const int32_t* __restrict__ order, int64_t N, double* __restrict__ xp,
                         int64_t ldxp) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= N * nr) return;
  const int64_t r = e / N, d = e - r * N;
  xp[r * ldxp + d] = x[r * ldx + 3 * (int64_t)order[d / 3] + d % 3];
}

// Several vectors: xi[d * nr + r] = x[r][3 order[d/3] + d%3] for rows d < N,
// zero for the pad rows [N, ldxp), so that the nr vectors' entries of a row
// share cache lines and pages.
__global__ void k_gather_il(int nr, const double* __restrict__ x, int64_t ldx,
                            const int32_t* __restrict__ order, int64_t N, int64_t ldxp,
                            double* __restrict__ xi) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ldxp * nr) return;
  const int64_t d = e / nr;
  const int r = (int)(e - d * nr);
  xi[e] = d < N ? x[r * ldx + 3 * (int64_t)order[d / 3] + d % 3] : 0.0;
}

constexpr int TILE = 2 * WAVE;  // rows per product tile: two rows per lane

// Stored matrix entries are FP64 or FP32 (T); the product computes in FP64.
// Pair<T> is the two-entry vector a lane loads (16 or 8 bytes); ld2 widens it.
template <typename T>
struct Pair;
template <>
struct Pair<double> {
  using type = double2;
};
template <>
struct Pair<float> {
  using type = float2;
};
template <typename T>
__device__ __forceinline__ typename Pair<T>::type ldp(const T* p) {
  return *reinterpret_cast<const typename Pair<T>::type*>(p);
}
template <typename T>
__device__ __forceinline__ double2 ld2(const T* p) {
  const typename Pair<T>::type v = ldp(p);
  return make_double2((double)v.x, (double)v.y);
}
// The single-vector kernels read each matrix entry once per product:
// non-temporal loads keep the entries from displacing the vectors and partial
// sums, which are reused, in the caches (0.667 -> 0.637 ms at icosphere L5).
// The matrix-core kernels keep plain loads: their lanes share cache lines of
// the panels, and non-temporal loads made them fetch 28% more.
template <typename T>
__device__ __forceinline__ typename Pair<T>::type ldp_nt(const T* p) {
  typedef T nv2 __attribute__((ext_vector_type(2)));
  const nv2 v = __builtin_nontemporal_load(reinterpret_cast<const nv2*>(p));
  typename Pair<T>::type r;
  r.x = v.x;
  r.y = v.y;
  return r;
}
template <typename T>
__device__ __forceinline__ double2 ld2_nt(const T* p) {
  const typename Pair<T>::type v = ldp_nt(p);
  return make_double2((double)v.x, (double)v.y);
}

// Phase A item: z = V_b^T x_s for a group of <= 8 columns; one wave. Lanes
// cover the aligned row window of V two rows at a time (16-byte loads of V and
// of the gathered x; pad rows of V are zero); NR right-hand sides at once,
// columns in sub-batches of CB. mv_a_cols does NC columns [l0, l0 + NC), NC
// known at compile time, so an item's last, partial sub-batch loads only its
// own columns (0.637 -> 0.631 ms per product at icosphere L5).
template <int NR, int NC, typename T>
__device__ __forceinline__ void mv_a_cols(const MvA& I, int l0, const T* __restrict__ V,
                                          const double* __restrict__ X, int64_t ldxp, int nr,
                                          double* __restrict__ z, int64_t ldz, int lane) {
  double acc[NC][NR];
#pragma unroll
  for (int c = 0; c < NC; c++)
#pragma unroll
    for (int r = 0; r < NR; r++) acc[c][r] = 0.0;
  for (int i = 2 * lane; i < I.ld; i += TILE) {
    double2 xv[NR], v[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) v[c] = ld2_nt(V + (size_t)(l0 + c) * I.ld + i);
#pragma unroll
    for (int r = 0; r < NR; r++)
      xv[r] = (r < nr) ? *reinterpret_cast<const double2*>(X + r * ldxp + i) : make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < NC; c++)
#pragma unroll
      for (int r = 0; r < NR; r++) acc[c][r] += v[c].x * xv[r].x + v[c].y * xv[r].y;
  }
#pragma unroll
  for (int c = 0; c < NC; c++)
#pragma unroll
    for (int r = 0; r < NR; r++) {
      const double sum = wave_sum(acc[c][r]);
      if (lane == 0 && r < nr) z[r * ldz + I.zoff + (l0 - I.l0) + c] = sum;
    }
}

template <int NR, typename T>
__device__ __forceinline__ void mv_a_item(const MvA& I, const T* __restrict__ far,
                                          const double* __restrict__ xp, int64_t ldxp, int nr,
                                          double* __restrict__ z, int64_t ldz) {
  constexpr int CB = (NR >= 16) ? 2 : ((NR >= 8) ? 4 : 8);
  const int lane = threadIdx.x & (WAVE - 1);
  const T* __restrict__ V = far + I.v_off;
  const double* __restrict__ X = xp + I.a0;
  for (int l0 = I.l0; l0 < I.l1; l0 += CB) {
    const int nc = min(CB, I.l1 - l0);
    switch (nc) {  // wave-uniform
      case 1: mv_a_cols<NR, 1, T>(I, l0, V, X, ldxp, nr, z, ldz, lane); break;
      case 2: mv_a_cols<NR, (CB >= 2 ? 2 : 1), T>(I, l0, V, X, ldxp, nr, z, ldz, lane); break;
      case 3: mv_a_cols<NR, (CB >= 3 ? 3 : 1), T>(I, l0, V, X, ldxp, nr, z, ldz, lane); break;
      case 4: mv_a_cols<NR, (CB >= 4 ? 4 : 1), T>(I, l0, V, X, ldxp, nr, z, ldz, lane); break;
      case 5: mv_a_cols<NR, (CB >= 5 ? 5 : 1), T>(I, l0, V, X, ldxp, nr, z, ldz, lane); break;
      case 6: mv_a_cols<NR, (CB >= 6 ? 6 : 1), T>(I, l0, V, X, ldxp, nr, z, ldz, lane); break;
      case 7: mv_a_cols<NR, (CB >= 7 ? 7 : 1), T>(I, l0, V, X, ldxp, nr, z, ldz, lane); break;
      default: mv_a_cols<NR, CB, T>(I, l0, V, X, ldxp, nr, z, ldz, lane); break;
    }
  }
}

// Phase B chunk: segments of one 128-row tile, each a column-major array of
// its rows [row_lo, row_hi) (even bounds) times its columns, stored back to
// back; lane L owns tile rows 2L and 2L+1 (acc0, acc1). A segment taller than
// half a wave is read with lane L on its own rows (16-byte loads; lanes
// outside the segment load a clamped in-segment address and discard it). A
// shorter one (single right-hand side) puts p = 64 / (len/2) columns side by
// side, so each load instruction covers p*len consecutive doubles; the p
// column groups are then summed with a lane tree and moved to the owning
// lanes. A tall segment's last partial batch issues its loads back to back
// too, rounded up to 4, 8 or 12 columns (the extra loads re-read the last
// column and are not added; a batch size fixed at compile time for each case
// cut 0.6% in FP64 and 1% in FP32 against re-reading up to 15 columns, and
// skipping the loads at run time cost 70% in FP32).
// Writes part[chunk][r][128].
// One short segment (len <= 64 rows, single right-hand side) of a phase-B
// chunk: g = len/2 lanes per column, p = 64/g >= 2 columns per load. Lane l
// reads column c0 + t p + l/g, rows 2(l mod g) and +1, at stream offset
// so + t p len + 2l -- consecutive lanes, consecutive addresses. Adds the
// segment's row sums to the owning lanes' acc0/acc1 (fixed summation order).
template <int UNR, typename T>
__device__ __forceinline__ void mv_b_grouped(const MvSeg& S, const T* __restrict__ stream,
                                             const double* __restrict__ src, double& acc0,
                                             double& acc1) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int len = S.row_hi - S.row_lo, g = len >> 1, p = WAVE / g;
  const int q = lane / g;
  const bool lact = q < p;
  const int ncol = S.c1 - S.c0;
  const int nsteps = (ncol + p - 1) / p;
  const int64_t step = (int64_t)p * len;
  const T* __restrict__ A = stream + S.so;
  const double* __restrict__ xs = src + S.soff + S.c0;
  double s0 = 0.0, s1 = 0.0;
  for (int t = 0; t < nsteps; t += UNR) {
    typename Pair<T>::type a[UNR];
    double xv[UNR];
#pragma unroll
    for (int u = 0; u < UNR; u++) {
      const int col = (t + u) * p + q;
      const bool ok = lact && col < ncol;
      a[u] = ldp_nt(A + (ok ? (int64_t)(t + u) * step + 2 * lane : 0));
      xv[u] = xs[ok ? col : 0];
      xv[u] = ok ? xv[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; u++) {
      s0 += (double)a[u].x * xv[u];
      s1 += (double)a[u].y * xv[u];
    }
  }
  // sum the p column groups: group q takes group q + off at level off
  for (int off = 1; off < p; off <<= 1) {
    const double o0 = __shfl(s0, (lane + off * g) & (WAVE - 1), WAVE);
    const double o1 = __shfl(s1, (lane + off * g) & (WAVE - 1), WAVE);
    if (q % (2 * off) == 0 && q + off < p) {
      s0 += o0;
      s1 += o1;
    }
  }
  // lanes [0, g) hold rows row_lo + 2l, +1: move them to lanes row_lo/2 + l
  const int from = lane - (S.row_lo >> 1);
  const double m0 = __shfl(s0, from & (WAVE - 1), WAVE);
  const double m1 = __shfl(s1, from & (WAVE - 1), WAVE);
  if (from >= 0 && from < g) {
    acc0 += m0;
    acc1 += m1;
  }
}

// One batch of B columns c .. c + B - 1 of a tall segment (B known at compile
// time); columns at or past c + nc re-read column c1 - 1 and are not added.
template <int NR, int B, typename T>
__device__ __forceinline__ void mv_b_batch(const T* __restrict__ A, int len, int c, int nc, int c1,
                                           const double* __restrict__ src, int64_t ld, int nr, bool act,
                                           double (&acc0)[NR], double (&acc1)[NR]) {
  typename Pair<T>::type a[B];
#pragma unroll
  for (int u = 0; u < B; u++) {
    const int cu = (u < nc) ? c + u : c1 - 1;
    a[u] = ldp_nt(A + (int64_t)cu * len);
  }
#pragma unroll
  for (int u = 0; u < B; u++) {
    a[u].x = act ? a[u].x : (T)0;
    a[u].y = act ? a[u].y : (T)0;
  }
#pragma unroll
  for (int r = 0; r < NR; r++) {
    if (r < nr) {
      const double* sr = src + r * ld + c;
#pragma unroll
      for (int u = 0; u < B; u++) {
        if (u < nc) {
          acc0[r] += (double)a[u].x * sr[u];
          acc1[r] += (double)a[u].y * sr[u];
        }
      }
    }
  }
}

template <int NR, int UNR, typename T>
__device__ __forceinline__ void mv_b_chunk(const MvChunk& C, int chunk,
                                           const MvSeg* __restrict__ segs,
                                           const T* __restrict__ stream,
                                           const double* __restrict__ z, int64_t ldz,
                                           const double* __restrict__ xp, int64_t ldxp, int nr,
                                           double* __restrict__ part) {
  const int L2 = 2 * (threadIdx.x & (WAVE - 1));
  double acc0[NR], acc1[NR];
#pragma unroll
  for (int r = 0; r < NR; r++) acc0[r] = acc1[r] = 0.0;
  for (int s = C.seg_lo; s < C.seg_hi; s++) {
    const MvSeg S = segs[s];
    const int len = S.row_hi - S.row_lo;
    if (NR == 1 && len <= WAVE) {
      // at most 8 loads per batch here: the x values are per lane too, and a
      // deeper batch raises the kernel's register count past 4 waves per SIMD
      mv_b_grouped<(UNR > 8 ? 8 : UNR), T>(S, stream, S.far ? z : xp, acc0[0], acc1[0]);
      continue;
    }
    const bool act = L2 >= S.row_lo && L2 < S.row_hi;
    const int Lc = min(max(L2, (int)S.row_lo), (int)S.row_hi - 2);
    const T* __restrict__ A = stream + S.so + (Lc - S.row_lo) - (int64_t)S.c0 * len;
    const double* __restrict__ src = (S.far ? z : xp) + S.soff;
    const int64_t ld = S.far ? ldz : ldxp;
    int c = S.c0;
    for (; c + UNR <= S.c1; c += UNR) mv_b_batch<NR, UNR, T>(A, len, c, UNR, S.c1, src, ld, nr, act, acc0, acc1);
    const int nc = S.c1 - c;  // last, partial batch (nc < UNR): loads rounded up to four columns
    if (nc > 0) {
      static_assert(UNR == 8 || UNR == 16, "partial batches assume 8 or 16 columns per batch");
      if (nc <= 4) mv_b_batch<NR, 4, T>(A, len, c, nc, S.c1, src, ld, nr, act, acc0, acc1);
      else if (nc <= 8) mv_b_batch<NR, 8, T>(A, len, c, nc, S.c1, src, ld, nr, act, acc0, acc1);
      else if (nc <= 12) mv_b_batch<NR, 12, T>(A, len, c, nc, S.c1, src, ld, nr, act, acc0, acc1);
      else mv_b_batch<NR, 16, T>(A, len, c, nc, S.c1, src, ld, nr, act, acc0, acc1);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; r++)
    if (r < nr)
      *reinterpret_cast<double2*>(part + ((size_t)chunk * NR + r) * TILE + L2) = make_double2(acc0[r], acc1[r]);
}

// Work units (phase-A items, chunks) go one per wave; MV_WPB independent waves
// share a workgroup (no LDS, no barriers) so more waves fit on a CU.
constexpr int MV_WPB = 1;

// Product launch 1: the phase-A items (largest first) and the dense-block
// chunks, which do not depend on z, in one grid so that neither leaves the
// other's tail idle.
template <int NR, int UNR, typename T>
__global__ __launch_bounds__(WAVE* MV_WPB) void k_mv1(const MvA* __restrict__ items, int nA,
                                                      int n_near_chunks,
                                                      const MvChunk* __restrict__ chunks,
                                                      const MvSeg* __restrict__ segs,
                                                      const T* __restrict__ far,
                                                      const T* __restrict__ stream,
                                                      const double* __restrict__ xp, int64_t ldxp,
                                                      int nr, double* __restrict__ z, int64_t ldz,
                                                      double* __restrict__ part) {
  // wave-uniform unit index: keeps descriptors and vector entries in scalar loads
  const int u = __builtin_amdgcn_readfirstlane(blockIdx.x * MV_WPB + threadIdx.x / WAVE);
  if (u < nA) {
    mv_a_item<NR, T>(items[u], far, xp, ldxp, nr, z, ldz);
  } else if (u < nA + n_near_chunks) {
    const int c = u - nA;
    mv_b_chunk<NR, UNR, T>(chunks[c], c, segs, stream, z, ldz, xp, ldxp, nr, part);
  }
}

// Product launch 2: the low-rank chunks (U z), chunk ids c_first + unit.
template <int NR, int UNR, typename T>
__global__ __launch_bounds__(WAVE* MV_WPB) void k_mv2(int c_first, int n,
                                                      const MvChunk* __restrict__ chunks,
                                                      const MvSeg* __restrict__ segs,
                                                      const T* __restrict__ stream,
                                                      const double* __restrict__ z, int64_t ldz,
                                                      const double* __restrict__ xp, int64_t ldxp,
                                                      int nr, double* __restrict__ part) {
  const int u = __builtin_amdgcn_readfirstlane(blockIdx.x * MV_WPB + threadIdx.x / WAVE);
  if (u >= n) return;
  const int c = c_first + u;
  mv_b_chunk<NR, UNR, T>(chunks[c], c, segs, stream, z, ldz, xp, ldxp, nr, part);
}

// ---------------------------------------------------------------------------
// Several right-hand sides (2..16): the two contractions V^T X and U Z (and
// D X) on the FP64 matrix cores. v_mfma_f64_16x16x4f64 computes
// D += A B with A 16x4, B 4x16; lane l holds A[l%16][l/16], B[l/16][l%16]
// and D[4v + l/16][l%16] in item v (v = 0..3). The right-hand sides are the
// 16 columns of B (lanes with l%16 >= nr carry zeros). To let every lane load
// four consecutive matrix rows with two 16-byte loads, the four products of a
// group take rows 4m + t (t = 0..3) in place of row m: a permutation of the
// summation (phase A) or of the output rows (phase B), undone when storing.

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Phase A, several vectors: z[zoff + c][:] = V[:, l0 + c]^T X for c < l1 - l0
// (<= 64 columns: four 16-column tiles). Per 16-row step lane l reads rows
// 4(l/16) .. +3 of column l%16 of each tile and the same rows of vector l%16.
// X and z hold a row's nr vector entries side by side; lanes of vectors past
// nr read the next row's (unused).
template <typename T>
__device__ __forceinline__ void mv_a_mfma(const MvA& I, const T* __restrict__ far,
                                          const double* __restrict__ xp, int64_t ldxp, int nr,
                                          double* __restrict__ z, int64_t ldz) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int kq = lane >> 4, cl = lane & 15;
  const int ncols = I.l1 - I.l0;
  const int ntile = (ncols + 15) >> 4;
  const bool rv = cl < nr;
  const double* __restrict__ X = xp + (int64_t)I.a0 * nr + cl;
  const T* Vc[4];
  bool cv[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int col = q * 16 + cl;
    cv[q] = col < ncols;
    Vc[q] = far + I.v_off + (int64_t)(I.l0 + min(col, ncols - 1)) * I.ld;
  }
  v4d acc[4];
#pragma unroll
  for (int q = 0; q < 4; q++) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < I.ld; i0 += 16) {
    const int r0 = i0 + 4 * kq;
    const bool p0 = r0 < I.ld, p1 = r0 + 2 < I.ld;  // ld and r0 even: pairs are whole
    const double* X0 = X + (int64_t)(p0 ? r0 : 0) * nr;
    const double* X1 = X + (int64_t)(p1 ? r0 + 2 : 0) * nr;
    double2 x0 = make_double2(X0[0], X0[nr]);
    double2 x1 = make_double2(X1[0], X1[nr]);
    const bool b0 = rv && p0, b1 = rv && p1;
    x0.x = b0 ? x0.x : 0.0;
    x0.y = b0 ? x0.y : 0.0;
    x1.x = b1 ? x1.x : 0.0;
    x1.y = b1 ? x1.y : 0.0;
    double2 a0[4], a1[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      if (q < ntile) {
        a0[q] = ld2(Vc[q] + (p0 ? r0 : 0));
        a1[q] = ld2(Vc[q] + (p1 ? r0 + 2 : 0));
      }
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      if (q < ntile) {
        const bool ok = cv[q];
        acc[q] = mfma4(ok ? a0[q].x : 0.0, x0.x, acc[q]);
        acc[q] = mfma4(ok ? a0[q].y : 0.0, x0.y, acc[q]);
        acc[q] = mfma4(ok ? a1[q].x : 0.0, x1.x, acc[q]);
        acc[q] = mfma4(ok ? a1[q].y : 0.0, x1.y, acc[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    if (q < ntile) {
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int col = q * 16 + 4 * v + kq;
        if (col < ncols && rv) z[(int64_t)(I.zoff + col) * nr + cl] = acc[q][v];
      }
    }
  }
}

// Phase B, several vectors: one chunk (segments of one 128-row tile). Per
// group of four columns c..c+3, lane l reads, of column c + l/16, the row
// pairs 64h + 2(l%16) and 64h + 32 + 2(l%16) in each 64-row half h the
// segment touches (so the 16 lanes of a column read 256 contiguous bytes per
// load), and entry c + l/16 of vector l%16. The four products of a half take
// the rows 64h + 2m, 64h + 2m + 1, 64h + 32 + 2m, 64h + 32 + 2m + 1 in place
// of row m of the 16-row operand; the stores undo it. Writes
// part[chunk][16][128].
//
// The work is a sequence of steps (segment, batch of 16 columns). The loads
// of step i+1 are issued before the products of step i, so a wave keeps a
// batch of loads in flight while its products run (software pipelining; two
// register sets in turn). Every step issues the same loads, also for a half
// the segment does not touch (clamped to the column's first row, a cache
// hit), so the compiler can wait for exactly one step's loads; after the last
// step one more, unused, batch is issued. The products and their order are
// those of the plain loop over segments and batches.
template <typename T>
struct MfmaSeg {  // one segment as this lane sees it (no flags: derived where used)
  const T* __restrict__ base;     // the segment's column block in the stream
  const double* __restrict__ Bp;  // its vectors (z or xp): column c's entry of this lane's at Bp[c * vs]
  int c0, c1, lo, hi;             // columns, tile rows [lo, hi)
  int vs;                         // entries per column in Bp (the number of vectors)
};

template <typename T>
__device__ __forceinline__ MfmaSeg<T> mfma_seg(const MvSeg& S, const T* __restrict__ stream,
                                               const double* __restrict__ z,
                                               const double* __restrict__ xp, int nr, int m16) {
  MfmaSeg<T> G;
  G.base = stream + S.so;
  G.Bp = (S.far ? z : xp) + (int64_t)S.soff * nr + m16;
  G.vs = nr;
  G.c0 = S.c0;
  G.c1 = S.c1;
  G.lo = S.row_lo;
  G.hi = S.row_hi;
  return G;
}

template <typename T>
struct MfmaStep {  // one step's loads, as loaded (FP32 entries widen at use)
  double bv[4];
  typename Pair<T>::type av[4][2][2];
};

// Row offset in the segment of this lane's k-th row pair (k = 0..3: half
// k/2, upper 32 rows of the half if k is odd); inside the segment iff in
// [0, len) (pairs are whole: segment bounds are even).
__device__ __forceinline__ int mfma_row(int lo, int m16, int k) {
  return 64 * (k >> 1) + 32 * (k & 1) + 2 * m16 - lo;
}

template <typename T>
__device__ __forceinline__ void mfma_load(MfmaStep<T>& B, const MfmaSeg<T>& G, int c, int kq,
                                          int m16) {
  const int len = G.hi - G.lo;
  int off[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int r = mfma_row(G.lo, m16, k);
    off[k] = (r >= 0 && r < len) ? r : 0;
  }
#pragma unroll
  for (int g = 0; g < 4; g++) {
    const int cc = min(c + 4 * g + kq, G.c1 - 1);
    const T* __restrict__ col = G.base + (int64_t)(cc - G.c0) * len;
    B.bv[g] = G.Bp[(int64_t)cc * G.vs];
    B.av[g][0][0] = ldp(col + off[0]);
    B.av[g][0][1] = ldp(col + off[1]);
    B.av[g][1][0] = ldp(col + off[2]);
    B.av[g][1][1] = ldp(col + off[3]);
  }
}

// s_waitcnt immediate (gfx9 encoding) that waits until at most n vector-memory
// loads are outstanding (expcnt and lgkmcnt left at their maxima).
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
constexpr int MFMA_STEP_LOADS = 20;  // per step: 4 vector entries + 16 matrix pairs

template <typename T>
__device__ __forceinline__ void mfma_step(v4d (&acc)[2][4], const MfmaStep<T>& B,
                                          const MfmaSeg<T>& G, int c, int kq, int m16, bool rv) {
  // This step's loads are done once at most the next step's are in flight.
  // Waiting here, before the branches over the halves, tells the compiler so
  // on every path (else it waits for all loads before reusing registers).
  __builtin_amdgcn_s_waitcnt(vmcnt_imm(MFMA_STEP_LOADS));
  const int len = G.hi - G.lo;
  bool q[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int r = mfma_row(G.lo, m16, k);
    q[k] = r >= 0 && r < len;
  }
  const bool h0 = G.lo < 64, h1 = G.hi > 64;  // halves the segment touches
#pragma unroll
  for (int g = 0; g < 4; g++) {
    const double b = (rv && c + 4 * g + kq < G.c1) ? B.bv[g] : 0.0;
    if (h0) {
      acc[0][0] = mfma4(q[0] ? (double)B.av[g][0][0].x : 0.0, b, acc[0][0]);
      acc[0][1] = mfma4(q[0] ? (double)B.av[g][0][0].y : 0.0, b, acc[0][1]);
      acc[0][2] = mfma4(q[1] ? (double)B.av[g][0][1].x : 0.0, b, acc[0][2]);
      acc[0][3] = mfma4(q[1] ? (double)B.av[g][0][1].y : 0.0, b, acc[0][3]);
    }
    if (h1) {
      acc[1][0] = mfma4(q[2] ? (double)B.av[g][1][0].x : 0.0, b, acc[1][0]);
      acc[1][1] = mfma4(q[2] ? (double)B.av[g][1][0].y : 0.0, b, acc[1][1]);
      acc[1][2] = mfma4(q[3] ? (double)B.av[g][1][1].x : 0.0, b, acc[1][2]);
      acc[1][3] = mfma4(q[3] ? (double)B.av[g][1][1].y : 0.0, b, acc[1][3]);
    }
  }
}

// First segment at or after t (< seg_hi) with columns, or seg_hi.
__device__ __forceinline__ int mfma_seg_from(int t, int seg_hi, const MvSeg* __restrict__ segs) {
  for (; t < seg_hi; t++)
    if (segs[t].c1 > segs[t].c0) break;
  return t;
}

template <typename T>
__device__ __forceinline__ void mv_b_mfma(const MvChunk& C, int chunk,
                                          const MvSeg* __restrict__ segs,
                                          const T* __restrict__ stream,
                                          const double* __restrict__ z, int64_t ldz,
                                          const double* __restrict__ xp, int64_t ldxp, int nr,
                                          double* __restrict__ part) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int kq = lane >> 4, m16 = lane & 15;
  const bool rv = m16 < nr;
  v4d acc[2][4];
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int t = 0; t < 4; t++) acc[h][t] = v4d{0.0, 0.0, 0.0, 0.0};
  int s = mfma_seg_from(C.seg_lo, C.seg_hi, segs);
  if (s < C.seg_hi) {
    // (Ga, ca) and (Gb, cb): the steps whose loads are in A and B
    MfmaSeg<T> Ga = mfma_seg<T>(segs[s], stream, z, xp, nr, m16), Gb;
    int ca = Ga.c0, cb;
    MfmaStep<T> A, B;
    mfma_load(A, Ga, ca, kq, m16);
    // advance (G, c) from segment s to the next step; false at the chunk's
    // end, where (Gn, cn) = (G, c + 16): a batch past the segment's columns,
    // whose loads (all clamped to its last column) are issued and unused, so
    // that every step waits for exactly one step's loads
    auto next = [&](const MfmaSeg<T>& G, int c, MfmaSeg<T>& Gn, int& cn) -> bool {
      if (c + 16 < G.c1 || (s = mfma_seg_from(s + 1, C.seg_hi, segs)) >= C.seg_hi) {
        Gn = G;
        cn = c + 16;
        return cn < G.c1;
      }
      Gn = mfma_seg<T>(segs[s], stream, z, xp, nr, m16);
      cn = Gn.c0;
      return true;
    };
    // (the exits wait for the unused loads, so that no path into the loop's
    // latch leaves loads in flight into registers the next step reuses)
    for (;;) {
      bool more = next(Ga, ca, Gb, cb);
      mfma_load(B, Gb, cb, kq, m16);
      mfma_step(acc, A, Ga, ca, kq, m16, rv);
      if (!more) {
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        break;
      }
      more = next(Gb, cb, Ga, ca);
      mfma_load(A, Ga, ca, kq, m16);
      mfma_step(acc, B, Gb, cb, kq, m16, rv);
      if (!more) {
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        break;
      }
    }
  }
  // lane holds vector m16 and, for operand row i = 4v + kq, tile rows
  // 64h + 2i + t (t = 0, 1) in acc[h][t][v] and 64h + 32 + 2i + t - 2 (t = 2, 3)
  if (rv) {
    double* __restrict__ out = part + ((size_t)chunk * 16 + m16) * TILE;
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int row = 64 * h + 8 * v + 2 * kq;
        *reinterpret_cast<double2*>(out + row) = make_double2(acc[h][0][v], acc[h][1][v]);
        *reinterpret_cast<double2*>(out + row + 32) = make_double2(acc[h][2][v], acc[h][3][v]);
      }
  }
}

template <typename T>
__global__ __launch_bounds__(WAVE) void k_mv1_mfma(const MvA* __restrict__ items, int nA,
                                                   int n_near_chunks,
                                                   const MvChunk* __restrict__ chunks,
                                                   const MvSeg* __restrict__ segs,
                                                   const T* __restrict__ far,
                                                   const T* __restrict__ stream,
                                                   const double* __restrict__ xp, int64_t ldxp,
                                                   int nr, double* __restrict__ z, int64_t ldz,
                                                   double* __restrict__ part) {
  const int u = __builtin_amdgcn_readfirstlane(blockIdx.x);
  if (u < nA) {
    mv_a_mfma(items[u], far, xp, ldxp, nr, z, ldz);
  } else if (u < nA + n_near_chunks) {
    const int c = u - nA;
    mv_b_mfma(chunks[c], c, segs, stream, z, ldz, xp, ldxp, nr, part);
  }
}

template <typename T>
__global__ __launch_bounds__(WAVE) void k_mv2_mfma(int c_first, int n,
                                                   const MvChunk* __restrict__ chunks,
                                                   const MvSeg* __restrict__ segs,
                                                   const T* __restrict__ stream,
                                                   const double* __restrict__ z, int64_t ldz,
                                                   const double* __restrict__ xp, int64_t ldxp,
                                                   int nr, double* __restrict__ part) {
  const int u = __builtin_amdgcn_readfirstlane(blockIdx.x);
  if (u >= n) return;
  const int c = c_first + u;
  mv_b_mfma(chunks[c], c, segs, stream, z, ldz, xp, ldxp, nr, part);
}

// FP32 copy of an FP64 array (reduced-precision storage of the arenas).
__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// Plain column-major block matrix -> stream segment (one workgroup per segment).
__global__ __launch_bounds__(256) void k_to_stream(const StreamTask* __restrict__ tasks,
                                                   double* __restrict__ stream) {
  const StreamTask T = tasks[blockIdx.x];
  const int len = T.row_hi - T.row_lo;
  const int64_t total = (int64_t)len * (T.c1 - T.c0);
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int64_t c = T.c0 + e / len;
    const int i = T.r0 + T.row_lo + (int)(e % len);
    stream[T.so + e] = (i >= 0 && i < T.ld) ? T.src[c * T.ld + i] : 0.0;
  }
}

// Stream segment -> plain column-major block matrix (rows outside [0, m) skipped).
template <typename E>
__global__ __launch_bounds__(256) void k_from_stream(const StreamTask* __restrict__ tasks,
                                                     const E* __restrict__ stream) {
  const StreamTask T = tasks[blockIdx.x];
  const int len = T.row_hi - T.row_lo;
  const int64_t total = (int64_t)len * (T.c1 - T.c0);
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int64_t c = T.c0 + e / len;
    const int i = T.r0 + T.row_lo + (int)(e % len);
    if (i >= 0 && i < T.ld) T.dst[c * T.ld + i] = (double)stream[T.so + e];
  }
}

// Sum the partials of each tile and scatter to the caller's order. The tile's
// chunks (dense-block chunks, then low-rank chunks) are dealt round-robin to
// RED_WAVES waves, which sum theirs in chunk order; wave 0 adds the waves'
// sums in wave order (a fixed order: results do not vary between calls).
constexpr int RED_WAVES = 4;
template <int NR>
__global__ __launch_bounds__(WAVE* RED_WAVES) void k_reduce(const int32_t* __restrict__ tile_near,
                                                            const int32_t* __restrict__ tile_far,
                                                            const double* __restrict__ part, int nr,
                                                            const int32_t* __restrict__ order,
                                                            int64_t N, double* __restrict__ y,
                                                            int64_t ldy) {
  __shared__ double2 red[RED_WAVES][WAVE];
  const int tile = blockIdx.x, w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
  const int L2 = 2 * lane;
  const int64_t row = (int64_t)tile * TILE + L2;
  const int n0 = tile_near[tile], nn = tile_near[tile + 1] - n0;
  const int f0 = tile_far[tile], n = nn + tile_far[tile + 1] - f0;
  constexpr int DEPTH = 4;  // loads in flight per lane
  for (int r = 0; r < nr; r++) {
    double s0 = 0.0, s1 = 0.0;
    for (int k = w; k < n; k += RED_WAVES * DEPTH) {
      double2 p[DEPTH];
#pragma unroll
      for (int j = 0; j < DEPTH; j++) {
        const int kk = k + j * RED_WAVES;
        const int c = kk < nn ? n0 + kk : f0 + (kk - nn);
        p[j] = kk < n ? *reinterpret_cast<const double2*>(part + ((size_t)c * NR + r) * TILE + L2)
                      : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int j = 0; j < DEPTH; j++) {
        s0 += p[j].x;
        s1 += p[j].y;
      }
    }
    red[w][lane] = make_double2(s0, s1);
    __syncthreads();
    if (w == 0 && row < N) {
      double t0 = 0.0, t1 = 0.0;
#pragma unroll
      for (int v = 0; v < RED_WAVES; v++) {
        t0 += red[v][lane].x;
        t1 += red[v][lane].y;
      }
      y[r * ldy + 3 * (int64_t)order[row / 3] + row % 3] = t0;
      if (row + 1 < N) y[r * ldy + 3 * (int64_t)order[(row + 1) / 3] + (row + 1) % 3] = t1;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Launchers.

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_gather(int nr, const double* x, int64_t ldx, const int32_t* order, int64_t N,
                         double* xp, int64_t ldxp, hipStream_t s) {
  if (nr > 1)  // several vectors: side by side, after the single-vector area
    hipLaunchKernelGGL(k_gather_il, dim3(blocks_for(ldxp * nr, 256)), dim3(256), 0, s, nr, x,
                       ldx, order, N, ldxp, xp + ldxp);
  else
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(N * nr, 256)), dim3(256), 0, s, nr, x, ldx, order,
                       N, xp, ldxp);
  return hipGetLastError();
}

template <int NR, int UNR, typename T>
static void mv_group(const ProductPlanDev& P, const T* far, const T* stream, const double* xp,
                     int64_t ldxp, int nr, double* z, int64_t ldz, double* part, double* y,
                     int64_t ldy, hipStream_t s, hipEvent_t* ev) {
  const int n1 = P.nA + P.n_near_chunks;
  if (n1 > 0)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mv1<NR, UNR, T>), dim3((n1 + MV_WPB - 1) / MV_WPB),
                       dim3(WAVE * MV_WPB), 0, s, P.items, P.nA, P.n_near_chunks, P.chunks, P.segs,
                       far, stream, xp, ldxp, nr, z, ldz, part);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (P.n_far_chunks > 0)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mv2<NR, UNR, T>), dim3((P.n_far_chunks + MV_WPB - 1) / MV_WPB),
                       dim3(WAVE * MV_WPB), 0, s, P.n_near_chunks, P.n_far_chunks, P.chunks, P.segs,
                       stream, z, ldz, xp, ldxp, nr, part);
  if (ev) (void)hipEventRecord(ev[1], s);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reduce<NR>), dim3(P.ntiles), dim3(WAVE * RED_WAVES), 0, s, P.tile_near,
                     P.tile_far, part, nr, P.order, P.N, y, ldy);
  if (ev) (void)hipEventRecord(ev[2], s);
}

template <typename T>
static void mv_group_mfma(const ProductPlanDev& P, const T* far, const T* stream, const double* xp,
                          int64_t ldxp, int nr, double* z, int64_t ldz, double* part, double* y,
                          int64_t ldy, hipStream_t s, hipEvent_t* ev) {
  const int n1 = P.nA + P.n_near_chunks;
  if (n1 > 0)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mv1_mfma<T>), dim3(n1), dim3(WAVE), 0, s, P.items, P.nA,
                       P.n_near_chunks, P.chunks, P.segs, far, stream, xp, ldxp, nr, z, ldz, part);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (P.n_far_chunks > 0)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_mv2_mfma<T>), dim3(P.n_far_chunks), dim3(WAVE), 0, s,
                       P.n_near_chunks, P.n_far_chunks, P.chunks, P.segs, stream, z, ldz, xp, ldxp,
                       nr, part);
  if (ev) (void)hipEventRecord(ev[1], s);
  hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reduce<16>), dim3(P.ntiles), dim3(WAVE * RED_WAVES), 0, s,
                     P.tile_near, P.tile_far, part, nr, P.order, P.N, y, ldy);
  if (ev) (void)hipEventRecord(ev[2], s);
}

// One pass over the matrix for nr <= 16 right-hand sides (xp already gathered),
// reading the FP64 arenas (prec 0) or their FP32 copies (prec 1).
// One vector: the vector-ALU kernels; two to sixteen: matrix cores.
hipError_t launch_matvec_group(const ProductPlanDev& P, int prec, int nr, const double* xp,
                               int64_t ldxp, double* z, int64_t ldz, double* part, double* y,
                               int64_t ldy, hipStream_t s, hipEvent_t* ev, int unroll) {
  if (prec == 1) {
    if (nr <= 1) {
      if (unroll >= 16)
        mv_group<1, 16, float>(P, P.far32, P.stream32, xp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
      else
        mv_group<1, 8, float>(P, P.far32, P.stream32, xp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
    } else {
      mv_group_mfma<float>(P, P.far32, P.stream32, xp + ldxp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
    }
  } else {
    if (nr <= 1) {
      if (unroll >= 16)
        mv_group<1, 16, double>(P, P.far, P.stream, xp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
      else
        mv_group<1, 8, double>(P, P.far, P.stream, xp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
    } else {
      mv_group_mfma<double>(P, P.far, P.stream, xp + ldxp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
    }
  }
  return hipGetLastError();
}

hipError_t launch_to_stream(const StreamTask* tasks, int ntasks, double* stream, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_to_stream, dim3(ntasks), dim3(256), 0, s, tasks, stream);
  return hipGetLastError();
}

hipError_t launch_from_stream(const StreamTask* tasks, int ntasks, const double* stream, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_from_stream<double>), dim3(ntasks), dim3(256), 0, s, tasks, stream);
  return hipGetLastError();
}
hipError_t launch_from_stream32(const StreamTask* tasks, int ntasks, const float* stream, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_from_stream<float>), dim3(ntasks), dim3(256), 0, s, tasks, stream);
  return hipGetLastError();
}

}  // namespace hm
