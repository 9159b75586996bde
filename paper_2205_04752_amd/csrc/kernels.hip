// CDNA4 (gfx950) kernels of the H-matrix path.
//
//   K1  k_near / k_self   dense (non-admissible) blocks entry by entry (Sec. 2.2)
//   K2  k_aca             ACA with partial pivoting on every admissible block
//                         (Sec. 2.2, Algorithm 1), one workgroup per block
//   --  k_compact         final low-rank arena (first k columns of the panels)
//   --  GMRES helpers     dots, column updates, norms
// (K3, the product, is in product.hip; the adaptive multiplication's kernels
// are in amvm.hip.)
//
// Entries: A[3i+a, 3j+b] = int_{tau_j} S_ab(c_i - y) ds_y with Kelvin's tensor
// S = c1 delta/|r| + c2 r r^T/|r|^3 (Sec. 4.1), collocation at the centroid c_i
// (Sec. 2 and Sec. 4.2). Off-diagonal: seven-point rule (geometry supplies the
// nodes and weights*area in cluster order). Self: tau_i split at c_i into three
// triangles in Duffy coordinates y = c + s[(p_m - c) + t(p_{m+1} - p_m)]; the
// product of kernel and Jacobian does not depend on s (|r| = s|d(t)|), so the
// 16-point rule in s integrates it exactly and only the 16 points in t remain.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <mutex>

#include "device_common.hpp"
#include "hmat_internal.hpp"

namespace hm {

// ---------------------------------------------------------------------------
// Entry generation.

// For collocation point x and triangle q (cluster position): e_b = sum_k w_k S_ab(x - y_k)
// for the fixed row component a, b = 0..2.
__device__ __forceinline__ void row3(const DevGeo& g, double x0, double x1, double x2, int a,
                                     int q, double& e0, double& e1, double& e2) {
  const int nt = g.nt;
  e0 = e1 = e2 = 0.0;
  double diag = 0.0;
#pragma unroll
  for (int k = 0; k < 7; k++) {
    const double r0 = x0 - g.q[(0 * 7 + k) * (size_t)nt + q];
    const double r1 = x1 - g.q[(1 * 7 + k) * (size_t)nt + q];
    const double r2 = x2 - g.q[(2 * 7 + k) * (size_t)nt + q];
    const double w = g.q[(3 * 7 + k) * (size_t)nt + q];
    const double inv = 1.0 / sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    const double ra = (a == 0) ? r0 : ((a == 1) ? r1 : r2);
    const double t = w * inv * inv * inv * ra;
    e0 += t * r0;
    e1 += t * r1;
    e2 += t * r2;
    diag += w * inv;
  }
  e0 *= g.c2;
  e1 *= g.c2;
  e2 *= g.c2;
  const double dd = g.c1 * diag;
  if (a == 0) e0 += dd; else if (a == 1) e1 += dd; else e2 += dd;
}

// Full symmetric 3x3 for collocation point x and triangle q (off-diagonal pair):
// s = {S00, S11, S22, S01, S02, S12}.
__device__ __forceinline__ void full3(const DevGeo& g, double x0, double x1, double x2, int q,
                                      double s[6]) {
  const int nt = g.nt;
  double d = 0.0, m00 = 0.0, m11 = 0.0, m22 = 0.0, m01 = 0.0, m02 = 0.0, m12 = 0.0;
#pragma unroll
  for (int k = 0; k < 7; k++) {
    const double r0 = x0 - g.q[(0 * 7 + k) * (size_t)nt + q];
    const double r1 = x1 - g.q[(1 * 7 + k) * (size_t)nt + q];
    const double r2 = x2 - g.q[(2 * 7 + k) * (size_t)nt + q];
    const double w = g.q[(3 * 7 + k) * (size_t)nt + q];
    const double inv = 1.0 / sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    const double w3 = w * inv * inv * inv;
    d += w * inv;
    m00 += w3 * r0 * r0;
    m11 += w3 * r1 * r1;
    m22 += w3 * r2 * r2;
    m01 += w3 * r0 * r1;
    m02 += w3 * r0 * r2;
    m12 += w3 * r1 * r2;
  }
  s[0] = g.c1 * d + g.c2 * m00;
  s[1] = g.c1 * d + g.c2 * m11;
  s[2] = g.c1 * d + g.c2 * m22;
  s[3] = g.c2 * m01;
  s[4] = g.c2 * m02;
  s[5] = g.c2 * m12;
}

// Self term, one angular point: sub-triangle m (0..2), Gauss node kt (0..15).
// Adds weight * (c1 delta/|d| + c2 d d^T/|d|^3) with weight = w_t |(p_m - c) x (p_{m+1} - p_m)|.
__device__ __forceinline__ void self_point(const DevGeo& g, int p, int m, int kt, double s[6]) {
  const int nt = g.nt;
  const double c0 = g.cen[p], c1v = g.cen[nt + p], c2v = g.cen[2 * nt + p];
  const int m1 = (m + 1) % 3;
  const double a0 = g.vtx[(m * 3 + 0) * (size_t)nt + p] - c0;
  const double a1 = g.vtx[(m * 3 + 1) * (size_t)nt + p] - c1v;
  const double a2 = g.vtx[(m * 3 + 2) * (size_t)nt + p] - c2v;
  const double b0 = g.vtx[(m1 * 3 + 0) * (size_t)nt + p] - g.vtx[(m * 3 + 0) * (size_t)nt + p];
  const double b1 = g.vtx[(m1 * 3 + 1) * (size_t)nt + p] - g.vtx[(m * 3 + 1) * (size_t)nt + p];
  const double b2 = g.vtx[(m1 * 3 + 2) * (size_t)nt + p] - g.vtx[(m * 3 + 2) * (size_t)nt + p];
  const double n0 = a1 * b2 - a2 * b1, n1 = a2 * b0 - a0 * b2, n2 = a0 * b1 - a1 * b0;
  const double jac = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  const double t = g.gl[kt], wt = g.gl[16 + kt] * jac;
  const double d0 = a0 + t * b0, d1 = a1 + t * b1, d2 = a2 + t * b2;
  const double inv = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const double w3 = wt * inv * inv * inv * g.c2;
  const double wd = wt * inv * g.c1;
  s[0] += wd + w3 * d0 * d0;
  s[1] += wd + w3 * d1 * d1;
  s[2] += wd + w3 * d2 * d2;
  s[3] += w3 * d0 * d1;
  s[4] += w3 * d0 * d2;
  s[5] += w3 * d1 * d2;
}

__device__ __forceinline__ double sym_get(const double s[6], int a, int b) {
  if (a == b) return s[a];
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return (lo == 0) ? (hi == 1 ? s[3] : s[4]) : s[5];
}

// The geometry with the Kelvin constants of the body of triangle p.
__device__ __forceinline__ DevGeo body_geo(const DevGeo& g, int p) {
  DevGeo b = g;
  b.c1 = g.kc[p];
  b.c2 = g.kc[g.nt + p];
  return b;
}

// K1: dense blocks, one workgroup per block, one thread per triangle pair.
// D is stored in the panel layout (column-major, leading dimension ld, front
// pad fp); consecutive threads take consecutive row triangles so the three
// rows of a pair land in contiguous memory.
__global__ __launch_bounds__(256) void k_near(DevGeo g0, const NearTask* __restrict__ tasks,
                                              double* __restrict__ D) {
  const NearTask T = tasks[blockIdx.x];
  const DevGeo g = body_geo(g0, T.t_off);
  const int ld = T.ld;
  double* __restrict__ Db = D + T.d_off + T.fp;
  const int npair = T.t_len * T.s_len;
  for (int idx = threadIdx.x; idx < npair; idx += blockDim.x) {
    const int p = idx % T.t_len, q = idx / T.t_len;
    const int ip = T.t_off + p, jq = T.s_off + q;
    if (ip == jq) continue;  // self entries: k_self
    double s[6];
    full3(g, g.cen[ip], g.cen[g.nt + ip], g.cen[2 * g.nt + ip], jq, s);
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
      for (int a = 0; a < 3; a++) Db[(size_t)(3 * q + b) * ld + 3 * p + a] = sym_get(s, a, b);
  }
}

// K1 self entries: one wave per triangle, 48 angular points over the lanes.
__global__ __launch_bounds__(256) void k_self(DevGeo g0, const SelfTask* __restrict__ tasks,
                                              double* __restrict__ D) {
  const int p = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  const int lane = threadIdx.x % WAVE;
  if (p >= g0.nt) return;
  const DevGeo g = body_geo(g0, p);
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (lane < 48) self_point(g, p, lane / 16, lane % 16, s);
#pragma unroll
  for (int c = 0; c < 6; c++)
    for (int o = WAVE / 2; o > 0; o >>= 1) s[c] += __shfl_xor(s[c], o, WAVE);
  if (lane == 0) {
    const SelfTask T = tasks[p];
    double* Db = D + T.d_off + T.fp;
    for (int b = 0; b < 3; b++)
      for (int a = 0; a < 3; a++) Db[(size_t)(3 * T.ploc + b) * T.ld + 3 * T.ploc + a] = sym_get(s, a, b);
  }
}

// Entries at arbitrary (row, col) DOF pairs in cluster numbering (p*3 + a).
__global__ void k_entries(DevGeo g0, int64_t n, const int64_t* __restrict__ rows,
                          const int64_t* __restrict__ cols, double* __restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int p = (int)(rows[k] / 3), a = (int)(rows[k] % 3);
  const DevGeo g = body_geo(g0, p);
  const int q = (int)(cols[k] / 3), b = (int)(cols[k] % 3);
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (p == q) {
    for (int m = 0; m < 3; m++)
      for (int kt = 0; kt < 16; kt++) self_point(g, p, m, kt, s);
  } else {
    full3(g, g.cen[p], g.cen[g.nt + p], g.cen[2 * g.nt + p], q, s);
  }
  out[k] = sym_get(s, a, b);
}

// ---------------------------------------------------------------------------
// Block-wide reductions for 256-thread workgroups. Two alternating LDS slot
// sets: a slot set is rewritten only after every thread has passed the
// barrier of the following reduction, so one barrier per reduction suffices.

constexpr int ACA_T = ACA_NWV * WAVE;            // workgroup of the ACA kernel (large blocks)
constexpr int ACA_WIDE_T = ACA_WIDE_NWV * WAVE;  // the same for launches of few blocks (one per CU)
constexpr int ACA_SMALL_T = WAVE;  // one wave per small block
constexpr int NW = 256 / WAVE;  // waves of a 256-thread workgroup

template <int NWV>
struct RedT {
  double d[2][3][NWV];
  int i[2][NWV];
};


template <int NWV>
__device__ __forceinline__ double blk_max(double v, RedT<NWV>& R, int& ph) {
  v = wave_max(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) R.d[ph][0][threadIdx.x / WAVE] = v;
  __syncthreads();
  double r = R.d[ph][0][0];
#pragma unroll
  for (int w = 1; w < NWV; w++) r = fmax(r, R.d[ph][0][w]);
  ph ^= 1;
  return r;
}
template <int NWV>
__device__ __forceinline__ int blk_min(int v, RedT<NWV>& R, int& ph) {
  v = wave_min(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) R.i[ph][threadIdx.x / WAVE] = v;
  __syncthreads();
  int r = R.i[ph][0];
#pragma unroll
  for (int w = 1; w < NWV; w++) r = min(r, R.i[ph][w]);
  ph ^= 1;
  return r;
}
template <int NWV>
__device__ __forceinline__ void blk_sum3(double& a, double& b, double& c, RedT<NWV>& R, int& ph) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if ((threadIdx.x & (WAVE - 1)) == 0) {
    R.d[ph][0][threadIdx.x / WAVE] = a;
    R.d[ph][1][threadIdx.x / WAVE] = b;
    R.d[ph][2][threadIdx.x / WAVE] = c;
  }
  __syncthreads();
  a = R.d[ph][0][0];
  b = R.d[ph][1][0];
  c = R.d[ph][2][0];
#pragma unroll
  for (int w = 1; w < NWV; w++) {
    a += R.d[ph][0][w];
    b += R.d[ph][1][w];
    c += R.d[ph][2][w];
  }
  ph ^= 1;
}

__device__ __forceinline__ bool in_z(const uint32_t* Z, int r) { return (Z[r >> 5] >> (r & 31)) & 1u; }

// ACA in the precision P of its panels, entries and remainders (FP64, or
// FP32 for FP32 builds); the norm update is FP64 either way. FUZZ: the
// relative width of an argmax tie (well above P's rounding); VANISH: a row
// remainder vanishes at max|v~| <= VANISH ||S_k||_F.
template <typename P>
struct AcaPrec;
template <>
struct AcaPrec<double> {
  static constexpr double FUZZ = 1e-10, VANISH = 1e-14;
};
template <>
struct AcaPrec<float> {
  static constexpr double FUZZ = 1e-6, VANISH = 1e-9;
};

// Fuzzy argmax over rows not in Z: lowest r with |u_r| >= (1 - FUZZ) max.
template <int TPB, typename P>
__device__ int argmax_free(const P* __restrict__ u, int m, const uint32_t* Z,
                           RedT<TPB / WAVE>& R, int& ph) {
  double mx = -1.0;
  for (int r = threadIdx.x; r < m; r += TPB)
    if (!in_z(Z, r)) mx = fmax(mx, (double)fabs(u[r]));
  mx = blk_max(mx, R, ph);
  const double thr = (1.0 - AcaPrec<P>::FUZZ) * mx;
  int cand = INT_MAX;
  for (int r = threadIdx.x; r < m; r += TPB)
    if (!in_z(Z, r) && (double)fabs(u[r]) >= thr) {
      cand = r;
      break;
    }
  return blk_min(cand, R, ph);
}

// Lowest unused row (not in Z) of the lowest of the three row classes
// (r mod 3: displacement component) not in `visited`; -1 if none.
template <int TPB>
__device__ int class_probe(const uint32_t* Z, int m, int visited, RedT<TPB / WAVE>& R, int& ph) {
  for (int c = 0; c < 3; c++) {
    if (visited & (1 << c)) continue;
    int cand = INT_MAX;
    for (int r = c + 3 * (int)threadIdx.x; r < m; r += 3 * TPB)
      if (!in_z(Z, r)) {
        cand = r;
        break;
      }
    const int best = blk_min(cand, R, ph);
    if (best < m) return best;
  }
  return -1;
}

// Row rule of the step-limited runs of the adaptive multiplication (no
// accuracy test that could send ACA to an unvisited component): the rows
// cycle through the three classes. After a step at row i, the next row comes
// from the first class c among i+1, i+2, i (mod 3) with rows outside Z: the
// fuzzy argmax over them of |u_l|, u_l the latest of the k crosses whose
// largest magnitude on them exceeds 1e-12 times its largest magnitude over
// all rows; the lowest of them if no cross qualifies. u_{k-1} is read from
// `ulast` (its LDS copy, or the panel), older crosses from the panel U.
// Returns -1 when Z holds every row.
template <int TPB, typename P>
__device__ int cycle_next(const P* U, const P* ulast, int k, int m, const uint32_t* Z,
                          int i, RedT<TPB / WAVE>& R, int& ph) {
  const int tid = threadIdx.x;
  for (int dc = 1; dc <= 3; dc++) {
    const int c = (i % 3 + dc) % 3;
    int cand = INT_MAX;
    for (int r = c + 3 * tid; r < m; r += 3 * TPB)
      if (!in_z(Z, r)) {
        cand = r;
        break;
      }
    const int lowest = blk_min(cand, R, ph);
    if (lowest >= m) continue;
    for (int l = k - 1; l >= 0; l--) {
      const P* __restrict__ u = (l == k - 1) ? ulast : U + (size_t)l * m;
      double all = 0.0, cls = 0.0;
      for (int r = tid; r < m; r += TPB) {
        const double a = fabs((double)u[r]);
        all = fmax(all, a);
        if (r % 3 == c && !in_z(Z, r)) cls = fmax(cls, a);
      }
      all = blk_max(all, R, ph);
      cls = blk_max(cls, R, ph);
      if (!(cls > 1e-12 * all)) continue;
      const double thr = (1.0 - AcaPrec<P>::FUZZ) * cls;
      cand = INT_MAX;
      for (int r = c + 3 * tid; r < m; r += 3 * TPB)
        if (!in_z(Z, r) && fabs((double)u[r]) >= thr) {
          cand = r;
          break;
        }
      return blk_min(cand, R, ph);
    }
    return lowest;
  }
  return -1;
}

// e_b -= sum_{l<k} coef[l] * P[l*ld + b] for b = 0..2 (one triangle's three
// rows or columns of a panel); four columns per step with separate sums, so
// twelve loads are in flight.
template <typename E>
__device__ __forceinline__ void sub_panel3(const E* __restrict__ coef, const E* P,
                                           int k, int ld, E& e0, E& e1, E& e2) {
  E a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0;
  E c0 = 0, c1 = 0, c2 = 0, d0 = 0, d1 = 0, d2 = 0;
  int l = 0;
  for (; l + 3 < k; l += 4) {
    const E* p0 = P + (size_t)l * ld;
    const E* p1 = p0 + ld;
    const E* p2 = p1 + ld;
    const E* p3 = p2 + ld;
    const E w0 = coef[l], w1 = coef[l + 1], w2 = coef[l + 2], w3 = coef[l + 3];
    a0 += w0 * p0[0];
    a1 += w0 * p0[1];
    a2 += w0 * p0[2];
    b0 += w1 * p1[0];
    b1 += w1 * p1[1];
    b2 += w1 * p1[2];
    c0 += w2 * p2[0];
    c1 += w2 * p2[1];
    c2 += w2 * p2[2];
    d0 += w3 * p3[0];
    d1 += w3 * p3[1];
    d2 += w3 * p3[2];
  }
  for (; l < k; l++) {
    const E* p0 = P + (size_t)l * ld;
    const E w0 = coef[l];
    a0 += w0 * p0[0];
    a1 += w0 * p0[1];
    a2 += w0 * p0[2];
  }
  e0 -= (a0 + b0) + (c0 + d0);
  e1 -= (a1 + b1) + (c1 + d1);
  e2 -= (a2 + b2) + (c2 + d2);
}

// As sub_panel3 (same loads, same partial sums for e_b), and also
// t_b = sum_{l<k} w[l] * P[l*ld + b] from the same loads (in FP64).
template <typename E>
__device__ __forceinline__ void sub_panel3w(const E* __restrict__ coef,
                                            const double* __restrict__ w, const E* P, int k,
                                            int ld, E& e0, E& e1, E& e2, double& t0,
                                            double& t1, double& t2) {
  E a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0;
  E c0 = 0, c1 = 0, c2 = 0, d0 = 0, d1 = 0, d2 = 0;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0, h0 = 0.0, h1 = 0.0, h2 = 0.0;
  int l = 0;
  for (; l + 3 < k; l += 4) {
    const E* p0 = P + (size_t)l * ld;
    const E* p1 = p0 + ld;
    const E* p2 = p1 + ld;
    const E* p3 = p2 + ld;
    const E x00 = p0[0], x01 = p0[1], x02 = p0[2];
    const E x10 = p1[0], x11 = p1[1], x12 = p1[2];
    const E x20 = p2[0], x21 = p2[1], x22 = p2[2];
    const E x30 = p3[0], x31 = p3[1], x32 = p3[2];
    const E w0 = coef[l], w1 = coef[l + 1], w2 = coef[l + 2], w3 = coef[l + 3];
    const double z0 = w[l], z1 = w[l + 1], z2 = w[l + 2], z3 = w[l + 3];
    a0 += w0 * x00;
    a1 += w0 * x01;
    a2 += w0 * x02;
    b0 += w1 * x10;
    b1 += w1 * x11;
    b2 += w1 * x12;
    c0 += w2 * x20;
    c1 += w2 * x21;
    c2 += w2 * x22;
    d0 += w3 * x30;
    d1 += w3 * x31;
    d2 += w3 * x32;
    f0 += z0 * (double)x00 + z2 * (double)x20;
    f1 += z0 * (double)x01 + z2 * (double)x21;
    f2 += z0 * (double)x02 + z2 * (double)x22;
    h0 += z1 * (double)x10 + z3 * (double)x30;
    h1 += z1 * (double)x11 + z3 * (double)x31;
    h2 += z1 * (double)x12 + z3 * (double)x32;
  }
  for (; l < k; l++) {
    const E* p0 = P + (size_t)l * ld;
    const E w0 = coef[l];
    const double z0 = w[l];
    const E x00 = p0[0], x01 = p0[1], x02 = p0[2];
    a0 += w0 * x00;
    a1 += w0 * x01;
    a2 += w0 * x02;
    f0 += z0 * (double)x00;
    f1 += z0 * (double)x01;
    f2 += z0 * (double)x02;
  }
  e0 -= (a0 + b0) + (c0 + d0);
  e1 -= (a1 + b1) + (c1 + d1);
  e2 -= (a2 + b2) + (c2 + d2);
  t0 = f0 + h0;
  t1 = f1 + h1;
  t2 = f2 + h2;
}

// As sub_panel3 (e_b -= sum_{l<k} coef[l] P[l*ld + b]), and from the same
// loads the dot products of panel columns l < c = k - 1 with column c (the
// cross whose norm-update term is pending), summed over the wave:
// pw[l * NWV] += sum over lanes of sum_b P[l*ld + b] P[c*ld + b] (pw: the
// wave's slot, NWV slots per column). Four columns per step; their four sums
// are reduced together (a reduce-scatter over lane bits 5 and 4, then a
// butterfly within 16 lanes): 7 exchanges instead of 4 x 6. Every lane of
// the wave calls it; an inactive lane (act = false) passes a valid P and
// contributes nothing. Columns past k are masked (addresses clamped).
template <int NWV, typename E>
__device__ __forceinline__ void sub_panel3_pend(const E* __restrict__ coef, const E* P, int k,
                                                int ld, bool act, E& e0, E& e1, E& e2,
                                                double* pw, int lane) {
  const int c = k - 1;
  const E* pc = P + (size_t)c * ld;
  const double y0 = act ? (double)pc[0] : 0.0, y1 = act ? (double)pc[1] : 0.0,
               y2 = act ? (double)pc[2] : 0.0;
  // the subtraction keeps sub_panel3's partial sums (four columns in four
  // sums, the tail column by column into the first), so v~ has its bits
  E a0 = 0, a1 = 0, a2 = 0, b0 = 0, b1 = 0, b2 = 0;
  E c0 = 0, c1 = 0, c2 = 0, d0 = 0, d1 = 0, d2 = 0;
  const bool hi32 = lane & 32, hi16 = lane & 16;
  const int mine = 2 * (lane >> 5) + ((lane >> 4) & 1);  // column (of the four) this lane's sum ends in
  for (int l = 0; l < k; l += 4) {
    const bool h1 = l + 1 < k, h2 = l + 2 < k, h3 = l + 3 < k;
    const E* p0 = P + (size_t)l * ld;
    const E* p1 = P + (size_t)min(l + 1, c) * ld;
    const E* p2 = P + (size_t)min(l + 2, c) * ld;
    const E* p3 = P + (size_t)min(l + 3, c) * ld;
    const E x00 = p0[0], x01 = p0[1], x02 = p0[2];
    const E x10 = h1 ? p1[0] : E(0), x11 = h1 ? p1[1] : E(0), x12 = h1 ? p1[2] : E(0);
    const E x20 = h2 ? p2[0] : E(0), x21 = h2 ? p2[1] : E(0), x22 = h2 ? p2[2] : E(0);
    const E x30 = h3 ? p3[0] : E(0), x31 = h3 ? p3[1] : E(0), x32 = h3 ? p3[2] : E(0);
    if (h3) {
      const E w0 = coef[l], w1 = coef[l + 1], w2 = coef[l + 2], w3 = coef[l + 3];
      a0 += w0 * x00;
      a1 += w0 * x01;
      a2 += w0 * x02;
      b0 += w1 * x10;
      b1 += w1 * x11;
      b2 += w1 * x12;
      c0 += w2 * x20;
      c1 += w2 * x21;
      c2 += w2 * x22;
      d0 += w3 * x30;
      d1 += w3 * x31;
      d2 += w3 * x32;
    } else {  // the last one to three columns, one after another into the first sums
      const E w0 = coef[l];
      a0 += w0 * x00;
      a1 += w0 * x01;
      a2 += w0 * x02;
      if (h1) {
        const E w1 = coef[l + 1];
        a0 += w1 * x10;
        a1 += w1 * x11;
        a2 += w1 * x12;
      }
      if (h2) {
        const E w2 = coef[l + 2];
        a0 += w2 * x20;
        a1 += w2 * x21;
        a2 += w2 * x22;
      }
    }
    const double s0 = l < c ? (double)x00 * y0 + (double)x01 * y1 + (double)x02 * y2 : 0.0;
    const double s1 = l + 1 < c ? (double)x10 * y0 + (double)x11 * y1 + (double)x12 * y2 : 0.0;
    const double s2 = l + 2 < c ? (double)x20 * y0 + (double)x21 * y1 + (double)x22 * y2 : 0.0;
    const double s3 = l + 3 < c ? (double)x30 * y0 + (double)x31 * y1 + (double)x32 * y2 : 0.0;
    // lanes 0-31 keep columns 0, 1 and lanes 32-63 columns 2, 3
    double ka = hi32 ? s2 : s0, kb = hi32 ? s3 : s1;
    ka += __shfl_xor(hi32 ? s0 : s2, 32, WAVE);
    kb += __shfl_xor(hi32 ? s1 : s3, 32, WAVE);
    // then lanes with bit 4 clear keep the first of their two, the others the second
    double t = hi16 ? kb : ka;
    t += __shfl_xor(hi16 ? ka : kb, 16, WAVE);
    t += __shfl_xor(t, 8, WAVE);
    t += __shfl_xor(t, 4, WAVE);
    t += __shfl_xor(t, 2, WAVE);
    t += __shfl_xor(t, 1, WAVE);
    if ((lane & 15) == 0 && l + mine < c) pw[(l + mine) * NWV] += t;
  }
  e0 -= (a0 + b0) + (c0 + d0);
  e1 -= (a1 + b1) + (c1 + d1);
  e2 -= (a2 + b2) + (c2 + d2);
}

// The pending cross term on its own, where no next step carries it (the
// block ends, or the next row is exactly zero): w_l = V[:, l] . V[:, c] for
// l < c (one wave per column, into wl), then sum_r U[r, c] (U[r, 0:c] w).
template <int TPB, typename E>
__device__ double pending_cross(const E* U, const E* V, int m, int n, int c, double* wl,
                                RedT<TPB / WAVE>& R, int& ph) {
  constexpr int NWV = TPB / WAVE;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const E* vc = V + (size_t)c * n;
  for (int l = wv; l < c; l += NWV) {
    const E* vl = V + (size_t)l * n;
    double a = 0.0;
    for (int r = lane; r < n; r += WAVE) a += (double)vl[r] * (double)vc[r];
    a = wave_sum(a);
    if (lane == 0) wl[l] = a;
  }
  __syncthreads();
  double x = 0.0, d1 = 0.0, d2 = 0.0;
  for (int r = tid; r < m; r += TPB) {
    double t = 0.0;
    for (int l = 0; l < c; l++) t += (double)U[r + (size_t)l * m] * wl[l];
    x += (double)U[r + (size_t)c * m] * t;
  }
  blk_sum3(x, d1, d2, R, ph);
  return x;
}

// The FP32 form of row3 (FP32 geometry copies, FP32 arithmetic): entries of
// admissible blocks in FP32 builds, where |r| >= dist(X_t, X_s) > 0.
__device__ __forceinline__ void row3f(const DevGeo& g, float x0, float x1, float x2, int a, int q,
                                      float& e0, float& e1, float& e2) {
  const int nt = g.nt;
  e0 = e1 = e2 = 0.0f;
  float diag = 0.0f;
  // not unrolled: the FP32 ACA kernels then fit three waves per SIMD (about
  // 164 VGPRs against 210; 9.4 -> 8.1 ms of ACA at icosphere L5, eps 1e-5).
  // The FP64 form stays unrolled: there the rolled loop saves too few
  // registers for a third wave and loses the overlap of the seven divisions.
#pragma unroll 1
  for (int k = 0; k < 7; k++) {
    const float r0 = x0 - g.q32[(0 * 7 + k) * (size_t)nt + q];
    const float r1 = x1 - g.q32[(1 * 7 + k) * (size_t)nt + q];
    const float r2 = x2 - g.q32[(2 * 7 + k) * (size_t)nt + q];
    const float w = g.q32[(3 * 7 + k) * (size_t)nt + q];
    const float inv = 1.0f / sqrtf(r0 * r0 + r1 * r1 + r2 * r2);
    const float ra = (a == 0) ? r0 : ((a == 1) ? r1 : r2);
    const float t = w * inv * inv * inv * ra;
    e0 += t * r0;
    e1 += t * r1;
    e2 += t * r2;
    diag += w * inv;
  }
  const float c2 = (float)g.c2;
  e0 *= c2;
  e1 *= c2;
  e2 *= c2;
  const float dd = (float)g.c1 * diag;
  if (a == 0) e0 += dd; else if (a == 1) e1 += dd; else e2 += dd;
}

// Three entries of row 3p+a, columns 3q..3q+2 (p, q cluster positions), in
// the ACA precision P.
template <typename P>
struct Ent;
template <>
struct Ent<double> {
  static __device__ __forceinline__ void row(const DevGeo& g, int p, int a, int q, double& e0, double& e1,
                                             double& e2) {
    const int nt = g.nt;
    row3(g, g.cen[p], g.cen[nt + p], g.cen[2 * nt + p], a, q, e0, e1, e2);
  }
};
template <>
struct Ent<float> {
  static __device__ __forceinline__ void row(const DevGeo& g, int p, int a, int q, float& e0, float& e1,
                                             float& e2) {
    const int nt = g.nt;
    row3f(g, g.cen32[p], g.cen32[nt + p], g.cen32[2 * nt + p], a, q, e0, e1, e2);
  }
};

// K2: ACA (Algorithm 1) on the DOF block of task blockIdx.x.
//   rows i_{k+1}: fuzzy argmax over rows not in Z of |u_k| (i_1 = 0);
//   columns j_k: fuzzy argmax of |v~_k|; v_k = v~_k / v~_k(j_k);
//   v~ vanishes if max|v~| = 0 (k = 0) or <= 1e-14 ||S_k||_F;
//   ||S_k||^2 = ||S_{k-1}||^2 + 2 sum_{l<k} (u_l.u_k)(v_l.v_k) + |u_k|^2 |v_k|^2 in FP64;
//   the accuracy test stops ACA only once rows of all three components
//   (row mod 3) are in Z; before that, the next row is the lowest unused row
//   of the first unvisited component, and a vanishing remainder there passes;
//   stop: |u_k||v_k| <= eps ||S_k|| (1), k = min(m,n) (2), Z full (3),
//   panel capacity reached (4: the host resumes the block from its saved
//   state with a larger capacity; the step's next row is chosen first),
//   no finite pivot (5: non-finite entries; reported as an error);
//   with T.cycle (the adaptive multiplication's step-limited runs, eps = 0)
//   the rows follow cycle_next instead of partial pivoting and the probes.
// Panels live in global memory (column-major U m x kcap, V n x kcap); the
// coefficient row U[i, 0:k] / V[j, 0:k], the weights w, the per-wave partial
// sums and the set Z are staged in LDS, and for m + n <= ACA_STAGE_MAX also
// the newest row v_k and column u_k (written to both; the step's later reads
// of them use the LDS copy).
// Each panel is read once per step. The cross term of cross c,
// sum_{l<c} (u_l . u_c)(v_l . v_c) = u_c . (U[:, 0:c] w) with w = V[:, 0:c]^T v_c,
// is formed during the next step: its row pass, which reads V[:, 0:c+1] for
// the subtraction, also forms w (v_c is a panel column by then), and its
// column pass, which reads U[:, 0:c+1], forms U[:, 0:c] w and the dot with
// u_c. The test of cross c is therefore settled one step late, with the
// next row chosen as if it failed (argmax |u_c|). When it passes, the step
// is dropped: ACA stops at rank c + 1, or (components not all visited) the
// speculative row leaves Z again and the step reruns at the probe row. The
// row's vanishing test waits for the settled norm the same way. Where no
// step follows (the block ends: k = min(m,n) or Z full) or the next row is
// exactly zero, the term is computed on its own (pending_cross). The
// decisions and crosses are those of the plain order; only the rounding of
// ||S_k|| differs.
template <int TPB, typename P>
__global__ __launch_bounds__(TPB) void k_aca(DevGeo g0, const AcaTask* __restrict__ tasks,
                                               int32_t* __restrict__ rank_out,
                                               int32_t* __restrict__ stop_out,
                                               double* __restrict__ ratio_out) {
  extern __shared__ double sh[];
  constexpr int NWV = TPB / WAVE;
  __shared__ RedT<NWV> R;
  const AcaTask T = tasks[blockIdx.x];
  const DevGeo g = body_geo(g0, T.t_off);
  const double eps = T.eps;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int m = 3 * T.t_len, n = 3 * T.s_len, kmax = min(m, n), kcap = T.kcap;
  P* __restrict__ U = static_cast<P*>(T.panel);
  P* __restrict__ V = U + (size_t)m * kcap;
  double* const wl = sh;             // weights w_l of the pending cross term
  double* const pw = sh + kcap;      // per wave: partial sums of V[:, l] . V[:, c]
  P* const coef = reinterpret_cast<P*>(sh + (1 + NWV) * kcap);
  const int cw = (kcap * (int)sizeof(P) + 7) / 8;  // coef in doubles
  uint32_t* Z = reinterpret_cast<uint32_t*>(sh + (1 + NWV) * kcap + cw);
  const int zw = (m + 31) >> 5;
  const bool stage = m + n <= ACA_STAGE_MAX;
  P* const vs = reinterpret_cast<P*>(sh + (1 + NWV) * kcap + cw + ((zw + 1) >> 1));  // staged v_k (n), then u_k (m)
  P* const us = vs + n;
  const int nt = g.nt;
  int ph = 0, k = 0, nZ = 0, i = 0, stop = 0, visited = 0, pending = 0;
  int pc = 0;                 // 1: the test of cross k - 1 is not settled yet
  double puu = 0.0, pvv = 0.0;  // |u|^2, |v|^2 of that cross
  double S2 = 0.0, ratio = 0.0;
  if (T.st) {  // resume
    const AcaState s0 = *T.st;
    k = s0.k;
    i = s0.i;
    nZ = s0.nZ;
    visited = s0.visited;
    pending = s0.pending;
    pc = s0.pc;
    S2 = s0.S2;
    ratio = s0.ratio;
    puu = s0.puu;
    pvv = s0.pvv;
    for (int w = tid; w < zw; w += TPB) Z[w] = T.zbits[w];
  } else {
    for (int w = tid; w < zw; w += TPB) Z[w] = 0u;
  }
  // settle the pending cross's test: S2 gets its terms; true if the test passes
  auto settle = [&](double cross) {
    S2 = S2 + 2.0 * cross + puu * pvv;
    const double lhs = sqrt(puu) * sqrt(pvv), rhs = eps * sqrt(S2);
    ratio = rhs > 0.0 ? lhs / rhs : INFINITY;
    pc = 0;
    return lhs <= rhs;
  };
  __syncthreads();
  for (;;) {
    for (int l = tid; l < k; l += TPB) coef[l] = U[i + (size_t)l * m];
    if (pc)
      for (int l = tid; l < k * NWV; l += TPB) pw[l] = 0.0;
    if (tid == 0) Z[i >> 5] |= (1u << (i & 31));
    nZ++;
    const int vis_before = visited;
    visited |= 1 << (i % 3);
    __syncthreads();
    // row i of the remainder into V[:, k]
    P* __restrict__ vk = V + (size_t)k * n;
    P* const vr = stage ? vs : vk;  // where this step reads v_k
    const int pi = T.t_off + i / 3, ai = i % 3;
    double mx = 0.0;
    if (pc) {
      // wave-uniform trip count: the dot products are summed over the wave
      for (int q0 = wv * WAVE; q0 < T.s_len; q0 += TPB) {
        const int q = q0 + lane;
        const bool act = q < T.s_len;
        P e0 = 0, e1 = 0, e2 = 0;
        if (act) Ent<P>::row(g, pi, ai, T.s_off + q, e0, e1, e2);
        sub_panel3_pend<NWV>(coef, V + 3 * (act ? q : 0), k, n, act, e0, e1, e2, pw + wv, lane);
        if (act) {
          vk[3 * q] = e0;
          vk[3 * q + 1] = e1;
          vk[3 * q + 2] = e2;
          if (stage) {
            vs[3 * q] = e0;
            vs[3 * q + 1] = e1;
            vs[3 * q + 2] = e2;
          }
          mx = fmax(mx, (double)fmax(fabs(e0), fmax(fabs(e1), fabs(e2))));
        }
      }
    } else {
      for (int q = tid; q < T.s_len; q += TPB) {
        P e0, e1, e2;
        Ent<P>::row(g, pi, ai, T.s_off + q, e0, e1, e2);
        sub_panel3(coef, V + 3 * q, k, n, e0, e1, e2);
        vk[3 * q] = e0;
        vk[3 * q + 1] = e1;
        vk[3 * q + 2] = e2;
        if (stage) {
          vs[3 * q] = e0;
          vs[3 * q + 1] = e1;
          vs[3 * q + 2] = e2;
        }
        mx = fmax(mx, (double)fmax(fabs(e0), fmax(fabs(e1), fabs(e2))));
      }
    }
    mx = blk_max(mx, R, ph);
    if (pc && !(mx > 0.0)) {
      // no pivot to normalise by: settle the pending cross on its own
      if (settle(pending_cross<TPB>(U, V, m, n, k - 1, wl, R, ph))) {
        if (vis_before == 7) { stop = 1; break; }
        // probe the first unvisited component instead of row i
        if (tid == 0) Z[i >> 5] &= ~(1u << (i & 31));
        __syncthreads();
        nZ--;
        visited = vis_before;
        pending = 1;
        i = class_probe<TPB>(Z, m, visited, R, ph);
        if (i < 0) { stop = 1; break; }
        continue;
      }
    }
    if (!pc) {
      const bool vanished = (k == 0) ? (mx == 0.0) : (mx <= AcaPrec<P>::VANISH * sqrt(S2));
      if (vanished) {
        if (nZ == m) {
          stop = 3;
          break;
        }
        if (pending && visited == 7) {  // the probe row of the last class is captured
          stop = 1;
          break;
        }
        if (T.cycle) {
          i = cycle_next<TPB>(U, U + (size_t)(k > 0 ? k - 1 : 0) * m, k, m, Z, i, R, ph);
          if (i < 0) i = m;  // unreachable: Z is not full here
        } else if (pending) {
          i = class_probe<TPB>(Z, m, visited, R, ph);
          if (i < 0) {
            stop = 1;
            break;
          }
        } else if (k == 0) {
          int cand = INT_MAX;
          for (int r = tid; r < m; r += TPB)
            if (!in_z(Z, r)) {
              cand = r;
              break;
            }
          i = blk_min(cand, R, ph);
        } else {
          i = argmax_free<TPB>(U + (size_t)(k - 1) * m, m, Z, R, ph);
        }
        if (i >= m) {
          stop = 5;
          break;
        }
        continue;
      }
    }
    const double thr = (1.0 - AcaPrec<P>::FUZZ) * mx;
    int cand = INT_MAX;
    for (int c = tid; c < n; c += TPB)
      if ((double)fabs(vr[c]) >= thr) {
        cand = c;
        break;
      }
    const int j = blk_min(cand, R, ph);
    if (j >= n) {  // no finite pivot (non-finite entries)
      stop = 5;
      break;
    }
    const P piv = vr[j];
    __syncthreads();  // every thread holds piv before vk is normalised in place
    double vv = 0.0;
    for (int c = tid; c < n; c += TPB) {
      const P v = vr[c] / piv;
      vk[c] = v;
      if (stage) vs[c] = v;
      vv += (double)v * (double)v;
    }
    const int pend = pc;  // this step also forms the pending cross term
    for (int l = tid; l < k; l += TPB) {
      double p = 0.0;
      if (pend && l < k - 1)
        for (int q = 0; q < NWV; q++) p += pw[l * NWV + q];
      wl[l] = p;
      coef[l] = V[j + (size_t)l * n];
    }
    __syncthreads();
    // column j of the remainder into U[:, k] (S is symmetric: A[3p+a, 3q+b] = S_ba),
    // and the pending cross term u_c . (U[:, 0:c] w), c = k - 1
    P* __restrict__ uk = U + (size_t)k * m;
    P* const ur = stage ? us : uk;  // where this step reads u_k
    const int qj = T.s_off + j / 3, bj = j % 3;
    double uu = 0.0, cross = 0.0;
    for (int p = tid; p < T.t_len; p += TPB) {
      const int ip = T.t_off + p;
      P e0, e1, e2;
      Ent<P>::row(g, ip, bj, qj, e0, e1, e2);
      if (pend) {
        double t0, t1, t2;
        sub_panel3w(coef, wl, U + 3 * p, k, m, e0, e1, e2, t0, t1, t2);
        const P* uc = U + (size_t)(k - 1) * m + 3 * p;
        cross += (double)uc[0] * t0 + (double)uc[1] * t1 + (double)uc[2] * t2;
      } else {
        sub_panel3(coef, U + 3 * p, k, m, e0, e1, e2);
      }
      uk[3 * p] = e0;
      uk[3 * p + 1] = e1;
      uk[3 * p + 2] = e2;
      if (stage) {
        us[3 * p] = e0;
        us[3 * p + 1] = e1;
        us[3 * p + 2] = e2;
      }
      uu += (double)e0 * (double)e0 + (double)e1 * (double)e1 + (double)e2 * (double)e2;
    }
    blk_sum3(uu, vv, cross, R, ph);
    if (pend) {
      if (settle(cross)) {
        if (vis_before == 7) { stop = 1; break; }  // rank k: this step is dropped
        // the accuracy test sends ACA to the first unvisited component: the
        // step reruns there, and row i leaves Z again
        if (tid == 0) Z[i >> 5] &= ~(1u << (i & 31));
        __syncthreads();
        nZ--;
        visited = vis_before;
        pending = 1;
        i = class_probe<TPB>(Z, m, visited, R, ph);
        if (i < 0) { stop = 1; break; }
        continue;
      }
      if (mx <= AcaPrec<P>::VANISH * sqrt(S2)) {  // row i vanishes: it stays in Z, no cross
        if (nZ == m) { stop = 3; break; }
        if (T.cycle)
          i = cycle_next<TPB>(U, U + (size_t)(k - 1) * m, k, m, Z, i, R, ph);
        else
          i = argmax_free<TPB>(U + (size_t)(k - 1) * m, m, Z, R, ph);
        if (i < 0 || i >= m) { stop = 5; break; }
        continue;
      }
    }
    if (tid == 0) {
      T.piv[k] = i;
      T.piv[kcap + k] = j;
    }
    k++;
    pending = 0;
    if (k == 1) {  // no earlier crosses: the test is settled at once
      puu = uu;
      pvv = vv;
      if (settle(0.0)) {
        if (visited == 7) { stop = 1; break; }
        pending = 1;
      }
    } else {
      puu = uu;
      pvv = vv;
      pc = 1;
      if (k == kmax || nZ == m) {  // no step follows to carry the cross term
        __syncthreads();
        if (settle(pending_cross<TPB>(U, V, m, n, k - 1, wl, R, ph))) {
          if (visited == 7) { stop = 1; break; }
          pending = 1;
        }
      }
    }
    if (k == kmax) { stop = 2; break; }
    if (nZ == m) { stop = 3; break; }
    // the next row (while the test of the new cross is pending: the row it
    // would take if the test fails)
    if (T.cycle) {
      i = cycle_next<TPB>(U, ur, k, m, Z, i, R, ph);
      if (i < 0) { stop = 3; break; }  // unreachable: Z is not full here
    } else if (pending) {
      i = class_probe<TPB>(Z, m, visited, R, ph);
      if (i < 0) { stop = 1; break; }
    } else {
      i = argmax_free<TPB>(ur, m, Z, R, ph);
      if (i >= m) {
        stop = 5;
        break;
      }
    }
    // panels full: the saved state holds the next row (and a pending test),
    // and the host resumes the block there with a larger capacity
    if (k == kcap) { stop = 4; break; }
    if (T.k_stop > 0 && k >= T.k_stop) {  // paused: the next step starts at row i
      stop = 6;
      break;
    }
  }
  if (tid == 0) {
    rank_out[T.blk] = k;
    stop_out[T.blk] = stop;
    ratio_out[T.blk] = ratio;
  }
  if (T.st) {
    __syncthreads();
    for (int w = tid; w < zw; w += TPB) T.zbits[w] = Z[w];
    if (tid == 0) *T.st = AcaState{k, i, nZ, stop, visited, pending, pc, 0, S2, ratio, puu, pvv};
  }
}

// V factors: the first k columns of the scratch panel, copied into the padded
// panel layout (pads were zeroed with the arena).
__global__ __launch_bounds__(256) void k_compact(const CopyTask* __restrict__ tasks) {
  const CopyTask T = tasks[blockIdx.x];
  const int64_t nv = (int64_t)T.n * T.k;
  for (int64_t e = threadIdx.x; e < nv; e += blockDim.x) {
    const int64_t c = e / T.n, i = e - c * T.n;
    T.dstV[c * T.ldv + T.fpv + i] = T.srcV[e];
  }
}

// ---------------------------------------------------------------------------
// GMRES helpers (FP64).

// Classical Gram-Schmidt pass h = Q^T w, w -= Q h in three launches:
// k_dots_part (partial dot products per block of rows and group of columns),
// k_dots_final (one wave per column sums the partials in a fixed order) and
// k_proj (the update, reading h).
//
// Workgroup (b, g) takes rows [b*DOT_ROWS, (b+1)*DOT_ROWS) (two per thread)
// and columns [g*DOT_COLS, (g+1)*DOT_COLS), and writes
// part[b*ncols + c] = sum over its rows of Q[i, c] w[i]. The column group's
// loads are independent, so each thread has 2*DOT_COLS of them in flight.
constexpr int DOT_ROWS = 512;
constexpr int DOT_COLS = 8;
__global__ __launch_bounds__(256) void k_dots_part(const double* __restrict__ Q, int64_t ldq,
                                                   int64_t n, int ncols,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ part) {
  __shared__ double red[NW][DOT_COLS];
  const int c0 = blockIdx.y * DOT_COLS;
  const int nc = min(DOT_COLS, ncols - c0);
  const int64_t i0 = (int64_t)blockIdx.x * DOT_ROWS + threadIdx.x;
  const int64_t i1 = i0 + 256;
  const double w0 = i0 < n ? w[i0] : 0.0, w1 = i1 < n ? w[i1] : 0.0;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  double acc[DOT_COLS];
#pragma unroll
  for (int c = 0; c < DOT_COLS; c++) {
    // columns past the group's last re-read it (not stored)
    const double* q = Q + (size_t)(c0 + min(c, nc - 1)) * ldq;
    acc[c] = (i0 < n ? q[i0] * w0 : 0.0) + (i1 < n ? q[i1] * w1 : 0.0);
  }
#pragma unroll
  for (int c = 0; c < DOT_COLS; c++) {
    const double t = wave_sum(acc[c]);
    if (lane == 0) red[wv][c] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < nc) {
    double t = 0.0;
    for (int k = 0; k < NW; k++) t += red[k][threadIdx.x];
    part[(size_t)blockIdx.x * ncols + c0 + threadIdx.x] = t;
  }
}

// hv[c] = sum_b part[b*ncols + c] (one wave per column: lanes stride over b,
// then a wave sum); the Hessenberg column acc takes hv (assign) or adds it.
__global__ __launch_bounds__(WAVE) void k_dots_final(const double* __restrict__ part, int nblk,
                                                     int ncols, double* __restrict__ hv,
                                                     double* __restrict__ acc, int assign) {
  const int c = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < nblk; b += WAVE) t += part[(size_t)b * ncols + c];
  t = wave_sum(t);
  if (threadIdx.x == 0) {
    hv[c] = t;
    acc[c] = assign ? t : acc[c] + t;
  }
}

// w -= Q[:, 0:ncols] hv. If normpart != nullptr, each workgroup writes the
// partial sum of squares of its updated rows to normpart[blockIdx.x].
__global__ __launch_bounds__(256) void k_proj(const double* __restrict__ Q, int64_t ldq, int64_t n,
                                              int ncols, const double* __restrict__ hv,
                                              double* __restrict__ w, double* __restrict__ normpart) {
  __shared__ double red[NW];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (i < n) {
    double s = 0.0;
#pragma unroll 8
    for (int c = 0; c < ncols; c++) s += Q[(size_t)c * ldq + i] * hv[c];
    const double v = w[i] - s;
    w[i] = v;
    sq = v * v;
  }
  if (normpart) {
    sq = wave_sum(sq);
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < NW; k++) t += red[k];
      normpart[blockIdx.x] = t;
    }
  }
}

// out = w / ||w|| with ||w|| = sqrt(sum of normpart[0:nblk]), summed by every
// workgroup in the same order (so all use the same value); workgroup 0 also
// stores the norm in *nrm. out is untouched when the norm is 0.
__global__ __launch_bounds__(256) void k_scale_norm(const double* __restrict__ w, int64_t n,
                                                    const double* __restrict__ normpart, int nblk,
                                                    double* __restrict__ nrm,
                                                    double* __restrict__ out,
                                                    const int32_t* __restrict__ order,
                                                    double* __restrict__ xp,
                                                    const double* __restrict__ col, int ncol,
                                                    double* __restrict__ col_host) {
  __shared__ double red[NW];
  __shared__ double dsh;
  double t = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) t += normpart[b];
  t = wave_sum(t);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = 0.0;
    for (int k = 0; k < NW; k++) u += red[k];
    dsh = sqrt(u);
    if (blockIdx.x == 0) *nrm = dsh;
  }
  __syncthreads();
  const double d = dsh;
  // col_host (host memory the device can write): col[0:ncol] and the norm
  if (col_host && blockIdx.x == 0) {
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) col_host[c] = col[c];
    if (threadIdx.x == 0) col_host[ncol] = d;
  }
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && d != 0.0) {
    out[i] = w[i] / d;
    // also the product's input in cluster order, xp[i] = out[3 order[i/3] + i%3]
    if (xp) xp[i] = w[3 * (int64_t)order[i / 3] + i % 3] / d;
  }
}

// Partial sums of squares: part[b] = sum over the rows of block b of w[i]^2.
__global__ __launch_bounds__(256) void k_sqnorm_part(const double* __restrict__ w, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double red[256 / WAVE];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double sq = i < n ? w[i] * w[i] : 0.0;
  sq = wave_sum(sq);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 256 / WAVE; k++) t += red[k];
    part[blockIdx.x] = t;
  }
}

// out[0] = sqrt(sum of part[0:nblk]) (one workgroup).
__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ part, int nblk,
                                                    double* __restrict__ out) {
  __shared__ double red[256 / WAVE];
  double t = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) t += part[b];
  t = wave_sum(t);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = 0.0;
    for (int k = 0; k < 256 / WAVE; k++) u += red[k];
    out[0] = sqrt(u);
  }
}

// out = w / *den (den on the device; out untouched if *den == 0).
__global__ void k_scale(const double* __restrict__ w, int64_t n, const double* __restrict__ den,
                        double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double d = *den;
  if (i < n && d != 0.0) out[i] = w[i] / d;
}

// x += Q[:, 0:ncols] y (y on the device)
__global__ __launch_bounds__(256) void k_add_comb(const double* __restrict__ Q, int64_t ldq,
                                                  int64_t n, int ncols,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < ncols; c++) s += Q[(size_t)c * ldq + i] * y[c];
  x[i] += s;
}

// r = b - r
__global__ void k_residual(const double* __restrict__ b, int64_t n, double* __restrict__ r) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - r[i];
}

// y += a x.
__global__ void k_axpy(double a, const double* __restrict__ x, int64_t n, double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers (host side).


hipError_t launch_self(const DevGeo& g, const SelfTask* tasks, double* D, hipStream_t s) {
  hipLaunchKernelGGL(k_self, dim3(blocks_for(g.nt, 4)), dim3(256), 0, s, g, tasks, D);
  return hipGetLastError();
}

hipError_t launch_near_only(const DevGeo& g, const NearTask* tasks, int ntasks, double* D,
                            hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_near, dim3(ntasks), dim3(256), 0, s, g, tasks, D);
  return hipGetLastError();
}

hipError_t launch_entries(const DevGeo& g, int64_t n, const int64_t* rows, const int64_t* cols,
                          double* out, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_entries, dim3(blocks_for(n, 128)), dim3(128), 0, s, g, n, rows, cols, out);
  return hipGetLastError();
}

// tasks[0, n_big): 256-thread workgroups (512 if `wide`); tasks[n_big,
// ntasks): blocks with at most ACA_SMALL_TRI triangles per side, one wave
// each. A one-wave block has no cross-wave barriers, and four times as many
// blocks fit on a CU. A launch of few large blocks (later capacity passes,
// the rounds of the adaptive multiplication) leaves most CUs idle; there a
// block's step is bound by the loads its own workgroup keeps in flight, and
// 512 threads keep twice as many. shmem_big / shmem_small: the largest
// aca_shmem of each part's tasks.
namespace {
// Dynamic LDS beyond 64 KiB must be allowed per kernel. Each ACA kernel is
// allowed the device's whole per-workgroup LDS (less its static part) once
// per device, so concurrent builds never lower the limit under one another.
std::mutex g_lds_mu;
uint32_t g_lds_set[64] = {};
hipError_t allow_full_lds(const void* f, int bit) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_lds_mu);
  if (g_lds_set[dev] & (1u << bit)) return hipSuccess;
  int a = 0, b = 0;
  if ((e = hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return e;
  if (hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) {
    (void)hipGetLastError();
    b = 0;
  }
  hipFuncAttributes fa{};
  if ((e = hipFuncGetAttributes(&fa, f)) != hipSuccess) return e;
  const int limit = std::min(std::max(a, b), 160 * 1024) - (int)fa.sharedSizeBytes;
  if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, limit)) != hipSuccess) return e;
  g_lds_set[dev] |= 1u << bit;
  return hipSuccess;
}
}  // namespace

template <typename P>
hipError_t launch_aca_t(const DevGeo& g, const AcaTask* tasks, int ntasks, int n_big, size_t shmem_big,
                        size_t shmem_small, bool wide, int32_t* rank, int32_t* stop, double* ratio,
                        hipStream_t s) {
  const int bits = sizeof(P) == 8 ? 0 : 3;
  if (shmem_big > 64 * 1024) {
    const void* f = wide ? reinterpret_cast<const void*>(&k_aca<ACA_WIDE_T, P>)
                         : reinterpret_cast<const void*>(&k_aca<ACA_T, P>);
    const hipError_t e = allow_full_lds(f, bits + (wide ? 1 : 0));
    if (e != hipSuccess) return e;
  }
  if (shmem_small > 64 * 1024) {
    const hipError_t e = allow_full_lds(reinterpret_cast<const void*>(&k_aca<ACA_SMALL_T, P>), bits + 2);
    if (e != hipSuccess) return e;
  }
  if (n_big > 0 && wide)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_aca<ACA_WIDE_T, P>), dim3(n_big), dim3(ACA_WIDE_T), shmem_big, s, g,
                       tasks, rank, stop, ratio);
  else if (n_big > 0)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_aca<ACA_T, P>), dim3(n_big), dim3(ACA_T), shmem_big, s, g, tasks,
                       rank, stop, ratio);
  if (ntasks > n_big)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_aca<ACA_SMALL_T, P>), dim3(ntasks - n_big), dim3(ACA_SMALL_T),
                       shmem_small, s, g, tasks + n_big, rank, stop, ratio);
  return hipGetLastError();
}

// fp32: panels, entries and remainders in FP32 (FP32 builds); else FP64.
hipError_t launch_aca(const DevGeo& g, const AcaTask* tasks, int ntasks, int n_big, size_t shmem_big,
                      size_t shmem_small, bool wide, bool fp32, int32_t* rank, int32_t* stop, double* ratio,
                      hipStream_t s) {
  return fp32 ? launch_aca_t<float>(g, tasks, ntasks, n_big, shmem_big, shmem_small, wide, rank, stop, ratio, s)
              : launch_aca_t<double>(g, tasks, ntasks, n_big, shmem_big, shmem_small, wide, rank, stop, ratio, s);
}

__global__ __launch_bounds__(256) void k_copy_spans(const SpanCopy* __restrict__ t) {
  const SpanCopy c = t[blockIdx.x];
  for (int64_t w = threadIdx.x; w < c.words; w += 256) c.dst[w] = c.src[w];
}

hipError_t launch_copy_spans(const SpanCopy* t, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy_spans, dim3(n), dim3(256), 0, s, t);
  return hipGetLastError();
}

// A block whose accuracy-controlled ACA reached full rank is stored exactly
// (a cross approximation is kept only as a compression, Sec. 2, and a
// full-rank run can end inexact when a remainder at rounding level is taken
// as a cross): U = B, V = I for n <= m, else U = I, V = B^T, entries as in the
// ACA passes (S symmetric: A[3p+a, 3q+b] = S_ba). One workgroup per block.
template <typename P>
__global__ __launch_bounds__(256) void k_exact(DevGeo g0, const ExactTask* __restrict__ tasks) {
  const ExactTask T = tasks[blockIdx.x];
  const DevGeo g = body_geo(g0, T.t_off);
  const int m = 3 * T.t_len, n = 3 * T.s_len, nt = g.nt;
  P* __restrict__ U = static_cast<P*>(T.panel);
  P* __restrict__ V = U + (size_t)m * T.kcap;
  if (n <= m) {
    for (int e = threadIdx.x; e < T.t_len * n; e += blockDim.x) {
      const int p = e % T.t_len, c = e / T.t_len, ip = T.t_off + p;
      double e0, e1, e2;
      row3(g, g.cen[ip], g.cen[nt + ip], g.cen[2 * nt + ip], c % 3, T.s_off + c / 3, e0, e1, e2);
      P* col = U + (size_t)c * m + 3 * p;
      col[0] = (P)e0;
      col[1] = (P)e1;
      col[2] = (P)e2;
    }
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) V[(size_t)(e / n) * n + e % n] = (e / n == e % n) ? P(1) : P(0);
  } else {
    for (int e = threadIdx.x; e < m * T.s_len; e += blockDim.x) {
      const int q = e % T.s_len, r = e / T.s_len, ip = T.t_off + r / 3;
      double e0, e1, e2;
      row3(g, g.cen[ip], g.cen[nt + ip], g.cen[2 * nt + ip], r % 3, T.s_off + q, e0, e1, e2);
      P* col = V + (size_t)r * n + 3 * q;
      col[0] = (P)e0;
      col[1] = (P)e1;
      col[2] = (P)e2;
    }
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) U[(size_t)(e / m) * m + e % m] = (e / m == e % m) ? P(1) : P(0);
  }
}

hipError_t launch_exact(const DevGeo& g, const ExactTask* tasks, int ntasks, bool fp32, hipStream_t s) {
  if (ntasks > 0 && fp32) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_exact<float>), dim3(ntasks), dim3(256), 0, s, g, tasks);
  if (ntasks > 0 && !fp32) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_exact<double>), dim3(ntasks), dim3(256), 0, s, g, tasks);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_compact32(const CopyTask32* __restrict__ tasks) {
  const CopyTask32 T = tasks[blockIdx.x];
  const int64_t nv = (int64_t)T.n * T.k;
  for (int64_t e = threadIdx.x; e < nv; e += blockDim.x) {
    const int64_t c = e / T.n, i = e - c * T.n;
    T.dstV[c * T.ldv + T.fpv + i] = (double)T.srcV[e];
  }
}

hipError_t launch_compact32(const CopyTask32* tasks, int ntasks, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_compact32, dim3(ntasks), dim3(256), 0, s, tasks);
  return hipGetLastError();
}

hipError_t launch_compact(const CopyTask* tasks, int ntasks, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_compact, dim3(ntasks), dim3(256), 0, s, tasks);
  return hipGetLastError();
}

// Scratch (doubles) for the partial dot products of launch_cgs_pass.
size_t dots_part_size(int64_t n, int ncols) { return (size_t)((n + DOT_ROWS - 1) / DOT_ROWS) * ncols; }

// One Gram-Schmidt pass: hv = Q[:, 0:ncols]^T w, acc = hv (assign) or
// acc += hv, w -= Q hv; with normpart, also the partial sums of squares of
// the new w (norm_part_size(n) doubles). part: dots_part_size(n, ncols).
hipError_t launch_cgs_pass(const double* Q, int64_t ldq, int64_t n, int ncols, double* w,
                           double* part, double* hv, double* acc, int assign, double* normpart,
                           hipStream_t s) {
  const int nblk = (int)((n + DOT_ROWS - 1) / DOT_ROWS);
  hipLaunchKernelGGL(k_dots_part, dim3(nblk, (ncols + DOT_COLS - 1) / DOT_COLS), dim3(256), 0, s, Q, ldq,
                     n, ncols, w, part);
  hipLaunchKernelGGL(k_dots_final, dim3(ncols), dim3(WAVE), 0, s, part, nblk, ncols, hv, acc, assign);
  hipLaunchKernelGGL(k_proj, dim3(blocks_for(n, 256)), dim3(256), 0, s, Q, ldq, n, ncols, hv, w,
                     normpart);
  return hipGetLastError();
}

// Partial-norm scratch (doubles) for n rows.
size_t norm_part_size(int64_t n) { return (size_t)((n + 255) / 256); }

// out = w / ||w|| from the partial sums of squares written by the last pass;
// *nrm = ||w||. With xp != nullptr, also xp[i] = out[3 order[i/3] + i%3]
// (out in cluster order; n a multiple of 3, order a permutation of n/3).
// With col_host != nullptr (pinned host memory), also col_host[0:ncol] =
// col[0:ncol] and col_host[ncol] = ||w||, written by the kernel itself.
hipError_t launch_scale_norm(const double* w, int64_t n, const double* normpart, double* nrm,
                             double* out, const int32_t* order, double* xp, const double* col,
                             int ncol, double* col_host, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_norm, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, n, normpart,
                     (int)blocks_for(n, 256), nrm, out, order, xp, col, ncol, col_host);
  return hipGetLastError();
}

// out[0] = ||w||_2 in two stages (normpart: norm_part_size(n) doubles).
hipError_t launch_norm(const double* w, int64_t n, double* normpart, double* out, hipStream_t s) {
  const int nblk = (int)blocks_for(n, 256);
  hipLaunchKernelGGL(k_sqnorm_part, dim3(nblk), dim3(256), 0, s, w, n, normpart);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, normpart, nblk, out);
  return hipGetLastError();
}

hipError_t launch_scale(const double* w, int64_t n, const double* den, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, n, den, out);
  return hipGetLastError();
}

hipError_t launch_add_comb(const double* Q, int64_t ldq, int64_t n, int ncols, const double* y,
                           double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_add_comb, dim3(blocks_for(n, 256)), dim3(256), 0, s, Q, ldq, n, ncols, y, x);
  return hipGetLastError();
}

hipError_t launch_residual(const double* b, int64_t n, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(blocks_for(n, 256)), dim3(256), 0, s, b, n, r);
  return hipGetLastError();
}

hipError_t launch_axpy(double a, const double* x, int64_t n, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, x, n, y);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free solve (hmat_solve_noalloc): one fixed
// array per device, loaded with the code object and held until the process
// ends. Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol); it passes the device address that
// hipGetSymbolAddress returns, resolved once per device with that device
// current.
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};
}  // namespace

hipError_t noalloc_workspace(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace hm
