// CDNA4 (gfx950) kernels of the H-matrix path.
//
//   K1  k_near / k_self   dense (non-admissible) blocks entry by entry (Sec. 2.2)
//   K2  k_aca             ACA with partial pivoting on every admissible block
//                         (Sec. 2.2, Algorithm 1), one workgroup per block
//   --  k_compact         final low-rank arena (first k columns of the panels)
//   K3  k_gather, k_mv1 (V^T x and dense blocks), k_mv2 (U z), k_reduce
//                         y = sum U_b (V_b^T x_s) + sum D_b x_s (Sec. 2)
//   --  GMRES helpers     dots, column updates, norms
//
// Entries: A[3i+a, 3j+b] = int_{tau_j} S_ab(c_i - y) ds_y with Kelvin's tensor
// S = c1 delta/|r| + c2 r r^T/|r|^3 (Sec. 4.1), collocation at the centroid c_i
// (Sec. 2 and Sec. 4.2). Off-diagonal: seven-point rule (geometry supplies the
// nodes and weights*area in cluster order). Self: tau_i split at c_i into three
// triangles in Duffy coordinates y = c + s[(p_m - c) + t(p_{m+1} - p_m)]; the
// product of kernel and Jacobian does not depend on s (|r| = s|d(t)|), so the
// 16-point rule in s integrates it exactly and only the 16 points in t remain.
#include <hip/hip_runtime.h>

#include <climits>

#include "hmat_internal.hpp"

namespace hm {

constexpr int WAVE = 64;

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

constexpr int ACA_T = 256;      // workgroup of the ACA kernel
constexpr int NW = 256 / WAVE;  // waves of a 256-thread workgroup

template <int NWV>
struct RedT {
  double d[2][2][NWV];
  int i[2][NWV];
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, WAVE));
  return v;
}

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
__device__ __forceinline__ void blk_sum2(double& a, double& b, RedT<NWV>& R, int& ph) {
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & (WAVE - 1)) == 0) {
    R.d[ph][0][threadIdx.x / WAVE] = a;
    R.d[ph][1][threadIdx.x / WAVE] = b;
  }
  __syncthreads();
  a = R.d[ph][0][0];
  b = R.d[ph][1][0];
#pragma unroll
  for (int w = 1; w < NWV; w++) {
    a += R.d[ph][0][w];
    b += R.d[ph][1][w];
  }
  ph ^= 1;
}

__device__ __forceinline__ bool in_z(const uint32_t* Z, int r) { return (Z[r >> 5] >> (r & 31)) & 1u; }

// Fuzzy argmax over rows not in Z: lowest r with |u_r| >= (1 - 1e-10) max.
template <int TPB>
__device__ int argmax_free(const double* __restrict__ u, int m, const uint32_t* Z,
                           RedT<TPB / WAVE>& R, int& ph) {
  double mx = -1.0;
  for (int r = threadIdx.x; r < m; r += TPB)
    if (!in_z(Z, r)) mx = fmax(mx, fabs(u[r]));
  mx = blk_max(mx, R, ph);
  const double thr = (1.0 - 1e-10) * mx;
  int cand = INT_MAX;
  for (int r = threadIdx.x; r < m; r += TPB)
    if (!in_z(Z, r) && fabs(u[r]) >= thr) {
      cand = r;
      break;
    }
  return blk_min(cand, R, ph);
}

// e_b -= sum_{l<k} coef[l] * P[l*ld + b] for b = 0..2 (one triangle's three
// rows or columns of a panel); four columns per step with separate sums, so
// twelve loads are in flight.
__device__ __forceinline__ void sub_panel3(const double* __restrict__ coef, const double* P,
                                           int k, int ld, double& e0, double& e1, double& e2) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
  int l = 0;
  for (; l + 3 < k; l += 4) {
    const double* p0 = P + (size_t)l * ld;
    const double* p1 = p0 + ld;
    const double* p2 = p1 + ld;
    const double* p3 = p2 + ld;
    const double w0 = coef[l], w1 = coef[l + 1], w2 = coef[l + 2], w3 = coef[l + 3];
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
    const double* p0 = P + (size_t)l * ld;
    const double w0 = coef[l];
    a0 += w0 * p0[0];
    a1 += w0 * p0[1];
    a2 += w0 * p0[2];
  }
  e0 -= (a0 + b0) + (c0 + d0);
  e1 -= (a1 + b1) + (c1 + d1);
  e2 -= (a2 + b2) + (c2 + d2);
}

// sum_r x[r] y[r] over r = lane, lane + 64, ... < n; four partial sums.
__device__ __forceinline__ double lane_dot(const double* x, const double* y, int n, int lane) {
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  int r = lane;
  for (; r + 3 * WAVE < n; r += 4 * WAVE) {
    a += x[r] * y[r];
    b += x[r + WAVE] * y[r + WAVE];
    c += x[r + 2 * WAVE] * y[r + 2 * WAVE];
    d += x[r + 3 * WAVE] * y[r + 3 * WAVE];
  }
  for (; r < n; r += WAVE) a += x[r] * y[r];
  return (a + b) + (c + d);
}

// K2: ACA (Algorithm 1) on the DOF block of task blockIdx.x.
//   rows i_{k+1}: fuzzy argmax over rows not in Z of |u_k| (i_1 = 0);
//   columns j_k: fuzzy argmax of |v~_k|; v_k = v~_k / v~_k(j_k);
//   v~ vanishes if max|v~| = 0 (k = 0) or <= 1e-14 ||S_k||_F;
//   ||S_k||^2 = ||S_{k-1}||^2 + 2 sum_{l<k} (u_l.u_k)(v_l.v_k) + |u_k|^2 |v_k|^2 in FP64;
//   stop: |u_k||v_k| <= eps ||S_k|| (1), k = min(m,n) (2), Z full (3),
//   panel capacity reached (4: the host re-runs the block with a larger capacity),
//   no finite pivot (5: non-finite entries; reported as an error).
// Panels live in global memory (column-major U m x kcap, V n x kcap); the
// coefficient row U[i, 0:k] / V[j, 0:k] and the set Z are staged in LDS.
template <int TPB>
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
  double* __restrict__ U = T.panel;
  double* __restrict__ V = T.panel + (size_t)m * kcap;
  double* coef = sh;
  uint32_t* Z = reinterpret_cast<uint32_t*>(sh + kcap);
  const int zw = (m + 31) >> 5;
  const int nt = g.nt;
  int ph = 0, k = 0, nZ = 0, i = 0, stop = 0;
  double S2 = 0.0, ratio = 0.0;
  if (T.st) {  // resume
    const AcaState s0 = *T.st;
    k = s0.k;
    i = s0.i;
    nZ = s0.nZ;
    S2 = s0.S2;
    ratio = s0.ratio;
    for (int w = tid; w < zw; w += TPB) Z[w] = T.zbits[w];
  } else {
    for (int w = tid; w < zw; w += TPB) Z[w] = 0u;
  }
  __syncthreads();
  for (;;) {
    for (int l = tid; l < k; l += TPB) coef[l] = U[i + (size_t)l * m];
    if (tid == 0) Z[i >> 5] |= (1u << (i & 31));
    nZ++;
    __syncthreads();
    // row i of the remainder into V[:, k]
    double* __restrict__ vk = V + (size_t)k * n;
    const int pi = T.t_off + i / 3, ai = i % 3;
    const double x0 = g.cen[pi], x1 = g.cen[nt + pi], x2 = g.cen[2 * nt + pi];
    double mx = 0.0;
    for (int q = tid; q < T.s_len; q += TPB) {
      double e0, e1, e2;
      row3(g, x0, x1, x2, ai, T.s_off + q, e0, e1, e2);
      sub_panel3(coef, V + 3 * q, k, n, e0, e1, e2);
      vk[3 * q] = e0;
      vk[3 * q + 1] = e1;
      vk[3 * q + 2] = e2;
      mx = fmax(mx, fmax(fabs(e0), fmax(fabs(e1), fabs(e2))));
    }
    mx = blk_max(mx, R, ph);
    const bool vanished = (k == 0) ? (mx == 0.0) : (mx <= 1e-14 * sqrt(S2));
    if (vanished) {
      if (nZ == m) {
        stop = 3;
        break;
      }
      if (k == 0) {
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
    const double thr = (1.0 - 1e-10) * mx;
    int cand = INT_MAX;
    for (int c = tid; c < n; c += TPB)
      if (fabs(vk[c]) >= thr) {
        cand = c;
        break;
      }
    const int j = blk_min(cand, R, ph);
    if (j >= n) {  // no finite pivot (non-finite entries)
      stop = 5;
      break;
    }
    const double piv = vk[j];
    __syncthreads();  // every thread holds piv before vk is normalised in place
    double vv = 0.0;
    for (int c = tid; c < n; c += TPB) {
      const double v = vk[c] / piv;
      vk[c] = v;
      vv += v * v;
    }
    for (int l = tid; l < k; l += TPB) coef[l] = V[j + (size_t)l * n];
    __syncthreads();
    // column j of the remainder into U[:, k] (S is symmetric: A[3p+a, 3q+b] = S_ba)
    double* __restrict__ uk = U + (size_t)k * m;
    const int qj = T.s_off + j / 3, bj = j % 3;
    double uu = 0.0;
    for (int p = tid; p < T.t_len; p += TPB) {
      const int ip = T.t_off + p;
      double e0, e1, e2;
      row3(g, g.cen[ip], g.cen[nt + ip], g.cen[2 * nt + ip], bj, qj, e0, e1, e2);
      sub_panel3(coef, U + 3 * p, k, m, e0, e1, e2);
      uk[3 * p] = e0;
      uk[3 * p + 1] = e1;
      uk[3 * p + 2] = e2;
      uu += e0 * e0 + e1 * e1 + e2 * e2;
    }
    blk_sum2(uu, vv, R, ph);
    // sum_{l<k} (u_l . u_k)(v_l . v_k): wave w takes l = w, w + NWV, ...
    double cr = 0.0;
    for (int l = wv; l < k; l += NWV) {
      const double* ul = U + (size_t)l * m;
      const double* vl = V + (size_t)l * n;
      const double a = lane_dot(ul, uk, m, lane), b = lane_dot(vl, vk, n, lane);
      cr += wave_sum(a) * wave_sum(b);
    }
    double cross = (lane == 0) ? cr : 0.0, dummy = 0.0;
    blk_sum2(cross, dummy, R, ph);
    if (tid == 0) {
      T.piv[k] = i;
      T.piv[kcap + k] = j;
    }
    k++;
    S2 = S2 + 2.0 * cross + uu * vv;
    const double lhs = sqrt(uu) * sqrt(vv), rhs = eps * sqrt(S2);
    ratio = rhs > 0.0 ? lhs / rhs : INFINITY;
    if (lhs <= rhs) { stop = 1; break; }
    if (k == kmax) { stop = 2; break; }
    if (nZ == m) { stop = 3; break; }
    if (k == kcap) { stop = 4; break; }
    i = argmax_free<TPB>(uk, m, Z, R, ph);
    if (i >= m) {
      stop = 5;
      break;
    }
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
    if (tid == 0) *T.st = AcaState{k, i, nZ, stop, S2, ratio};
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

// Phase A item: z = V_b^T x_s for a group of <= 8 columns; one wave. Lanes
// cover the aligned row window of V two rows at a time (16-byte loads of V and
// of the gathered x; pad rows of V are zero); NR right-hand sides at once,
// columns in sub-batches of CB.
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
    double acc[CB][NR];
#pragma unroll
    for (int c = 0; c < CB; c++)
#pragma unroll
      for (int r = 0; r < NR; r++) acc[c][r] = 0.0;
    for (int i = 2 * lane; i < I.ld; i += TILE) {
      double2 xv[NR], v[CB];
#pragma unroll
      for (int c = 0; c < CB; c++)  // columns past l1 re-read the last one (not accumulated)
        v[c] = ld2(V + (size_t)(l0 + min(c, nc - 1)) * I.ld + i);
#pragma unroll
      for (int r = 0; r < NR; r++)
        xv[r] = (r < nr) ? *reinterpret_cast<const double2*>(X + r * ldxp + i) : make_double2(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < CB; c++) {
        if (c < nc) {
#pragma unroll
          for (int r = 0; r < NR; r++) acc[c][r] += v[c].x * xv[r].x + v[c].y * xv[r].y;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CB; c++)
#pragma unroll
      for (int r = 0; r < NR; r++) {
        const double sum = wave_sum(acc[c][r]);
        if (lane == 0 && c < nc && r < nr) z[r * ldz + I.zoff + (l0 - I.l0) + c] = sum;
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
// lanes. A segment's last partial batch re-reads in-segment data without
// accumulating it, so every batch issues its UNR loads back to back. Writes
// part[chunk][r][128].
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
      a[u] = ldp(A + (ok ? (int64_t)(t + u) * step + 2 * lane : 0));
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
      mv_b_grouped<UNR, T>(S, stream, S.far ? z : xp, acc0[0], acc1[0]);
      continue;
    }
    const bool act = L2 >= S.row_lo && L2 < S.row_hi;
    const int Lc = min(max(L2, (int)S.row_lo), (int)S.row_hi - 2);
    const T* __restrict__ A = stream + S.so + (Lc - S.row_lo) - (int64_t)S.c0 * len;
    const double* __restrict__ src = (S.far ? z : xp) + S.soff;
    const int64_t ld = S.far ? ldz : ldxp;
    for (int c = S.c0; c < S.c1; c += UNR) {
      const int nc = min(UNR, S.c1 - c);
      typename Pair<T>::type a[UNR];
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        const int cu = (u < nc) ? c + u : S.c1 - 1;
        a[u] = ldp(A + (int64_t)cu * len);
      }
#pragma unroll
      for (int u = 0; u < UNR; u++) {
        a[u].x = act ? a[u].x : (T)0;
        a[u].y = act ? a[u].y : (T)0;
      }
      if (nc == UNR) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
          if (r < nr) {
            const double* sr = src + r * ld + c;
#pragma unroll
            for (int u = 0; u < UNR; u++) {
              acc0[r] += (double)a[u].x * sr[u];
              acc1[r] += (double)a[u].y * sr[u];
            }
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < NR; r++) {
          if (r < nr) {
            const double* sr = src + r * ld + c;
#pragma unroll
            for (int u = 0; u < UNR; u++) {
              if (u < nc) {
                acc0[r] += (double)a[u].x * sr[u];
                acc1[r] += (double)a[u].y * sr[u];
              }
            }
          }
        }
      }
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

// Phase A, several vectors: z[:, zoff + c] = V[:, l0 + c]^T X for c < l1 - l0
// (<= 64 columns: four 16-column tiles). Per 16-row step lane l reads rows
// 4(l/16) .. +3 of column l%16 of each tile and the same rows of vector l%16.
template <typename T>
__device__ __forceinline__ void mv_a_mfma(const MvA& I, const T* __restrict__ far,
                                          const double* __restrict__ xp, int64_t ldxp, int nr,
                                          double* __restrict__ z, int64_t ldz) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int kq = lane >> 4, cl = lane & 15;
  const int ncols = I.l1 - I.l0;
  const int ntile = (ncols + 15) >> 4;
  const bool rv = cl < nr;
  const double* __restrict__ X = xp + (int64_t)min(cl, nr - 1) * ldxp + I.a0;
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
    double2 x0 = *reinterpret_cast<const double2*>(X + (p0 ? r0 : 0));
    double2 x1 = *reinterpret_cast<const double2*>(X + (p1 ? r0 + 2 : 0));
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
        if (col < ncols && rv) z[(int64_t)cl * ldz + I.zoff + col] = acc[q][v];
      }
    }
  }
}

// Phase B, several vectors: one chunk (segments of one 128-row tile). Per
// group of four columns c..c+3, lane l reads rows 4(l%16) .. +3 of column
// c + l/16 in each 64-row half the segment touches, and entry c + l/16 of
// vector l%16. Product t of a half accumulates tile rows 64h + 4m + t.
// Writes part[chunk][16][128].
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
  for (int s = C.seg_lo; s < C.seg_hi; s++) {
    const MvSeg S = segs[s];
    const int len = S.row_hi - S.row_lo;
    const double* __restrict__ Bp =
        (S.far ? z + (int64_t)min(m16, nr - 1) * ldz : xp + (int64_t)min(m16, nr - 1) * ldxp) + S.soff;
    const bool h0 = S.row_lo < 64, h1 = S.row_hi > 64;  // halves the segment touches
    // this lane's rows in each half, relative to the segment (pairs are whole: bounds are even)
    const int R0 = 4 * m16 - S.row_lo, R1 = 64 + 4 * m16 - S.row_lo;
    const bool q00 = R0 >= 0 && R0 < len, q01 = R0 + 2 >= 0 && R0 + 2 < len;
    const bool q10 = R1 >= 0 && R1 < len, q11 = R1 + 2 >= 0 && R1 + 2 < len;
    // batches of 16 columns (four groups of four): all loads first
    for (int c = S.c0; c < S.c1; c += 16) {
      double bv[4];
      double2 av[4][2][2];
#pragma unroll
      for (int g = 0; g < 4; g++) {
        const int cc = c + 4 * g + kq;
        const bool cok = cc < S.c1;
        const int ccl = cok ? cc : S.c1 - 1;
        const T* __restrict__ col = stream + S.so + (int64_t)(ccl - S.c0) * len;
        bv[g] = Bp[ccl];
        bv[g] = (cok && rv) ? bv[g] : 0.0;
        if (h0) {
          av[g][0][0] = ld2(col + (q00 ? R0 : 0));
          av[g][0][1] = ld2(col + (q01 ? R0 + 2 : 0));
        }
        if (h1) {
          av[g][1][0] = ld2(col + (q10 ? R1 : 0));
          av[g][1][1] = ld2(col + (q11 ? R1 + 2 : 0));
        }
      }
#pragma unroll
      for (int g = 0; g < 4; g++) {
        if (h0) {
          acc[0][0] = mfma4(q00 ? av[g][0][0].x : 0.0, bv[g], acc[0][0]);
          acc[0][1] = mfma4(q00 ? av[g][0][0].y : 0.0, bv[g], acc[0][1]);
          acc[0][2] = mfma4(q01 ? av[g][0][1].x : 0.0, bv[g], acc[0][2]);
          acc[0][3] = mfma4(q01 ? av[g][0][1].y : 0.0, bv[g], acc[0][3]);
        }
        if (h1) {
          acc[1][0] = mfma4(q10 ? av[g][1][0].x : 0.0, bv[g], acc[1][0]);
          acc[1][1] = mfma4(q10 ? av[g][1][0].y : 0.0, bv[g], acc[1][1]);
          acc[1][2] = mfma4(q11 ? av[g][1][1].x : 0.0, bv[g], acc[1][2]);
          acc[1][3] = mfma4(q11 ? av[g][1][1].y : 0.0, bv[g], acc[1][3]);
        }
      }
    }
  }
  // lane holds vector m16, tile rows 64h + 16v + 4kq + t in acc[h][t][v]
  if (rv) {
    double* __restrict__ out = part + ((size_t)chunk * 16 + m16) * TILE;
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int row = 64 * h + 16 * v + 4 * kq;
        *reinterpret_cast<double2*>(out + row) = make_double2(acc[h][0][v], acc[h][1][v]);
        *reinterpret_cast<double2*>(out + row + 2) = make_double2(acc[h][2][v], acc[h][3][v]);
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

// Adaptive multiplication (Algorithm 2): dense-block products and the
// rank-two look-ahead contributions (A^_k - A_k)_b x_s, one workgroup per block.
__global__ __launch_bounds__(256) void k_dense_mv(const DenseMvTask* __restrict__ tasks,
                                                  const double* __restrict__ D,
                                                  const double* __restrict__ xp,
                                                  double* __restrict__ out) {
  const DenseMvTask T = tasks[blockIdx.x];
  const double* __restrict__ Db = D + T.d_off;
  const double* __restrict__ xs = xp + T.col0;
  for (int r = threadIdx.x; r < T.m; r += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < T.n; c++) acc += Db[(size_t)c * T.m + r] * xs[c];
    out[T.out + r] = acc;
  }
}

__global__ __launch_bounds__(256) void k_lowrank_delta(const DeltaTask* __restrict__ tasks,
                                                       const double* __restrict__ xp,
                                                       double* __restrict__ out) {
  __shared__ double red[2][256 / WAVE];
  const DeltaTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nl = T.r1 - T.r0;  // 1 or 2
  double w[2] = {0.0, 0.0};
  for (int l = 0; l < nl; l++) {
    const double* __restrict__ v = T.V + (size_t)(T.r0 + l) * T.n;
    double a = 0.0;
    for (int c = tid; c < T.n; c += blockDim.x) a += v[c] * xp[T.col0 + c];
    a = wave_sum(a);
    if (lane == 0) red[l][wv] = a;
  }
  __syncthreads();
  for (int l = 0; l < nl; l++) {
    double t = 0.0;
    for (int q = 0; q < 256 / WAVE; q++) t += red[l][q];
    w[l] = t;
  }
  for (int r = tid; r < T.m; r += blockDim.x) {
    double acc = 0.0;
    for (int l = 0; l < nl; l++) acc += T.U[(size_t)(T.r0 + l) * T.m + r] * w[l];
    out[T.out + r] = acc;
  }
}

hipError_t launch_dense_mv(const DenseMvTask* tasks, int n, const double* D, const double* xp,
                           double* out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_dense_mv, dim3(n), dim3(256), 0, s, tasks, D, xp, out);
  return hipGetLastError();
}

hipError_t launch_lowrank_delta(const DeltaTask* tasks, int n, const double* xp, double* out,
                                hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_lowrank_delta, dim3(n), dim3(256), 0, s, tasks, xp, out);
  return hipGetLastError();
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
__global__ __launch_bounds__(256) void k_from_stream(const StreamTask* __restrict__ tasks,
                                                     const double* __restrict__ stream) {
  const StreamTask T = tasks[blockIdx.x];
  const int len = T.row_hi - T.row_lo;
  const int64_t total = (int64_t)len * (T.c1 - T.c0);
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int64_t c = T.c0 + e / len;
    const int i = T.r0 + T.row_lo + (int)(e % len);
    if (i >= 0 && i < T.ld) T.dst[c * T.ld + i] = stream[T.so + e];
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
// GMRES helpers (FP64).

// Two-stage Q^T w: workgroup b takes rows [b*DOT_ROWS, (b+1)*DOT_ROWS) and writes
// part[b*ncols + c] = sum over its rows of Q[i, c] w[i]; k_proj sums over b.
constexpr int DOT_ROWS = 512;
__global__ __launch_bounds__(256) void k_dots_part(const double* __restrict__ Q, int64_t ldq,
                                                   int64_t n, int ncols,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ part) {
  extern __shared__ double red[];  // [NW][ncols]
  const int64_t i0 = (int64_t)blockIdx.x * DOT_ROWS + threadIdx.x;
  const int64_t i1 = i0 + 256;
  const double w0 = i0 < n ? w[i0] : 0.0, w1 = i1 < n ? w[i1] : 0.0;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  for (int c = 0; c < ncols; c++) {
    const double* q = Q + (size_t)c * ldq;
    double s = (i0 < n ? q[i0] * w0 : 0.0) + (i1 < n ? q[i1] * w1 : 0.0);
    s = wave_sum(s);
    if (lane == 0) red[wv * ncols + c] = s;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    double t = 0.0;
    for (int k = 0; k < NW; k++) t += red[k * ncols + c];
    part[(size_t)blockIdx.x * ncols + c] = t;
  }
}

// w -= Q[:, 0:ncols] h, where h[c] = sum_b part[b*ncols + c] (the partial dot
// products of k_dots_part, summed here by every workgroup into LDS). Block 0
// also folds h into the Hessenberg column acc (acc = h if assign, else
// acc += h). If normpart != nullptr, each workgroup writes the partial sum of
// squares of its updated rows to normpart[blockIdx.x].
constexpr int PROJ_MAX_COLS = 1025;
__global__ __launch_bounds__(256) void k_proj(const double* __restrict__ Q, int64_t ldq, int64_t n,
                                              int ncols, const double* __restrict__ part, int nblk,
                                              double* __restrict__ w, double* __restrict__ acc,
                                              int assign, double* __restrict__ normpart) {
  __shared__ double hs[PROJ_MAX_COLS];
  __shared__ double red[256 / WAVE];
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < nblk; b++) t += part[(size_t)b * ncols + c];
    hs[c] = t;
    if (acc && blockIdx.x == 0) acc[c] = assign ? t : acc[c] + t;
  }
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int c = 0; c < ncols; c++) s += Q[(size_t)c * ldq + i] * hs[c];
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
      for (int k = 0; k < 256 / WAVE; k++) t += red[k];
      normpart[blockIdx.x] = t;
    }
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

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

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

hipError_t launch_aca(const DevGeo& g, const AcaTask* tasks, int ntasks, size_t shmem,
                      int32_t* rank, int32_t* stop, double* ratio, hipStream_t s) {
  if (shmem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_aca<ACA_T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
  }
  if (ntasks > 0)
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_aca<ACA_T>), dim3(ntasks), dim3(ACA_T), shmem, s, g, tasks,
                       rank, stop, ratio);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_compact(const CopyTask* tasks, int ntasks, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_compact, dim3(ntasks), dim3(256), 0, s, tasks);
  return hipGetLastError();
}

hipError_t launch_gather(int nr, const double* x, int64_t ldx, const int32_t* order, int64_t N,
                         double* xp, int64_t ldxp, hipStream_t s) {
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
      mv_group_mfma<float>(P, P.far32, P.stream32, xp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
    }
  } else {
    if (nr <= 1) {
      if (unroll >= 16)
        mv_group<1, 16, double>(P, P.far, P.stream, xp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
      else
        mv_group<1, 8, double>(P, P.far, P.stream, xp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
    } else {
      mv_group_mfma<double>(P, P.far, P.stream, xp, ldxp, nr, z, ldz, part, y, ldy, s, ev);
    }
  }
  return hipGetLastError();
}

hipError_t launch_to_stream(const StreamTask* tasks, int ntasks, double* stream, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_to_stream, dim3(ntasks), dim3(256), 0, s, tasks, stream);
  return hipGetLastError();
}

hipError_t launch_from_stream(const StreamTask* tasks, int ntasks, const double* stream, hipStream_t s) {
  if (ntasks > 0) hipLaunchKernelGGL(k_from_stream, dim3(ntasks), dim3(256), 0, s, tasks, stream);
  return hipGetLastError();
}

// Scratch (doubles) for the partial dot products of launch_dots_part.
size_t dots_part_size(int64_t n, int ncols) { return (size_t)((n + DOT_ROWS - 1) / DOT_ROWS) * ncols; }

// part[b][c] = partial Q[:, c] . w over row block b (c < ncols); returns the block count.
int launch_dots_part(const double* Q, int64_t ldq, int64_t n, int ncols, const double* w,
                     double* part, hipStream_t s) {
  const int nblk = (int)((n + DOT_ROWS - 1) / DOT_ROWS);
  hipLaunchKernelGGL(k_dots_part, dim3(nblk), dim3(256), sizeof(double) * NW * ncols, s, Q, ldq, n,
                     ncols, w, part);
  return nblk;
}

// Partial-norm scratch (doubles) for n rows.
size_t norm_part_size(int64_t n) { return (size_t)((n + 255) / 256); }

hipError_t launch_proj(const double* Q, int64_t ldq, int64_t n, int ncols, const double* part,
                       int nblk, double* w, double* acc, int assign, double* normpart, hipStream_t s) {
  hipLaunchKernelGGL(k_proj, dim3(blocks_for(n, 256)), dim3(256), 0, s, Q, ldq, n, ncols, part, nblk,
                     w, acc, assign, normpart);
  return hipGetLastError();
}

// out[0] = ||w||_2 in two stages (normpart: norm_part_size(n) doubles).
hipError_t launch_norm(const double* w, int64_t n, double* normpart, double* out, hipStream_t s) {
  const int nblk = (int)blocks_for(n, 256);
  hipLaunchKernelGGL(k_sqnorm_part, dim3(nblk), dim3(256), 0, s, w, n, normpart);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, normpart, nblk, out);
  return hipGetLastError();
}

hipError_t launch_norm_final(const double* normpart, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, s, normpart, (int)blocks_for(n, 256), out);
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

}  // namespace hm
