// Device side of the adaptive matrix-vector multiplication (Algorithm 2,
// Sec. 3): the dense-block products of b_0, the look-ahead contributions
// d_b = (A^_k - A_k)_b x_s, the estimator's row errors, and the marking of
// P_k (step 3 b), so that a round sends only a few scalars and the order of
// the candidate blocks to the host.
//
// Marking, as the host would do it: rows in decreasing |e_i| (ties: lower row
// first); along them, every block with |(d_b)_i| >= tau joins P_k (blocks of
// a row in canonical order); stop after the first row at which
// ||sum_{b not in P_k} d_b|| <= (1 - theta) gamma_k. Here:
//   1. the rows are radix-sorted by (|e_i| descending, i ascending), giving
//      each row its rank in that order;
//   2. a block's key is the smallest rank among its rows with
//      |(d_b)_i| >= tau: the row at which it would join. Sorting the blocks by
//      (key, block) gives the order in which they join, and blocks with equal
//      keys join at the same row;
//   3. rest = e - sum of the joined d_b changes only in the rows of the
//      joining block. All rows of one leaf cluster lie in the same admissible
//      blocks, so a workgroup per leaf sorts that list by join position once
//      and runs rest_i through it in that order. Each step stores
//      rest_i^2(after) - rest_i^2(before) and rest_i(after);
//   4. ||rest||^2 after the first p blocks is gamma^2 plus the prefix sum of
//      the per-block changes. A scan over the sorted blocks finds the first
//      row boundary at which that sum falls below the goal, and the exact
//      norm of rest there, summed in a fixed order, confirms it.
// All reductions run in a fixed order, so every result is deterministic.
#include <hip/hip_runtime.h>

#include <hipcub/device/device_radix_sort.hpp>

#include <climits>

#include "device_common.hpp"
#include "hmat_internal.hpp"

namespace hm {

// ---------------------------------------------------------------------------
// b_0 and the look-ahead contributions, one workgroup per block.

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

// d_b for the listed blocks, list[j] = {block, r0, r1, source}: the window
// [r0, r1) with r1 = min(r0 + look, crosses available), the count read from
// avail (source 0) or avail2 (source 1), or r1 as given (source 2); a block
// without a window gets has_d = 0. tmpl[f] holds the block's panels, output
// offset, sizes and column offset (its r0, r1 are unused).
__global__ __launch_bounds__(256) void k_lowrank_delta(const DeltaTask* __restrict__ tmpl,
                                                       const int4* __restrict__ list,
                                                       const int32_t* __restrict__ avail,
                                                       const int32_t* __restrict__ avail2, int look,
                                                       const double* __restrict__ xp,
                                                       double* __restrict__ out, char* __restrict__ has_d) {
  __shared__ double red[2][256 / WAVE];
  const int4 L = list[blockIdx.x];
  const DeltaTask T = tmpl[L.x];
  const int r0 = L.y, r1 = L.w == 2 ? L.z : min(r0 + look, (L.w == 1 ? avail2 : avail)[L.x]);
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  if (tid == 0) has_d[L.x] = r1 > r0 ? 1 : 0;
  if (r1 <= r0) return;
  const int nl = r1 - r0;  // 1 or 2
  double w[2] = {0.0, 0.0};
  for (int l = 0; l < nl; l++) {
    const double* __restrict__ v = T.V + (size_t)(r0 + l) * T.n;
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
    for (int l = 0; l < nl; l++) acc += T.U[(size_t)(r0 + l) * T.m + r] * w[l];
    out[T.out + r] = acc;
  }
}

// The round's ACA tasks: out[j] = base[list[j].x] paused at list[j].y crosses.
__global__ void k_amvm_aca_tasks(const AcaTask* __restrict__ base, const int2* __restrict__ list, int n,
                                 AcaTask* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  AcaTask t = base[list[j].x];
  t.k_stop = list[j].y;
  out[j] = t;
}

// ---------------------------------------------------------------------------
// Estimator and marking.

constexpr int LEAF_T = 128;  // threads of the per-leaf kernels
constexpr int SCAN_T = 1024;

// Fixed-order sum of one value per thread over a workgroup of NT threads.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < NT / WAVE; q++) t += red[q];
  __syncthreads();
  return t;  // valid in thread 0
}

// Row errors e_i = sum over the leaf's blocks with a window, canonical order,
// of d_b[i]; the row sort keys; and per-leaf partial sums of e^2 and (b+e)^2.
__global__ __launch_bounds__(LEAF_T) void k_amvm_rows(const AmvmLeaf* __restrict__ leaves,
                                                      const int32_t* __restrict__ lblk,
                                                      const char* __restrict__ has_d,
                                                      const int64_t* __restrict__ dbase,
                                                      const double* __restrict__ d,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ e,
                                                      uint64_t* __restrict__ rkey,
                                                      int32_t* __restrict__ rval,
                                                      double* __restrict__ part) {
  extern __shared__ int64_t lb[];  // the leaf's blocks with a window (canonical order): dbase
  __shared__ double red[LEAF_T / WAVE];
  __shared__ int wcnt[LEAF_T / WAVE];
  const AmvmLeaf L = leaves[blockIdx.x];
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  int nk = 0;
  for (int q0 = 0; q0 < L.nb; q0 += LEAF_T) {  // ordered compaction
    const int q = q0 + threadIdx.x;
    int64_t o = -1;
    if (q < L.nb) {
      const int32_t f = lblk[L.b0 + q];
      if (has_d[f]) o = dbase[f];
    }
    const uint64_t bal = __ballot(o >= 0);
    if (lane == 0) wcnt[wv] = __popcll(bal);
    __syncthreads();
    int off = nk, tot = 0;
    for (int w = 0; w < LEAF_T / WAVE; w++) {
      off += w < wv ? wcnt[w] : 0;
      tot += wcnt[w];
    }
    if (o >= 0) lb[off + __popcll(bal & ((1ull << lane) - 1))] = o;
    nk += tot;
    __syncthreads();
  }
  double g = 0.0, h = 0.0;
  for (int r = threadIdx.x; r < L.nr; r += LEAF_T) {
    const int64_t i = L.r0 + r;
    double s = 0.0;
#pragma unroll 8
    for (int q = 0; q < nk; q++) s += d[lb[q] + i];
    e[i] = s;
    rkey[i] = ~(uint64_t)__double_as_longlong(fabs(s));  // descending |e|
    rval[i] = (int32_t)i;
    g += s * s;
    const double t = b[i] + s;
    h += t * t;
  }
  g = block_sum<LEAF_T>(g, red);
  h = block_sum<LEAF_T>(h, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = g;
    part[2 * blockIdx.x + 1] = h;
  }
}

// ctl->g2 = gamma_k^2 = ||e||^2, ctl->bh2 = ||b + e||^2 (fixed order over leaves).
__global__ __launch_bounds__(256) void k_amvm_norms(const double* __restrict__ part, int nl,
                                                    AmvmCtl* __restrict__ ctl) {
  __shared__ double red[256 / WAVE];
  double g = 0.0, h = 0.0;
  for (int l = threadIdx.x; l < nl; l += 256) {
    g += part[2 * l];
    h += part[2 * l + 1];
  }
  g = block_sum<256>(g, red);
  h = block_sum<256>(h, red);
  if (threadIdx.x == 0) {
    ctl->g2 = g;
    ctl->bh2 = h;
    ctl->ncand = 0;
    ctl->p_cand = 0;
    ctl->exact2 = 0.0;
  }
}

__global__ void k_amvm_rowrank(const int32_t* __restrict__ sorted_rows, int64_t n,
                               int32_t* __restrict__ rank) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < n) rank[sorted_rows[j]] = (int32_t)j;
}

// Block keys, one workgroup per admissible block: (first qualifying row rank)
// << 32 | block, or (N << 32) | block when no row qualifies or the block has
// no window. tau = (1 - theta) gamma_k / den with den = sqrt(c_sp M N). (A
// workgroup, not a wave: the largest blocks have thousands of rows.)
__global__ __launch_bounds__(256) void k_amvm_keys(const AmvmCtl* __restrict__ ctl, double theta, double den,
                                                   const char* __restrict__ has_d,
                                                   const int64_t* __restrict__ doff,
                                                   const int64_t* __restrict__ r0,
                                                   const int32_t* __restrict__ mrow,
                                                   const double* __restrict__ d,
                                                   const int32_t* __restrict__ rank, int64_t n,
                                                   uint64_t* __restrict__ key) {
  __shared__ int red[256 / WAVE];
  const int f = blockIdx.x;
  int best = INT_MAX;
  if (has_d[f]) {
    const double tau = (1.0 - theta) * sqrt(ctl->g2) / den;
    const double* __restrict__ df = d + doff[f];
    const int32_t* __restrict__ rk = rank + r0[f];
    const int m = mrow[f];
#pragma unroll 4
    for (int r = threadIdx.x; r < m; r += 256) {
      const double v = df[r];
      const int q = rk[r];
      if (fabs(v) >= tau) best = min(best, q);
    }
    best = wave_min(best);
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = best;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int w = 1; w < 256 / WAVE; w++) best = min(best, red[w]);
  }
  if (threadIdx.x == 0) key[f] = ((uint64_t)(best == INT_MAX ? n : best) << 32) | (uint32_t)f;
}

// Sorted keys -> order of the candidate blocks (sf), join positions (pos,
// INT_MAX for blocks that never join) and their count.
__global__ void k_amvm_pos(const uint64_t* __restrict__ skey, int nf, int64_t n, int32_t* __restrict__ sf,
                           int32_t* __restrict__ pos, AmvmCtl* __restrict__ ctl) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nf) return;
  const uint64_t k = skey[j];
  const int32_t f = (int32_t)(uint32_t)k;
  const bool cand = (int64_t)(k >> 32) < n;
  sf[j] = f;
  pos[f] = cand ? j : INT_MAX;
  if (cand && (j + 1 == nf || (int64_t)(skey[j + 1] >> 32) >= n)) ctl->ncand = j + 1;
}

// Per leaf: its candidate blocks sorted by join position (also stored to
// lsorted[b0 ..], parallel to the leaf's block list, with the count in lcount), then rest_i through them in that
// order: dsq = rest^2(after) - rest^2(before), restv = rest(after), stored at
// the block's entry of row i.
__global__ __launch_bounds__(LEAF_T) void k_amvm_rest(const AmvmLeaf* __restrict__ leaves,
                                                      const int32_t* __restrict__ lblk,
                                                      const int32_t* __restrict__ pos,
                                                      const int64_t* __restrict__ dbase,
                                                      const double* __restrict__ d,
                                                      const double* __restrict__ e,
                                                      int32_t* __restrict__ lsorted,
                                                      int32_t* __restrict__ lcount,
                                                      double* __restrict__ dsq,
                                                      double* __restrict__ restv) {
  extern __shared__ int64_t sm[];
  __shared__ int cnt;
  const AmvmLeaf L = leaves[blockIdx.x];
  int64_t* cb = sm;                      // [nb] compacted: dbase
  int64_t* sb = sm + L.nb;               // [nb] sorted: dbase
  int32_t* cp = (int32_t*)(sm + 2 * L.nb);  // [nb] compacted: pos
  int32_t* cf = cp + L.nb;               // [nb] compacted: block
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < L.nb; q += LEAF_T) {
    const int32_t f = lblk[L.b0 + q];
    const int32_t p = pos[f];
    if (p != INT_MAX) {
      const int slot = atomicAdd(&cnt, 1);
      cp[slot] = p;
      cf[slot] = f;
      cb[slot] = dbase[f];
    }
  }
  __syncthreads();
  const int nc = cnt;
  // positions are distinct: the rank of each is the count of smaller ones
  for (int q = threadIdx.x; q < nc; q += LEAF_T) {
    const int32_t p = cp[q];
    int rk = 0;
    for (int t = 0; t < nc; t++) rk += cp[t] < p ? 1 : 0;
    sb[rk] = cb[q];
    lsorted[L.b0 + rk] = cf[q];
  }
  if (threadIdx.x == 0) lcount[blockIdx.x] = nc;
  __syncthreads();
  for (int r = threadIdx.x; r < L.nr; r += LEAF_T) {
    const int64_t i = L.r0 + r;
    double rest = e[i];
#pragma unroll 4
    for (int q = 0; q < nc; q++) {
      const int64_t o = sb[q] + i;
      const double nr = rest - d[o];
      dsq[o] = nr * nr - rest * rest;
      restv[o] = nr;
      rest = nr;
    }
  }
}

// ds[j] = sum over the rows of the j-th candidate block of its dsq (one
// workgroup per candidate, fixed order).
__global__ __launch_bounds__(256) void k_amvm_blockdelta(const AmvmCtl* __restrict__ ctl,
                                                         const int32_t* __restrict__ sf,
                                                         const int64_t* __restrict__ doff,
                                                         const int32_t* __restrict__ mrow,
                                                         const double* __restrict__ dsq,
                                                         double* __restrict__ ds) {
  __shared__ double red[256 / WAVE];
  const int j = blockIdx.x;
  if (j >= ctl->ncand) return;
  const int32_t f = sf[j];
  const double* __restrict__ v = dsq + doff[f];
  const int m = mrow[f];
  double s = 0.0;
#pragma unroll 4
  for (int r = threadIdx.x; r < m; r += 256) s += v[r];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) ds[j] = s;
}

// First row boundary p > from (p = number of blocks in P_k, a boundary when
// block p lies in a later row than block p-1, or p = ncand) at which
// gamma^2 + sum_{j<p} ds[j] <= goal^2 (1 + 1e-6), goal = (1 - theta) gamma;
// ncand when there is none. One workgroup, inclusive scan per chunk.
__global__ __launch_bounds__(SCAN_T) void k_amvm_scan(AmvmCtl* __restrict__ ctl, const double* __restrict__ ds,
                                                      const uint64_t* __restrict__ skey, double theta,
                                                      int32_t from) {
  __shared__ double wt[SCAN_T / WAVE];
  __shared__ int first;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
  const int nc = ctl->ncand;
  const double g2 = ctl->g2;
  const double goal = (1.0 - theta) * sqrt(g2);
  const double lim = goal * goal * (1.0 + 1e-6);
  double carry = 0.0;
  if (tid == 0) first = INT_MAX;
  __syncthreads();
  for (int c0 = 0; c0 < nc; c0 += SCAN_T) {
    const int j = c0 + tid;
    double v = j < nc ? ds[j] : 0.0;
    for (int o = 1; o < WAVE; o <<= 1) {
      const double u = __shfl_up(v, o, WAVE);
      if (lane >= o) v += u;
    }
    if (lane == WAVE - 1) wt[wv] = v;
    __syncthreads();
    double off = carry;
    for (int q = 0; q < wv; q++) off += wt[q];
    double tot = carry;
    for (int q = 0; q < SCAN_T / WAVE; q++) tot += wt[q];
    const double S = g2 + (off + v);
    if (j < nc && j + 1 > from) {
      const bool boundary = j + 1 == nc || (skey[j + 1] >> 32) != (skey[j] >> 32);
      if (boundary && S <= lim) atomicMin(&first, j);
    }
    __syncthreads();
    if (first != INT_MAX) break;
    carry = tot;
  }
  if (tid == 0) ctl->p_cand = first == INT_MAX ? nc : first + 1;
}

// Load the leaf's sorted candidate list and count those before position p.
__device__ __forceinline__ int leaf_prefix(const AmvmLeaf& L, int nc, const int32_t* __restrict__ lsorted,
                                           const int32_t* __restrict__ pos, const int64_t* __restrict__ dbase,
                                           int32_t p, int64_t* sb, int* cnt) {
  if (threadIdx.x == 0) *cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int q = threadIdx.x; q < nc; q += LEAF_T) {
    const int32_t f = lsorted[L.b0 + q];
    sb[q] = dbase[f];
    mine += pos[f] < p ? 1 : 0;
  }
  if (mine) atomicAdd(cnt, mine);
  __syncthreads();
  return *cnt;  // sorted by position: the first cnt entries
}

// Exact ||rest||^2 after the first p_cand blocks: per-leaf partial sums.
__global__ __launch_bounds__(LEAF_T) void k_amvm_exact(const AmvmCtl* __restrict__ ctl,
                                                       const AmvmLeaf* __restrict__ leaves,
                                                       const int32_t* __restrict__ lsorted,
                                                       const int32_t* __restrict__ lcount,
                                                       const int32_t* __restrict__ pos,
                                                       const int64_t* __restrict__ dbase,
                                                       const double* __restrict__ e,
                                                       const double* __restrict__ restv,
                                                       double* __restrict__ part) {
  extern __shared__ int64_t sb[];
  __shared__ int cnt;
  __shared__ double red[LEAF_T / WAVE];
  const AmvmLeaf L = leaves[blockIdx.x];
  const int32_t p = ctl->p_cand;
  const int n = leaf_prefix(L, lcount[blockIdx.x], lsorted, pos, dbase, p, sb, &cnt);
  double s = 0.0;
  for (int r = threadIdx.x; r < L.nr; r += LEAF_T) {
    const int64_t i = L.r0 + r;
    const double v = n > 0 ? restv[sb[n - 1] + i] : e[i];
    s += v * v;
  }
  s = block_sum<LEAF_T>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_amvm_exact_sum(const double* __restrict__ part, int nl,
                                                        AmvmCtl* __restrict__ ctl) {
  __shared__ double red[256 / WAVE];
  double s = 0.0;
  for (int l = threadIdx.x; l < nl; l += 256) s += part[l];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) ctl->exact2 = s;
}

// A_{k+1} = A^_k on the first p blocks: b_i += d_b[i] in join order.
__global__ __launch_bounds__(LEAF_T) void k_amvm_update(const AmvmLeaf* __restrict__ leaves,
                                                        const int32_t* __restrict__ lsorted,
                                                        const int32_t* __restrict__ lcount,
                                                        const int32_t* __restrict__ pos,
                                                        const int64_t* __restrict__ dbase,
                                                        const double* __restrict__ d, int32_t p,
                                                        double* __restrict__ b) {
  extern __shared__ int64_t sb[];
  __shared__ int cnt;
  const AmvmLeaf L = leaves[blockIdx.x];
  const int n = leaf_prefix(L, lcount[blockIdx.x], lsorted, pos, dbase, p, sb, &cnt);
  if (n == 0) return;
  for (int r = threadIdx.x; r < L.nr; r += LEAF_T) {
    const int64_t i = L.r0 + r;
    double v = b[i];
#pragma unroll 8
    for (int q = 0; q < n; q++) v += d[sb[q] + i];
    b[i] = v;
  }
}

// y[3 order[t] + a] = b[3 t + a]: the result in the caller's order.
__global__ void k_amvm_out(const double* __restrict__ b, const int32_t* __restrict__ order, int64_t n,
                           double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[3 * (int64_t)order[i / 3] + i % 3] = b[i];
}

// ---------------------------------------------------------------------------
// Launchers.

hipError_t launch_dense_mv(const DenseMvTask* tasks, int n, const double* D, const double* xp,
                           double* out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_dense_mv, dim3(n), dim3(256), 0, s, tasks, D, xp, out);
  return hipGetLastError();
}

hipError_t launch_lowrank_delta(const DeltaTask* tmpl, const int4* list, int n, const int32_t* avail,
                                const int32_t* avail2, int look, const double* xp, double* out, char* has_d,
                                hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_lowrank_delta, dim3(n), dim3(256), 0, s, tmpl, list, avail, avail2, look, xp, out, has_d);
  return hipGetLastError();
}

hipError_t launch_amvm_aca_tasks(const AcaTask* base, const int2* list, int n, AcaTask* out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_amvm_aca_tasks, dim3(blocks_for(n, 256)), dim3(256), 0, s, base, list, n, out);
  return hipGetLastError();
}

size_t amvm_sort_bytes(int64_t n, int nf) {
  size_t a = 0, b = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0, 64);
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr, nf, 0, 64);
  return std::max<size_t>(std::max(a, b), 1);
}

size_t amvm_leaf_shmem(int nbmax) { return 32 * (size_t)std::max(nbmax, 1); }

hipError_t launch_amvm_estimate(const AmvmDev& A, double theta, double den, hipStream_t s) {
  const int nl = A.n_leaves;
  hipLaunchKernelGGL(k_amvm_rows, dim3(nl), dim3(LEAF_T), 8 * (size_t)std::max(A.nbmax, 1), s, A.leaves, A.lblk,
                     A.has_d, A.dbase, A.d, A.b, A.e, A.rkey, A.rval, A.part);
  hipLaunchKernelGGL(k_amvm_norms, dim3(1), dim3(256), 0, s, A.part, nl, A.ctl);
  size_t tb = A.sort_bytes;
  hipError_t err = hipcub::DeviceRadixSort::SortPairs(A.sort_tmp, tb, A.rkey, A.rkey + A.n, A.rval, A.rval + A.n,
                                                      (int)A.n, 0, 64, s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_amvm_rowrank, dim3(blocks_for(A.n, 256)), dim3(256), 0, s, A.rval + A.n, A.n, A.rank);
  if (A.nf == 0) return hipGetLastError();  // no admissible blocks: nothing to mark
  hipLaunchKernelGGL(k_amvm_keys, dim3(A.nf), dim3(256), 0, s, A.ctl, theta, den, A.has_d, A.doff, A.r0, A.mrow,
                     A.d, A.rank, A.n, A.bkey);
  int bits = 32;
  while (bits < 64 && ((int64_t)1 << (bits - 32)) <= A.n) bits++;
  tb = A.sort_bytes;
  err = hipcub::DeviceRadixSort::SortKeys(A.sort_tmp, tb, A.bkey, A.bkey + A.nf, A.nf, 0, bits, s);
  if (err != hipSuccess) return err;
  const uint64_t* skey = A.bkey + A.nf;
  hipLaunchKernelGGL(k_amvm_pos, dim3(blocks_for(A.nf, 256)), dim3(256), 0, s, skey, A.nf, A.n, A.sf, A.pos, A.ctl);
  hipLaunchKernelGGL(k_amvm_rest, dim3(nl), dim3(LEAF_T), amvm_leaf_shmem(A.nbmax), s, A.leaves, A.lblk, A.pos,
                     A.dbase, A.d, A.e, A.lsorted, A.lcount, A.dsq, A.restv);
  hipLaunchKernelGGL(k_amvm_blockdelta, dim3(A.nf), dim3(256), 0, s, A.ctl, A.sf, A.doff, A.mrow, A.dsq, A.ds);
  return hipGetLastError();
}

hipError_t launch_amvm_stop(const AmvmDev& A, double theta, int32_t from, hipStream_t s) {
  if (A.nf == 0) return hipGetLastError();  // ncand = p_cand = 0 from k_amvm_norms
  hipLaunchKernelGGL(k_amvm_scan, dim3(1), dim3(SCAN_T), 0, s, A.ctl, A.ds, A.bkey + A.nf, theta, from);
  hipLaunchKernelGGL(k_amvm_exact, dim3(A.n_leaves), dim3(LEAF_T), 8 * (size_t)std::max(A.nbmax, 1), s, A.ctl,
                     A.leaves, A.lsorted, A.lcount, A.pos, A.dbase, A.e, A.restv, A.part);
  hipLaunchKernelGGL(k_amvm_exact_sum, dim3(1), dim3(256), 0, s, A.part, A.n_leaves, A.ctl);
  return hipGetLastError();
}

hipError_t launch_amvm_update(const AmvmDev& A, int32_t p, hipStream_t s) {
  if (p > 0)
    hipLaunchKernelGGL(k_amvm_update, dim3(A.n_leaves), dim3(LEAF_T), 8 * (size_t)std::max(A.nbmax, 1), s,
                       A.leaves, A.lsorted, A.lcount, A.pos, A.dbase, A.d, p, A.b);
  return hipGetLastError();
}

hipError_t launch_amvm_out(const double* b, const int32_t* order, int64_t n, double* y, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_amvm_out, dim3(blocks_for(n, 256)), dim3(256), 0, s, b, order, n, y);
  return hipGetLastError();
}

}  // namespace hm
