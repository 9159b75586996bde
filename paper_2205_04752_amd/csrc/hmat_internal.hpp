// Internal declarations shared by the host planner, the kernels and the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "hmat.h"

namespace hm {

// Task and descriptor records handed to the kernels (plain data, identical
// layout on host and device).

// Geometry in cluster order p (see Geometry below). Kelvin tensor
// S = c1 delta/|r| + c2 r r^T/|r|^3 with c1 = cK (3 - 4 nu), c2 = cK,
// cK = (1+nu)/(8 pi E (1-nu)) (Sec. 4.1). kc holds c1 and c2 per triangle
// (several bodies with their own E, nu may share one geometry); a kernel
// copies the constants of the body it works on into c1, c2, which the entry
// functions read.
struct DevGeo {
  const double* cen;  // [3][nt]
  const double* q;    // [4][7][nt]: x, y, z, weight*area
  const double* vtx;  // [9][nt]: p0x p0y p0z p1x ... p2z
  const double* gl;   // [2][16] Gauss-Legendre nodes and weights on [0,1]
  const double* kc;   // [2][nt]: c1, c2 of the triangle's body
  const float* cen32; // FP32 copies of cen and q (FP32 ACA only; else null)
  const float* q32;
  int32_t nt;
  int32_t pad;
  double c1, c2;
};

// Row alignment of the stored block matrices. A V panel whose rows are the
// global DOFs [R0, R0 + M) keeps row i of column c at base + c*ld + fp + i,
// with fp = R0 mod PANEL_ALIGN, ld a multiple of PANEL_ALIGN >= fp + M and base
// a multiple of PANEL_ALIGN: global DOF g sits at an address congruent to g
// modulo PANEL_ALIGN doubles, so a lane reads the row pair (2j, 2j+1) with one
// 16-byte load. The product-order stream widens block row ranges to even rows
// the same way (STREAM_ALIGN) and starts every segment on a 128-byte line
// (SEG_START_ALIGN), so no line is shared by two segments. Pad entries are zero.
constexpr int PANEL_ALIGN = 2;       // doubles (16 bytes)
constexpr int STREAM_ALIGN = 2;      // doubles (16 bytes)
constexpr int SEG_START_ALIGN = 16;  // doubles (128 bytes)
// ACA runs one 256-thread workgroup per block, or one wave per block for
// blocks with at most ACA_SMALL_TRI triangles on either side (the launch
// takes the large blocks first, then the small ones).
constexpr int ACA_SMALL_TRI = 64;
constexpr int ACA_NWV = 4;       // waves of the ACA workgroup for large blocks
constexpr int ACA_WIDE_NWV = 8;  // the same in launches of few blocks (one per CU)
// Adaptive multiplication: admissible blocks with m + n >= AMVM_AHEAD_ROWS run
// their look-ahead ACA steps one round ahead, on a stream of their own.
constexpr int64_t AMVM_AHEAD_ROWS = 2048;
// Adaptive multiplication: blocks with at most AMVM_SMALL_TRI triangles on both
// sides resume ACA one wave each (two steps per round: a workgroup would idle;
// 256 against 64, 128 and 512 cut the ellipsoid's AMVM 53 -> 45 ms).
constexpr int AMVM_SMALL_TRI = 256;
// A block with m + n <= ACA_STAGE_MAX keeps the newest row and column of
// its remainder in LDS as well as in the panels, so the pivot searches,
// the normalisation and the norm update of a step read them from LDS.
constexpr int ACA_STAGE_MAX = 7936;
// Size (doubles) of the per-device workspace of the allocation-free solve:
// 32 MiB, enough for GMRES(50) at 61440 DOF (Krylov basis, work vector,
// partial sums and Hessenberg columns).
constexpr size_t NOALLOC_DOUBLES = size_t(4) << 20;
// Dynamic LDS (bytes) of the ACA kernel for one block and a workgroup of
// nwv waves, panel entries of esize bytes: the cross-term weights (kcap
// doubles), the per-wave partial sums of V^T v_c (kcap * nwv doubles), the
// coefficient row (kcap entries, padded to a double), the row set Z (m bits,
// in 32-bit words, padded to a double) and, if staged, the newest row and
// column (n + m entries).
inline size_t aca_shmem(int kcap, int64_t m, int64_t n, int nwv, int esize = 8) {
  const size_t zw = (size_t)((m + 31) / 32);
  return 8 * (size_t)kcap * (1 + nwv) + 8 * (((size_t)kcap * esize + 7) / 8) + 8 * ((zw + 1) / 2) +
         (m + n <= ACA_STAGE_MAX ? (size_t)esize * (size_t)(m + n) : 0);
}

// Dense (non-admissible) block at d_off in the near arena (m = 3 t_len rows).
struct NearTask {
  int32_t t_off, t_len, s_off, s_len;
  int64_t d_off;
  int32_t ld, fp;
};

// Self entry of cluster position p: lives in the diagonal dense block at d_off
// with leading dimension ld and front pad fp, local triangle index ploc.
struct SelfTask {
  int64_t d_off;
  int32_t ld, fp, ploc, pad;
};

// ACA task: scratch panels U (m x kcap) then V (n x kcap), plain column-major, at `panel`.
// Resumable ACA state of one block (adaptive multiplication): steps taken,
// next pivot row, rows used, last stop code (6: paused), row classes visited
// (bit c: a row of component c was used), accuracy test passed while a class
// was unvisited, ||S_k||_F^2, last stop ratio.
struct AcaState {
  int32_t k, i, nZ, stop, visited, pending;
  int32_t pc, pad;  // pc = 1: the test of cross k - 1 is not settled (its |u|^2, |v|^2 in puu, pvv)
  double S2, ratio, puu, pvv;
};

struct AcaTask {
  int32_t t_off, t_len, s_off, s_len;
  void* panel;    // U (m x kcap) then V (n x kcap), column-major, in the ACA precision
  int32_t* piv;   // [2][kcap]: pivot rows, pivot columns
  int32_t kcap;
  int32_t blk;    // index into the far-block result arrays
  double eps;     // ACA accuracy of the block's body
  AcaState* st;   // null: start from scratch; else resume from and save to *st
  uint32_t* zbits;  // with st: the block's set Z of used rows, (m + 31) / 32 words
  int32_t k_stop;   // > 0: pause (stop code 6) once k reaches k_stop
  int32_t cycle;    // 1: class-cycling rows (step-limited runs of the adaptive multiplication)
};

// Adaptive multiplication: out[out + r] = (D x)_r for a dense block (D plain
// column-major m x n at d_off of the dense staging arena, x entries from
// xp[col0 ...]).
struct DenseMvTask {
  int64_t d_off, out;
  int32_t m, n, col0, pad;
};

// Adaptive multiplication: out[out + r] = sum_{l in [r0, r1)} U[r, l] (V[:, l] . x)
// for one admissible block's ACA panels (U m x ldk, V n x ldk, column-major).
struct DeltaTask {
  const double* U;
  const double* V;
  int64_t out;
  int32_t m, n, r0, r1, col0, pad;
};

// Adaptive multiplication, marking on the device: a leaf cluster's rows
// [r0, r0 + nr) all lie in the same admissible blocks, listed (canonical
// order) at lblk[b0 .. b0 + nb).
struct AmvmLeaf {
  int64_t r0, b0;
  int32_t nr, nb;
};

// Scalars of one round, kept on the device.
struct AmvmCtl {
  double g2;      // gamma_k^2 = ||b^_k - b_k||^2
  double bh2;     // ||b^_k||^2
  double exact2;  // ||rest||^2 after the first p_cand candidate blocks
  int32_t ncand;  // blocks that would join P_k if marking ran through every row
  int32_t p_cand; // candidate size of P_k
};

// Device arrays of the marking (see amvm.hip). n rows, nf admissible blocks;
// rkey/rval and bkey hold the sort input followed by its output.
struct AmvmDev {
  const AmvmLeaf* leaves;
  int n_leaves, nbmax, nf, pad;
  int64_t n;
  const int32_t* lblk;
  const char* has_d;
  const int64_t *dbase, *doff, *r0;  // dbase = doff - r0: entry of row i at dbase + i
  const int32_t* mrow;
  const double* d;
  double *b, *e, *part, *dsq, *restv, *ds;
  uint64_t *rkey, *bkey;
  int32_t *rval, *rank, *sf, *pos, *lsorted, *lcount;
  AmvmCtl* ctl;
  void* sort_tmp;
  size_t sort_bytes;
};

// One contiguous copy of `words` 32-bit words (the panels and pivots of a
// block carried into the next, larger ACA pass).
struct SpanCopy {
  const uint32_t* src;
  uint32_t* dst;
  int64_t words;
};

// A block whose ACA reached full rank, stored exactly in its panels (U m x
// kcap, V n x kcap): U = B, V = I for n <= m, else U = I, V = B^T.
struct ExactTask {
  int32_t t_off, t_len, s_off, s_len;
  void* panel;
  int32_t kcap, pad;
};

// Compaction of the V factors: copy the first k columns of a scratch panel
// (n x kcap, leading dimension n) into the panel layout above.
struct CopyTask {
  const double* srcV;
  double* dstV;  // column c, row i at dstV[c*ldv + fpv + i]
  int32_t n, k, ldv, fpv;
};

// The same from an FP32 panel into an FP64 staging buffer (FP32 ACA).
struct CopyTask32 {
  const float* srcV;
  double* dstV;
  int32_t n, k, ldv, fpv;
};

// Product, phase A: z[zoff + l - l0] = V[:, l] . xp[window] for l in [l0, l1).
// The window is the aligned row range [a0, a0 + ld) of V (global DOFs).
// Right-hand sides per pass over the matrix. With nr > 1 of them, the
// product's gathered input and its Vᵀx results hold a row's nr vector entries
// side by side (entry (row, r) at row * nr + r).
constexpr int MV_MAX_NR = 16;

struct MvA {
  int64_t v_off;  // V base (row a0 of column 0) in the far arena
  int32_t ld, l0, l1, a0;
  int32_t zoff, pad;
};

// Product, phase B. The U factors and the dense blocks are stored in the order
// phase B reads them ("stream" arena): 128-row tile by tile, and within a tile
// segment by segment, each segment being one block's rows [row_lo, row_hi) of
// the tile (multiples of 16) times its columns [c0, c1), column by column. The
// slice of column c starts at so + (c - c0) * (row_hi - row_lo); the vector
// entry for column c is src[soff + c] with src = z (far) or xp (near).
struct MvSeg {
  int64_t so;
  int32_t c0, c1, soff;
  int16_t row_lo, row_hi;
  int32_t far;  // 1: low-rank block (vector z); 0: dense block (vector xp)
  int32_t pad;
};

// Copy between a plain column-major block matrix (leading dimension ld = its
// row count m) and one stream segment. Tile row r is block row r0 + r; rows
// outside [0, m) are zero in the stream.
struct StreamTask {
  const double* src;
  double* dst;
  int64_t so;
  int32_t ld, r0, row_lo, row_hi, c0, c1;
};

struct MvChunk {
  int32_t tile, seg_lo, seg_hi, pad;
};

// Device pointers and sizes of a product plan (passed to the launchers).
// Chunks: dense-block chunks [0, n_near_chunks), then low-rank chunks.
struct ProductPlanDev {
  const MvA* items;
  const MvChunk* chunks;
  const MvSeg* segs;
  const int32_t* tile_near;  // [ntiles + 1] chunk ranges per tile
  const int32_t* tile_far;   // [ntiles + 1]
  const int32_t* order;
  const double* far;         // V panels
  const double* stream;      // U factors and dense blocks in product order
  const float* far32;        // FP32 copies of the two (reduced-precision storage), or null
  const float* stream32;
  int32_t nA, n_near_chunks, n_far_chunks, ntiles;
  int64_t N;
};

// ----------------------------------------------------------------------------
// Host planner (planner.cpp).

struct Cluster {
  int32_t off, len, son0, son1, level;
  double lo[3], hi[3];  // box of the vertices of the cluster's triangles
};

struct BlockRec {
  int32_t t, s;  // cluster ids
  int32_t far;
};

struct Plan {
  int32_t nt = 0;
  std::vector<int32_t> order;  // cluster position -> caller's triangle
  std::vector<Cluster> cl;
  std::vector<BlockRec> blk;   // canonical order (row_off, col_off)
  int32_t csp = 0, depth = 0;
};

struct HostGeometry {  // cluster order, SoA as in DevGeo
  std::vector<double> cen, q, vtx, gl;
};

// Returns HMAT_OK or HMAT_EINVAL with a message.
hmat_status validate_mesh(const hmat_mesh* mesh, std::string& err);
hmat_status validate_params(double E, double nu, double eta, int32_t leaf, double eps,
                            std::string& err);
void make_plan(const hmat_mesh* mesh, double eta, int32_t leaf, Plan& plan);
void make_geometry(const hmat_mesh* mesh, const Plan& plan, HostGeometry& g);
void gauss_legendre_unit(int n, double* x, double* w);  // rule on [0,1]

// Cap on the ACA panel memory of builds made by the calling thread (0: the
// default, a quarter of the free device memory). Used by the request server,
// whose workers build concurrently.
void set_thread_aca_budget(int64_t bytes);
// A request server starts (true) or ends (false): while any runs, freed
// device memory is kept in the pool up to 64 GiB instead of 4 GiB (see
// init_pool in api.cpp).
void serving_pool(bool begin);
void radon7(double bary[7][3], double w[7]);
// Indices of `key` in decreasing key order, equal keys in increasing index
// order (stable radix sort; planner.cpp).
std::vector<int32_t> order_desc_stable(const std::vector<uint64_t>& key);

}  // namespace hm
