// Internal declarations shared by the HIP translation units of librelsim.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "relsim.h"

namespace relsim {

// Constants handed to every particle/grid kernel by value.
struct KParams {
  int dim, nx, ny, nz, ncells, nspecies, nbins, nonrel;
  int tx, ty, tz;     // tile extents of the particle kernels' cell order (powers of two dividing nx, ny, nz)
  int sty, stz;       // y and z extents of the push passes' segment tiles (powers of two dividing ny, nz)
  int ltx, lty, ltz;  // their base-2 logarithms
  int ntx, nty;       // tiles along x and y
  int gx, gxy;        // strides of the ghosted field copies: nx + 2, (nx + 2)(ny + 2)
  int nghost;         // points of a ghosted field copy
  double dx, dy, dz, dt, c, theta, V;
  double inv_dx, inv_dy, inv_dz, inv_c, inv_c2, inv_V;
  double q[8], m[8], beta[8];
  // the same constants rounded to FP32 once on the host (mixed precision)
  float f_dt, f_inv_c, f_inv_c2, f_inv_V, f_inv_dx, f_inv_dy, f_inv_dz;
  float f_q[8], f_beta[8];
};

// Offsets (in bytes) of the regions carved out of the caller's workspace.
struct Layout {
  size_t S, cnt, pre, total, scan_tmp, dirc, err, gm_V, gm_t, gm_b, gm_r, gm_part, gm_small, red_part;
  size_t gs_k0, gs_k1, gs_v0, gs_v1, gs_hist, stB, stE, sink, kin_part, push_ke, end;
};

constexpr int kMaxRestart = 64;
constexpr int kDotBlocks = 1024;    // blocks of the multi-dot reduction
constexpr int kRedBlocks = 1024;    // blocks of the energy reductions
constexpr int kSinkSlots = 512;     // per-lane store sinks of the particle kernels (power of two), 32 B each

// Moments per cell: 2D 81 mass moments + 12 current moments; 3D 3 x 81 mass
// moments (one set per z-monomial type) plus 2 x 12 current moments.
inline int n_cell_moments(int dim) { return dim == 3 ? 3 * 81 + 2 * 12 : 81 + 12; }

// Per-cell moments in memory (93 per cell in 2D, 267 in 3D): blocks of 64
// consecutive cells, each block holding its moments as 64-cell rows, moment
// m of cell c at ((c / 64) nmom + m) 64 + c % 64.  A deposit wave (8 or 16
// consecutive cells) then writes its moment pieces inside one block, a few
// DRAM pages, instead of one page per moment plane; the assembly's wave (64
// consecutive nodes) still reads 256 contiguous bytes per moment.  Room:
// ncells rounded up to a multiple of 64.
constexpr int kMomBlock = 64;
template <int DIM>
__host__ __device__ inline size_t mom_index(int m, int c) {
  constexpr size_t NM = DIM == 3 ? 267 : 93;
  return ((size_t)(c >> 6) * NM + (size_t)m) * kMomBlock + (size_t)(c & (kMomBlock - 1));
}

inline int n_dirs(int dim) { return dim == 3 ? 27 : 9; }

// Mass-matrix storage.  The node-pair block of the linearised current is
// symmetric in the pair, M_{g,g'} = M_{g',g} as one 3x3 block (Sec. 2: both
// are sums of W_g W_g' alpha_p over the same particles), so of the 3^dim
// offsets only the upper half in the offset order (x fastest) is stored:
// slot h in [0, m_slots) of node g holds M_{g, g+delta(m_centre + h)}; the
// block of the mirrored offset -delta at node g is slot h of node g - delta.
template <int DIM>
__host__ __device__ constexpr int m_slots() { return DIM == 3 ? 14 : 5; }
template <int DIM>
__host__ __device__ constexpr int m_centre() { return DIM == 3 ? 13 : 4; }

// Node order of the field solve's per-node kernels (S4 operator, curls,
// right-hand side, update): 64-node chunks of x-rows, the rows taken in slabs
// of kStrip consecutive z-planes swept along y, z fastest inside a slab.  A
// node reads rows k-1 and j-1 (the mirrored mass-matrix slots, the curl
// cubes); in this order they were read one and kStrip rows earlier and are
// still in the L2, where the plain order read the row at k-1 a whole z-plane
// earlier.  The chunks in flight stay within kStrip planes.  In 2D it is the
// plain order.  Blocks of 256 threads take 4 chunks.
constexpr int kStrip = 4;
inline int grid_node_blocks(int nx, int ny, int nz) { return (((nx + 63) >> 6) * ny * nz + 3) >> 2; }
// chunk L (of the grid's ((nx + 63) / 64) ny nz), lane in [0, 64) -> node
// (i, j, k) and its linear index, or -1 past the grid
__device__ __forceinline__ int strip_node(int nx, int ny, int nz, int L, int lane, int &i, int &j, int &k) {
  const int nxc = (nx + 63) >> 6;
  const int xc = L % nxc, q = L / nxc;
  const int S = nz % kStrip == 0 ? kStrip : 1;
  const int per = S * ny;
  const int kb = q / per, r = q - kb * per;
  j = r / S;
  k = kb * S + (r - j * S);
  i = xc * 64 + lane;
  return (i < nx && k < nz) ? i + nx * (j + ny * k) : -1;
}

// Packed records: a ghosted field point (three components and a pad) or a
// particle's (u_x, u_y, u_z, w); a particle's (off_x, off_y).
template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T x, y, z, w;
};
template <typename T>
struct alignas(2 * sizeof(T)) V2 {
  T x, y;
};

// ---- particle kernels (particles.hip) ----
// Particle arrays of one buffer set (element type T = float or double):
// 2D: xy [n] of (off_x, off_y), uw [n] of (u_x, u_y, u_z, w); 3D: xy [n] of
// 8-value records (off_x, off_y, off_z, 0, u_x, u_y, u_z, w), uw and z unused.
struct PartPtrs {
  const int32_t *bin_start;
  void *xy;
  void *uw;
  void *z;
  const void *gbar = nullptr;  // per-particle gbar of the energy-conserving variant, or null
};

// Ghosted, component-interleaved copy of a grid vector field (SoA FP64 on
// nodes or centres) in the particle arithmetic type: point (i, j, k) with
// i in [-1, nx], ... at (i + 1) + gx (j + 1) [+ gxy (k + 1)], 4 values each.
void launch_stage_field(const KParams &kp, int prec, const double *F, void *out, hipStream_t st);
void launch_deposit_cells(const KParams &kp, int prec, int group, const PartPtrs &pp, const void *Bst, void *S,
                          hipStream_t st);
void launch_assemble(const KParams &kp, int prec, int mass_fp32, const void *S, double *J, void *M,
                     hipStream_t st);
// `sink`: kSinkSlots * 64 * 32 bytes of workspace that lanes without a
// particle store into (contents meaningless)
// The push passes give each wave `cells` consecutive cells of one grid row
// (a power of two dividing nx); push_lds_bytes is the LDS one wave stages.
// count_moves: only read the particles and write each one's move (dirc) and
// the per-(move, bin) counts (first pass of the re-sort); else push in place
size_t push_lds_bytes(const KParams &kp, int prec, int cells);
void launch_push(const KParams &kp, int prec, int cells, const PartPtrs &pp, const void *Est, const void *Bst,
                 uint8_t *dirc, uint16_t *cnt, int32_t *err, int count_moves, void *sink, hipStream_t st);
// The energy-conserving variant's fixed-point pass: pushes each particle
// with pp.gbar (gamma(u^n) if null) without touching the state, writes
// gbar_next = (gamma(u^n) + gamma(u^{n+1}))/2 and raises *chg to the bits of
// max |gbar_next - gbar| / gbar.
void launch_gamma_mean(const KParams &kp, int prec, int cells, const PartPtrs &pp, const void *Est,
                       const void *Bst, int32_t *err, void *sink, void *gbar_next, unsigned long long *chg,
                       hipStream_t st);
// one secant step per particle of the energy-conserving fixed point
void launch_gamma_secant(int prec, int n, const void *g, void *Fg, void *gp, void *rp, int first, hipStream_t st);
void launch_sort_offsets(const KParams &kp, const uint16_t *cnt, uint16_t *pre, int32_t *total, int32_t *err,
                         hipStream_t st);
void launch_scan(const int32_t *in, int32_t *out, int n, int32_t *tmp, hipStream_t st);
size_t scan_tmp_elems(int n);
// second pass of the re-sort: push src again and write the new state into
// out in the new bin order, each in the cell of its recorded move (err bit
// 8: a recomputed position further than rounding outside that cell; *clamps
// += particles within rounding outside it, put on its face).  kep[w] gets
// the FP64 kinetic energy of the particles wave w pushed (ncells / cells
// waves; w in the segment order).
void launch_push_scatter(const KParams &kp, int prec, int cells, const PartPtrs &src, const void *Est,
                         const void *Bst, const uint8_t *dirc, const uint16_t *pre, const int32_t *bin_start_new,
                         const PartPtrs &out, int ntot, int32_t *err, unsigned long long *clamps, int32_t *perm,
                         void *sink, double *kep, hipStream_t st);
// cell[p] for every particle from the bin ranges
void launch_fill_cells(const KParams &kp, const int32_t *bin_start, int32_t *cell, hipStream_t st);
// partials: one double per block of 64/group cells (at most ncells)
void launch_kinetic(const KParams &kp, int prec, int group, const PartPtrs &pp, double *partials, hipStream_t st);

// ---- general stable sort by bin (sort.hip) ----
size_t gsort_tmp_elems(int64_t n);  // int32 elements of scratch for the histograms
void launch_gsort(const KParams &kp, int prec, int64_t n, const int32_t *cell, const uint8_t *species, const PartPtrs &src,
                  int32_t *keys0, int32_t *keys1, int32_t *vals0, int32_t *vals1, int32_t *hist, int32_t *scan_tmp,
                  int32_t *err, int32_t *bin_start_out, int32_t *cell_out, const PartPtrs &out, hipStream_t st);

// ---- adjoint kernels (adjoint.hip), FP64 particle state ----
struct AdjInPtrs {
  const int32_t *bin_start = nullptr;
  const int32_t *cell = nullptr;
  const double *xy = nullptr;  // 2D: [n] (off_x, off_y); 3D: [n] 8-value records
  const double *uw = nullptr;  // 2D: [n] (u_x, u_y, u_z, w); unused in 3D
  const double *z = nullptr;   // unused
};
void launch_push_adjoint(const KParams &kp, const AdjInPtrs &in, int n, const double *Eth, const double *B,
                         const int32_t *new_index, const double *lx_in, const double *lu_in, double *lx_out,
                         double *lu_out, double *lEth, double *lB, hipStream_t st);
void launch_deposit_adjoint(const KParams &kp, const AdjInPtrs &in, int n, const double *B, const double *Eth,
                            const double *mu, double *lx_out, double *lu_out, double *lB, hipStream_t st);
void launch_adj_rhs(size_t n3, double theta, double cdt, const double *lth, const double *lE1, const double *ccn_lB1,
                    double *out, hipStream_t st);
void launch_adj_finish(size_t n3, double theta, double ctdt, const double *lE1, const double *lB1, const double *mu,
                       const double *cnc_mu, double *lEn, double *lBn, hipStream_t st);

// ---- field kernels (field.hip) ----
void launch_curl(const KParams &kp, const double *in, double *out, int to_centres, hipStream_t st);
// M: the stored half of the mass matrix, float if mass_fp32, else double
void launch_apply_A_tail(const KParams &kp, int mass_fp32, const void *M, const double *x, const double *t,
                         double *out, hipStream_t st);
void launch_apply_AT_tail(const KParams &kp, int mass_fp32, const void *M, const double *x, const double *t,
                          double *out, hipStream_t st);
void launch_rhs(const KParams &kp, const double *En, const double *Bn, const double *J, double *out, hipStream_t st);
void launch_field_update(const KParams &kp, const double *En, const double *Bn, const double *Eth, double *En1,
                         double *Bn1, hipStream_t st);
// out[k] = sum_i V[k][i] * w[i] for k < nvec (V rows of length n with stride ld)
// written to partials[blocks][nvec]; then reduced into res[nvec] (device).
void launch_mdot(const double *V, size_t ld, int nvec, const double *w, size_t n, double *partials, double *res,
                 hipStream_t st);
// w -= sum_k h[k] V[k]  (h on the device)
void launch_maxpy(const double *V, size_t ld, int nvec, const double *h, double *w, size_t n, hipStream_t st);
// w -= sum_k h[k] V[k] (k < nvec), then res[0..nvec] = (V[k] . w for k <
// nvec, w . w), reading the basis once; returns 0 (and launches nothing)
// for nvec > 32, where the caller takes launch_maxpy and launch_mdot.
int launch_maxpy_dot(const double *V, size_t ld, int nvec, const double *h, double *w, size_t n, double *partials,
                     double *res, hipStream_t st);
// w = (w - sum_k h[k] V[k]) / hn, hn = sqrt(h[nvec] - sum_k h[k]^2), left
// unscaled when that difference is at most 1e-4 h[nvec]; h[nvec + 1] = hn,
// or 0 when unscaled
void launch_maxpy_scale(const double *V, size_t ld, int nvec, double *h, double *w, size_t n, hipStream_t st);
// y = a * x + b * y  (scalars from the host)
void launch_axpby(double a, const double *x, double b, double *y, size_t n, hipStream_t st);
void launch_sumsq_partials(const double *x, size_t n, double *partials, hipStream_t st);
void launch_reduce_partials(const double *partials, int nparts, int nvec, double *res, hipStream_t st);
// res[0] = sum of in[0..n) in a fixed order (tmp: kRedBlocks doubles)
void launch_reduce_long(const double *in, int n, double *tmp, double *res, hipStream_t st);

}  // namespace relsim
