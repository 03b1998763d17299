// Particle kernels of the semi-implicit step for gfx950: moment deposit
// (S1-S3), node assembly of J-hat and M, push (S6) with the stable re-sort
// by bin in two passes (count the moves; push again and write each particle
// in its new place), and the kinetic-energy reduction (S7).
//
// Work decomposition.  The deposit and the kinetic-energy reduction split a
// 64-lane wavefront into 64/G lane groups; each group owns one cell and walks
// that cell's particles (both species, contiguous because particles are
// sorted by bin = cell * nspecies + species) G at a time, so loads are
// coalesced and every particle of a group sees the same neighbourhood of
// grid values.  The two push passes instead give a wave a segment of
// consecutive cells of one grid row and walk its particles 64 at a time
// across cell boundaries, with the segment's fields staged in LDS (no lane
// idles because one cell holds more particles than its neighbours).  Cells
// and segments are visited tile by tile (2D tiles of up to 16 x 8 cells, 3D
// of up to 16 x 4 x 4), so that neighbouring cells, whose particles exchange
// places in the re-sort, are processed close together in time; workgroups
// are remapped so that each XCD (and its L2) works on one contiguous band.
// The next rounds' particle loads are issued before the current round is
// computed.
//
// Deposit formulation.  For a particle with in-cell offsets f_d, the CIC
// node weights are products of (1 - f_d) or f_d, so the weight product of an
// ordered node pair (a, b) of the cell's corners depends only on the per-dim
// monomial type t_d = a_d + b_d in {0,1,2}: (1-f)^2, f(1-f), f^2.  Hence
//   M_{g,g'} = sum over cells c containing g and g' of S_c[t(g,g',c)],
//   S_c[t][k] = V^-1 sum_{p in c} (w q beta / gbar) prod_d mono_{t_d}(f_d) alpha_k,
// and J-hat likewise from per-corner sums.  In 2D (93 moments per cell) the
// lanes of a group split the cell's particles and their partial moments are
// then added in fixed lane order (registers, then one LDS transpose); in 3D
// (267 moments) the 4 lanes of a group split the moments instead and share
// each particle's quantities through LDS.  A second kernel assembles every
// node's J-hat and 9/27 M blocks from the 4/8 surrounding cells by a
// fixed-order gather.  No float atomics: results are deterministic, and
// M_{g,g'} == M_{g',g} bit for bit.
#include <climits>

#include "relsim_internal.h"

namespace relsim {
namespace {

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Consecutive workgroups are dispatched to the 8 XCDs round robin; remap so
  // that each XCD (and its L2) works on one contiguous slice of the grid.
  const int q = nb >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7) * q + (b >> 3);
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Grid coordinates of the cell visited by processing slot `slot`: tiles in
// row-major order, cells row-major inside a tile (power-of-two tile extents
// dividing the grid).
__device__ __forceinline__ void slot_coords(const KParams &kp, int slot, int &i, int &j, int &k) {
  const int lt = kp.ltx + kp.lty + kp.ltz;
  const int tile = slot >> lt, r = slot & ((1 << lt) - 1);
  const int lx = r & (kp.tx - 1), ly = (r >> kp.ltx) & (kp.ty - 1), lz = r >> (kp.ltx + kp.lty);
  const int t2 = tile / kp.ntx;
  const int tiz = t2 / kp.nty;
  i = ((tile - t2 * kp.ntx) << kp.ltx) + lx;
  j = ((t2 - tiz * kp.nty) << kp.lty) + ly;
  k = (tiz << kp.ltz) + lz;
}

// Reciprocal and reciprocal square root: the hardware instructions (1 ulp)
// in FP32, correctly rounded in FP64.
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }

// S7's relativistic kinetic term w m |u|^2 / (gamma + 1) in FP64, gamma =
// sqrt(1 + v), v = |u|^2 / c^2, given y ~ 1 / gamma from the push.  In FP64
// the quotient is formed directly.  From an FP32 y (relative error about
// 1e-7): two Newton steps for the square root, gamma <- gamma + (1 + v -
// gamma^2) y / 2, and two for the reciprocal of d = gamma + 1 from its FP32
// estimate, r <- r + r (1 - d r); each step squares the relative error, which
// ends within a few units of FP64 rounding (checked against exact arithmetic
// over |u| / c from 1e-4 to 3e3 with 3-ulp FP32 estimates: worst 3.2e-16).
// All full-rate FMAs, where the correctly rounded FP64 square root and
// division take twice as many instructions, two of them quarter rate.
__device__ __forceinline__ double kinetic_rel(double wmuu, double v, double) { return wmuu / (sqrt(1.0 + v) + 1.0); }
__device__ __forceinline__ double kinetic_rel(double wmuu, double v, float y32) {
  const double t = 1.0 + v;
  const double y = y32, hy = 0.5 * y;
  double g = t * y;
  g = fma(fma(-g, g, t), hy, g);
  g = fma(fma(-g, g, t), hy, g);
  const double d = g + 1.0;
  double r = (double)__builtin_amdgcn_rcpf((float)d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return wmuu * r;
}

// alpha = (I - [b]x + b b^T) / (1 + |b|^2), row-major, as its numerator
// (written to a) and the returned scale 1 / (1 + |b|^2); the kernels fold
// the scale into their per-particle coefficients.
template <typename T>
__device__ __forceinline__ T alpha_num(T bx, T by, T bz, T a[9]) {
  a[0] = T(1) + bx * bx;
  a[1] = bz + bx * by;
  a[2] = bx * bz - by;
  a[3] = bx * by - bz;
  a[4] = T(1) + by * by;
  a[5] = bx + by * bz;
  a[6] = by + bx * bz;
  a[7] = by * bz - bx;
  a[8] = T(1) + bz * bz;
  return rcp_t(a[0] + by * by + bz * bz);
}

// Particle-side view of the kernel constants in the arithmetic type T
// (precomputed on the host: no divisions or conversions in the kernels).
// The charges and betas of species 0 and 1 are also held by value (read
// once from the kernel arguments): a per-particle load of them inside a
// round would make the round wait for every load issued before it,
// prefetches included.
template <typename T>
struct PC;
template <>
struct PC<float> {
  float dt, invc, invc2, invV, idx, idy, idz;
  float q0, q1, b0, b1;
  const float *q, *beta;
  __device__ explicit PC(const KParams &kp)
      : dt(kp.f_dt), invc(kp.f_inv_c), invc2(kp.f_inv_c2), invV(kp.f_inv_V), idx(kp.f_inv_dx), idy(kp.f_inv_dy),
        idz(kp.f_inv_dz), q0(kp.f_q[0]), q1(kp.f_q[1]), b0(kp.f_beta[0]), b1(kp.f_beta[1]), q(kp.f_q),
        beta(kp.f_beta) {}
};
template <>
struct PC<double> {
  double dt, invc, invc2, invV, idx, idy, idz;
  double q0, q1, b0, b1;
  const double *q, *beta;
  __device__ explicit PC(const KParams &kp)
      : dt(kp.dt), invc(kp.inv_c), invc2(kp.inv_c2), invV(kp.inv_V), idx(kp.inv_dx), idy(kp.inv_dy),
        idz(kp.inv_dz), q0(kp.q[0]), q1(kp.q[1]), b0(kp.beta[0]), b1(kp.beta[1]), q(kp.q), beta(kp.beta) {}
};



// Ghosted copy of a SoA FP64 grid field (one thread per ghosted point).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_stage_field(KParams kp, const double *__restrict__ F,
                                                     V4<T> *__restrict__ out) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= kp.nghost) return;
  const int gi = g % kp.gx, gj = (g / kp.gx) % (kp.ny + 2);
  const int i = wrapi(gi - 1, kp.nx), j = wrapi(gj - 1, kp.ny);
  const int k = DIM == 3 ? wrapi(g / kp.gxy - 1, kp.nz) : 0;
  const size_t N = (size_t)kp.ncells, id = (size_t)i + (size_t)kp.nx * ((size_t)j + (size_t)kp.ny * k);
  V4<T> v;
  v.x = (T)F[id];
  v.y = (T)F[N + id];
  v.z = (T)F[2 * N + id];
  v.w = T(0);
  out[g] = v;
}

// Index of grid point (i, j, k) in a ghosted copy, i in [-1, nx] etc.
template <int DIM>
__device__ __forceinline__ int gidx(const KParams &kp, int i, int j, int k) {
  return (i + 1) + kp.gx * (j + 1) + (DIM == 3 ? kp.gxy * (k + 1) : 0);
}

// The 3^DIM block of cell-centre B values around the cell with ghosted
// index gc, staged in LDS by the G lanes of the cell's group (centre t at
// shift (t % 3 - 1, t / 3 % 3 - 1, t / 9 - 1) from the cell).  The caller
// synchronises the block before the first gather.
template <typename T, int G, int DIM>
__device__ __forceinline__ void stage_B_block(const KParams &kp, const V4<T> *__restrict__ Bs, int gc, int gl,
                                              V4<T> *blk) {
  constexpr int NB = DIM == 3 ? 27 : 9;
#pragma unroll
  for (int t = gl; t < NB; t += G)
    blk[t] = Bs[gc + (t % 3 - 1) + kp.gx * ((t / 3) % 3 - 1) + (DIM == 3 ? kp.gxy * (t / 9 - 1) : 0)];
}

// B at the particle from the 2^DIM cell centres around it (lower corner at
// shift -1 or 0 per dimension), read from an LDS block of centres in which
// bc points at the particle's cell and (sy, sz) are the y and z strides.
// A field point without the pad of V4: the 3D deposit's B blocks in LDS (12
// instead of 16 bytes per point in FP32, 16.2 -> 14.5 KB per wave, which
// lets 11 instead of 9 waves share a CU's 160 KB: 3 % faster on the
// 256 x 128 x 128 sheet, 7 % on 128 x 64 x 64)
template <typename T>
struct P3 {
  T x, y, z;
};
template <typename T, int DIM, typename PT = V4<T>>
__device__ __forceinline__ void gather_B(const PT *bc, int sy, int sz, T fx, T fy, T fz, T &Bx, T &By,
                                         T &Bz) {
  constexpr int NCEN = DIM == 3 ? 8 : 4;
  const bool hx = fx >= T(0.5), hy = fy >= T(0.5), hz = DIM == 3 && fz >= T(0.5);
  const T gx = hx ? fx - T(0.5) : fx + T(0.5);
  const T gy = hy ? fy - T(0.5) : fy + T(0.5);
  const T gz = hz ? fz - T(0.5) : fz + T(0.5);
  const PT *const b0 = bc - (hx ? 0 : 1) - (hy ? 0 : sy) - ((DIM == 3 && !hz) ? sz : 0);
#pragma unroll
  for (int a = 0; a < NCEN; ++a) {
    const PT b = b0[(a & 1) + ((a & 2) ? sy : 0) + ((a & 4) ? sz : 0)];
    T wt = ((a & 1) ? gx : T(1) - gx) * ((a & 2) ? gy : T(1) - gy);
    if constexpr (DIM == 3) wt *= (a & 4) ? gz : T(1) - gz;
    Bx = a == 0 ? wt * b.x : Bx + wt * b.x;
    By = a == 0 ? wt * b.y : By + wt * b.y;
    Bz = a == 0 ? wt * b.z : Bz + wt * b.z;
  }
}

// Per-lane cell bookkeeping shared by the particle kernels.
struct CellSpan {
  int cell, ci, cj, ck, pbeg, pend;
  int gc;        // ghosted field index of the cell's lower node / its centre
  int bound[8];  // first particle of species s (the cell's end for s >= nspecies)
  bool valid;
};

// The cell of processing slot blk * (64/G) + grp and its particle range.
template <int G>
__device__ __forceinline__ CellSpan slot_span(const KParams &kp, const int32_t *__restrict__ bin_start, int blk,
                                              int grp) {
  const int slot = blk * (64 / G) + grp;
  const bool valid = slot < kp.ncells;
  CellSpan cs;
  cs.valid = valid;
  slot_coords(kp, valid ? slot : 0, cs.ci, cs.cj, cs.ck);
  cs.cell = cs.ci + kp.nx * (cs.cj + kp.ny * cs.ck);
  cs.gc = (cs.ci + 1) + kp.gx * (cs.cj + 1) + kp.gxy * (kp.dim == 3 ? cs.ck + 1 : 0);
  const int S = kp.nspecies, b0 = cs.cell * S;
#pragma unroll
  for (int s = 0; s < 8; ++s) cs.bound[s] = valid ? bin_start[b0 + (s < S ? s : S)] : 0;
  cs.pbeg = cs.bound[0];
  cs.pend = valid ? bin_start[b0 + S] : 0;
  return cs;
}

// Wave-uniform number of rounds: max over the wave of ceil(count / G).
template <int G>
__device__ __forceinline__ int wave_rounds(int count) {
  int r = (count + G - 1) / G;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) r = max(r, __shfl_xor(r, o));
  // every lane holds the maximum now; as a scalar, loops over rounds
  // branch uniformly
  return __builtin_amdgcn_readfirstlane(r);
}

// Species of particle p of the cell (particles of a cell are ordered by
// species), with its charge and beta.  The two-species case selects between
// values passed in (q0, q1, b0, b1), not between loads: the compiler may
// turn a select of two loads into one load from a selected address, which
// pins the operands in memory.  Other species counts read the tables qt, bt.
template <typename T>
__device__ __forceinline__ int species_sel(const KParams &kp, const CellSpan &cs, int p, T q0, T q1, T b0, T b1,
                                          const T *qt, const T *bt, T &q, T &beta) {
  if (kp.nspecies == 2) {
    const bool s1 = p >= cs.bound[1];
    q = s1 ? q1 : q0;
    beta = s1 ? b1 : b0;
    return s1 ? 1 : 0;
  }
  int s = 0;
#pragma unroll
  for (int s2 = 1; s2 < 8; ++s2) s = p >= cs.bound[s2] ? s2 : s;
  q = qt[s];
  beta = bt[s];
  return s;
}

template <typename T>
__device__ __forceinline__ int species_of(const KParams &kp, const PC<T> &pc, const CellSpan &cs, int p,
                                         const T (*tab)[8], T &q, T &beta) {
  return species_sel<T>(kp, cs, p, pc.q0, pc.q1, pc.b0, pc.b1, tab[0], tab[1], q, beta);
}

// Per-species charge and beta in LDS (row 0: q, row 1: beta), for species
// counts other than two: read inside a round from LDS, since a load from
// memory there would wait for the next rounds' prefetched loads too.  The
// caller synchronises before the first use.
template <typename T>
__device__ __forceinline__ void fill_species_table(const PC<T> &pc, T (*tab)[8], int lane) {
  if (lane < 8) {
    tab[0][lane] = pc.q[lane];
    tab[1][lane] = pc.beta[lane];
  }
}

// One particle's state as loaded from the SoA arrays.
template <typename T>
struct PRec {
  T fx, fy, fz, ux, uy, uz, w;
  T g;  // gbar of the energy-conserving variant (loaded only there)
};

// Index a lane loads for particle p of a cell ending at pend: lanes past
// the end read a valid neighbour instead of branching, so that the loads stay
// unconditional and the next round's loads are in flight while the current
// round computes.  Only used when the wave has particles (n > 0).
__device__ __forceinline__ int load_index(int p, int pend) { return p < pend ? p : (pend > 0 ? pend - 1 : 0); }

// Rounds start on 64-byte boundaries (lanes before the cell's first particle
// idle), so that each load or store instruction of a lane group covers whole
// 32-byte memory sectors: a sector split between two instructions is
// transferred twice.
template <typename T, int G>
constexpr int round_align() {
  return (64 / (int)sizeof(T)) < G ? 64 / (int)sizeof(T) : G;
}

// 2D: (off_x, off_y) in xy[p] and (u_x, u_y, u_z, w) in uw[p].  3D: one
// 8-value record per particle at xy (two V4: (off_x, off_y, off_z, 0) and
// (u_x, u_y, u_z, w)), so that a particle is one aligned 32-byte block in
// FP32 (a whole memory sector) and the re-sort writes whole sectors; uw and
// zz are unused in 3D.
template <typename T>
__device__ __forceinline__ const V4<T> *rec3(const V2<T> *xy) {
  return reinterpret_cast<const V4<T> *>(xy);
}
template <typename T>
__device__ __forceinline__ V4<T> *rec3(V2<T> *xy) {
  return reinterpret_cast<V4<T> *>(xy);
}

template <typename T, int DIM>
__device__ __forceinline__ void load_rec(int p, int pend, const V2<T> *__restrict__ xy, const V4<T> *__restrict__ uw,
                                         const T *__restrict__ zz, PRec<T> &r) {
  const int q = load_index(p, pend);
  V4<T> b;
  if constexpr (DIM == 3) {
    const V4<T> *R = rec3<T>(xy) + 2 * (size_t)q;
    const V4<T> a = R[0];
    b = R[1];
    r.fx = a.x;
    r.fy = a.y;
    r.fz = a.z;
  } else {
    const V2<T> a = xy[q];
    b = uw[q];
    r.fx = a.x;
    r.fy = a.y;
  }
  r.ux = b.x;
  r.uy = b.y;
  r.uz = b.z;
  r.w = b.w;
}

// Store one particle's state at slot q of the record arrays (3D: one
// 8-value record), or into the lane's sink slot when `to_sink`.
template <typename T, int DIM>
__device__ __forceinline__ void store_rec(bool to_sink, size_t q, V2<T> *__restrict__ xy, V4<T> *__restrict__ uw,
                                          T *__restrict__ zz, void *sink, T fx, T fy, T fz, T ux, T uy, T uz, T w) {
  V4<T> b;
  b.x = ux;
  b.y = uy;
  b.z = uz;
  b.w = w;
  if constexpr (DIM == 3) {
    V4<T> a;
    a.x = fx;
    a.y = fy;
    a.z = fz;
    a.w = T(0);
    // both halves of a sink store go to the lane's one slot
    V4<T> *R = to_sink ? reinterpret_cast<V4<T> *>(sink) : rec3<T>(xy) + 2 * q;
    const int h = to_sink ? 0 : 1;
    R[0] = a;
    R[h] = b;
  } else {
    V2<T> a;
    a.x = fx;
    a.y = fy;
    *(to_sink ? reinterpret_cast<V2<T> *>(sink) : xy + q) = a;
    *(to_sink ? reinterpret_cast<V4<T> *>(sink) : uw + q) = b;
  }
}

// The energy-conserving variant gives gbar per particle (in the particle
// arithmetic type, in the particles' order); its kernels load it beside the
// record (GB).  1 / gbar of S2: that value, or 1 / gamma(u^n).
template <bool GB, typename T>
__device__ __forceinline__ void load_gbar(int p, int pend, const T *__restrict__ gb, PRec<T> &r) {
  if constexpr (GB) r.g = gb[load_index(p, pend)];
}

template <bool GB, typename T>
__device__ __forceinline__ T inv_gbar(const KParams &kp, const PC<T> &pc, const PRec<T> &r, T ux, T uy, T uz) {
  if constexpr (GB)
    return kp.nonrel ? T(1) : T(1) / r.g;
  else
    return kp.nonrel ? T(1) : rsqrt_t(T(1) + (ux * ux + uy * uy + uz * uz) * pc.invc2);
}

// ---------------------------------------------------------------------------
// S1-S3: per-cell moments
// ---------------------------------------------------------------------------
// 2D: the G lanes of a group split the cell's particles; each lane sums all
// 93 moments (81 mass, 12 current) of its particles, and the group's G
// partial sums are then added in fixed lane order.
template <typename T, int G, bool GB>
__global__ __launch_bounds__(64) void k_deposit_cells(KParams kp, const int32_t *__restrict__ bin_start,
                                                      const V2<T> *__restrict__ xy,
                                                      const V4<T> *__restrict__ uw,
                                                      const V4<T> *__restrict__ Bs, T *__restrict__ S,
                                                      const T *__restrict__ gb) {
  constexpr int NACC = 93;  // 81 mass moments + 12 current moments
  constexpr int CH = 32;    // moments per LDS transpose chunk (keeps LDS off the occupancy limit)
  __shared__ T red[64 * (CH + 1)];
  __shared__ V4<T> bsh[64 / G][9];
  __shared__ T stab[2][8];
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const CellSpan cs = slot_span<G>(kp, bin_start, blk, grp);
  const PC<T> pc(kp);

  stage_B_block<T, G, 2>(kp, Bs, cs.gc, gl, bsh[grp]);
  fill_species_table<T>(pc, stab, lane);
  __syncthreads();
  const int pal = cs.pbeg & ~(round_align<T, G>() - 1);
  const int rounds = wave_rounds<G>(cs.pend - pal);

  T acc[NACC];
#pragma unroll
  for (int k = 0; k < NACC; ++k) acc[k] = T(0);
  PRec<T> cur{}, nxt{};
  int p = pal + gl;
  if (rounds > 0) {
    load_rec<T, 2>(p, cs.pend, xy, uw, nullptr, cur);
    load_gbar<GB>(p, cs.pend, gb, cur);
  }
  __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 2
  for (int r = 0; r < rounds; ++r) {
    const int pn = p + G;
    load_rec<T, 2>(pn, cs.pend, xy, uw, nullptr, nxt);
    load_gbar<GB>(pn, cs.pend, gb, nxt);
    if (p >= cs.pbeg && p < cs.pend) {
      const T fx = cur.fx, fy = cur.fy;
      const T ux = cur.ux, uy = cur.uy, uz = cur.uz, wp = cur.w;
      T qs, bs;
      species_of<T>(kp, pc, cs, p, stab, qs, bs);
      T Bx, By, Bz;
      gather_B<T, 2>(bsh[grp] + 4, 3, 9, fx, fy, T(0), Bx, By, Bz);
      const T igb = inv_gbar<GB>(kp, pc, cur, ux, uy, uz);
      const T kb = bs * igb * pc.invc;
      T a[9];
      const T inv = alpha_num<T>(kb * Bx, kb * By, kb * Bz, a);
      // current and mass coefficients with the alpha scale folded in; the
      // mass coefficient rides on the x monomials
      const T cJ = wp * qs * igb * pc.invV * inv;
      const T cM = cJ * bs;
      T psiJ[3];
      psiJ[0] = cJ * (a[0] * ux + a[1] * uy + a[2] * uz);
      psiJ[1] = cJ * (a[3] * ux + a[4] * uy + a[5] * uz);
      psiJ[2] = cJ * (a[6] * ux + a[7] * uy + a[8] * uz);
      const T nx0 = T(1) - fx, ny0 = T(1) - fy;
      const T mx[3] = {cM * (nx0 * nx0), cM * (nx0 * fx), cM * (fx * fx)};
      const T my[3] = {ny0 * ny0, ny0 * fy, fy * fy};
#pragma unroll
      for (int m = 0; m < 9; ++m) {
        const T wgt = mx[m % 3] * my[m / 3];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[m * 9 + k] += wgt * a[k];
      }
#pragma unroll
      for (int cxy = 0; cxy < 4; ++cxy) {
        const T wgt = ((cxy & 1) ? fx : nx0) * ((cxy & 2) ? fy : ny0);
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[81 + cxy * 3 + k] += wgt * psiJ[k];
      }
    }
    cur = nxt;
    p = pn;
  }
  // group reduction, CH moments at a time: registers -> LDS transpose ->
  // G-term sums in fixed lane order
#pragma unroll
  for (int c0 = 0; c0 < NACC; c0 += CH) {
#pragma unroll
    for (int k = 0; k < CH; ++k)
      if (c0 + k < NACC) red[lane * (CH + 1) + k] = acc[c0 + k];
    __syncthreads();
    const int kend = NACC - c0 < CH ? NACC - c0 : CH;
    for (int k = gl; k < kend; k += G) {
      T s = T(0);
#pragma unroll 8
      for (int j = 0; j < G; ++j) s += red[(grp * G + j) * (CH + 1) + k];
      if (cs.valid) S[mom_index<2>(c0 + k, cs.cell)] = s;
    }
    __syncthreads();
  }
}

// 3D: the cell's 267 moments are split over the 4 lanes of its group rather
// than its particles: lane t (t = 0, 1, 2) accumulates the 81 mass moments
// of z-monomial type t over all of the cell's particles, lane 3 the 24
// current moments (8 corners x 3 components).  Each round, every lane
// computes the per-particle quantities of one particle and shares them with
// its group through LDS; each lane then adds the 4 particles of the round to
// its own moments.  The per-particle work (B gather, alpha) is done once
// instead of once per z-monomial type, and no cross-lane reduction is
// needed: each moment is summed by one lane, in particle order.  All lanes
// run one instruction stream, acc[m * 9 + k] += X[m % 3] Z Y[m / 3] P[k],
// on operands read from a lane-dependent place:
//   lanes 0-2: X = ((1-f_x)^2, (1-f_x) f_x, f_x^2), Y likewise in y,
//              Z = mono_t(f_z), P = the 9 alpha-weighted mass coefficients;
//   lane 3:    X = (1-f_x, f_x, 0), Y = (1-f_y, f_y, 0), Z = 1,
//              P = (current x (1-f_z), current x f_z, 0, 0, 0),
// so lane 3 uses 24 of its 81 accumulators.
template <typename T, bool GB>
__global__ __launch_bounds__(64) void k_deposit_split3(KParams kp, const int32_t *__restrict__ bin_start,
                                                       const V2<T> *__restrict__ xy,
                                                       const V4<T> *__restrict__ uw, const T *__restrict__ zz,
                                                       const V4<T> *__restrict__ Bs, T *__restrict__ S,
                                                       const T *__restrict__ gb) {
  constexpr int G = 4;
  // per producing lane: operand blocks (X0 X1 X2 Y0) (Y1 Y2 P0 P1) (P2..P5)
  // (P6 P7 P8 -) for the mass lanes [0] and the current lane [1], and Z
  __shared__ V4<T> sh[2][4][64];
  __shared__ T zsh[4][64];
  __shared__ P3<T> bsh[64 / G][27];
  __shared__ T stab[2][8];
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  // blocks in launch order, not banded per XCD: the moment stores then
  // interleave over the XCDs (measured 5 % faster on the 256 x 128 x 128
  // sheet than XCD bands, 1 % on 128 x 64 x 64)
  const int blk = (int)blockIdx.x;
  const CellSpan cs = slot_span<G>(kp, bin_start, blk, grp);
  const PC<T> pc(kp);
#pragma unroll
  for (int t = gl; t < 27; t += G) {
    const V4<T> b = Bs[cs.gc + (t % 3 - 1) + kp.gx * ((t / 3) % 3 - 1) + kp.gxy * (t / 9 - 1)];
    bsh[grp][t] = P3<T>{b.x, b.y, b.z};
  }
  fill_species_table<T>(pc, stab, lane);
  __syncthreads();
  const bool isJ = gl == 3;
  const V4<T> *const mine = &sh[isJ ? 1 : 0][0][0];

  T acc[81];
#pragma unroll
  for (int k = 0; k < 81; ++k) acc[k] = T(0);
  // rounds start at the cell's first particle: with few particles per cell
  // an aligned start costs more rounds than it saves in memory sectors
  const int pal = cs.pbeg;
  const int rounds = wave_rounds<G>(cs.pend - pal);
  PRec<T> cur{}, nxt{};
  int p = pal + gl;
  if (rounds > 0) load_rec<T, 3>(p, cs.pend, xy, uw, zz, cur);
  if (GB && rounds > 0) load_gbar<GB>(p, cs.pend, gb, cur);
  __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 1
  for (int r = 0; r < rounds; ++r) {
    const int pn = p + G;
    load_rec<T, 3>(pn, cs.pend, xy, uw, zz, nxt);
    load_gbar<GB>(pn, cs.pend, gb, nxt);
    {
      // this lane's particle (lanes outside the cell's range contribute 0)
      const bool pv = p >= cs.pbeg && p < cs.pend;
      const T fx = cur.fx, fy = cur.fy, fz = cur.fz;
      const T ux = cur.ux, uy = cur.uy, uz = cur.uz;
      T qs, bs;
      species_of<T>(kp, pc, cs, p, stab, qs, bs);
      T Bx, By, Bz;
      gather_B<T, 3, P3<T>>(bsh[grp] + 13, 3, 9, fx, fy, fz, Bx, By, Bz);
      T igb;
      if constexpr (GB)
        igb = inv_gbar<GB>(kp, pc, cur, ux, uy, uz);
      else
        igb = kp.nonrel ? T(1) : rsqrt_t(T(1) + (ux * ux + uy * uy + uz * uz) * pc.invc2);
      const T kb = bs * igb * pc.invc;
      T a[9];
      const T inv = alpha_num<T>(kb * Bx, kb * By, kb * Bz, a);
      const T cJ = pv ? cur.w * qs * igb * pc.invV * inv : T(0);
      const T cM = cJ * bs;
      const T j0 = cJ * (a[0] * ux + a[1] * uy + a[2] * uz);
      const T j1 = cJ * (a[3] * ux + a[4] * uy + a[5] * uz);
      const T j2 = cJ * (a[6] * ux + a[7] * uy + a[8] * uz);
      const T nx0 = T(1) - fx, ny0 = T(1) - fy, nz0 = T(1) - fz;
      V4<T> m0, m1, m2, m3, c0, c1, c2, c3;
      m0.x = nx0 * nx0;
      m0.y = nx0 * fx;
      m0.z = fx * fx;
      m0.w = ny0 * ny0;
      m1.x = ny0 * fy;
      m1.y = fy * fy;
      m1.z = cM * a[0];
      m1.w = cM * a[1];
      m2.x = cM * a[2];
      m2.y = cM * a[3];
      m2.z = cM * a[4];
      m2.w = cM * a[5];
      m3.x = cM * a[6];
      m3.y = cM * a[7];
      m3.z = cM * a[8];
      m3.w = T(0);
      c0.x = nx0;
      c0.y = fx;
      c0.z = T(0);
      c0.w = ny0;
      c1.x = fy;
      c1.y = T(0);
      c1.z = j0 * nz0;
      c1.w = j1 * nz0;
      c2.x = j2 * nz0;
      c2.y = j0 * fz;
      c2.z = j1 * fz;
      c2.w = j2 * fz;
      c3.x = T(0);
      c3.y = T(0);
      c3.z = T(0);
      c3.w = T(0);
      __syncthreads();  // the previous round's reads are done
      sh[0][0][lane] = m0;
      sh[0][1][lane] = m1;
      sh[0][2][lane] = m2;
      sh[0][3][lane] = m3;
      sh[1][0][lane] = c0;
      sh[1][1][lane] = c1;
      sh[1][2][lane] = c2;
      sh[1][3][lane] = c3;
      zsh[0][lane] = nz0 * nz0;
      zsh[1][lane] = nz0 * fz;
      zsh[2][lane] = fz * fz;
      zsh[3][lane] = T(1);
      __syncthreads();
    }
#pragma unroll 1
    for (int j = 0; j < G; ++j) {
      const int src = grp * G + j;
      const V4<T> v0 = mine[src], v1 = mine[64 + src], v2 = mine[128 + src], v3 = mine[192 + src];
      const T Z = zsh[gl][src];
      const T XZ[3] = {v0.x * Z, v0.y * Z, v0.z * Z};
      const T Y[3] = {v0.w, v1.x, v1.y};
      const T P[9] = {v1.z, v1.w, v2.x, v2.y, v2.z, v2.w, v3.x, v3.y, v3.z};
#pragma unroll
      for (int m = 0; m < 9; ++m) {
        const T wgt = XZ[m % 3] * Y[m / 3];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[m * 9 + k] += wgt * P[k];
      }
    }
    cur = nxt;
    p = pn;
  }
  if (!cs.valid) return;
  // moment (block row) layout: see mom_index
  T *const base = S + mom_index<3>(0, cs.cell);
  if (!isJ) {
    T *const q = base + (size_t)(gl * 81) * kMomBlock;
#pragma unroll
    for (int e = 0; e < 81; ++e) q[(size_t)e * kMomBlock] = acc[e];
  } else {
    // accumulator (x + 3 y) * 9 + k holds the current of corner (x, y, k / 3)
    // along k % 3
    T *const q = base + (size_t)243 * kMomBlock;
#pragma unroll
    for (int e = 0; e < 81; ++e) {
      const int m = e / 9, k = e % 9, x = m % 3, y = m / 3;
      if (x < 2 && y < 2 && k < 6) q[(size_t)((k / 3) * 12 + (x + 2 * y) * 3 + k % 3) * kMomBlock] = acc[e];
    }
  }
}

// ---------------------------------------------------------------------------
// J-hat and M at nodes from the per-cell moments (fixed-order gather).  Both
// are summed in FP64; J-hat is stored in FP64 and M in MT (double, or float
// on request in mixed precision, where the moments are already FP32).
// ---------------------------------------------------------------------------
template <typename T, int DIM, typename MT>
__global__ __launch_bounds__(256) void k_assemble(KParams kp, const T *__restrict__ S, double *__restrict__ J,
                                                  MT *__restrict__ M) {
  constexpr int NSLOT = m_slots<DIM>(), CEN = m_centre<DIM>();
  constexpr int NCORN = DIM == 3 ? 8 : 4;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int g = blk * blockDim.x + threadIdx.x;
  if (g >= kp.ncells) return;
  const size_t N = (size_t)kp.ncells;
  const int i = g % kp.nx, j = (g / kp.nx) % kp.ny, k = g / (kp.nx * kp.ny);
  // cells having node g as corner a: c = g - a
  int cidx[NCORN];
#pragma unroll
  for (int a = 0; a < NCORN; ++a) {
    const int ii = wrapi(i - (a & 1), kp.nx);
    const int jj = wrapi(j - ((a >> 1) & 1), kp.ny);
    const int kk = DIM == 3 ? wrapi(k - ((a >> 2) & 1), kp.nz) : 0;
    cidx[a] = ii + kp.nx * (jj + kp.ny * kk);
  }
  // the stored half of the offsets (the other half is the same blocks seen
  // from the other node of each pair)
#pragma unroll
  for (int h = 0; h < NSLOT; ++h) {
    const int off = CEN + h;
    const int dx = off % 3 - 1, dy = (off / 3) % 3 - 1, dz = DIM == 3 ? off / 9 - 1 : 0;
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
#pragma unroll
    for (int a = 0; a < NCORN; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      const int bx = ax + dx, by = ay + dy, bz = az + dz;
      if (bx < 0 || bx > 1 || by < 0 || by > 1) continue;
      if (DIM == 3 && (bz < 0 || bz > 1)) continue;
      const int mono = (ax + bx) + 3 * (ay + by);
      const int base = DIM == 3 ? (az + bz) * 81 + mono * 9 : mono * 9;
#pragma unroll
      for (int q = 0; q < 9; ++q) acc[q] += (double)S[mom_index<DIM>(base + q, cidx[a])];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) M[((size_t)h * 9 + q) * N + g] = (MT)acc[q];
  }
  double jacc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < NCORN; ++a) {
    const int cxy = (a & 1) + 2 * ((a >> 1) & 1);
    const int base = DIM == 3 ? 243 + ((a >> 2) & 1) * 12 + cxy * 3 : 81 + cxy * 3;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      jacc[q] += (double)S[mom_index<DIM>(base + q, cidx[a])];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) J[(size_t)q * N + g] = jacc[q];
}

// ---------------------------------------------------------------------------
// S6: push, cell crossing, and per-(bin, move) counts for the re-sort
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int cross_cell(T &f, int &bad) {
  // f is the new offset in cell units; bring it back into [0,1) with one
  // cell move.  A value rounding to exactly 1 after the correction from
  // below is the left face of the cell (offset 0, no move).
  // (written with selects only: no divergent branches)
  const bool up = f >= T(1), dn = f < T(0);
  int m = up ? 1 : (dn ? -1 : 0);
  f = up ? f - T(1) : (dn ? f + T(1) : f);
  const bool edge = dn && f == T(1);
  m = edge ? 0 : m;
  f = edge ? T(0) : f;
  const bool out = !(f >= T(0) && f < T(1));  // moved more than one cell, or non-finite
  bad = out ? 1 : bad;
  f = out ? T(0) : f;
  return m;
}

// Offset along one dimension relative to the cell the counting pass placed
// the particle in (move m), from its new offset f relative to the old cell:
// the same arithmetic as cross_cell for that move, so the result is the
// counting pass's bit for bit when the push is recomputed identically.
// Should compiled code ever round the recomputation differently, a particle
// within rounding of a face is put on that face inside the counted cell;
// anything further off (a disagreement a rounding difference cannot
// explain) sets off.
// The counting pass's own rule for an offset just below 0 whose correction
// rounds to exactly 1 (no move, offset 0; see cross_cell) gives move 0 and a
// negative f here: that particle is placed at 0 as the first pass placed it.
// Any other placement onto the face (within rounding outside the cell) sets
// clamp; the scatter counts those particles.
template <typename T>
__device__ __forceinline__ T place_offset(T f, int m, int &off, int &clamp) {
  constexpr T below1 = sizeof(T) == 4 ? T(0x1.fffffep-1) : T(0x1.fffffffffffffp-1);
  constexpr T tol = T(1e-4);
  T g = m > 0 ? f - T(1) : (m < 0 ? f + T(1) : f);
  const bool edge = m == 0 && f < T(0) && f + T(1) == T(1);
  const bool lo = !(g >= T(0)), hi = g >= T(1);  // lo includes NaN
  off = ((lo && !(g > -tol)) || (hi && !(g < T(1) + tol))) ? 1 : off;
  clamp = ((lo && !edge) || hi) ? 1 : clamp;
  return lo ? T(0) : (hi ? below1 : g);
}

// Lanes past their cell's end store into a per-lane slot of a small sink in
// the workspace instead of branching around the stores: with unconditional
// stores the compiler can count them, and the wait for the next round's
// loads does not also wait for this round's stores to complete.
template <typename T>
__device__ __forceinline__ T *sink_slot(void *sink, int lane) {
  return reinterpret_cast<T *>(sink) + (((blockIdx.x & (kSinkSlots - 1)) << 6) + lane);
}

// Where a lane finds the fields of its particle's cell: the LDS regions of
// cell-centre B values and E_theta node values staged for the wave's row
// segment (see Segment), as pointers to the cell's centre and lower node.
template <typename T>
struct CellFields {
  const V4<T> *bc;  // B at the cell's centre; y and z strides by, bz
  const V4<T> *e0;  // E_theta at the cell's lower corner node; strides ey, ez
  int by, bz, ey, ez;
};

// S6 for one particle: u^{n+1} = 2 alpha (u^n + beta E_p) - u^n (alpha from
// B^n at the particle, E_p from the cell's corner values of E_theta) and the
// offsets advanced by dt u^{n+1} / gamma^{n+1} in cell units, not yet brought
// back into [0, 1).  Every kernel that pushes calls this one function, so
// that they all round identically.
template <typename T, int DIM, bool GB = false>
__device__ __forceinline__ void push_one(const KParams &kp, const PC<T> &pc, const CellFields<T> &cf, T bs,
                                         const PRec<T> &cur, T &fx, T &fy, T &fz, T &nx, T &ny, T &nz, T &ign) {
  constexpr int NCORN = DIM == 3 ? 8 : 4;
  fx = cur.fx;
  fy = cur.fy;
  fz = DIM == 3 ? cur.fz : T(0);
  const T ux = cur.ux, uy = cur.uy, uz = cur.uz;
  T Bx, By, Bz;
  gather_B<T, DIM>(cf.bc, cf.by, cf.bz, fx, fy, fz, Bx, By, Bz);
  const T igb = inv_gbar<GB>(kp, pc, cur, ux, uy, uz);
  const T kb = bs * igb * pc.invc;
  T a[9];
  const T inv2 = T(2) * alpha_num<T>(kb * Bx, kb * By, kb * Bz, a);
  T Ex, Ey, Ez;
#pragma unroll
  for (int c = 0; c < NCORN; ++c) {
    const V4<T> e = cf.e0[(c & 1) + ((c & 2) ? cf.ey : 0) + ((c & 4) ? cf.ez : 0)];
    T wgt = ((c & 1) ? fx : T(1) - fx) * ((c & 2) ? fy : T(1) - fy);
    if constexpr (DIM == 3) wgt *= (c & 4) ? fz : T(1) - fz;
    Ex = c == 0 ? wgt * e.x : Ex + wgt * e.x;
    Ey = c == 0 ? wgt * e.y : Ey + wgt * e.y;
    Ez = c == 0 ? wgt * e.z : Ez + wgt * e.z;
  }
  const T vx = ux + bs * Ex, vy = uy + bs * Ey, vz = uz + bs * Ez;
  // u^{n+1} = 2 alpha v - u^n, alpha = (numerator a) / (1 + |b|^2)
  const T ubx = a[0] * vx + a[1] * vy + a[2] * vz;
  const T uby = a[3] * vx + a[4] * vy + a[5] * vz;
  const T ubz = a[6] * vx + a[7] * vy + a[8] * vz;
  nx = inv2 * ubx - ux;
  ny = inv2 * uby - uy;
  nz = inv2 * ubz - uz;
  ign = kp.nonrel ? T(1) : rsqrt_t(T(1) + (nx * nx + ny * ny + nz * nz) * pc.invc2);
  const T dtg = pc.dt * ign;
  fx += dtg * nx * pc.idx;
  fy += dtg * ny * pc.idy;
  if constexpr (DIM == 3) fz += dtg * nz * pc.idz;
}

// ---------------------------------------------------------------------------
// Push passes: a flat walk over a row segment.
// A wave owns C consecutive cells of one grid row (C divides nx) and walks
// their particles, contiguous in memory because they are sorted by bin, 64
// at a time across cell boundaries.  Lanes are not tied to a cell, so a cell
// holding more particles than the others costs no idle lanes (with a lane
// group per cell, a wave's rounds are set by its fullest cell).  The wave
// first stages in LDS what its particles can touch: the starts of the
// segment's C * nspecies bins, the cell-centre B values around the segment,
// the E_theta node values of the segment and the species table; a lane
// finds its particle's bin by a binary search over the bin starts.
// ---------------------------------------------------------------------------
template <typename T, int DIM>
struct Segment {
  int C, nb;         // cells and bins of the segment
  int c0, i0, j, k;  // first cell and its coordinates
  V4<T> *Bg;         // (C + 2) x 3 [x 3] cell centres from (i0 - 1, j - 1, k - 1), x fastest
  V4<T> *Eg;         // (C + 1) x 2 [x 2] nodes from (i0, j, k)
  T (*stab)[8];      // species charge and beta
  double *mtab;      // species mass (FP64)
  int *binb;         // nb + 1 bin starts, then INT_MAX up to a power of two
  int *keys;         // nb x NDIR counters (counting pass) or run bases (scatter)
};

// Smallest power of two >= nb (nb >= 1).
__host__ __device__ constexpr int pow2_at_least(int nb) {
  int q = 1;
  while (q < nb) q <<= 1;
  return q;
}

// Slots of the staged bin starts: nb + 1 starts, padded to a power of two so
// that the bin search needs no bounds check.
__host__ __device__ constexpr int binb_slots(int nb) { return nb + 1 > pow2_at_least(nb) ? nb + 1 : pow2_at_least(nb); }

// LDS bytes of a segment of C cells with S species.
template <typename T, int DIM>
__host__ __device__ constexpr size_t segment_lds_bytes(int C, int S) {
  return sizeof(V4<T>) * ((size_t)(C + 2) * 3 * (DIM == 3 ? 3 : 1) + (size_t)(C + 1) * 2 * (DIM == 3 ? 2 : 1)) +
         sizeof(T) * 16 + sizeof(double) * 8 + sizeof(int) * (size_t)binb_slots(C * S) +
         sizeof(int) * (size_t)C * S * (DIM == 3 ? 27 : 9);
}

template <typename T, int DIM>
__device__ __forceinline__ Segment<T, DIM> stage_segment(const KParams &kp, int C, int wave, const PC<T> &pc,
                                                         const int32_t *__restrict__ bin_start,
                                                         const V4<T> *__restrict__ Es, const V4<T> *__restrict__ Bs,
                                                         unsigned char *smem, int lane) {
  Segment<T, DIM> sg;
  const int S = kp.nspecies;
  sg.C = C;
  sg.nb = C * S;
  // segments are visited tile by tile (tiles of max(tx, C) x sty x stz cells,
  // segments row-major inside a tile), as the other particle kernels visit
  // cells: the destinations of neighbouring sources are then written close
  // together in time
  const int TX = C > kp.tx ? C : kp.tx;
  const int spr = TX / C, per_tile = spr * kp.sty * kp.stz;
  const int tile = wave / per_tile, r = wave - tile * per_tile;
  const int ntx = kp.nx / TX, nty = kp.ny / kp.sty;
  const int t2 = tile / ntx;
  sg.i0 = (tile - t2 * ntx) * TX + (r % spr) * C;
  sg.j = (t2 % nty) * kp.sty + (r / spr) % kp.sty;
  sg.k = DIM == 3 ? (t2 / nty) * kp.stz + r / (spr * kp.sty) : 0;
  sg.c0 = sg.i0 + kp.nx * (sg.j + kp.ny * sg.k);
  const int W = C + 2, nB = W * 3 * (DIM == 3 ? 3 : 1), nE = (C + 1) * 2 * (DIM == 3 ? 2 : 1);
  sg.Bg = reinterpret_cast<V4<T> *>(smem);
  sg.Eg = sg.Bg + nB;
  sg.stab = reinterpret_cast<T(*)[8]>(sg.Eg + nE);
  sg.mtab = reinterpret_cast<double *>(sg.stab + 2);
  sg.binb = reinterpret_cast<int *>(sg.mtab + 8);
  sg.keys = sg.binb + binb_slots(sg.nb);
  // centre (i0 - 1 + a, j - 1 + b, k - 1 + c) sits at ghosted index
  // (i0 + a) + gx (j + b) + gxy (k + c); the staged rows are (b, c), x
  // fastest
  constexpr int RB = DIM == 3 ? 9 : 3, RE = DIM == 3 ? 4 : 2;
  const int WE = C + 1;
  auto b_at = [&](int r, int a) {
    return Bs[(sg.i0 + a) + kp.gx * (sg.j + r % 3) + (DIM == 3 ? kp.gxy * (sg.k + r / 3) : 0)];
  };
  auto e_at = [&](int r, int a) { return Es[gidx<DIM>(kp, sg.i0 + a, sg.j + r % 2, sg.k + r / 2)]; };
  const int nbb = binb_slots(sg.nb);
  auto bin_at = [&](int t) { return t <= sg.nb ? bin_start[sg.c0 * S + t] : INT_MAX; };
  // One lane per x position of every staged row: all of the first 64
  // positions' loads are in registers before any of them is stored, so that
  // the staging waits for one round trip to memory instead of one per row
  // (a wave holds a few hundred particles: a round trip per row would be a
  // sizeable part of its time), and no lane divides by the row length.
  // Rows longer than 64 and bin starts past the first 64 finish in plain
  // loops.
  V4<T> vb[RB], ve[RE];
  int vn = 0;
  const T tq = pc.q[lane & 7], tbeta = pc.beta[lane & 7];
  const double tm = kp.m[lane & 7];
  if (lane < W) {
#pragma unroll
    for (int r = 0; r < RB; ++r) vb[r] = b_at(r, lane);
  }
  if (lane < WE) {
#pragma unroll
    for (int r = 0; r < RE; ++r) ve[r] = e_at(r, lane);
  }
  if (lane < nbb) vn = bin_at(lane);
  if (lane < W) {
#pragma unroll
    for (int r = 0; r < RB; ++r) sg.Bg[r * W + lane] = vb[r];
  }
  if (lane < WE) {
#pragma unroll
    for (int r = 0; r < RE; ++r) sg.Eg[r * WE + lane] = ve[r];
  }
  if (lane < nbb) sg.binb[lane] = vn;
  for (int a = lane + 64; a < W; a += 64)
    for (int r = 0; r < RB; ++r) sg.Bg[r * W + a] = b_at(r, a);
  for (int a = lane + 64; a < WE; a += 64)
    for (int r = 0; r < RE; ++r) sg.Eg[r * WE + a] = e_at(r, a);
  for (int t = lane + 64; t < nbb; t += 64) sg.binb[t] = bin_at(t);
  if (lane < 8) {
    sg.stab[0][lane] = tq;
    sg.stab[1][lane] = tbeta;
    sg.mtab[lane] = tm;
  }
  return sg;
}

// Bin (within the segment) of particle p, binb[0] <= p < binb[nb]: the last
// b with binb[b] <= p, by binary search over the staged bin starts.  The
// starts are padded with INT_MAX up to a power of two, so every probe reads
// a valid slot and the search is straight-line code (a wave-uniform number
// of steps, no lane-dependent branch).
__device__ __forceinline__ int segment_bin(const int *binb, int nb, int p) {
  int lo = 0;
  for (int step = pow2_at_least(nb) >> 1; step > 0; step >>= 1) {
    const int m = lo + step;
    lo = binb[m] <= p ? m : lo;
  }
  return lo;
}

// Charge and beta of species s: selected between values for two species
// (the compiler may turn a select of two loads into one load from a
// selected address), else from the LDS table.
template <typename T>
__device__ __forceinline__ void species_consts(int S, int s, T q0, T q1, T b0, T b1, const T (*tab)[8], T &q,
                                               T &beta) {
  if (S == 2) {
    q = s ? q1 : q0;
    beta = s ? b1 : b0;
  } else {
    q = tab[0][s];
    beta = tab[1][s];
  }
}

// Where the lane's particle finds its fields: cell lc of the segment.
template <typename T, int DIM>
__device__ __forceinline__ CellFields<T> segment_fields(const Segment<T, DIM> &sg, int lc) {
  CellFields<T> cf;
  cf.by = sg.C + 2;
  cf.bz = 3 * (sg.C + 2);
  cf.ey = sg.C + 1;
  cf.ez = 2 * (sg.C + 1);
  cf.bc = sg.Bg + (lc + 1) + cf.by + (DIM == 3 ? cf.bz : 0);
  cf.e0 = sg.Eg + lc;
  return cf;
}

// Push pass.  COUNT: the first pass of the re-sort; the particles are only
// read: each one's move (dirc) and the per-(bin, move) counts are written,
// and k_push_scatter later recomputes the push and writes the new state in
// the new order.  !COUNT: push in place with no re-sort; offsets stay
// relative to the old cell, in [-1, 2).
// GB selects the Lorentz factor of S2 and what the pass does:
//   0  gamma(u^n); count the moves (COUNT) or push in place
//   1  gbar from gb; as 0
//   2  gbar from gb; leave the state alone and write, per particle, the next
//      fixed-point value gnx = (gamma(u^n) + gamma(u^{n+1}))/2 of the
//      energy-conserving variant, and into *chg the largest
//      |gnx - gbar| / gbar (as the bits of a non-negative double, so that
//      an integer atomic max orders them; infinite if not finite)
//   3  as 2 with gbar = gamma(u^n) (the iteration's start; gb unused)
template <typename T, int DIM, bool COUNT, int GB>
__global__ __launch_bounds__(64) void k_push(KParams kp, int C, const int32_t *__restrict__ bin_start,
                                             V2<T> *__restrict__ xy, V4<T> *__restrict__ uw, T *__restrict__ zz,
                                             const V4<T> *__restrict__ Es, const V4<T> *__restrict__ Bs,
                                             uint8_t *__restrict__ dirc, uint16_t *__restrict__ cnt,
                                             int32_t *__restrict__ err, void *__restrict__ sink,
                                             const T *__restrict__ gb, T *__restrict__ gnx,
                                             unsigned long long *__restrict__ chg) {
  constexpr int NDIR = DIM == 3 ? 27 : 9;
  constexpr bool LOADG = GB == 1 || GB == 2;
  constexpr bool TRIAL = GB >= 2;
  static_assert(!(TRIAL && COUNT), "a fixed-point pass counts nothing");
  extern __shared__ __attribute__((aligned(32))) unsigned char smem[];
  const int lane = threadIdx.x;
  const PC<T> pc(kp);
  const Segment<T, DIM> sg =
      stage_segment<T, DIM>(kp, C, xcd_remap(blockIdx.x, gridDim.x), pc, bin_start, Es, Bs, smem, lane);
  if constexpr (COUNT)
    for (int t = lane; t < sg.nb * NDIR; t += 64) sg.keys[t] = 0;
  __syncthreads();
  const int S = kp.nspecies;
  const T sq0 = pc.q0, sq1 = pc.q1, sb0 = pc.b0, sb1 = pc.b1;
  T *const sinkT = sink_slot<T>(sink, lane);
  uint8_t *const sinkB = sink_slot<uint8_t>(sink, lane);
  const int p0 = __builtin_amdgcn_readfirstlane(sg.binb[0]);
  const int p1 = __builtin_amdgcn_readfirstlane(sg.binb[sg.nb]);
  // rounds start on 64-byte boundaries (lanes before p0 idle)
  const int pal = p0 & ~(round_align<T, 64>() - 1);
  const int rounds = __builtin_amdgcn_readfirstlane(p1 > p0 ? (p1 - pal + 63) >> 6 : 0);
  PRec<T> cur{}, nxt{};
  int p = pal + lane;
  int bad = 0;
  double dmax = 0.0;
  if (rounds > 0) {
    load_rec<T, DIM>(p, p1, xy, uw, zz, cur);
    load_gbar<LOADG>(p, p1, gb, cur);
  }
  // enter the loop with nothing in flight, so the loop's waits only count
  // its own loads and stores
  __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 2
  for (int r = 0; r < rounds; ++r) {
    const int pn = p + 64;
    load_rec<T, DIM>(pn, p1, xy, uw, zz, nxt);
    load_gbar<LOADG>(pn, p1, gb, nxt);
    // lanes outside [p0, p1) compute on a valid particle's copy and store
    // into the sink
    const bool pv = p >= p0 && p < p1;
    const int b = segment_bin(sg.binb, sg.nb, min(max(p, p0), p1 - 1));
    const int lc = S == 2 ? b >> 1 : b / S, s = b - lc * S;
    T qs, bs;
    species_consts<T>(S, s, sq0, sq1, sb0, sb1, sg.stab, qs, bs);
    T fx, fy, fz, nx, ny, nz;
    T ign;
    push_one<T, DIM, LOADG>(kp, pc, segment_fields(sg, lc), bs, cur, fx, fy, fz, nx, ny, nz, ign);
    if constexpr (TRIAL) {
      const T g0 = kp.nonrel ? T(1) : sqrt(T(1) + (cur.ux * cur.ux + cur.uy * cur.uy + cur.uz * cur.uz) * pc.invc2);
      const T g1 = kp.nonrel ? T(1) : sqrt(T(1) + (nx * nx + ny * ny + nz * nz) * pc.invc2);
      const T gm = T(0.5) * (g0 + g1);
      const T gin = GB == 2 ? cur.g : g0;
      *(pv ? gnx + p : sinkT) = gm;
      const double d = fabs((double)gm - (double)gin) / (double)gin;
      dmax = pv ? (d <= dmax ? dmax : (d == d ? d : __builtin_inf())) : dmax;
    } else if constexpr (COUNT) {
      int flag = 0;
      const int mx = cross_cell<T>(fx, flag);
      const int my = cross_cell<T>(fy, flag);
      const int mz = DIM == 3 ? cross_cell<T>(fz, flag) : 0;
      bad |= pv ? flag : 0;
      const int dir = (mx + 1) + 3 * (my + 1) + (DIM == 3 ? 9 * (mz + 1) : 0);
      *(pv ? dirc + p : sinkB) = (uint8_t)dir;
      if (pv) atomicAdd(&sg.keys[b * NDIR + dir], 1);  // integer: order-independent
    } else {
      // no re-sort: offsets stay relative to the old cell, in [-1, 2)
      bool ok = fx >= T(-1) && fx < T(2) && fy >= T(-1) && fy < T(2);
      if constexpr (DIM == 3) ok = ok && fz >= T(-1) && fz < T(2);
      bad |= (pv && !ok) ? 1 : 0;
      store_rec<T, DIM>(!pv, (size_t)p, xy, uw, zz, sink_slot<V4<T>>(sink, lane), fx, fy, fz, nx, ny, nz, cur.w);
    }
    cur = nxt;
    p = pn;
  }
  if (__ballot(bad) && lane == 0) atomicOr(err, 1);
  if constexpr (TRIAL) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o));
    // one atomic per wave on a single address serialises (tens of thousands
    // of waves); a wave whose value is not above the one already stored has
    // nothing to add, so it reads first and skips the atomic
    const unsigned long long v = (unsigned long long)__double_as_longlong(dmax);
    if (lane == 0 && v > __hip_atomic_load(chg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(chg, v);
  }
  if constexpr (COUNT) {
    __syncthreads();
    // counts out in [move][bin] order: one lane per bin, consecutive bins
    // per move
    const size_t nbins = (size_t)kp.nbins;
    bool over = false;  // a move class beyond the 16-bit counters
    for (int bin = lane; bin < sg.nb; bin += 64) {
#pragma unroll
      for (int dir = 0; dir < NDIR; ++dir) {
        const int v = sg.keys[bin * NDIR + dir];
        over = over || v > 65535;
        cnt[(size_t)dir * nbins + (size_t)sg.c0 * S + bin] = (uint16_t)(v > 65535 ? 65535 : v);
      }
    }
    if (over) atomicOr(err, 2);
  }
}

// ---------------------------------------------------------------------------
// re-sort, step 2: per destination bin, the offset of each incoming move
// class in source order (sources are earlier in the old order iff their cell
// index is smaller), and the bin total.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int source_shift(int r, int c, int n) {
  // r-th smallest of the wrapped coordinates {c-1, c, c+1} -> its shift
  if (c == 0) return r == 0 ? 0 : (r == 1 ? 1 : -1);
  if (c == n - 1) return r == 0 ? 1 : (r == 1 ? -1 : 0);
  return r - 1;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_sort_offsets(KParams kp, const uint16_t *__restrict__ cnt,
                                                      uint16_t *__restrict__ pre, int32_t *__restrict__ total,
                                                      int32_t *__restrict__ err) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= kp.nbins) return;
  const int S = kp.nspecies;
  const int cell = d / S, s = d % S;
  const int ci = cell % kp.nx, cj = (cell / kp.nx) % kp.ny, ck = cell / (kp.nx * kp.ny);
  const size_t nb = (size_t)kp.nbins;
  int run = 0;
  const int NZ = DIM == 3 ? 3 : 1;
  for (int rz = 0; rz < NZ; ++rz) {
    const int sz = DIM == 3 ? source_shift(rz, ck, kp.nz) : 0;
    for (int ry = 0; ry < 3; ++ry) {
      const int sy = source_shift(ry, cj, kp.ny);
      for (int rx = 0; rx < 3; ++rx) {
        const int sx = source_shift(rx, ci, kp.nx);
        const int src = wrapi(ci + sx, kp.nx) + kp.nx * (wrapi(cj + sy, kp.ny) + kp.ny * (DIM == 3 ? wrapi(ck + sz, kp.nz) : 0));
        const int dir = (1 - sx) + 3 * (1 - sy) + (DIM == 3 ? 9 * (1 - sz) : 0);
        const int c16 = cnt[(size_t)dir * nb + (size_t)src * S + s];
        pre[(size_t)dir * nb + d] = (uint16_t)(run > 65535 ? 65535 : run);
        run += c16;
      }
    }
  }
  if (run > 65535) atomicOr(err, 2);
  total[d] = run;
}

// One round of the pushing scatter for particle p of the segment, on
// record buffer (cur, dc), which it then refills with the round three
// ahead; see k_push_scatter.
template <typename T, int DIM, bool PERM, bool GB>
__device__ __forceinline__ void scatter_round(const KParams &kp, const PC<T> &pc, const Segment<T, DIM> &sg,
                                              int p1, int lane, unsigned long long lt, int ntot,
                                              const V2<T> *__restrict__ xy, const V4<T> *__restrict__ uw,
                                              const T *__restrict__ zz, const T *__restrict__ gb,
                                              const uint8_t *__restrict__ dirc,
                                              V2<T> *__restrict__ xo, V4<T> *__restrict__ uo, T *__restrict__ zo,
                                              int32_t *__restrict__ perm, void *__restrict__ sink, T q0, T q1,
                                              T b0, T b1, double m0, double m1, int &p, int &bad, int &nclamp,
                                              double &ke, PRec<T> &cur, uint8_t &dc) {
  constexpr int NDIR = DIM == 3 ? 27 : 9;
  constexpr int DBITS = DIM == 3 ? 5 : 4;  // bits of a move code
  const int S = kp.nspecies;
  const int dcur = dc;
  const bool pv = p < p1;
  const int b = segment_bin(sg.binb, sg.nb, min(p, p1 - 1));
  const int lc = S == 2 ? b >> 1 : b / S, s = b - lc * S;
  T qs, bs;
  species_consts<T>(S, s, q0, q1, b0, b1, sg.stab, qs, bs);
  T fx, fy, fz, nx, ny, nz, ign;
  push_one<T, DIM, GB>(kp, pc, segment_fields(sg, lc), bs, cur, fx, fy, fz, nx, ny, nz, ign);
  // S7's kinetic term of the pushed particle, in FP64 whatever T:
  // w m c^2 (gamma - 1) = w m |u|^2 / (gamma + 1), or w m |u|^2 / 2 without
  // relativity
  {
    const double ux = nx, uy = ny, uz = nz;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double wm = (double)cur.w * (S == 2 ? (s ? m1 : m0) : sg.mtab[s]);
    const double term = kp.nonrel ? 0.5 * wm * uu : kinetic_rel(wm * uu, uu * kp.inv_c2, ign);
    ke += pv ? term : 0.0;
  }
  // the new state goes where the counting pass counted it (move dcur),
  // with its offsets taken relative to that cell
  int off = 0, clamp = 0;
  fx = place_offset<T>(fx, dcur % 3 - 1, off, clamp);
  fy = place_offset<T>(fy, (dcur / 3) % 3 - 1, off, clamp);
  if constexpr (DIM == 3) fz = place_offset<T>(fz, dcur / 9 - 1, off, clamp);
  bad |= (pv && off) ? 4 : 0;
  nclamp += __popcll(__ballot(pv && clamp));  // wave-uniform
  // lanes of this round with the same (bin, move) key: the bin's particles
  // occupy the contiguous lanes [f, l) of the round, so only the move code
  // needs matching, one ballot per bit
  const int rb = p - lane;
  const int f = sg.binb[b] - rb, l = sg.binb[b + 1] - rb;
  const unsigned long long fmask = f <= 0 ? ~0ull : (~0ull << f);
  const unsigned long long lmask = l <= 0 ? 0ull : (l >= 64 ? ~0ull : ((1ull << l) - 1ull));
  unsigned long long same = __ballot(pv) & fmask & lmask;
#pragma unroll
  for (int bit = 0; bit < DBITS; ++bit) {
    const bool on = (dcur >> bit) & 1;
    const unsigned long long ones = __ballot(on);
    same &= on ? ones : ~ones;
  }
  const int key = pv ? b * NDIR + dcur : 0;
  int pos = 0;
  if (pv) pos = sg.keys[key] + __popcll(same & lt);
  __builtin_amdgcn_wave_barrier();
  // the highest lane of each key advances that key's base
  if (pv && (same >> lane) == 1ull) sg.keys[key] += __popcll(same);
  // only reachable out of range when a bin overflowed the 16-bit
  // counters (flagged); lanes past the end store into the sink
  const bool ok = pv && pos >= 0 && pos < ntot;
  bad |= (pv && !ok) ? 2 : 0;
  store_rec<T, DIM>(!ok, (size_t)(ok ? pos : 0), xo, uo, zo, sink_slot<V4<T>>(sink, lane), fx, fy, fz, nx, ny, nz,
                    cur.w);
  if constexpr (PERM) *(ok ? perm + p : sink_slot<int32_t>(sink, lane)) = pos;
  __builtin_amdgcn_wave_barrier();
  load_rec<T, DIM>(p + 3 * 64, p1, xy, uw, zz, cur);
  load_gbar<GB>(p + 3 * 64, p1, gb, cur);
  dc = dirc[load_index(p + 3 * 64, p1)];
  p += 64;
}

// ---------------------------------------------------------------------------
// re-sort, step 3: push again and scatter, stably, into the back buffers.
// The wave walks its row segment as the counting pass did.  It first
// resolves, for every (bin, move) key of the segment, where that class's run
// starts in the new order (new bin start of the destination + offset of this
// source among the destination's sources).  In the loop every particle is
// pushed once more (push_one, as in the counting pass; its offsets are
// taken relative to the cell of the recorded move, see place_offset), and
// its new state is written at that base plus its rank among the same-key
// lanes of earlier rounds and lower lanes of this round.  The particle state
// is thus read twice and written once per step.
// ---------------------------------------------------------------------------
template <typename T, int DIM, bool PERM, bool GB>
__global__ __launch_bounds__(64) void k_push_scatter(KParams kp, int C, const int32_t *__restrict__ bin_start,
                                                     const V2<T> *__restrict__ xy,
                                                     const V4<T> *__restrict__ uw, const T *__restrict__ zz,
                                                     const V4<T> *__restrict__ Es, const V4<T> *__restrict__ Bs,
                                                     const uint8_t *__restrict__ dirc,
                                                     const uint16_t *__restrict__ pre,
                                                     const int32_t *__restrict__ bsn, V2<T> *__restrict__ xo,
                                                     V4<T> *__restrict__ uo, T *__restrict__ zo, int ntot,
                                                     int32_t *__restrict__ err,
                                                     unsigned long long *__restrict__ clamps,
                                                     int32_t *__restrict__ perm, void *__restrict__ sink,
                                                     const T *__restrict__ gb, double *__restrict__ kep) {
  constexpr int NDIR = DIM == 3 ? 27 : 9;
  extern __shared__ __attribute__((aligned(32))) unsigned char smem[];
  const int lane = threadIdx.x;
  const PC<T> pc(kp);
  const Segment<T, DIM> sg =
      stage_segment<T, DIM>(kp, C, xcd_remap(blockIdx.x, gridDim.x), pc, bin_start, Es, Bs, smem, lane);
  const int S = kp.nspecies;
  const size_t nbins = (size_t)kp.nbins;
  // one lane per bin of the segment, all moves at once: the 2 NDIR loads
  // of a lane are in flight together, and for each move the lanes read
  // consecutive destination bins
  for (int b0 = 0; b0 < sg.nb; b0 += 64) {
    // lanes past the segment's bins compute (and do not store) its last
    // bin's keys, so that every address is a valid one
    const bool on = b0 + lane < sg.nb;
    const int bin = on ? b0 + lane : sg.nb - 1;
    const int lc = S == 2 ? bin >> 1 : bin / S, s = bin - lc * S;
    int v[NDIR];
#pragma unroll
    for (int dir = 0; dir < NDIR; ++dir) {
      const int mx = dir % 3 - 1, my = (dir / 3) % 3 - 1, mz = dir / 9 - 1;
      const int dc = wrapi(sg.i0 + lc + mx, kp.nx) +
                     kp.nx * (wrapi(sg.j + my, kp.ny) + kp.ny * (DIM == 3 ? wrapi(sg.k + mz, kp.nz) : 0));
      const int d = dc * S + s;
      v[dir] = bsn[d] + (int)pre[(size_t)dir * nbins + d];
    }
    if (on) {
#pragma unroll
      for (int dir = 0; dir < NDIR; ++dir) sg.keys[bin * NDIR + dir] = v[dir];
    }
  }
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int p0 = __builtin_amdgcn_readfirstlane(sg.binb[0]);
  const int p1 = __builtin_amdgcn_readfirstlane(sg.binb[sg.nb]);
  const int rounds = __builtin_amdgcn_readfirstlane(p1 > p0 ? (p1 - p0 + 63) >> 6 : 0);
  // Three record buffers in rotation: while one round is pushed and
  // stored, the loads of the next two are in flight.  Each round refills
  // its own buffer with the round three ahead once it has been used, so no
  // buffer is ever copied into another (a copy would wait for its loads).
  // The loop runs whole groups of three rounds, so every pass through it
  // issues the same loads in the same order and its waits stay exact; the
  // last one or two rounds follow it.
  PRec<T> rb0{}, rb1{}, rb2{};
  uint8_t db0 = 0, db1 = 0, db2 = 0;
  int p = p0 + lane, bad = 0, nclamp = 0;
  double ke = 0.0;  // this lane's kinetic energy of the pushed particles
  if (rounds > 0) {
    load_rec<T, DIM>(p, p1, xy, uw, zz, rb0);
    load_gbar<GB>(p, p1, gb, rb0);
    db0 = dirc[load_index(p, p1)];
    load_rec<T, DIM>(p + 64, p1, xy, uw, zz, rb1);
    load_gbar<GB>(p + 64, p1, gb, rb1);
    db1 = dirc[load_index(p + 64, p1)];
    load_rec<T, DIM>(p + 128, p1, xy, uw, zz, rb2);
    load_gbar<GB>(p + 128, p1, gb, rb2);
    db2 = dirc[load_index(p + 128, p1)];
  }
  // enter the loop with nothing in flight, so that the waits in the loop
  // count only the loop's own loads and stores
  __builtin_amdgcn_s_waitcnt(0);
  const T sq0 = pc.q0, sq1 = pc.q1, sb0 = pc.b0, sb1 = pc.b1;
  const double sm0 = kp.m[0], sm1 = kp.m[1];
#define RELSIM_SCATTER_ROUND(rb, db)                                                                            \
  scatter_round<T, DIM, PERM, GB>(kp, pc, sg, p1, lane, lt, ntot, xy, uw, zz, gb, dirc, xo, uo, zo, perm, sink, \
                                  sq0, sq1, sb0, sb1, sm0, sm1, p, bad, nclamp, ke, rb, db)
  int r = 0;
#pragma unroll 1
  for (; r + 3 <= rounds; r += 3) {
    RELSIM_SCATTER_ROUND(rb0, db0);
    RELSIM_SCATTER_ROUND(rb1, db1);
    RELSIM_SCATTER_ROUND(rb2, db2);
  }
  if (r < rounds) RELSIM_SCATTER_ROUND(rb0, db0);
  if (r + 1 < rounds) RELSIM_SCATTER_ROUND(rb1, db1);
#undef RELSIM_SCATTER_ROUND
  const int ball = __ballot(bad & 2) ? 2 : 0;
  const int balm = __ballot(bad & 4) ? 8 : 0;
  if ((ball | balm) && lane == 0) atomicOr(err, ball | balm);
  if (nclamp && lane == 0) atomicAdd(clamps, (unsigned long long)nclamp);
  // the wave's kinetic energy, summed in a fixed butterfly (every lane ends
  // with the same value), one partial per segment
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ke += __shfl_xor(ke, o);
  if (lane == 0) kep[xcd_remap(blockIdx.x, gridDim.x)] = ke;
}

// ---------------------------------------------------------------------------
// cell id of every particle from the bin ranges (one wave per cell)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_fill_cells(KParams kp, const int32_t *__restrict__ bin_start,
                                                   int32_t *__restrict__ cell) {
  const int c = blockIdx.x;
  const int b = bin_start[c * kp.nspecies], e = bin_start[(c + 1) * kp.nspecies];
  for (int p = b + (int)threadIdx.x; p < e; p += 64) cell[p] = c;
}

// ---------------------------------------------------------------------------
// S7 kinetic part: per-block FP64 partial sums (fixed order)
// ---------------------------------------------------------------------------
template <typename T, int DIM, int G>
__global__ __launch_bounds__(64) void k_kinetic(KParams kp, const int32_t *__restrict__ bin_start,
                                                const V4<T> *__restrict__ uw, double *__restrict__ partials) {
  // one block per 64/G cells in slot order; block b writes partials[b]
  __shared__ double red[64];
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const CellSpan cs = slot_span<G>(kp, bin_start, blk, grp);
  const double invc2 = kp.inv_c2;
  const int S = kp.nspecies;
  double acc = 0.0;
  for (int p = cs.pbeg + gl; p < cs.pend; p += G) {
    int s = 0;
    if (S == 2) {
      s = p >= cs.bound[1] ? 1 : 0;
    } else {
#pragma unroll
      for (int s2 = 1; s2 < 8; ++s2)
        if (p >= cs.bound[s2]) s = s2;
    }
    // 3D: uw points at the records, whose second half is (u, w)
    const V4<T> r = DIM == 3 ? uw[2 * (size_t)p + 1] : uw[p];
    const double ux = r.x, uy = r.y, uz = r.z;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double wm = (double)r.w * kp.m[s];
    // (gamma - 1) c^2 = |u|^2 / (sqrt(1 + |u|^2/c^2) + 1), without cancellation
    acc += kp.nonrel ? 0.5 * wm * uu : wm * uu / (sqrt(1.0 + uu * invc2) + 1.0);
  }
  red[lane] = acc;
  __syncthreads();
  for (int o = 32; o >= 1; o >>= 1) {
    if (lane < o) red[lane] += red[lane + o];
    __syncthreads();
  }
  if (lane == 0) partials[blk] = red[0];
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (three-phase: block scans, scan of block sums, add)
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 2 * kScanBlock;

__device__ __forceinline__ int block_exclusive_scan(int v, int *lds, int &total) {
  // inclusive warp scan via shuffles, then across waves through LDS
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  if (wid == 0) {
    const int nw = blockDim.x >> 6;
    int t = lane < nw ? lds[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(t, o);
      if (lane >= o) t += y;
    }
    if (lane < nw) lds[64 + lane] = t;
  }
  __syncthreads();
  const int wprefix = wid > 0 ? lds[64 + wid - 1] : 0;
  total = lds[64 + (blockDim.x >> 6) - 1];
  __syncthreads();
  return wprefix + x - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                            int n, int32_t *__restrict__ bsum) {
  __shared__ int lds[128];
  const size_t base = (size_t)blockIdx.x * kScanItems;
  const size_t i0 = base + 2 * threadIdx.x;
  const int a = i0 < (size_t)n ? in[i0] : 0;
  const int b = i0 + 1 < (size_t)n ? in[i0 + 1] : 0;
  int total;
  const int ex = block_exclusive_scan(a + b, lds, total);
  if (i0 < (size_t)n) out[i0] = ex;
  if (i0 + 1 < (size_t)n) out[i0 + 1] = ex + a;
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_top(int32_t *__restrict__ bsum, int nb, int32_t *__restrict__ out,
                                                         int n) {
  __shared__ int lds[128];
  int carry = 0;
  for (int base = 0; base < nb; base += kScanBlock) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int total;
    const int ex = block_exclusive_scan(v, lds, total);
    if (i < nb) bsum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(256) void k_scan_add(int32_t *__restrict__ out, int n, const int32_t *__restrict__ bsum) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < (size_t)n) out[i] += bsum[i / kScanItems];
}

template <typename T>
const T *cp(const void *p) {
  return static_cast<const T *>(p);
}
template <typename T>
T *mp(void *p) {
  return static_cast<T *>(p);
}

template <typename T, int G>
void deposit_impl(const KParams &kp, const PartPtrs &pp, const void *Bst, void *S, hipStream_t st) {
  const int nblk = (kp.ncells + (64 / G) - 1) / (64 / G);
  if (pp.gbar)
    hipLaunchKernelGGL((k_deposit_cells<T, G, true>), dim3(nblk), dim3(64), 0, st, kp, pp.bin_start,
                       cp<V2<T>>(pp.xy), cp<V4<T>>(pp.uw), cp<V4<T>>(Bst), mp<T>(S), cp<T>(pp.gbar));
  else
    hipLaunchKernelGGL((k_deposit_cells<T, G, false>), dim3(nblk), dim3(64), 0, st, kp, pp.bin_start,
                       cp<V2<T>>(pp.xy), cp<V4<T>>(pp.uw), cp<V4<T>>(Bst), mp<T>(S), nullptr);
}

template <typename T>
void deposit3_impl(const KParams &kp, const PartPtrs &pp, const void *Bst, void *S, hipStream_t st) {
  const int nblk = (kp.ncells + 15) / 16;
  if (pp.gbar)
    hipLaunchKernelGGL((k_deposit_split3<T, true>), dim3(nblk), dim3(64), 0, st, kp, pp.bin_start,
                       cp<V2<T>>(pp.xy), cp<V4<T>>(pp.uw), cp<T>(pp.z), cp<V4<T>>(Bst), mp<T>(S), cp<T>(pp.gbar));
  else
    hipLaunchKernelGGL((k_deposit_split3<T, false>), dim3(nblk), dim3(64), 0, st, kp, pp.bin_start,
                       cp<V2<T>>(pp.xy), cp<V4<T>>(pp.uw), cp<T>(pp.z), cp<V4<T>>(Bst), mp<T>(S), nullptr);
}

template <typename T, int DIM, bool COUNT, int GB>
void push_launch(const KParams &kp, int C, const PartPtrs &pp, const void *Est, const void *Bst, uint8_t *dirc,
                 uint16_t *cnt, int32_t *err, void *sink, void *gnx, unsigned long long *chg, hipStream_t st) {
  const int nblk = kp.ncells / C;
  const size_t lds = segment_lds_bytes<T, DIM>(C, kp.nspecies);
  hipLaunchKernelGGL((k_push<T, DIM, COUNT, GB>), dim3(nblk), dim3(64), lds, st, kp, C, pp.bin_start,
                     mp<V2<T>>(pp.xy), mp<V4<T>>(pp.uw), mp<T>(pp.z), cp<V4<T>>(Est), cp<V4<T>>(Bst), dirc, cnt, err,
                     sink, cp<T>(pp.gbar), mp<T>(gnx), chg);
}

template <typename T, int DIM>
void push_impl(const KParams &kp, int C, const PartPtrs &pp, const void *Est, const void *Bst, uint8_t *dirc,
               uint16_t *cnt, int32_t *err, int count_moves, void *sink, hipStream_t st) {
  if (pp.gbar) {
    if (count_moves)
      push_launch<T, DIM, true, 1>(kp, C, pp, Est, Bst, dirc, cnt, err, sink, nullptr, nullptr, st);
    else
      push_launch<T, DIM, false, 1>(kp, C, pp, Est, Bst, dirc, cnt, err, sink, nullptr, nullptr, st);
  } else {
    if (count_moves)
      push_launch<T, DIM, true, 0>(kp, C, pp, Est, Bst, dirc, cnt, err, sink, nullptr, nullptr, st);
    else
      push_launch<T, DIM, false, 0>(kp, C, pp, Est, Bst, dirc, cnt, err, sink, nullptr, nullptr, st);
  }
}

template <typename T, int DIM>
void gamma_mean_impl(const KParams &kp, int C, const PartPtrs &pp, const void *Est, const void *Bst, int32_t *err,
                     void *sink, void *gnx, unsigned long long *chg, hipStream_t st) {
  if (pp.gbar)
    push_launch<T, DIM, false, 2>(kp, C, pp, Est, Bst, nullptr, nullptr, err, sink, gnx, chg, st);
  else
    push_launch<T, DIM, false, 3>(kp, C, pp, Est, Bst, nullptr, nullptr, err, sink, gnx, chg, st);
}

template <typename T, int DIM, bool PERM, bool GB>
void scatter_launch(const KParams &kp, int C, const PartPtrs &src, const void *Est, const void *Bst,
                    const uint8_t *dirc, const uint16_t *pre, const int32_t *bsn, const PartPtrs &out, int ntot,
                    int32_t *err, unsigned long long *clamps, int32_t *perm, void *sink, double *kep,
                    hipStream_t st) {
  const int nblk = kp.ncells / C;
  const size_t lds = segment_lds_bytes<T, DIM>(C, kp.nspecies);
  hipLaunchKernelGGL((k_push_scatter<T, DIM, PERM, GB>), dim3(nblk), dim3(64), lds, st, kp, C, src.bin_start,
                     cp<V2<T>>(src.xy), cp<V4<T>>(src.uw), cp<T>(src.z), cp<V4<T>>(Est), cp<V4<T>>(Bst), dirc, pre,
                     bsn, mp<V2<T>>(out.xy), mp<V4<T>>(out.uw), mp<T>(out.z), ntot, err, clamps, perm, sink,
                     cp<T>(src.gbar), kep);
}

template <typename T, int DIM>
void scatter_impl(const KParams &kp, int C, const PartPtrs &src, const void *Est, const void *Bst,
                  const uint8_t *dirc, const uint16_t *pre, const int32_t *bsn, const PartPtrs &out, int ntot,
                  int32_t *err, unsigned long long *cl, int32_t *perm, void *sink, double *kep, hipStream_t st) {
  if (src.gbar) {
    if (perm)
      scatter_launch<T, DIM, true, true>(kp, C, src, Est, Bst, dirc, pre, bsn, out, ntot, err, cl, perm, sink, kep,
                                         st);
    else
      scatter_launch<T, DIM, false, true>(kp, C, src, Est, Bst, dirc, pre, bsn, out, ntot, err, cl, perm, sink,
                                          kep, st);
  } else {
    if (perm)
      scatter_launch<T, DIM, true, false>(kp, C, src, Est, Bst, dirc, pre, bsn, out, ntot, err, cl, perm, sink,
                                          kep, st);
    else
      scatter_launch<T, DIM, false, false>(kp, C, src, Est, Bst, dirc, pre, bsn, out, ntot, err, cl, perm, sink,
                                           kep, st);
  }
}

template <typename T, int DIM, int G>
void kinetic_impl(const KParams &kp, const PartPtrs &pp, double *partials, hipStream_t st) {
  const int nblk = (kp.ncells + (64 / G) - 1) / (64 / G);
  // 3D: the momenta are the second half of each record in xy
  hipLaunchKernelGGL((k_kinetic<T, DIM, G>), dim3(nblk), dim3(64), 0, st, kp, pp.bin_start,
                     cp<V4<T>>(DIM == 3 ? pp.xy : pp.uw), partials);
}

// Dispatch over (precision, dim, group) to the template instances.
template <template <typename, int, int> class F, typename... A>
void dispatch(int prec, int dim, int group, A &&...args) {
#define RELSIM_CASE(TT, DD, GG) \
  if (dim == DD && group == GG) return F<TT, DD, GG>::run(args...);
  if (prec == RELSIM_MIXED) {
    RELSIM_CASE(float, 2, 4) RELSIM_CASE(float, 2, 8) RELSIM_CASE(float, 2, 16) RELSIM_CASE(float, 2, 32)
    RELSIM_CASE(float, 2, 64) RELSIM_CASE(float, 3, 4) RELSIM_CASE(float, 3, 8) RELSIM_CASE(float, 3, 16)
    RELSIM_CASE(float, 3, 32) RELSIM_CASE(float, 3, 64)
  } else {
    RELSIM_CASE(double, 2, 4) RELSIM_CASE(double, 2, 8) RELSIM_CASE(double, 2, 16) RELSIM_CASE(double, 2, 32)
    RELSIM_CASE(double, 2, 64) RELSIM_CASE(double, 3, 4) RELSIM_CASE(double, 3, 8) RELSIM_CASE(double, 3, 16)
    RELSIM_CASE(double, 3, 32) RELSIM_CASE(double, 3, 64)
  }
#undef RELSIM_CASE
}

template <typename T, int D, int G>
struct KineticF {
  template <typename... A>
  static void run(A &&...a) { kinetic_impl<T, D, G>(a...); }
};

}  // namespace

void launch_stage_field(const KParams &kp, int prec, const double *F, void *out, hipStream_t st) {
  const int nblk = (kp.nghost + 255) / 256;
  if (prec == RELSIM_MIXED) {
    if (kp.dim == 2)
      hipLaunchKernelGGL((k_stage_field<float, 2>), dim3(nblk), dim3(256), 0, st, kp, F, mp<V4<float>>(out));
    else
      hipLaunchKernelGGL((k_stage_field<float, 3>), dim3(nblk), dim3(256), 0, st, kp, F, mp<V4<float>>(out));
  } else {
    if (kp.dim == 2)
      hipLaunchKernelGGL((k_stage_field<double, 2>), dim3(nblk), dim3(256), 0, st, kp, F, mp<V4<double>>(out));
    else
      hipLaunchKernelGGL((k_stage_field<double, 3>), dim3(nblk), dim3(256), 0, st, kp, F, mp<V4<double>>(out));
  }
}

void launch_deposit_cells(const KParams &kp, int prec, int group, const PartPtrs &pp, const void *Bst, void *S,
                          hipStream_t st) {
  const bool f = prec == RELSIM_MIXED;
  if (kp.dim == 3) return f ? deposit3_impl<float>(kp, pp, Bst, S, st) : deposit3_impl<double>(kp, pp, Bst, S, st);
  switch (group) {
    case 4: return f ? deposit_impl<float, 4>(kp, pp, Bst, S, st) : deposit_impl<double, 4>(kp, pp, Bst, S, st);
    case 8: return f ? deposit_impl<float, 8>(kp, pp, Bst, S, st) : deposit_impl<double, 8>(kp, pp, Bst, S, st);
    case 16: return f ? deposit_impl<float, 16>(kp, pp, Bst, S, st) : deposit_impl<double, 16>(kp, pp, Bst, S, st);
    case 32: return f ? deposit_impl<float, 32>(kp, pp, Bst, S, st) : deposit_impl<double, 32>(kp, pp, Bst, S, st);
    case 64: return f ? deposit_impl<float, 64>(kp, pp, Bst, S, st) : deposit_impl<double, 64>(kp, pp, Bst, S, st);
  }
}

template <typename T, typename MT>
void assemble_as(const KParams &kp, const void *S, double *J, void *M, hipStream_t st) {
  const int nblk = (kp.ncells + 255) / 256;
  if (kp.dim == 2)
    hipLaunchKernelGGL((k_assemble<T, 2, MT>), dim3(nblk), dim3(256), 0, st, kp, cp<T>(S), J, mp<MT>(M));
  else
    hipLaunchKernelGGL((k_assemble<T, 3, MT>), dim3(nblk), dim3(256), 0, st, kp, cp<T>(S), J, mp<MT>(M));
}

void launch_assemble(const KParams &kp, int prec, int mass_fp32, const void *S, double *J, void *M,
                     hipStream_t st) {
  if (prec != RELSIM_MIXED)
    assemble_as<double, double>(kp, S, J, M, st);
  else if (mass_fp32)
    assemble_as<float, float>(kp, S, J, M, st);
  else
    assemble_as<float, double>(kp, S, J, M, st);
}

size_t push_lds_bytes(const KParams &kp, int prec, int cells) {
  const bool f = prec == RELSIM_MIXED;
  if (kp.dim == 3)
    return f ? segment_lds_bytes<float, 3>(cells, kp.nspecies) : segment_lds_bytes<double, 3>(cells, kp.nspecies);
  return f ? segment_lds_bytes<float, 2>(cells, kp.nspecies) : segment_lds_bytes<double, 2>(cells, kp.nspecies);
}

void launch_push(const KParams &kp, int prec, int cells, const PartPtrs &pp, const void *Est, const void *Bst,
                 uint8_t *dirc, uint16_t *cnt, int32_t *err, int count_moves, void *sink, hipStream_t st) {
  const bool f = prec == RELSIM_MIXED;
  if (kp.dim == 3)
    return f ? push_impl<float, 3>(kp, cells, pp, Est, Bst, dirc, cnt, err, count_moves, sink, st)
             : push_impl<double, 3>(kp, cells, pp, Est, Bst, dirc, cnt, err, count_moves, sink, st);
  return f ? push_impl<float, 2>(kp, cells, pp, Est, Bst, dirc, cnt, err, count_moves, sink, st)
           : push_impl<double, 2>(kp, cells, pp, Est, Bst, dirc, cnt, err, count_moves, sink, st);
}

void launch_gamma_mean(const KParams &kp, int prec, int cells, const PartPtrs &pp, const void *Est,
                       const void *Bst, int32_t *err, void *sink, void *gbar_next, unsigned long long *chg,
                       hipStream_t st) {
  const bool f = prec == RELSIM_MIXED;
  if (kp.dim == 3)
    return f ? gamma_mean_impl<float, 3>(kp, cells, pp, Est, Bst, err, sink, gbar_next, chg, st)
             : gamma_mean_impl<double, 3>(kp, cells, pp, Est, Bst, err, sink, gbar_next, chg, st);
  return f ? gamma_mean_impl<float, 2>(kp, cells, pp, Est, Bst, err, sink, gbar_next, chg, st)
           : gamma_mean_impl<double, 2>(kp, cells, pp, Est, Bst, err, sink, gbar_next, chg, st);
}

namespace {
// Per-particle secant step of the energy-conserving fixed point (FP64
// residuals and slopes whatever T, the history kept in T); see
// relsim_gamma_secant.
template <typename T>
__global__ __launch_bounds__(256) void k_gamma_secant(int n, const T *__restrict__ g, T *__restrict__ Fg,
                                                      T *__restrict__ gp, T *__restrict__ rp, int first) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double gd = (double)g[i];
  const double r = (double)Fg[i] - gd;
  if (!first) {
    const double dg = gd - (double)gp[i];
    const double slope = (r - (double)rp[i]) / (dg == 0.0 ? 1.0 : dg);
    const bool use = fabs(dg) > 1e-12 * gd && slope <= -0.1 && slope >= -10.0;
    const double nxt = use ? gd - r / slope : gd + r;
    Fg[i] = (T)(nxt < 1.0 ? 1.0 : nxt);  // a NaN passes through (and fails the caller's test)
  }
  gp[i] = (T)gd;  // exact: gd is g[i]
  rp[i] = (T)r;
}
}  // namespace

void launch_gamma_secant(int prec, int n, const void *g, void *Fg, void *gp, void *rp, int first, hipStream_t st) {
  if (n <= 0) return;
  const int nb = (n + 255) / 256;
  if (prec == RELSIM_MIXED)
    hipLaunchKernelGGL(k_gamma_secant<float>, dim3(nb), dim3(256), 0, st, n, cp<float>(g), mp<float>(Fg),
                       mp<float>(gp), mp<float>(rp), first);
  else
    hipLaunchKernelGGL(k_gamma_secant<double>, dim3(nb), dim3(256), 0, st, n, cp<double>(g), mp<double>(Fg),
                       mp<double>(gp), mp<double>(rp), first);
}

void launch_sort_offsets(const KParams &kp, const uint16_t *cnt, uint16_t *pre, int32_t *total, int32_t *err,
                         hipStream_t st) {
  const int nblk = (kp.nbins + 255) / 256;
  if (kp.dim == 2)
    hipLaunchKernelGGL((k_sort_offsets<2>), dim3(nblk), dim3(256), 0, st, kp, cnt, pre, total, err);
  else
    hipLaunchKernelGGL((k_sort_offsets<3>), dim3(nblk), dim3(256), 0, st, kp, cnt, pre, total, err);
}

size_t scan_tmp_elems(int n) { return (size_t)(n + kScanItems - 1) / kScanItems + 1; }

void launch_scan(const int32_t *in, int32_t *out, int n, int32_t *tmp, hipStream_t st) {
  const int nb = (n + kScanItems - 1) / kScanItems;
  if (nb > 0) hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kScanBlock), 0, st, in, out, n, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, st, tmp, nb, out, n);
  if (nb > 1) hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, st, out, n, tmp);
}

void launch_push_scatter(const KParams &kp, int prec, int cells, const PartPtrs &src, const void *Est,
                         const void *Bst, const uint8_t *dirc, const uint16_t *pre, const int32_t *bin_start_new,
                         const PartPtrs &out, int ntot, int32_t *err, unsigned long long *clamps, int32_t *perm,
                         void *sink, double *kep, hipStream_t st) {
  const bool f = prec == RELSIM_MIXED;
  if (kp.dim == 3)
    return f ? scatter_impl<float, 3>(kp, cells, src, Est, Bst, dirc, pre, bin_start_new, out, ntot, err, clamps,
                                      perm, sink, kep, st)
             : scatter_impl<double, 3>(kp, cells, src, Est, Bst, dirc, pre, bin_start_new, out, ntot, err, clamps,
                                       perm, sink, kep, st);
  return f ? scatter_impl<float, 2>(kp, cells, src, Est, Bst, dirc, pre, bin_start_new, out, ntot, err, clamps,
                                    perm, sink, kep, st)
           : scatter_impl<double, 2>(kp, cells, src, Est, Bst, dirc, pre, bin_start_new, out, ntot, err, clamps,
                                     perm, sink, kep, st);
}

void launch_fill_cells(const KParams &kp, const int32_t *bin_start, int32_t *cell, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_cells, dim3(kp.ncells), dim3(64), 0, st, kp, bin_start, cell);
}

void launch_kinetic(const KParams &kp, int prec, int group, const PartPtrs &pp, double *partials, hipStream_t st) {
  dispatch<KineticF>(prec, kp.dim, group, kp, pp, partials, st);
}

}  // namespace relsim
