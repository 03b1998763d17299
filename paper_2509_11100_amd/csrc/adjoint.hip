// Hand-written adjoint (reverse mode) of one step, FP64 only.
//
// Forward step of one particle (S1, S2, S6), positions in physical units:
//   B_p = sum_c W_c(x) B^n_c, gbar = gamma(u), b = beta B_p/(gbar c),
//   alpha(b) = (I - [b]x + b b^T)/(1 + b^2), E_p = sum_g W_g(x) E_th_g,
//   z = u + beta E_p, ubar = alpha z, u' = 2 ubar - u, x' = x + dt u'/gamma(u').
// The deposit (S3) enters the linearised objective only through
//   Jbar = Jhat + M E_th = V^-1 sum_p w q W_g ubar_p / gbar_p,
// so its adjoint is, per particle, the derivative of
//   Phi_p = K_p mu_p^T alpha (u + beta E_p),  K_p = -4 pi th dt w q / (V gbar),
// with mu = A^-T lambda_{E_th} gathered at the particle: two node gathers and
// one outer product per particle, no 9 x 9 x offset scatter.
// Gradients of the CIC weights are piecewise constant (one-sided at a node,
// taken from the particle's own cell).  Grid adjoints are accumulated with
// FP64 atomics, after summing the lanes of one cell within the wave (the
// particles are bin-sorted, so a wave holds few cells): one atomic per grid
// entry and cell instead of one per particle.
#include "relsim_internal.h"

namespace relsim {
namespace {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct PState {
  int s;
  double q, beta, m;
  int ci, cj, ck;
  double f[3];
  double u[3];
  double w;
};

template <int DIM>
__device__ __forceinline__ PState load_particle(const KParams &kp, const int32_t *__restrict__ bin_start,
                                                const int32_t *__restrict__ cell, const double *__restrict__ xy,
                                                const double *__restrict__ uw, const double *__restrict__ zz, int p) {
  PState st;
  const int c = cell[p];
  const int S = kp.nspecies;
  int s = 0;
  for (int s2 = 1; s2 < S; ++s2)
    if (p >= bin_start[c * S + s2]) s = s2;
  st.s = s;
  st.q = kp.q[0];
  st.beta = kp.beta[0];
  st.m = kp.m[0];
#pragma unroll
  for (int s2 = 1; s2 < 8; ++s2)
    if (s == s2) {
      st.q = kp.q[s2];
      st.beta = kp.beta[s2];
      st.m = kp.m[s2];
    }
  st.ci = c % kp.nx;
  st.cj = (c / kp.nx) % kp.ny;
  st.ck = c / (kp.nx * kp.ny);
  if (DIM == 3) {
    // one 8-value record per particle at xy: (off_x, off_y, off_z, 0, u_x, u_y, u_z, w)
    const double *r = xy + 8 * (size_t)p;
    st.f[0] = r[0];
    st.f[1] = r[1];
    st.f[2] = r[2];
    st.u[0] = r[4];
    st.u[1] = r[5];
    st.u[2] = r[6];
    st.w = r[7];
  } else {
    st.f[0] = xy[2 * (size_t)p];
    st.f[1] = xy[2 * (size_t)p + 1];
    st.f[2] = 0.0;
    st.u[0] = uw[4 * (size_t)p];
    st.u[1] = uw[4 * (size_t)p + 1];
    st.u[2] = uw[4 * (size_t)p + 2];
    st.w = uw[4 * (size_t)p + 3];
  }
  return st;
}

// CIC stencil of the 2^DIM nodes (shift 0) or centres (shift 1/2) around a
// particle: linear indices, weights and weight gradients (physical units).
template <int DIM>
struct Stencil {
  int idx[8];
  double wt[8];
  double grad[8][3];
};

template <int DIM>
__device__ __forceinline__ void stencil(const KParams &kp, const PState &st, bool centres, Stencil<DIM> &S) {
  int lo[3];
  double g[3];
  const int ext[3] = {kp.nx, kp.ny, kp.nz};
  const int base[3] = {st.ci, st.cj, st.ck};
  const double inv[3] = {kp.inv_dx, kp.inv_dy, kp.inv_dz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= DIM) {
      lo[d] = 0;
      g[d] = 0.0;
      continue;
    }
    const double f = st.f[d];
    if (!centres) {
      lo[d] = base[d];
      g[d] = f;  // weight of the upper node
    } else {
      const bool hi = f >= 0.5;
      lo[d] = hi ? base[d] : base[d] - 1;
      g[d] = hi ? f - 0.5 : f + 0.5;
    }
  }
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a) {
    const int o[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
    double wd[3], dw[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      wd[d] = d < DIM ? (o[d] ? g[d] : 1.0 - g[d]) : 1.0;
      dw[d] = d < DIM ? (o[d] ? inv[d] : -inv[d]) : 0.0;
    }
    S.wt[a] = wd[0] * wd[1] * wd[2];
    S.grad[a][0] = dw[0] * wd[1] * wd[2];
    S.grad[a][1] = wd[0] * dw[1] * wd[2];
    S.grad[a][2] = wd[0] * wd[1] * dw[2];
    const int ii = wrapi(lo[0] + o[0], kp.nx);
    const int jj = wrapi(lo[1] + o[1], kp.ny);
    const int kk = DIM == 3 ? wrapi(lo[2] + o[2], ext[2]) : 0;
    S.idx[a] = ii + kp.nx * (jj + kp.ny * kk);
  }
}

__device__ __forceinline__ void alpha_of(const double b[3], double a[9]) {
  const double inv = 1.0 / (1.0 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  a[0] = (1.0 + b[0] * b[0]) * inv;
  a[1] = (b[2] + b[0] * b[1]) * inv;
  a[2] = (b[0] * b[2] - b[1]) * inv;
  a[3] = (b[0] * b[1] - b[2]) * inv;
  a[4] = (1.0 + b[1] * b[1]) * inv;
  a[5] = (b[0] + b[1] * b[2]) * inv;
  a[6] = (b[1] + b[0] * b[2]) * inv;
  a[7] = (b[1] * b[2] - b[0]) * inv;
  a[8] = (1.0 + b[2] * b[2]) * inv;
}

// d<la, alpha(b)>/db for a 3x3 cotangent la (row-major).
__device__ __forceinline__ void alpha_vjp(const double b[3], const double a[9], const double la[9], double lb[3]) {
  const double inv = 1.0 / (1.0 + b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  double la_a = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) la_a += la[k] * a[k];
  // -d<la, [b]x>/db
  const double cx = la[5] - la[7], cy = la[6] - la[2], cz = la[1] - la[3];
  // (la + la^T) b
  double sb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) sb[i] = (la[3 * i] + la[i]) * b[0] + (la[3 * i + 1] + la[3 + i]) * b[1] +
                                     (la[3 * i + 2] + la[6 + i]) * b[2];
  lb[0] = (cx + sb[0] - 2.0 * la_a * b[0]) * inv;
  lb[1] = (cy + sb[1] - 2.0 * la_a * b[1]) * inv;
  lb[2] = (cz + sb[2] - 2.0 * la_a * b[2]) * inv;
}

__device__ __forceinline__ void atomic_add3(double *g, size_t N, int idx, double wt, const double v[3]) {
  atomicAdd(&g[idx], wt * v[0]);
  atomicAdd(&g[N + idx], wt * v[1]);
  atomicAdd(&g[2 * N + idx], wt * v[2]);
}

// Butterfly sum over the 64 lanes of a wave (every lane gets the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Lanes of one cell are summed in the wave before the atomics when the cell
// has at least this many of the wave's lanes; sparser cells add per lane.
constexpr int kSegMin = 16;

// Linear index of the point (ci + ox, cj + oy, ck + oz), periodic.
template <int DIM>
__device__ __forceinline__ int grid_index(const KParams &kp, int ci, int cj, int ck, int ox, int oy, int oz) {
  return wrapi(ci + ox, kp.nx) + kp.nx * (wrapi(cj + oy, kp.ny) + kp.ny * (DIM == 3 ? wrapi(ck + oz, kp.nz) : 0));
}

// g[k N + .] += the lanes' node-stencil contributions wt[a] v[k] (node a of
// the lane's cell) and, with the centre stencil, wt[a] v[k] at the centre
// (cell + a - 1 + h) (h: the lane's upper-half flags).  Lanes of one cell are
// summed over the wave first (per node or centre slot of that cell), then
// one lane per slot adds with an atomic; `active` lanes only.
template <int DIM>
__device__ void add_stencil(const KParams &kp, double *__restrict__ g, bool active, int cell, int ci, int cj, int ck,
                            const Stencil<DIM> &S, bool centres, const double (&hf)[3], const double v[3]) {
  constexpr int NA = 1 << DIM, NS = DIM == 3 ? 27 : 9;
  const size_t N = (size_t)kp.ncells;
  const int lane = threadIdx.x & 63;
  int h[3] = {0, 0, 0};
  if (centres) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) h[d] = hf[d] >= 0.5 ? 1 : 0;
  }
  bool pending = active;
  unsigned long long todo = __ballot(pending);
  while (todo) {
    const int leader = __builtin_amdgcn_readfirstlane(__ffsll((long long)todo) - 1);
    const int c = __shfl(cell, leader);
    const bool mine = pending && cell == c;
    const unsigned long long seg = __ballot(mine);
    if (__popcll(seg) >= kSegMin) {
      const int li = __shfl(ci, leader), lj = __shfl(cj, leader), lk = __shfl(ck, leader);
      // slots of the cell: its 2^DIM nodes, or the 3^DIM centres around it
      for (int sl = 0; sl < (centres ? NS : NA); ++sl) {
        int o[3], a = 0;
        bool hit = mine;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int sd = centres ? (sl / (d == 0 ? 1 : (d == 1 ? 3 : 9))) % 3 : (sl >> d) & 1;
          // the lane's stencil corner that lands on this slot
          const int ad = centres ? sd - h[d] : sd;
          if (d < DIM) {
            hit = hit && ad >= 0 && ad <= 1;
            a += (ad & 1) << d;
          }
          o[d] = centres ? sd - 1 : sd;
        }
        const double w = hit ? S.wt[a] : 0.0;
        const double t0 = wave_sum(w * v[0]), t1 = wave_sum(w * v[1]), t2 = wave_sum(w * v[2]);
        if (lane == leader) {
          const int id = grid_index<DIM>(kp, li, lj, lk, o[0], o[1], o[2]);
          atomicAdd(&g[id], t0);
          atomicAdd(&g[N + id], t1);
          atomicAdd(&g[2 * N + id], t2);
        }
      }
    } else if (mine) {
#pragma unroll
      for (int a = 0; a < NA; ++a) atomic_add3(g, N, S.idx[a], S.wt[a], v);
    }
    pending = pending && !mine;
    todo = __ballot(pending);
  }
}

struct AdjIn {
  const int32_t *bin_start, *cell;
  const double *xy, *uw, *z;  // packed (off_x, off_y), (u_x, u_y, u_z, w); off_z
};

template <int DIM>
__global__ __launch_bounds__(256) void k_push_adjoint(KParams kp, AdjIn in, int n, const double *__restrict__ Eth,
                                                      const double *__restrict__ B, const int32_t *__restrict__ new_index,
                                                      const double *__restrict__ lx_in, const double *__restrict__ lu_in,
                                                      double *__restrict__ lx_out, double *__restrict__ lu_out,
                                                      double *__restrict__ lEth, double *__restrict__ lB) {
  // every lane stays to the end (the grid sums are wave-wide); lanes past
  // the particles compute on the last one and add nothing
  const int p0 = blockIdx.x * 256 + threadIdx.x;
  const bool act = p0 < n;
  const int p = act ? p0 : n - 1;
  const size_t N = (size_t)kp.ncells;
  const PState st = load_particle<DIM>(kp, in.bin_start, in.cell, in.xy, in.uw, in.z, p);
  const int cell = in.cell[p];
  const double c2 = kp.c * kp.c;
  Stencil<DIM> sc, sn;
  stencil<DIM>(kp, st, true, sc);
  stencil<DIM>(kp, st, false, sn);
  double Bp[3] = {0, 0, 0}, Ep[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Bp[k] += sc.wt[a] * B[k * N + sc.idx[a]];
      Ep[k] += sn.wt[a] * Eth[k * N + sn.idx[a]];
    }
  const double *u = st.u;
  const double gb = kp.nonrel ? 1.0 : sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / c2);
  const double kb = st.beta / (gb * kp.c);
  const double b[3] = {kb * Bp[0], kb * Bp[1], kb * Bp[2]};
  double a[9];
  alpha_of(b, a);
  const double z[3] = {u[0] + st.beta * Ep[0], u[1] + st.beta * Ep[1], u[2] + st.beta * Ep[2]};
  double ub[3], un[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ub[i] = a[3 * i] * z[0] + a[3 * i + 1] * z[1] + a[3 * i + 2] * z[2];
    un[i] = 2.0 * ub[i] - u[i];
  }
  const double gn = kp.nonrel ? 1.0 : sqrt(1.0 + (un[0] * un[0] + un[1] * un[1] + un[2] * un[2]) / c2);
  // incoming cotangents (new order -> this particle)
  const int q = new_index ? new_index[p] : p;
  double lxp[3] = {0, 0, 0}, lun[3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) lxp[d] = lx_in[(size_t)d * n + q];
#pragma unroll
  for (int k = 0; k < 3; ++k) lun[k] = lu_in[(size_t)k * n + q];
  // x' = x + dt u'/gamma(u'):  d(u/gamma)/du = (I - u u^T/(c^2 gamma^2))/gamma
  {
    double ulx = 0.0;
    for (int d = 0; d < DIM; ++d) ulx += un[d] * lxp[d];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double lk = k < DIM ? lxp[k] : 0.0;
      lun[k] += kp.dt * (kp.nonrel ? lk : (lk - un[k] * ulx / (c2 * gn * gn)) / gn);
    }
  }
  // u' = 2 ubar - u, ubar = alpha z
  const double lub[3] = {2.0 * lun[0], 2.0 * lun[1], 2.0 * lun[2]};
  double lu[3] = {-lun[0], -lun[1], -lun[2]};
  double la[9], lz[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) la[3 * i + j] = lub[i] * z[j];
#pragma unroll
  for (int j = 0; j < 3; ++j) lz[j] = a[j] * lub[0] + a[3 + j] * lub[1] + a[6 + j] * lub[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) lu[k] += lz[k];
  const double lEp[3] = {st.beta * lz[0], st.beta * lz[1], st.beta * lz[2]};
  double lx[3] = {lxp[0], lxp[1], lxp[2]};
#pragma unroll
  for (int a2 = 0; a2 < (1 << DIM); ++a2) {
    const int id = sn.idx[a2];
    const double e = Eth[id] * lEp[0] + Eth[N + id] * lEp[1] + Eth[2 * N + id] * lEp[2];
#pragma unroll
    for (int d = 0; d < DIM; ++d) lx[d] += sn.grad[a2][d] * e;
  }
  add_stencil<DIM>(kp, lEth, act, cell, st.ci, st.cj, st.ck, sn, false, st.f, lEp);
  // alpha(b(B_p, gbar))
  double lb[3];
  alpha_vjp(b, a, la, lb);
  const double lBp[3] = {kb * lb[0], kb * lb[1], kb * lb[2]};
  if (!kp.nonrel) {
    const double lgb = -(b[0] * lb[0] + b[1] * lb[1] + b[2] * lb[2]) / gb;
#pragma unroll
    for (int k = 0; k < 3; ++k) lu[k] += lgb * u[k] / (gb * c2);
  }
#pragma unroll
  for (int a2 = 0; a2 < (1 << DIM); ++a2) {
    const int id = sc.idx[a2];
    const double e = B[id] * lBp[0] + B[N + id] * lBp[1] + B[2 * N + id] * lBp[2];
#pragma unroll
    for (int d = 0; d < DIM; ++d) lx[d] += sc.grad[a2][d] * e;
  }
  add_stencil<DIM>(kp, lB, act, cell, st.ci, st.cj, st.ck, sc, true, st.f, lBp);
  if (act) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) lx_out[(size_t)d * n + p] = lx[d];
#pragma unroll
    for (int k = 0; k < 3; ++k) lu_out[(size_t)k * n + p] = lu[k];
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_deposit_adjoint(KParams kp, AdjIn in, int n, const double *__restrict__ B,
                                                         const double *__restrict__ Eth, const double *__restrict__ mu,
                                                         double *__restrict__ lx_out, double *__restrict__ lu_out,
                                                         double *__restrict__ lB) {
  const int p0 = blockIdx.x * 256 + threadIdx.x;
  const bool act = p0 < n;
  const int p = act ? p0 : n - 1;
  const size_t N = (size_t)kp.ncells;
  const PState st = load_particle<DIM>(kp, in.bin_start, in.cell, in.xy, in.uw, in.z, p);
  const int cell = in.cell[p];
  const double c2 = kp.c * kp.c;
  Stencil<DIM> sc, sn;
  stencil<DIM>(kp, st, true, sc);
  stencil<DIM>(kp, st, false, sn);
  double Bp[3] = {0, 0, 0}, Ep[3] = {0, 0, 0}, mp[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Bp[k] += sc.wt[a] * B[k * N + sc.idx[a]];
      Ep[k] += sn.wt[a] * Eth[k * N + sn.idx[a]];
      mp[k] += sn.wt[a] * mu[k * N + sn.idx[a]];
    }
  const double *u = st.u;
  const double gb = kp.nonrel ? 1.0 : sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / c2);
  const double kb = st.beta / (gb * kp.c);
  const double b[3] = {kb * Bp[0], kb * Bp[1], kb * Bp[2]};
  double a[9];
  alpha_of(b, a);
  const double z[3] = {u[0] + st.beta * Ep[0], u[1] + st.beta * Ep[1], u[2] + st.beta * Ep[2]};
  double ub[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) ub[i] = a[3 * i] * z[0] + a[3 * i + 1] * z[1] + a[3 * i + 2] * z[2];
  const double K = -4.0 * M_PI * kp.theta * kp.dt * st.w * st.q / (kp.V * gb);
  const double phi = K * (mp[0] * ub[0] + mp[1] * ub[1] + mp[2] * ub[2]);
  // d/d mu_p and d/d z
  const double lmp[3] = {K * ub[0], K * ub[1], K * ub[2]};
  double lz[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) lz[j] = K * (a[j] * mp[0] + a[3 + j] * mp[1] + a[6 + j] * mp[2]);
  double lu[3] = {lz[0], lz[1], lz[2]};
  const double lEp[3] = {st.beta * lz[0], st.beta * lz[1], st.beta * lz[2]};
  double lx[3] = {0, 0, 0};
#pragma unroll
  for (int a2 = 0; a2 < (1 << DIM); ++a2) {
    const int id = sn.idx[a2];
    const double e = Eth[id] * lEp[0] + Eth[N + id] * lEp[1] + Eth[2 * N + id] * lEp[2] + mu[id] * lmp[0] +
                     mu[N + id] * lmp[1] + mu[2 * N + id] * lmp[2];
#pragma unroll
    for (int d = 0; d < DIM; ++d) lx[d] += sn.grad[a2][d] * e;
  }
  // d/d alpha = K mu_p z^T
  double la[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) la[3 * i + j] = K * mp[i] * z[j];
  double lb[3];
  alpha_vjp(b, a, la, lb);
  const double lBp[3] = {kb * lb[0], kb * lb[1], kb * lb[2]};
  if (!kp.nonrel) {
    // gbar enters through b and through K
    const double lgb = -(b[0] * lb[0] + b[1] * lb[1] + b[2] * lb[2]) / gb - phi / gb;
#pragma unroll
    for (int k = 0; k < 3; ++k) lu[k] += lgb * u[k] / (gb * c2);
  }
#pragma unroll
  for (int a2 = 0; a2 < (1 << DIM); ++a2) {
    const int id = sc.idx[a2];
    const double e = B[id] * lBp[0] + B[N + id] * lBp[1] + B[2 * N + id] * lBp[2];
#pragma unroll
    for (int d = 0; d < DIM; ++d) lx[d] += sc.grad[a2][d] * e;
  }
  add_stencil<DIM>(kp, lB, act, cell, st.ci, st.cj, st.ck, sc, true, st.f, lBp);
  if (act) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) lx_out[(size_t)d * n + p] += lx[d];
#pragma unroll
    for (int k = 0; k < 3; ++k) lu_out[(size_t)k * n + p] += lu[k];
  }
}

// rhs of the transposed solve: l_th + l_E1/theta - c dt C_CN l_B1  (curl precomputed in t)
__global__ __launch_bounds__(256) void k_adj_rhs(size_t n3, double theta, double cdt, const double *__restrict__ lth,
                                                 const double *__restrict__ lE1, const double *__restrict__ ccn_lB1,
                                                 double *__restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n3) return;
  out[i] = lth[i] + lE1[i] / theta - cdt * ccn_lB1[i];
}

// l_En = -(1-theta)/theta l_E1 + mu ;  l_Bn += l_B1 + c theta dt C_NC mu (curl precomputed)
__global__ __launch_bounds__(256) void k_adj_finish(size_t n3, double theta, double ctdt, const double *__restrict__ lE1,
                                                    const double *__restrict__ lB1, const double *__restrict__ mu,
                                                    const double *__restrict__ cnc_mu, double *__restrict__ lEn,
                                                    double *__restrict__ lBn) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n3) return;
  lEn[i] += -(1.0 - theta) / theta * lE1[i] + mu[i];
  lBn[i] += lB1[i] + ctdt * cnc_mu[i];
}

}  // namespace

void launch_push_adjoint(const KParams &kp, const AdjInPtrs &in, int n, const double *Eth, const double *B,
                         const int32_t *new_index, const double *lx_in, const double *lu_in, double *lx_out,
                         double *lu_out, double *lEth, double *lB, hipStream_t st) {
  if (n <= 0) return;
  AdjIn a{in.bin_start, in.cell, in.xy, in.uw, in.z};
  const int nb = (n + 255) / 256;
  if (kp.dim == 2)
    hipLaunchKernelGGL(k_push_adjoint<2>, dim3(nb), dim3(256), 0, st, kp, a, n, Eth, B, new_index, lx_in, lu_in, lx_out,
                       lu_out, lEth, lB);
  else
    hipLaunchKernelGGL(k_push_adjoint<3>, dim3(nb), dim3(256), 0, st, kp, a, n, Eth, B, new_index, lx_in, lu_in, lx_out,
                       lu_out, lEth, lB);
}

void launch_deposit_adjoint(const KParams &kp, const AdjInPtrs &in, int n, const double *B, const double *Eth,
                            const double *mu, double *lx_out, double *lu_out, double *lB, hipStream_t st) {
  if (n <= 0) return;
  AdjIn a{in.bin_start, in.cell, in.xy, in.uw, in.z};
  const int nb = (n + 255) / 256;
  if (kp.dim == 2)
    hipLaunchKernelGGL(k_deposit_adjoint<2>, dim3(nb), dim3(256), 0, st, kp, a, n, B, Eth, mu, lx_out, lu_out, lB);
  else
    hipLaunchKernelGGL(k_deposit_adjoint<3>, dim3(nb), dim3(256), 0, st, kp, a, n, B, Eth, mu, lx_out, lu_out, lB);
}

void launch_adj_rhs(size_t n3, double theta, double cdt, const double *lth, const double *lE1, const double *ccn_lB1,
                    double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_rhs, dim3((n3 + 255) / 256), dim3(256), 0, st, n3, theta, cdt, lth, lE1, ccn_lB1, out);
}

void launch_adj_finish(size_t n3, double theta, double ctdt, const double *lE1, const double *lB1, const double *mu,
                       const double *cnc_mu, double *lEn, double *lBn, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_finish, dim3((n3 + 255) / 256), dim3(256), 0, st, n3, theta, ctdt, lE1, lB1, mu, cnc_mu, lEn,
                     lBn);
}

}  // namespace relsim
