// Grid kernels of the implicit field solve (S4-S5), all FP64: discrete curls,
// the S4 operator, right-hand side, field update, and the BLAS-1 pieces of
// restarted GMRES (multi-dot, multi-axpy, norms) with fixed-order reductions.
//
// Both curls use one stencil shape: the difference along d averaged over the
// transverse corners of a 2x2(x2) cube.  Nodes -> centre of cell (i,j,k)
// reads the cube of nodes starting at (i,j,k); centres -> node (i,j,k) reads
// the cube of cells starting at (i-1,j-1,k-1).  That makes C_CN the exact
// transpose of C_NC on the periodic grid.
#include "relsim_internal.h"

namespace relsim {
namespace {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7) * q + (b >> 3);
}

// Cube of 2^DIM values of the three components starting at (i0, j0, k0).
template <int DIM>
__device__ __forceinline__ void load_cube(const KParams &kp, const double *__restrict__ F, int i0, int j0, int k0,
                                          double c[3][8]) {
  const size_t N = (size_t)kp.ncells;
  const int x0 = wrapi(i0, kp.nx), x1 = wrapi(i0 + 1, kp.nx);
  const int y0 = wrapi(j0, kp.ny), y1 = wrapi(j0 + 1, kp.ny);
  const int z0 = DIM == 3 ? wrapi(k0, kp.nz) : 0, z1 = DIM == 3 ? wrapi(k0 + 1, kp.nz) : 0;
#pragma unroll
  for (int a = 0; a < (DIM == 3 ? 8 : 4); ++a) {
    const size_t id = (size_t)((a & 1) ? x1 : x0) +
                      (size_t)kp.nx * ((size_t)((a & 2) ? y1 : y0) + (size_t)kp.ny * ((a & 4) ? z1 : z0));
    c[0][a] = F[id];
    c[1][a] = F[N + id];
    c[2][a] = F[2 * N + id];
  }
}

// curl of the cube: (dy Fz - dz Fy, dz Fx - dx Fz, dx Fy - dy Fx)
template <int DIM>
__device__ __forceinline__ void cube_curl(const KParams &kp, const double c[3][8], double out[3]) {
  const double ax = kp.inv_dx / (DIM == 3 ? 4.0 : 2.0);
  const double ay = kp.inv_dy / (DIM == 3 ? 4.0 : 2.0);
  const double az = kp.inv_dz / 4.0;
  double d[3][3];  // d[comp][dim]
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if constexpr (DIM == 2) {
      d[q][0] = ax * ((c[q][1] - c[q][0]) + (c[q][3] - c[q][2]));
      d[q][1] = ay * ((c[q][2] - c[q][0]) + (c[q][3] - c[q][1]));
      d[q][2] = 0.0;
    } else {
      d[q][0] = ax * ((c[q][1] - c[q][0]) + (c[q][3] - c[q][2]) + (c[q][5] - c[q][4]) + (c[q][7] - c[q][6]));
      d[q][1] = ay * ((c[q][2] - c[q][0]) + (c[q][3] - c[q][1]) + (c[q][6] - c[q][4]) + (c[q][7] - c[q][5]));
      d[q][2] = az * ((c[q][4] - c[q][0]) + (c[q][5] - c[q][1]) + (c[q][6] - c[q][2]) + (c[q][7] - c[q][3]));
    }
  }
  out[0] = d[2][1] - d[1][2];
  out[1] = d[0][2] - d[2][0];
  out[2] = d[1][0] - d[0][1];
}

template <int DIM>
__global__ __launch_bounds__(256) void k_curl(KParams kp, const double *__restrict__ in, double *__restrict__ out,
                                              int shift) {
  int i, j, k;
  const int g = strip_node(kp.nx, kp.ny, kp.nz, xcd_remap(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6),
                           (int)(threadIdx.x & 63), i, j, k);
  if (g < 0) return;
  double c[3][8], r[3];
  load_cube<DIM>(kp, in, i - shift, j - shift, k - shift, c);
  cube_curl<DIM>(kp, c, r);
  const size_t N = (size_t)kp.ncells;
  out[g] = r[0];
  out[N + g] = r[1];
  out[2 * N + g] = r[2];
}

// Linear index of node (i + dx, j + dy, k + dz), periodic.
template <int DIM>
__device__ __forceinline__ size_t node_at(const KParams &kp, int i, int j, int k, int dx, int dy, int dz) {
  return (size_t)wrapi(i + dx, kp.nx) +
         (size_t)kp.nx * ((size_t)wrapi(j + dy, kp.ny) + (size_t)kp.ny * (DIM == 3 ? wrapi(k + dz, kp.nz) : 0));
}

// (M x)_g, or (M^T x)_g with TR (each 3x3 block transposed), from the stored
// half of the blocks: slot h of node g couples x at g + delta(h), and for
// h > 0 the same slot of node g - delta(h) couples x at g - delta(h)
// (M_{g,g-delta} = M_{g-delta,g}).  MT is M's storage type (double, or
// float on request in mixed precision); the products and sums are FP64.
template <int DIM, bool TR, typename MT>
__device__ __forceinline__ void apply_M(const KParams &kp, const MT *__restrict__ M,
                                        const double *__restrict__ x, int g, int i, int j, int k, double mx[3]) {
  constexpr int NSLOT = m_slots<DIM>(), CEN = m_centre<DIM>();
  const size_t N = (size_t)kp.ncells;
#pragma unroll
  for (int h = 0; h < NSLOT; ++h) {
    const int off = CEN + h;
    const int dx = off % 3 - 1, dy = (off / 3) % 3 - 1, dz = DIM == 3 ? off / 9 - 1 : 0;
#pragma unroll
    for (int side = 0; side < (h ? 2 : 1); ++side) {
      // side 0: own block times x at g + delta; side 1: the neighbour's
      // block times x at g - delta
      const size_t id = side ? node_at<DIM>(kp, i, j, k, -dx, -dy, -dz) : node_at<DIM>(kp, i, j, k, dx, dy, dz);
      const double x0 = x[id], x1 = x[N + id], x2 = x[2 * N + id];
      const MT *Mo = M + (size_t)h * 9 * N + (side ? id : (size_t)g);
      double m[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) m[q] = (double)Mo[q * N];
      if constexpr (!TR) {
        mx[0] += m[0] * x0 + m[1] * x1 + m[2] * x2;
        mx[1] += m[3] * x0 + m[4] * x1 + m[5] * x2;
        mx[2] += m[6] * x0 + m[7] * x1 + m[8] * x2;
      } else {
        mx[0] += m[0] * x0 + m[3] * x1 + m[6] * x2;
        mx[1] += m[1] * x0 + m[4] * x1 + m[7] * x2;
        mx[2] += m[2] * x0 + m[5] * x1 + m[8] * x2;
      }
    }
  }
}

// out = x + a^2 C_CN t + b M x, with t = C_NC x precomputed; with TR the
// transposed operator, x + a^2 C_CN t + b M^T x (the curl-curl term is
// symmetric, C_CN being the transpose of C_NC)
template <int DIM, bool TR, typename MT>
__global__ __launch_bounds__(256) void k_apply_A_tail(KParams kp, const MT *__restrict__ M,
                                                      const double *__restrict__ x, const double *__restrict__ t,
                                                      double *__restrict__ out) {
  int i, j, k;
  const int g = strip_node(kp.nx, kp.ny, kp.nz, xcd_remap(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6),
                           (int)(threadIdx.x & 63), i, j, k);
  if (g < 0) return;
  const size_t N = (size_t)kp.ncells;
  double c[3][8], cc[3];
  load_cube<DIM>(kp, t, i - 1, j - 1, k - 1, c);
  cube_curl<DIM>(kp, c, cc);
  const double a = kp.c * kp.theta * kp.dt;
  const double b = 4.0 * M_PI * kp.theta * kp.dt;
  double mx[3] = {0.0, 0.0, 0.0};
  apply_M<DIM, TR, MT>(kp, M, x, g, i, j, k, mx);
#pragma unroll
  for (int q = 0; q < 3; ++q) out[q * N + g] = x[q * N + g] + a * a * cc[q] + b * mx[q];
}

template <int DIM>
__global__ __launch_bounds__(256) void k_rhs(KParams kp, const double *__restrict__ En, const double *__restrict__ Bn,
                                             const double *__restrict__ J, double *__restrict__ out) {
  int i, j, k;
  const int g = strip_node(kp.nx, kp.ny, kp.nz, xcd_remap(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6),
                           (int)(threadIdx.x & 63), i, j, k);
  if (g < 0) return;
  const size_t N = (size_t)kp.ncells;
  double c[3][8], cc[3];
  load_cube<DIM>(kp, Bn, i - 1, j - 1, k - 1, c);
  cube_curl<DIM>(kp, c, cc);
  const double a = kp.c * kp.theta * kp.dt;
  const double b = 4.0 * M_PI * kp.theta * kp.dt;
#pragma unroll
  for (int q = 0; q < 3; ++q) out[q * N + g] = En[q * N + g] + a * cc[q] - b * J[q * N + g];
}

template <int DIM>
__global__ __launch_bounds__(256) void k_field_update(KParams kp, const double *__restrict__ En,
                                                      const double *__restrict__ Bn, const double *__restrict__ Eth,
                                                      double *__restrict__ En1, double *__restrict__ Bn1) {
  int i, j, k;
  const int g = strip_node(kp.nx, kp.ny, kp.nz, xcd_remap(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6),
                           (int)(threadIdx.x & 63), i, j, k);
  if (g < 0) return;
  const size_t N = (size_t)kp.ncells;
  double c[3][8], cc[3];
  load_cube<DIM>(kp, Eth, i, j, k, c);
  cube_curl<DIM>(kp, c, cc);
  const double th = kp.theta;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    Bn1[q * N + g] = Bn[q * N + g] - kp.c * kp.dt * cc[q];
    En1[q * N + g] = (Eth[q * N + g] - (1.0 - th) * En[q * N + g]) / th;
  }
}

// ---- BLAS-1 with fixed-order reductions ----
__device__ __forceinline__ double block_sum_256(double v, double *lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return r;
}

// Multi-dot partial sums: block b owns one contiguous chunk of the vectors
// and writes, for each vector v_k, the sum of v_k[i] w[i] over its chunk
// (each thread in index order, then a fixed-order block sum).  The vectors
// are taken kMdotBatch at a time with one accumulator each per thread, so w
// is read once per batch and a thread has a batch of independent loads in
// flight (one vector per pass left the kernel latency-bound).
constexpr int kMdotBatch = 8;
__global__ __launch_bounds__(256) void k_mdot(const double *__restrict__ V, size_t ld, int nvec,
                                              const double *__restrict__ w, size_t n, double *__restrict__ partials) {
  __shared__ double lds[4][kMdotBatch];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const size_t beg = (size_t)blockIdx.x * chunk;
  const size_t end = beg + chunk < n ? beg + chunk : n;
  for (int k0 = 0; k0 < nvec; k0 += kMdotBatch) {
    const int kn = nvec - k0 < kMdotBatch ? nvec - k0 : kMdotBatch;
    double acc[kMdotBatch];
#pragma unroll
    for (int q = 0; q < kMdotBatch; ++q) acc[q] = 0.0;
    for (size_t i = beg + threadIdx.x; i < end; i += 256) {
      const double wi = w[i];
#pragma unroll
      for (int q = 0; q < kMdotBatch; ++q)
        if (q < kn) acc[q] += V[(size_t)(k0 + q) * ld + i] * wi;
    }
#pragma unroll
    for (int q = 0; q < kMdotBatch; ++q) {
      double v = acc[q];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) lds[wid][q] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < kn) {
      const int q = threadIdx.x;
      partials[(size_t)blockIdx.x * nvec + k0 + q] = (lds[0][q] + lds[1][q]) + (lds[2][q] + lds[3][q]);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ partials, int nparts, int nvec,
                                                         double *__restrict__ res) {
  __shared__ double lds[4];
  const int kv = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) acc += partials[(size_t)b * nvec + kv];
  const double s = block_sum_256(acc, lds);
  if (threadIdx.x == 0) res[kv] = s;
}

// Sums of consecutive chunks of a long array of partial sums, one block per
// chunk, in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_chunks(const double *__restrict__ in, int n, int chunk,
                                                       double *__restrict__ out) {
  __shared__ double lds[4];
  const int b0 = blockIdx.x * chunk;
  const int b1 = b0 + chunk < n ? b0 + chunk : n;
  double acc = 0.0;
  for (int i = b0 + threadIdx.x; i < b1; i += 256) acc += in[i];
  const double s = block_sum_256(acc, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_maxpy(const double *__restrict__ V, size_t ld, int nvec,
                                               const double *__restrict__ h, double *__restrict__ w, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = w[i];
  for (int kv = 0; kv < nvec; ++kv) acc -= h[kv] * V[(size_t)kv * ld + i];
  w[i] = acc;
}

// The two halves of an Arnoldi step's second Gram-Schmidt pass, each fused
// with its neighbour so that the basis is read once per half:
//
// k_maxpy_dot: w -= sum_k h[k] V[k], then the partial sums (per block, as in
// k_mdot) of V[k] . w for k < nvec and of w . w, all from one read of the
// nvec basis vectors (held in registers between the update and the dots).
// The update rounds as k_maxpy's and the sums are taken in k_mdot's order.
template <int NV>
__global__ __launch_bounds__(256) void k_maxpy_dot(const double *__restrict__ V, size_t ld, int nvec,
                                                   const double *__restrict__ h, double *__restrict__ w, size_t n,
                                                   double *__restrict__ partials) {
  __shared__ double lds[4][NV + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const size_t beg = (size_t)blockIdx.x * chunk;
  const size_t end = beg + chunk < n ? beg + chunk : n;
  double hk[NV], acc[NV + 1];
#pragma unroll
  for (int q = 0; q < NV; ++q) hk[q] = q < nvec ? h[q] : 0.0;
#pragma unroll
  for (int q = 0; q <= NV; ++q) acc[q] = 0.0;
  for (size_t i = beg + threadIdx.x; i < end; i += 256) {
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = q < nvec ? V[(size_t)q * ld + i] : 0.0;
    double wi = w[i];
#pragma unroll
    for (int q = 0; q < NV; ++q)
      if (q < nvec) wi -= hk[q] * v[q];
    w[i] = wi;
#pragma unroll
    for (int q = 0; q < NV; ++q)
      if (q < nvec) acc[q] += v[q] * wi;
    acc[NV] += wi * wi;
  }
#pragma unroll
  for (int q = 0; q <= NV; ++q) {
    if (q < nvec || q == NV) {
      double v = acc[q];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) lds[wid][q] = v;
    }
  }
  __syncthreads();
  // partials[b][0..nvec]: the dots, then w . w
  if ((int)threadIdx.x <= nvec) {
    const int q = (int)threadIdx.x == nvec ? NV : threadIdx.x;
    partials[(size_t)blockIdx.x * (nvec + 1) + threadIdx.x] = (lds[0][q] + lds[1][q]) + (lds[2][q] + lds[3][q]);
  }
}

// k_maxpy_scale: w = (w - sum_k h[k] V[k]) / hn, with hn = sqrt(ww - sum_k
// h[k]^2) and ww = h[nvec] (the norm of w after the update, from the
// orthogonality of the basis).  When the difference has cancelled (at most
// 1e-4 ww) w is left unscaled, for the host to normalise by an explicit
// norm.  h[nvec + 1] receives hn, or 0 when w was left unscaled.
__global__ __launch_bounds__(256) void k_maxpy_scale(const double *__restrict__ V, size_t ld, int nvec,
                                                     double *__restrict__ h, double *__restrict__ w, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s2 = 0.0;
  for (int kv = 0; kv < nvec; ++kv) s2 += h[kv] * h[kv];
  const double ww = h[nvec], hn2 = ww - s2;
  const bool ok = hn2 > 1e-4 * ww;
  const double hn = ok ? sqrt(hn2) : 0.0;
  const double a = ok ? 1.0 / hn : 1.0;
  double acc = w[i];
  for (int kv = 0; kv < nvec; ++kv) acc -= h[kv] * V[(size_t)kv * ld + i];
  w[i] = a * acc;
  if (i == 0) h[nvec + 1] = hn;
}

__global__ __launch_bounds__(256) void k_axpby(double a, const double *__restrict__ x, double b, double *__restrict__ y,
                                               size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

__global__ __launch_bounds__(256) void k_sumsq(const double *__restrict__ x, size_t n, double *__restrict__ partials) {
  __shared__ double lds[4];
  const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const size_t beg = (size_t)blockIdx.x * chunk;
  const size_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  for (size_t i = beg + threadIdx.x; i < end; i += 256) acc += x[i] * x[i];
  const double s = block_sum_256(acc, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

inline int grid_of(size_t n) { return (int)((n + 255) / 256); }
// blocks of the per-node kernels (strip node order)
inline int node_blocks(const KParams &kp) { return grid_node_blocks(kp.nx, kp.ny, kp.nz); }

}  // namespace

void launch_curl(const KParams &kp, const double *in, double *out, int to_centres, hipStream_t st) {
  const int shift = to_centres ? 0 : 1;
  if (kp.dim == 2)
    hipLaunchKernelGGL(k_curl<2>, dim3(node_blocks(kp)), dim3(256), 0, st, kp, in, out, shift);
  else
    hipLaunchKernelGGL(k_curl<3>, dim3(node_blocks(kp)), dim3(256), 0, st, kp, in, out, shift);
}

template <bool TR, typename MT>
void launch_apply_tail(const KParams &kp, const MT *M, const double *x, const double *t, double *out,
                       hipStream_t st) {
  if (kp.dim == 2)
    hipLaunchKernelGGL((k_apply_A_tail<2, TR, MT>), dim3(node_blocks(kp)), dim3(256), 0, st, kp, M, x, t, out);
  else
    hipLaunchKernelGGL((k_apply_A_tail<3, TR, MT>), dim3(node_blocks(kp)), dim3(256), 0, st, kp, M, x, t, out);
}

void launch_apply_A_tail(const KParams &kp, int mass_fp32, const void *M, const double *x, const double *t,
                         double *out, hipStream_t st) {
  if (mass_fp32)
    launch_apply_tail<false>(kp, static_cast<const float *>(M), x, t, out, st);
  else
    launch_apply_tail<false>(kp, static_cast<const double *>(M), x, t, out, st);
}

void launch_apply_AT_tail(const KParams &kp, int mass_fp32, const void *M, const double *x, const double *t,
                          double *out, hipStream_t st) {
  if (mass_fp32)
    launch_apply_tail<true>(kp, static_cast<const float *>(M), x, t, out, st);
  else
    launch_apply_tail<true>(kp, static_cast<const double *>(M), x, t, out, st);
}

void launch_rhs(const KParams &kp, const double *En, const double *Bn, const double *J, double *out, hipStream_t st) {
  if (kp.dim == 2)
    hipLaunchKernelGGL(k_rhs<2>, dim3(node_blocks(kp)), dim3(256), 0, st, kp, En, Bn, J, out);
  else
    hipLaunchKernelGGL(k_rhs<3>, dim3(node_blocks(kp)), dim3(256), 0, st, kp, En, Bn, J, out);
}

void launch_field_update(const KParams &kp, const double *En, const double *Bn, const double *Eth, double *En1,
                         double *Bn1, hipStream_t st) {
  if (kp.dim == 2)
    hipLaunchKernelGGL(k_field_update<2>, dim3(node_blocks(kp)), dim3(256), 0, st, kp, En, Bn, Eth, En1, Bn1);
  else
    hipLaunchKernelGGL(k_field_update<3>, dim3(node_blocks(kp)), dim3(256), 0, st, kp, En, Bn, Eth, En1, Bn1);
}

void launch_mdot(const double *V, size_t ld, int nvec, const double *w, size_t n, double *partials, double *res,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_mdot, dim3(kDotBlocks), dim3(256), 0, st, V, ld, nvec, w, n, partials);
  hipLaunchKernelGGL(k_reduce_partials, dim3(nvec), dim3(256), 0, st, partials, kDotBlocks, nvec, res);
}

void launch_maxpy(const double *V, size_t ld, int nvec, const double *h, double *w, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_maxpy, dim3(grid_of(n)), dim3(256), 0, st, V, ld, nvec, h, w, n);
}

int launch_maxpy_dot(const double *V, size_t ld, int nvec, const double *h, double *w, size_t n, double *partials,
                     double *res, hipStream_t st) {
  if (nvec <= 8)
    hipLaunchKernelGGL(k_maxpy_dot<8>, dim3(kDotBlocks), dim3(256), 0, st, V, ld, nvec, h, w, n, partials);
  else if (nvec <= 16)
    hipLaunchKernelGGL(k_maxpy_dot<16>, dim3(kDotBlocks), dim3(256), 0, st, V, ld, nvec, h, w, n, partials);
  else if (nvec <= 32)
    hipLaunchKernelGGL(k_maxpy_dot<32>, dim3(kDotBlocks), dim3(256), 0, st, V, ld, nvec, h, w, n, partials);
  else
    return 0;
  hipLaunchKernelGGL(k_reduce_partials, dim3(nvec + 1), dim3(256), 0, st, partials, kDotBlocks, nvec + 1, res);
  return 1;
}

void launch_maxpy_scale(const double *V, size_t ld, int nvec, double *h, double *w, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_maxpy_scale, dim3(grid_of(n)), dim3(256), 0, st, V, ld, nvec, h, w, n);
}

void launch_axpby(double a, const double *x, double b, double *y, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_of(n)), dim3(256), 0, st, a, x, b, y, n);
}

void launch_sumsq_partials(const double *x, size_t n, double *partials, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(kRedBlocks), dim3(256), 0, st, x, n, partials);
}

void launch_reduce_partials(const double *partials, int nparts, int nvec, double *res, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(nvec), dim3(256), 0, st, partials, nparts, nvec, res);
}

void launch_reduce_long(const double *in, int n, double *tmp, double *res, hipStream_t st) {
  const int chunk = (n + kRedBlocks - 1) / kRedBlocks;
  hipLaunchKernelGGL(k_reduce_chunks, dim3(kRedBlocks), dim3(256), 0, st, in, n, chunk > 0 ? chunk : 1, tmp);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, st, tmp, kRedBlocks, 1, res);
}

}  // namespace relsim
