// General stable sort of particles by bin = cell * nspecies + species, for
// particles in arbitrary order (initial loading, or after external edits).
// Least-significant-digit radix sort of (bin, index) pairs with 4-bit digits:
// per pass, a per-block digit histogram (digit-major, block-minor, so that the
// exclusive scan yields stable global offsets), then a scatter that ranks
// equal digits inside the block by wave ballots.  The particle arrays are
// then gathered through the sorted indices and bin_start is rebuilt from the
// sorted keys.  The per-step re-sort after a push does not use this path.
#include "relsim_internal.h"

namespace relsim {
namespace {

constexpr int kRsBlock = 256;
constexpr int kRsBits = 4;
constexpr int kRsDigits = 1 << kRsBits;

__global__ __launch_bounds__(256) void k_make_keys(KParams kp, int n, const int32_t *__restrict__ cell,
                                                   const uint8_t *__restrict__ species, int32_t *__restrict__ keys,
                                                   int32_t *__restrict__ vals, int32_t *__restrict__ err) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c = cell[i];
  const int s = species ? (int)species[i] : 0;
  if (c < 0 || c >= kp.ncells || s >= kp.nspecies) {
    atomicOr(err, 4);
    keys[i] = 0;
  } else {
    keys[i] = c * kp.nspecies + s;
  }
  vals[i] = i;
}

__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const int32_t *__restrict__ keys, int n, int shift,
                                                      int32_t *__restrict__ hist, int nblk) {
  __shared__ int cnt[kRsDigits];
  if (threadIdx.x < kRsDigits) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int i = blockIdx.x * kRsBlock + threadIdx.x;
  if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kRsDigits - 1)], 1);
  __syncthreads();
  if (threadIdx.x < kRsDigits) hist[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const int32_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                                         int n, int shift, const int32_t *__restrict__ offs, int nblk,
                                                         int32_t *__restrict__ kout, int32_t *__restrict__ vout) {
  __shared__ int wcnt[kRsBlock / 64][kRsDigits];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int i = blockIdx.x * kRsBlock + threadIdx.x;
  const bool v = i < n;
  const int key = v ? kin[i] : 0;
  const int dg = (key >> shift) & (kRsDigits - 1);
  // lanes of this wave holding the same digit
  unsigned long long same = __ballot(v);
#pragma unroll
  for (int b = 0; b < kRsBits; ++b) {
    const unsigned long long ones = __ballot(v && ((dg >> b) & 1));
    same &= ((dg >> b) & 1) ? ones : ~ones;
  }
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int rank_w = __popcll(same & lt);
  if (threadIdx.x < (kRsBlock / 64) * kRsDigits) (&wcnt[0][0])[threadIdx.x] = 0;
  __syncthreads();
  if (v && rank_w == 0) wcnt[wid][dg] = __popcll(same);
  __syncthreads();
  if (v) {
    int before = 0;
    for (int w2 = 0; w2 < wid; ++w2) before += wcnt[w2][dg];
    const int pos = offs[dg * nblk + blockIdx.x] + before + rank_w;
    kout[pos] = key;
    vout[pos] = vin[i];
  }
}

__global__ __launch_bounds__(256) void k_bin_bounds(const int32_t *__restrict__ keys, int n, int nbins,
                                                    int32_t *__restrict__ bin_start) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j > n) return;
  // bins (prev, cur] start at j, where prev is the key before j (-1 at 0)
  // and cur is the key at j (nbins past the end)
  const int prev = j == 0 ? -1 : keys[j - 1];
  const int cur = j == n ? nbins : keys[j];
  for (int b = prev + 1; b <= cur; ++b) bin_start[b] = j;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(KParams kp, int n, const int32_t *__restrict__ idx,
                                                const int32_t *__restrict__ keys, const V2<T> *__restrict__ xy,
                                                const V4<T> *__restrict__ uw, const T *__restrict__ zz,
                                                int32_t *__restrict__ cell_out, V2<T> *__restrict__ xo,
                                                V4<T> *__restrict__ uo, T *__restrict__ zo) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int i = idx[j];
  if (kp.dim == 3) {
    // one 8-value record per particle, at xy (two V4)
    const V4<T> *R = reinterpret_cast<const V4<T> *>(xy) + 2 * (size_t)i;
    V4<T> *O = reinterpret_cast<V4<T> *>(xo) + 2 * (size_t)j;
    O[0] = R[0];
    O[1] = R[1];
  } else {
    xo[j] = xy[i];
    uo[j] = uw[i];
  }
  cell_out[j] = keys[j] / kp.nspecies;
}

}  // namespace

size_t gsort_tmp_elems(int64_t n) { return (size_t)kRsDigits * (size_t)((n + kRsBlock - 1) / kRsBlock) + 1; }

void launch_gsort(const KParams &kp, int prec, int64_t n64, const int32_t *cell, const uint8_t *species,
                  const PartPtrs &src, int32_t *keys0, int32_t *keys1, int32_t *vals0, int32_t *vals1, int32_t *hist,
                  int32_t *scan_tmp, int32_t *err, int32_t *bin_start_out, int32_t *cell_out, const PartPtrs &out,
                  hipStream_t st) {
  const int n = (int)n64;
  const int g256 = (n + 255) / 256;
  if (n > 0) hipLaunchKernelGGL(k_make_keys, dim3(g256), dim3(256), 0, st, kp, n, cell, species, keys0, vals0, err);
  int bits = 0;
  while ((1ll << bits) < (long long)kp.nbins) ++bits;
  const int nblk = (n + kRsBlock - 1) / kRsBlock;
  int32_t *ka = keys0, *kb = keys1, *va = vals0, *vb = vals1;
  for (int shift = 0; shift < bits && n > 0; shift += kRsBits) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kRsBlock), 0, st, ka, n, shift, hist, nblk);
    launch_scan(hist, hist, kRsDigits * nblk, scan_tmp, st);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kRsBlock), 0, st, ka, va, n, shift, hist, nblk, kb, vb);
    int32_t *t = ka;
    ka = kb;
    kb = t;
    t = va;
    va = vb;
    vb = t;
  }
  hipLaunchKernelGGL(k_bin_bounds, dim3((n + 1 + 255) / 256), dim3(256), 0, st, ka, n, kp.nbins, bin_start_out);
  if (n == 0) return;
  if (prec == RELSIM_MIXED)
    hipLaunchKernelGGL(k_gather<float>, dim3(g256), dim3(256), 0, st, kp, n, va, ka, (const V2<float> *)src.xy,
                       (const V4<float> *)src.uw, (const float *)src.z, cell_out, (V2<float> *)out.xy,
                       (V4<float> *)out.uw, (float *)out.z);
  else
    hipLaunchKernelGGL(k_gather<double>, dim3(g256), dim3(256), 0, st, kp, n, va, ka, (const V2<double> *)src.xy,
                       (const V4<double> *)src.uw, (const double *)src.z, cell_out, (V2<double> *)out.xy,
                       (V4<double> *)out.uw, (double *)out.z);
}

}  // namespace relsim
