// C ABI of librelsim: parameter validation, workspace carving, per-kernel
// timing, the host side of restarted GMRES, and the entry points declared in
// include/relsim.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "relsim_internal.h"

using namespace relsim;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct TimedLaunch {
  int name;
  hipEvent_t a, b;
};

}  // namespace

struct relsim_ctx {
  relsim_params p;
  KParams kp;
  Layout L;
  hipStream_t st;
  char *ws;
  int device;
  std::string err;
  double *host;  // pinned scratch for small device-to-host copies
  // kinetic-energy partials of the last push with re-sort (one per wave of
  // its second pass), or 0 when no such push has happened since the last
  // call that could change the particle state
  int push_ke_parts = 0;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> pool;
  std::vector<TimedLaunch> pending;
  std::vector<std::string> names;
  std::map<std::string, int> name_id;
  std::vector<double> ms;
  std::vector<int64_t> count;

  template <typename X>
  X *at(size_t off) const {
    return reinterpret_cast<X *>(ws + off);
  }
};

namespace {

int fail(relsim_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(relsim_ctx *c, hipError_t e, const char *where) {
  return fail(c, RELSIM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_CHECK(c, expr)                        \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
  } while (0)

int name_index(relsim_ctx *c, const char *name) {
  auto it = c->name_id.find(name);
  if (it != c->name_id.end()) return it->second;
  const int id = (int)c->names.size();
  c->names.push_back(name);
  c->name_id[name] = id;
  c->ms.push_back(0.0);
  c->count.push_back(0);
  return id;
}

void harvest(relsim_ctx *c) {
  if (c->pending.empty()) return;
  // a failed synchronisation shows up as failed elapsed-time queries below
  (void)hipStreamSynchronize(c->st);
  for (auto &t : c->pending) {
    float v = 0.f;
    if (hipEventElapsedTime(&v, t.a, t.b) == hipSuccess) {
      c->ms[t.name] += v;
      c->count[t.name] += 1;
    }
    c->pool.push_back(t.a);
    c->pool.push_back(t.b);
  }
  c->pending.clear();
}

// Run `f` (which enqueues one kernel or a short fixed sequence) bracketed by
// events when timing is on.
template <typename F>
void timed(relsim_ctx *c, const char *name, F &&f) {
  if (!c->timing) {
    f();
    return;
  }
  if (c->pool.size() < 2) harvest(c);
  TimedLaunch t;
  t.name = name_index(c, name);
  t.b = c->pool.back();
  c->pool.pop_back();
  t.a = c->pool.back();
  c->pool.pop_back();
  // timing is best effort: a failed record leaves the launch itself intact
  // (its error, if any, is reported by launch_status)
  (void)hipEventRecord(t.a, c->st);
  f();
  (void)hipEventRecord(t.b, c->st);
  c->pending.push_back(t);
}

int validate(const relsim_params *p, std::string &msg) {
  if (!p) return msg = "null params", RELSIM_EINVAL;
  if (p->dim != 2 && p->dim != 3) return msg = "dim must be 2 or 3", RELSIM_EINVAL;
  if (p->nx < 3 || p->ny < 3 || (p->dim == 3 && p->nz < 3)) return msg = "every grid extent must be >= 3", RELSIM_EINVAL;
  const double nc = (double)p->nx * p->ny * (p->dim == 3 ? p->nz : 1);
  if (nc * std::max(1, p->nspecies) >= 2147483647.0) return msg = "too many cells", RELSIM_EINVAL;
  if (!(p->dx > 0) || !(p->dy > 0) || (p->dim == 3 && !(p->dz > 0))) return msg = "cell sizes must be > 0", RELSIM_EINVAL;
  if (!(p->dt > 0) || !std::isfinite(p->dt)) return msg = "dt must be finite and > 0", RELSIM_EINVAL;
  if (!(p->c > 0) || !std::isfinite(p->c)) return msg = "c must be finite and > 0", RELSIM_EINVAL;
  if (!(p->theta >= 0.5 && p->theta <= 1.0)) return msg = "theta must lie in [1/2, 1]", RELSIM_EINVAL;
  if (p->precision != RELSIM_FP64 && p->precision != RELSIM_MIXED) return msg = "unknown precision", RELSIM_EINVAL;
  if (p->nspecies < 1 || p->nspecies > 8) return msg = "nspecies must be 1..8", RELSIM_EINVAL;
  for (int s = 0; s < p->nspecies; ++s)
    if (!(p->m[s] > 0) || !std::isfinite(p->q[s])) return msg = "species mass must be > 0, charge finite", RELSIM_EINVAL;
  if (p->max_particles < 0 || p->max_particles >= 2147483647LL) return msg = "max_particles must be < 2^31", RELSIM_EINVAL;
  if (p->gmres_restart < 1 || p->gmres_restart > kMaxRestart) return msg = "gmres_restart must be 1..64", RELSIM_EINVAL;
  if (p->gmres_maxit < 1) return msg = "gmres_maxit must be >= 1", RELSIM_EINVAL;
  if (!(p->gmres_rtol > 0)) return msg = "gmres_rtol must be > 0", RELSIM_EINVAL;
  if (p->group != 0 && p->group != 4 && p->group != 8 && p->group != 16 && p->group != 32 && p->group != 64)
    return msg = "group must be 0, 4, 8, 16, 32 or 64", RELSIM_EINVAL;
  if (p->mass_fp32 != 0 && (p->mass_fp32 != 1 || p->precision != RELSIM_MIXED))
    return msg = "mass_fp32 must be 0, or 1 with mixed precision", RELSIM_EINVAL;
  return RELSIM_OK;
}

Layout make_layout(const relsim_params *p) {
  Layout L{};
  const size_t nc = (size_t)p->nx * p->ny * (p->dim == 3 ? p->nz : 1);
  const size_t nb = nc * p->nspecies;
  const size_t es = p->precision == RELSIM_MIXED ? 4 : 8;
  const size_t np = (size_t)std::max<int64_t>(p->max_particles, 1);
  const size_t nd = (size_t)n_dirs(p->dim);
  const size_t n3 = 3 * nc;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.S = take((size_t)n_cell_moments(p->dim) * ((nc + kMomBlock - 1) / kMomBlock * kMomBlock) * es);
  L.cnt = take(nd * nb * 2);
  L.pre = take(nd * nb * 2);
  L.total = take(nb * 4);
  L.scan_tmp = take(std::max(scan_tmp_elems((int)nb + 1), scan_tmp_elems((int)gsort_tmp_elems(np))) * 4 + 64);
  L.dirc = take(np);
  L.err = take(64);
  L.gm_V = take((size_t)(p->gmres_restart + 1) * n3 * 8);
  L.gm_t = take(n3 * 8);
  L.gm_b = take(n3 * 8);
  L.gm_r = take(n3 * 8);
  L.gm_part = take((size_t)kDotBlocks * (kMaxRestart + 2) * 8);
  L.gm_small = take(4 * (kMaxRestart + 2) * 8);
  L.red_part = take((size_t)kRedBlocks * 8 * 4);
  L.gs_k0 = take(np * 4);
  L.gs_k1 = take(np * 4);
  L.gs_v0 = take(np * 4);
  L.gs_v1 = take(np * 4);
  L.gs_hist = take(gsort_tmp_elems(np) * 4);
  const size_t ng = (size_t)(p->nx + 2) * (p->ny + 2) * (p->dim == 3 ? p->nz + 2 : 1);
  L.stB = take(ng * 4 * es);
  L.stE = take(ng * 4 * es);
  L.sink = take((size_t)kSinkSlots * 64 * 32);
  L.kin_part = take(nc * 8);
  L.push_ke = take(nc * 8);
  L.end = o;
  return L;
}

KParams make_kparams(const relsim_params *p) {
  KParams k{};
  k.dim = p->dim;
  k.nx = p->nx;
  k.ny = p->ny;
  k.nz = p->dim == 3 ? p->nz : 1;
  k.ncells = k.nx * k.ny * k.nz;
  k.nspecies = p->nspecies;
  k.nbins = k.ncells * k.nspecies;
  k.nonrel = p->nonrelativistic ? 1 : 0;
  // largest power-of-two tile extents (up to 16 x 8 in 2D, 16 x 4 x 4 in 3D)
  // that divide the grid.  A wave of the 3D deposit then takes 16 cells of
  // one row, so each of its 267 moment stores writes 64 contiguous bytes
  // (with 8 x 2 cells, two 32-byte pieces whose neighbours another tile
  // writes much later: the counters showed 1.47x the moment bytes written,
  // and the deposit was 8-16 % slower)
  auto tile = [](int n, int cap) {
    int t = cap;
    while (t > 1 && n % t != 0) t >>= 1;
    return t;
  };
  k.tx = tile(k.nx, 16);
  k.ty = tile(k.ny, p->dim == 3 ? 4 : 8);
  k.tz = p->dim == 3 ? tile(k.nz, 4) : 1;
  // the push passes visit their row segments in taller tiles (2D 32 rows,
  // 3D 16 rows x 4 layers): the re-sort then writes each destination bin's
  // runs from the rows above and below it closer together in time, so more
  // of its partly written lines are completed in L2 before they go to HBM
  // (measured against 8 to 512 rows: 5-6 % off the scatter on both grids)
  k.sty = tile(k.ny, p->dim == 3 ? 16 : 32);
  k.stz = p->dim == 3 ? tile(k.nz, 4) : 1;
  auto lg = [](int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
  };
  k.ltx = lg(k.tx);
  k.lty = lg(k.ty);
  k.ltz = lg(k.tz);
  k.ntx = k.nx / k.tx;
  k.nty = k.ny / k.ty;
  k.dx = p->dx;
  k.dy = p->dy;
  k.dz = p->dim == 3 ? p->dz : 1.0;
  k.dt = p->dt;
  k.c = p->c;
  k.theta = p->theta;
  k.V = k.dx * k.dy * (p->dim == 3 ? k.dz : 1.0);
  k.inv_dx = 1.0 / k.dx;
  k.inv_dy = 1.0 / k.dy;
  k.inv_dz = 1.0 / k.dz;
  k.inv_c = 1.0 / k.c;
  k.inv_c2 = 1.0 / (k.c * k.c);
  k.inv_V = 1.0 / k.V;
  k.gx = k.nx + 2;
  k.gxy = k.gx * (k.ny + 2);
  k.nghost = k.gxy * (p->dim == 3 ? k.nz + 2 : 1);
  for (int s = 0; s < 8; ++s) {
    k.q[s] = s < p->nspecies ? p->q[s] : 0.0;
    k.m[s] = s < p->nspecies ? p->m[s] : 1.0;
    k.beta[s] = s < p->nspecies ? p->q[s] * p->dt / (2.0 * p->m[s]) : 0.0;
    k.f_q[s] = (float)k.q[s];
    k.f_beta[s] = (float)k.beta[s];
  }
  k.f_dt = (float)k.dt;
  k.f_inv_c = (float)k.inv_c;
  k.f_inv_c2 = (float)k.inv_c2;
  k.f_inv_V = (float)k.inv_V;
  k.f_inv_dx = (float)k.inv_dx;
  k.f_inv_dy = (float)k.inv_dy;
  k.f_inv_dz = (float)k.inv_dz;
  return k;
}

enum KernelKind { K_DEPOSIT, K_PUSH, K_SCATTER, K_OTHER };

// Cells per wave of the push passes: the widest power of two dividing nx
// whose segment holds about `rounds` rounds of 64 particles, while the grid
// still gives 2048 waves and the segment's LDS stays within 8 KB (more
// starts to limit occupancy).  The counting pass wants 8 rounds, the
// pushing scatter 4: measured on the 1024 x 512 sheet (128 particles per
// cell: segments of 4 and 2 cells) and the 256 x 128 x 128 sheet (16 per
// cell: 16 cells, LDS-bound, for both).
int choose_cells(const relsim_ctx *c, int64_t n, KernelKind k) {
  const double rounds = k == K_SCATTER ? 4.0 : 8.0;
  const size_t lds = 8192;
  const double mean = (double)n / (double)c->kp.ncells;
  int C = 1;
  while (C < 64 && 2.0 * C * mean <= rounds * 64.0 && c->kp.nx % (2 * C) == 0 &&
         c->kp.ncells / (2 * C) >= 2048 && push_lds_bytes(c->kp, c->p.precision, 2 * C) <= lds)
    C *= 2;
  return C;
}

// Lanes per cell for the deposit and the kinetic-energy kernel: the largest
// power of two in [gmin, 64] not above mean_occupancy / rounds, where
// `rounds` is the number of G-wide rounds per cell the kernel wants, then
// widened until the launch has at least 512 waves (2 per CU) on small
// grids.  The 2D deposit amortises its per-cell reduction over many rounds
// (16 in FP32; 32 in FP64, whose register-bound occupancy favours narrower
// groups) and may go down to 4 lanes.  (The 3D deposit always splits a
// cell's moments over 4 lanes and takes no group.)
int choose_group(const relsim_params &p, const KParams &kp, int64_t n, KernelKind k = K_OTHER) {
  if (p.group) return p.group;
  const bool fp64 = p.precision == RELSIM_FP64;
  double rounds = 4.0;
  if (k == K_DEPOSIT) rounds = fp64 ? 32.0 : 16.0;
  const double mean = (double)n / (double)kp.ncells;
  int g = k == K_DEPOSIT ? 4 : 8;
  while (g < 64 && 2.0 * g <= mean / rounds) g *= 2;
  while (g < 64 && (double)kp.ncells * g < 512.0 * 64.0) g *= 2;
  return g;
}

int choose_group(const relsim_ctx *c, int64_t n, KernelKind k = K_OTHER) { return choose_group(c->p, c->kp, n, k); }

PartPtrs front(const relsim_particles *pt) {
  PartPtrs pp;
  pp.bin_start = pt->bin_start;
  pp.xy = pt->xy;
  pp.uw = pt->uw;
  pp.z = pt->z;
  return pp;
}

PartPtrs back(const relsim_particles *pt) {
  PartPtrs pp;
  pp.bin_start = pt->bin_start_back;
  pp.xy = pt->xy_back;
  pp.uw = pt->uw_back;
  pp.z = pt->z_back;
  return pp;
}

void swap_sets(relsim_particles *pt) {
  std::swap(pt->bin_start, pt->bin_start_back);
  std::swap(pt->cell, pt->cell_back);
  std::swap(pt->xy, pt->xy_back);
  std::swap(pt->uw, pt->uw_back);
  std::swap(pt->z, pt->z_back);
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// 2D: xy (2 T per particle) and uw (4 T); 3D: one 8-T record per particle
// in xy (uw and z unused).  Records must be aligned to their size.
bool records_ok(int dim, size_t es, const void *xy, const void *uw) {
  if (dim == 3) return xy && aligned(xy, 8 * es);
  return xy && uw && aligned(xy, 2 * es) && aligned(uw, 4 * es);
}

int check_particles(relsim_ctx *c, const relsim_particles *pt, bool need_back) {
  if (!pt) return fail(c, RELSIM_EINVAL, "null particles");
  if (pt->n < 0 || pt->n > c->p.max_particles) return fail(c, RELSIM_EINVAL, "particle count outside [0, max_particles]");
  const size_t es = c->p.precision == RELSIM_MIXED ? 4 : 8;
  if (!pt->bin_start || !records_ok(c->p.dim, es, pt->xy, pt->uw))
    return fail(c, RELSIM_EINVAL, "null particle array, or records not aligned to their size");
  if (need_back && (!pt->bin_start_back || !pt->cell_back || !records_ok(c->p.dim, es, pt->xy_back, pt->uw_back)))
    return fail(c, RELSIM_EINVAL, "null back-buffer particle array, or records not aligned to their size");
  return RELSIM_OK;
}

// Deferred error flags raised by kernels (bit 0: move > 1 cell or non-finite
// position; bit 1: bin over 65535 particles; bit 2: bad cell/species id).
int check_flags(relsim_ctx *c) {
  HIP_CHECK(c, hipMemcpyAsync(c->host, c->at<int32_t>(c->L.err), sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
  HIP_CHECK(c, hipStreamSynchronize(c->st));
  int32_t f;
  std::memcpy(&f, c->host, sizeof(f));
  if (f == 0) return RELSIM_OK;
  HIP_CHECK(c, hipMemsetAsync(c->at<int32_t>(c->L.err), 0, sizeof(int32_t), c->st));
  if (f & 1) return fail(c, RELSIM_ERANGE, "a particle moved more than one cell in a step, or its position is not finite");
  if (f & 2) return fail(c, RELSIM_ERANGE, "a (cell, species) bin holds more than 65535 particles");
  if (f & 8) return fail(c, RELSIM_EINTERNAL, "the re-sort's second push pass put a particle further than rounding outside the cell its first pass counted");
  return fail(c, RELSIM_EINVAL, "cell index or species id out of range in relsim_sort input");
}

int launch_status(relsim_ctx *c, const char *where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, where);
  return RELSIM_OK;
}

// S7 on the device: the kinetic energy into res[0] (per-block partials in
// kpart, one per 64/G cells, then a fixed-order reduction through
// part[0..kRedBlocks)), the sums of |E|^2 and |B|^2 into res[1], res[2]
// (partials in part[kRedBlocks..3 kRedBlocks)).
int kinetic_partials(const KParams &kp, int G) { return (kp.ncells + (64 / G) - 1) / (64 / G); }

void enqueue_kinetic(const KParams &kp, int prec, int G, const PartPtrs &pp, double *kpart, double *part, double *res,
                     hipStream_t st) {
  launch_kinetic(kp, prec, G, pp, kpart, st);
  launch_reduce_long(kpart, kinetic_partials(kp, G), part, res, st);
}

void enqueue_field_energy(const KParams &kp, const double *E, const double *B, double *part, double *res,
                          hipStream_t st) {
  const size_t n3 = 3 * (size_t)kp.ncells;
  launch_sumsq_partials(E, n3, part + kRedBlocks, st);
  launch_reduce_partials(part + kRedBlocks, kRedBlocks, 1, res + 1, st);
  launch_sumsq_partials(B, n3, part + 2 * kRedBlocks, st);
  launch_reduce_partials(part + 2 * kRedBlocks, kRedBlocks, 1, res + 2, st);
}

// kinetic, electric, magnetic and total energy from the three device sums
__host__ __device__ void finish_energy(const KParams &kp, const double sums[3], double out[4]) {
  const double f = kp.V / (8.0 * M_PI);
  out[0] = sums[0];
  out[1] = f * sums[1];
  out[2] = f * sums[2];
  out[3] = out[0] + out[1] + out[2];
}

// Count of particles the pushing scatter put on a face of their counted cell
// (8 bytes in the flag slot, after the fixed-point pass's change).
unsigned long long *clamp_counter(relsim_ctx *c) {
  return reinterpret_cast<unsigned long long *>(c->at<char>(c->L.err) + 16);
}

// device -> host copy of k doubles into c->host, synchronising
int fetch(relsim_ctx *c, const double *dev, int k) {
  HIP_CHECK(c, hipMemcpyAsync(c->host, dev, sizeof(double) * k, hipMemcpyDeviceToHost, c->st));
  HIP_CHECK(c, hipStreamSynchronize(c->st));
  return RELSIM_OK;
}

// out = A x   (uses gm_t as the curl scratch)
void apply_A(relsim_ctx *c, const void *M, const double *x, double *out) {
  double *t = c->at<double>(c->L.gm_t);
  timed(c, "curl_nc", [&] { launch_curl(c->kp, x, t, 1, c->st); });
  timed(c, "apply_A", [&] { launch_apply_A_tail(c->kp, c->p.mass_fp32, M, x, t, out, c->st); });
}

// out = A^T x
void apply_AT(relsim_ctx *c, const void *M, const double *x, double *out) {
  double *t = c->at<double>(c->L.gm_t);
  timed(c, "curl_nc", [&] { launch_curl(c->kp, x, t, 1, c->st); });
  timed(c, "apply_AT", [&] { launch_apply_AT_tail(c->kp, c->p.mass_fp32, M, x, t, out, c->st); });
}

int norm2(relsim_ctx *c, const double *x, size_t n, double *out) {
  double *part = c->at<double>(c->L.red_part);
  double *res = c->at<double>(c->L.gm_small) + 3 * (kMaxRestart + 2);
  timed(c, "sumsq", [&] {
    launch_sumsq_partials(x, n, part, c->st);
    launch_reduce_partials(part, kRedBlocks, 1, res, c->st);
  });
  int rc = fetch(c, res, 1);
  if (rc) return rc;
  *out = std::sqrt(c->host[0]);
  return RELSIM_OK;
}

}  // namespace

extern "C" {

size_t relsim_workspace_bytes(const relsim_params *p) {
  std::string msg;
  if (validate(p, msg) != RELSIM_OK) return 0;
  return make_layout(p).end;
}

int relsim_init(const relsim_params *p, void *hip_stream, void *workspace, size_t workspace_bytes, relsim_ctx **out) {
  if (!out) return RELSIM_EINVAL;
  *out = nullptr;
  std::string msg;
  const int v = validate(p, msg);
  if (v != RELSIM_OK) return v;
  const Layout L = make_layout(p);
  if (!workspace || workspace_bytes < L.end) return RELSIM_EINVAL;
  relsim_ctx *c = new (std::nothrow) relsim_ctx();
  if (!c) return RELSIM_EINVAL;
  // an error that earlier calls of other code left pending in this thread
  // (HIP keeps the last one until it is read) is not this call's: clear it
  // before the check at the end
  (void)hipGetLastError();
  c->p = *p;
  if (c->p.dim == 2) c->p.nz = 1;
  c->kp = make_kparams(&c->p);
  c->L = L;
  c->st = (hipStream_t)hip_stream;
  c->ws = (char *)workspace;
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipHostMalloc((void **)&c->host, 4096, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return RELSIM_EHIP;
  }
  for (int i = 0; i < 4096; ++i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) break;
    c->pool.push_back(e);
  }
  if (hipMemsetAsync(c->at<int32_t>(L.err), 0, 64, c->st) != hipSuccess) {
    relsim_finalize(c);
    return RELSIM_EHIP;
  }
  // processing order of the particle kernels: tile-major slot -> cell table
  if (hipGetLastError() != hipSuccess) {
    relsim_finalize(c);
    return RELSIM_EHIP;
  }
  *out = c;
  return RELSIM_OK;
}

void relsim_finalize(relsim_ctx *c) {
  if (!c) return;
  // teardown is best effort: nothing can be reported after this call
  (void)hipStreamSynchronize(c->st);
  for (auto &t : c->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->host) (void)hipHostFree(c->host);
  delete c;
}

int relsim_sort(relsim_ctx *c, relsim_particles *pt) {
  if (!c) return RELSIM_EINVAL;
  int rc = check_particles(c, pt, true);
  if (rc) return rc;
  if (!pt->cell) return fail(c, RELSIM_EINVAL, "relsim_sort needs the cell array");
  if (c->p.nspecies > 1 && !pt->species) return fail(c, RELSIM_EINVAL, "relsim_sort needs species ids");
  timed(c, "general_sort", [&] {
    launch_gsort(c->kp, c->p.precision, pt->n, pt->cell, pt->species, front(pt), c->at<int32_t>(c->L.gs_k0),
                 c->at<int32_t>(c->L.gs_k1), c->at<int32_t>(c->L.gs_v0), c->at<int32_t>(c->L.gs_v1),
                 c->at<int32_t>(c->L.gs_hist), c->at<int32_t>(c->L.scan_tmp), c->at<int32_t>(c->L.err),
                 pt->bin_start_back, pt->cell_back, back(pt), c->st);
  });
  c->push_ke_parts = 0;
  rc = launch_status(c, "relsim_sort");
  if (rc) return rc;
  rc = check_flags(c);
  if (rc) return rc;
  swap_sets(pt);
  return RELSIM_OK;
}

int relsim_deposit_moments(relsim_ctx *c, const relsim_particles *pt, const double *B_n, double *Jhat, void *M) {
  return relsim_deposit_moments_ec(c, pt, B_n, nullptr, Jhat, M);
}

int relsim_deposit_moments_ec(relsim_ctx *c, const relsim_particles *pt, const double *B_n, const void *gbar,
                              double *Jhat, void *M) {
  if (!c) return RELSIM_EINVAL;
  int rc = check_particles(c, pt, false);
  if (rc) return rc;
  if (!B_n || !Jhat || !M) return fail(c, RELSIM_EINVAL, "null grid array");
  if (!aligned(M, c->p.mass_fp32 ? 4 : 8)) return fail(c, RELSIM_EINVAL, "M not aligned to its element size");
  if (gbar && !aligned(gbar, c->p.precision == RELSIM_MIXED ? 4 : 8))
    return fail(c, RELSIM_EINVAL, "gbar not aligned to its element size");
  const int G = choose_group(c, pt->n, K_DEPOSIT);
  void *S = c->at<char>(c->L.S);
  void *stB = c->at<char>(c->L.stB);
  PartPtrs pp = front(pt);
  pp.gbar = gbar;
  timed(c, "stage_fields", [&] { launch_stage_field(c->kp, c->p.precision, B_n, stB, c->st); });
  timed(c, "deposit_cells", [&] { launch_deposit_cells(c->kp, c->p.precision, G, pp, stB, S, c->st); });
  timed(c, "assemble_nodes", [&] { launch_assemble(c->kp, c->p.precision, c->p.mass_fp32, S, Jhat, M, c->st); });
  return launch_status(c, "relsim_deposit_moments");
}

int relsim_push(relsim_ctx *c, relsim_particles *pt, const double *E_theta, const double *B_n, int32_t resort,
                int32_t *new_index) {
  return relsim_push_ec(c, pt, E_theta, B_n, nullptr, resort, new_index);
}

int relsim_gamma_secant(relsim_ctx *c, int64_t n, const void *gbar, void *gbar_next, void *g_prev, void *r_prev,
                        int first) {
  if (!c) return RELSIM_EINVAL;
  if (n < 0 || n > c->p.max_particles) return fail(c, RELSIM_EINVAL, "particle count out of range");
  if (n == 0) return RELSIM_OK;
  if (!gbar || !gbar_next || !g_prev || !r_prev) return fail(c, RELSIM_EINVAL, "null array");
  const size_t es = c->p.precision == RELSIM_MIXED ? 4 : 8;
  if (!aligned(gbar, es) || !aligned(gbar_next, es) || !aligned(g_prev, es) || !aligned(r_prev, es))
    return fail(c, RELSIM_EINVAL, "array not aligned to its element size");
  if (gbar == gbar_next) return fail(c, RELSIM_EINVAL, "gbar and gbar_next must not alias");
  timed(c, "gamma_secant", [&] {
    launch_gamma_secant(c->p.precision, (int)n, gbar, gbar_next, g_prev, r_prev, first, c->st);
  });
  return launch_status(c, "relsim_gamma_secant");
}

int relsim_push_ec(relsim_ctx *c, relsim_particles *pt, const double *E_theta, const double *B_n, const void *gbar,
                   int32_t resort, int32_t *new_index) {
  if (!c) return RELSIM_EINVAL;
  int rc = check_particles(c, pt, resort != 0);
  if (rc) return rc;
  if (!E_theta || !B_n) return fail(c, RELSIM_EINVAL, "null grid array");
  if (gbar && !aligned(gbar, c->p.precision == RELSIM_MIXED ? 4 : 8))
    return fail(c, RELSIM_EINVAL, "gbar not aligned to its element size");
  PartPtrs pp = front(pt);
  pp.gbar = gbar;
  const int cells = choose_cells(c, pt->n, K_PUSH);
  const int cells_s = choose_cells(c, pt->n, K_SCATTER);
  uint8_t *dirc = c->at<uint8_t>(c->L.dirc);
  uint16_t *cnt = c->at<uint16_t>(c->L.cnt);
  uint16_t *pre = c->at<uint16_t>(c->L.pre);
  int32_t *total = c->at<int32_t>(c->L.total);
  int32_t *err = c->at<int32_t>(c->L.err);
  void *stB = c->at<char>(c->L.stB);
  void *stE = c->at<char>(c->L.stE);
  timed(c, "stage_fields", [&] {
    launch_stage_field(c->kp, c->p.precision, B_n, stB, c->st);
    launch_stage_field(c->kp, c->p.precision, E_theta, stE, c->st);
  });
  // with resort the first pass only counts the moves, and the second pushes
  // again, writing the new state straight into its new place
  timed(c, resort ? "push_count" : "push", [&] {
    launch_push(c->kp, c->p.precision, cells, pp, stE, stB, dirc, cnt, err, resort ? 1 : 0,
                c->at<char>(c->L.sink), c->st);
  });
  if (resort) {
    timed(c, "sort_offsets", [&] { launch_sort_offsets(c->kp, cnt, pre, total, err, c->st); });
    timed(c, "sort_scan", [&] {
      launch_scan(total, pt->bin_start_back, c->kp.nbins, c->at<int32_t>(c->L.scan_tmp), c->st);
    });
    timed(c, "push_scatter", [&] {
      launch_push_scatter(c->kp, c->p.precision, cells_s, pp, stE, stB, dirc, pre, pt->bin_start_back, back(pt),
                          (int)pt->n, err, clamp_counter(c), new_index, c->at<char>(c->L.sink),
                          c->at<double>(c->L.push_ke), c->st);
    });
    rc = launch_status(c, "relsim_push");
    if (rc) return rc;
    swap_sets(pt);
    c->push_ke_parts = c->kp.ncells / cells_s;
    return RELSIM_OK;
  }
  c->push_ke_parts = 0;
  return launch_status(c, "relsim_push");
}

int relsim_gamma_mean(relsim_ctx *c, const relsim_particles *pt, const double *E_theta, const double *B_n,
                      const void *gbar, void *gbar_next, double *max_rel_change) {
  if (!c) return RELSIM_EINVAL;
  int rc = check_particles(c, pt, false);
  if (rc) return rc;
  if (!E_theta || !B_n) return fail(c, RELSIM_EINVAL, "null grid array");
  if (!gbar_next || !max_rel_change) return fail(c, RELSIM_EINVAL, "null gbar_next or max_rel_change");
  const size_t es = c->p.precision == RELSIM_MIXED ? 4 : 8;
  if ((gbar && !aligned(gbar, es)) || !aligned(gbar_next, es))
    return fail(c, RELSIM_EINVAL, "gbar not aligned to its element size");
  if (gbar && gbar == gbar_next) return fail(c, RELSIM_EINVAL, "gbar and gbar_next must not alias");
  const int cells = choose_cells(c, pt->n, K_PUSH);
  int32_t *err = c->at<int32_t>(c->L.err);
  // the 8 bytes after the error flags (both in the 64-byte flag slot)
  unsigned long long *chg = reinterpret_cast<unsigned long long *>(c->at<char>(c->L.err) + 8);
  void *stB = c->at<char>(c->L.stB);
  void *stE = c->at<char>(c->L.stE);
  PartPtrs pp = front(pt);
  pp.gbar = gbar;
  HIP_CHECK(c, hipMemsetAsync(chg, 0, sizeof(unsigned long long), c->st));
  timed(c, "stage_fields", [&] {
    launch_stage_field(c->kp, c->p.precision, B_n, stB, c->st);
    launch_stage_field(c->kp, c->p.precision, E_theta, stE, c->st);
  });
  timed(c, "gamma_mean", [&] {
    launch_gamma_mean(c->kp, c->p.precision, cells, pp, stE, stB, err, c->at<char>(c->L.sink), gbar_next, chg,
                      c->st);
  });
  rc = launch_status(c, "relsim_gamma_mean");
  if (rc) return rc;
  HIP_CHECK(c, hipMemcpyAsync(c->host, chg, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->st));
  HIP_CHECK(c, hipStreamSynchronize(c->st));
  std::memcpy(max_rel_change, c->host, sizeof(double));
  return RELSIM_OK;
}

int relsim_placement_clamps(relsim_ctx *c, int64_t *count) {
  if (!c || !count) return RELSIM_EINVAL;
  unsigned long long *d = reinterpret_cast<unsigned long long *>(c->at<char>(c->L.err) + 16);
  HIP_CHECK(c, hipMemcpyAsync(c->host, d, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->st));
  HIP_CHECK(c, hipStreamSynchronize(c->st));
  unsigned long long v;
  std::memcpy(&v, c->host, sizeof(v));
  HIP_CHECK(c, hipMemsetAsync(d, 0, sizeof(unsigned long long), c->st));
  *count = (int64_t)v;
  return RELSIM_OK;
}

int relsim_fill_cells(relsim_ctx *c, relsim_particles *pt) {
  if (!c) return RELSIM_EINVAL;
  int rc = check_particles(c, pt, false);
  if (rc) return rc;
  if (!pt->cell) return fail(c, RELSIM_EINVAL, "null cell array");
  launch_fill_cells(c->kp, pt->bin_start, pt->cell, c->st);
  return launch_status(c, "relsim_fill_cells");
}

int relsim_energy(relsim_ctx *c, const relsim_particles *pt, const double *E, const double *B, double out[4]) {
  if (!c) return RELSIM_EINVAL;
  int rc = check_particles(c, pt, false);
  if (rc) return rc;
  if (!E || !B || !out) return fail(c, RELSIM_EINVAL, "null argument");
  rc = check_flags(c);
  if (rc) return rc;
  const int G = choose_group(c, pt->n);
  double *part = c->at<double>(c->L.red_part);
  double *res = c->at<double>(c->L.gm_small);
  timed(c, "kinetic", [&] {
    enqueue_kinetic(c->kp, c->p.precision, G, front(pt), c->at<double>(c->L.kin_part), part, res, c->st);
  });
  timed(c, "field_energy", [&] { enqueue_field_energy(c->kp, E, B, part, res, c->st); });
  rc = launch_status(c, "relsim_energy");
  if (rc) return rc;
  rc = fetch(c, res, 3);
  if (rc) return rc;
  finish_energy(c->kp, c->host, out);
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(out[i])) return fail(c, RELSIM_ENONFINITE, "energy is not finite");
  return RELSIM_OK;
}

int relsim_energy_pushed(relsim_ctx *c, const double *E, const double *B, double out[4]) {
  if (!c) return RELSIM_EINVAL;
  if (!E || !B || !out) return fail(c, RELSIM_EINVAL, "null argument");
  if (c->push_ke_parts <= 0)
    return fail(c, RELSIM_EINVAL, "relsim_energy_pushed needs a relsim_push with resort since the last sort");
  int rc = check_flags(c);
  if (rc) return rc;
  double *part = c->at<double>(c->L.red_part);
  double *res = c->at<double>(c->L.gm_small);
  timed(c, "kinetic_reduce", [&] {
    launch_reduce_long(c->at<double>(c->L.push_ke), c->push_ke_parts, part, res, c->st);
  });
  timed(c, "field_energy", [&] { enqueue_field_energy(c->kp, E, B, part, res, c->st); });
  rc = launch_status(c, "relsim_energy_pushed");
  if (rc) return rc;
  rc = fetch(c, res, 3);
  if (rc) return rc;
  finish_energy(c->kp, c->host, out);
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(out[i])) return fail(c, RELSIM_ENONFINITE, "energy is not finite");
  return RELSIM_OK;
}

int relsim_curl_nc(relsim_ctx *c, const double *in, double *out) {
  if (!c || !in || !out) return RELSIM_EINVAL;
  timed(c, "curl_nc", [&] { launch_curl(c->kp, in, out, 1, c->st); });
  return launch_status(c, "relsim_curl_nc");
}

int relsim_curl_cn(relsim_ctx *c, const double *in, double *out) {
  if (!c || !in || !out) return RELSIM_EINVAL;
  timed(c, "curl_cn", [&] { launch_curl(c->kp, in, out, 0, c->st); });
  return launch_status(c, "relsim_curl_cn");
}

int relsim_apply_A(relsim_ctx *c, const void *M, const double *x, double *out) {
  if (!c || !M || !x || !out) return RELSIM_EINVAL;
  if (x == out) return fail(c, RELSIM_EINVAL, "relsim_apply_A cannot work in place");
  apply_A(c, M, x, out);
  return launch_status(c, "relsim_apply_A");
}

}  // extern "C"

// Restarted GMRES for A x = b (or A^T x = b) from the initial guess in x.
// b must live in the workspace slot gm_b.  Returns RELSIM_OK, or
// RELSIM_ENOTCONVERGED with the last iterate in x.
static int gmres_solve(relsim_ctx *c, const void *M, bool transpose, double *x, int32_t *iters, double *rel_resid) {
  const size_t n3 = 3 * (size_t)c->kp.ncells;
  const int m = c->p.gmres_restart;
  double *V = c->at<double>(c->L.gm_V);
  double *b = c->at<double>(c->L.gm_b);
  double *r = c->at<double>(c->L.gm_r);
  double *part = c->at<double>(c->L.gm_part);
  double *hdev = c->at<double>(c->L.gm_small);
  double *ydev = hdev + (kMaxRestart + 2);
  double *h1dev = hdev, *h2dev = hdev + 2 * (kMaxRestart + 2);
  auto op = [&](const double *in, double *out) {
    if (transpose)
      apply_AT(c, M, in, out);
    else
      apply_A(c, M, in, out);
  };
  int rc;
  double bnorm;
  rc = norm2(c, b, n3, &bnorm);
  if (rc) return rc;
  if (!std::isfinite(bnorm)) return fail(c, RELSIM_ENONFINITE, "right-hand side is not finite");
  const double tol = c->p.gmres_rtol * bnorm;
  int total_it = 0;
  double rel = 0.0;
  bool converged = false;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  for (;;) {
    // true residual r = b - A x
    op(x, r);
    timed(c, "axpby", [&] { launch_axpby(1.0, b, -1.0, r, n3, c->st); });
    double beta;
    rc = norm2(c, r, n3, &beta);
    if (rc) return rc;
    if (!std::isfinite(beta)) return fail(c, RELSIM_ENONFINITE, "GMRES residual is not finite");
    rel = bnorm > 0 ? beta / bnorm : 0.0;
    if (beta <= tol) {
      converged = true;
      break;
    }
    if (total_it >= c->p.gmres_maxit) break;
    timed(c, "axpby", [&] { launch_axpby(1.0 / beta, r, 0.0, V, n3, c->st); });
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jdone = 0;
    for (int j = 0; j < m; ++j) {
      double *vj = V + (size_t)j * n3;
      double *w = V + (size_t)(j + 1) * n3;
      op(vj, w);
      // classical Gram-Schmidt, twice, with the coefficients staying on the
      // device: h1, then the correction h2, whose entry j + 1 is |w|^2 after
      // the first pass.  The first pass's update and the second pass's dots
      // share one read of the basis, and the second update normalises w by
      // |w| = sqrt(|w|^2 - |h2|^2) (entry j + 2, 0 if that cancelled and w
      // was left as it is); one copy to the host per Arnoldi step.
      timed(c, "mdot", [&] { launch_mdot(V, n3, j + 1, w, n3, part, h1dev, c->st); });
      int fused = 0;
      timed(c, "maxpy_dot", [&] { fused = launch_maxpy_dot(V, n3, j + 1, h1dev, w, n3, part, h2dev, c->st); });
      if (!fused) {
        timed(c, "maxpy", [&] { launch_maxpy(V, n3, j + 1, h1dev, w, n3, c->st); });
        timed(c, "mdot", [&] { launch_mdot(V, n3, j + 2, w, n3, part, h2dev, c->st); });
      }
      timed(c, "maxpy", [&] { launch_maxpy_scale(V, n3, j + 1, h2dev, w, n3, c->st); });
      rc = fetch(c, hdev, (int)(h2dev - hdev) + j + 3);
      if (rc) return rc;
      const double *h1 = c->host, *h2 = c->host + (h2dev - hdev);
      std::vector<double> h(h1, h1 + j + 1);
      for (int k = 0; k <= j; ++k) h[k] += h2[k];
      double hn = h2[j + 2];
      const bool scaled = hn > 0.0;
      if (!scaled) {
        rc = norm2(c, w, n3, &hn);
        if (rc) return rc;
      }
      if (!std::isfinite(hn)) return fail(c, RELSIM_ENONFINITE, "GMRES Arnoldi vector is not finite");
      for (int k = 0; k <= j; ++k) H[(size_t)k * m + j] = h[k];
      H[(size_t)(j + 1) * m + j] = hn;
      for (int k = 0; k < j; ++k) {
        const double a = H[(size_t)k * m + j], bb = H[(size_t)(k + 1) * m + j];
        H[(size_t)k * m + j] = cs[k] * a + sn[k] * bb;
        H[(size_t)(k + 1) * m + j] = -sn[k] * a + cs[k] * bb;
      }
      const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
      const double den = std::hypot(a, bb);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? bb / den : 0.0;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total_it;
      jdone = j + 1;
      const bool last = std::fabs(g[j + 1]) <= tol || hn == 0.0 || j == m - 1 || total_it >= c->p.gmres_maxit;
      if (last) break;
      if (!scaled) timed(c, "axpby", [&] { launch_axpby(1.0 / hn, w, 0.0, w, n3, c->st); });
    }
    // y = H^-1 g (upper triangular), x += V y
    for (int k = jdone - 1; k >= 0; --k) {
      double s = g[k];
      for (int l = k + 1; l < jdone; ++l) s -= H[(size_t)k * m + l] * y[l];
      y[k] = H[(size_t)k * m + k] != 0.0 ? s / H[(size_t)k * m + k] : 0.0;
    }
    for (int k = 0; k < jdone; ++k) c->host[k] = -y[k];
    HIP_CHECK(c, hipMemcpyAsync(ydev, c->host, sizeof(double) * jdone, hipMemcpyHostToDevice, c->st));
    timed(c, "maxpy", [&] { launch_maxpy(V, n3, jdone, ydev, x, n3, c->st); });
    // the copy reads c->host; make sure it finished before the host buffer is reused
    HIP_CHECK(c, hipStreamSynchronize(c->st));
  }
  if (iters) *iters = total_it;
  if (rel_resid) *rel_resid = rel;
  if (!converged) return fail(c, RELSIM_ENOTCONVERGED, "GMRES reached gmres_maxit before gmres_rtol");
  return RELSIM_OK;
}

extern "C" {

}  // extern "C"

// S4-S5 from E^n (guess == false) or from E_theta's contents (guess == true).
static int field_solve(relsim_ctx *c, const void *M, const double *Jhat, const double *E_n, const double *B_n,
                       double *E_theta, double *E_np1, double *B_np1, int32_t *iters, double *rel_resid,
                       bool guess) {
  if (!c) return RELSIM_EINVAL;
  if (!M || !Jhat || !E_n || !B_n || !E_theta || !E_np1 || !B_np1) return fail(c, RELSIM_EINVAL, "null grid array");
  if (E_theta == E_n || E_theta == E_np1 || B_np1 == B_n) return fail(c, RELSIM_EINVAL, "aliased solve arguments");
  int rc = check_flags(c);
  if (rc) return rc;
  const size_t n3 = 3 * (size_t)c->kp.ncells;
  double *b = c->at<double>(c->L.gm_b);
  timed(c, "rhs", [&] { launch_rhs(c->kp, E_n, B_n, Jhat, b, c->st); });
  if (!guess) HIP_CHECK(c, hipMemcpyAsync(E_theta, E_n, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->st));
  const int solved = gmres_solve(c, M, false, E_theta, iters, rel_resid);
  if (solved != RELSIM_OK && solved != RELSIM_ENOTCONVERGED) return solved;
  timed(c, "field_update", [&] { launch_field_update(c->kp, E_n, B_n, E_theta, E_np1, B_np1, c->st); });
  rc = launch_status(c, guess ? "relsim_field_solve_guess" : "relsim_field_solve");
  if (rc) return rc;
  return solved;
}

extern "C" {

int relsim_field_solve(relsim_ctx *c, const void *M, const double *Jhat, const double *E_n, const double *B_n,
                       double *E_theta, double *E_np1, double *B_np1, int32_t *iters, double *rel_resid) {
  return field_solve(c, M, Jhat, E_n, B_n, E_theta, E_np1, B_np1, iters, rel_resid, false);
}

int relsim_field_solve_guess(relsim_ctx *c, const void *M, const double *Jhat, const double *E_n,
                             const double *B_n, double *E_theta, double *E_np1, double *B_np1, int32_t *iters,
                             double *rel_resid) {
  return field_solve(c, M, Jhat, E_n, B_n, E_theta, E_np1, B_np1, iters, rel_resid, true);
}

int relsim_apply_AT(relsim_ctx *c, const void *M, const double *x, double *out) {
  if (!c || !M || !x || !out) return RELSIM_EINVAL;
  if (x == out) return fail(c, RELSIM_EINVAL, "relsim_apply_AT cannot work in place");
  apply_AT(c, M, x, out);
  return launch_status(c, "relsim_apply_AT");
}

static AdjInPtrs adj_inputs(const relsim_particles *pt) {
  AdjInPtrs a;
  a.bin_start = pt->bin_start;
  a.cell = pt->cell;
  a.xy = (const double *)pt->xy;
  a.uw = (const double *)pt->uw;
  a.z = (const double *)pt->z;
  return a;
}

int relsim_push_adjoint(relsim_ctx *c, const relsim_particles *state_n, const double *E_theta, const double *B_n,
                        const int32_t *new_index, const double *lam_x_in, const double *lam_u_in, double *lam_x_out,
                        double *lam_u_out, double *lam_E_theta, double *lam_B_n) {
  if (!c) return RELSIM_EINVAL;
  if (c->p.precision != RELSIM_FP64) return fail(c, RELSIM_EINVAL, "the adjoint needs RELSIM_FP64");
  int rc = check_particles(c, state_n, false);
  if (rc) return rc;
  if (!state_n->cell || !E_theta || !B_n || !lam_x_in || !lam_u_in || !lam_x_out || !lam_u_out || !lam_E_theta ||
      !lam_B_n)
    return fail(c, RELSIM_EINVAL, "null argument");
  timed(c, "push_adjoint", [&] {
    launch_push_adjoint(c->kp, adj_inputs(state_n), (int)state_n->n, E_theta, B_n, new_index, lam_x_in, lam_u_in,
                        lam_x_out, lam_u_out, lam_E_theta, lam_B_n, c->st);
  });
  return launch_status(c, "relsim_push_adjoint");
}

int relsim_field_solve_adjoint(relsim_ctx *c, const void *M, const double *lam_E_theta, const double *lam_E_np1,
                               const double *lam_B_np1, double *mu, double *lam_E_n, double *lam_B_n, int32_t *iters,
                               double *rel_resid) {
  if (!c) return RELSIM_EINVAL;
  if (!M || !lam_E_theta || !lam_E_np1 || !lam_B_np1 || !mu || !lam_E_n || !lam_B_n)
    return fail(c, RELSIM_EINVAL, "null grid array");
  int rc = check_flags(c);
  if (rc) return rc;
  const size_t n3 = 3 * (size_t)c->kp.ncells;
  const double th = c->kp.theta;
  double *b = c->at<double>(c->L.gm_b);
  double *t = c->at<double>(c->L.gm_t);
  // rhs = l_th + l_E1/theta - c dt C_NC^T l_B1, with C_NC^T = C_CN
  timed(c, "curl_cn", [&] { launch_curl(c->kp, lam_B_np1, t, 0, c->st); });
  timed(c, "adj_rhs", [&] { launch_adj_rhs(n3, th, c->kp.c * c->kp.dt, lam_E_theta, lam_E_np1, t, b, c->st); });
  HIP_CHECK(c, hipMemsetAsync(mu, 0, n3 * sizeof(double), c->st));
  const int solved = gmres_solve(c, M, true, mu, iters, rel_resid);
  if (solved != RELSIM_OK && solved != RELSIM_ENOTCONVERGED) return solved;
  // l_En += -(1-theta)/theta l_E1 + mu ; l_Bn += l_B1 + c theta dt C_CN^T mu, with C_CN^T = C_NC
  timed(c, "curl_nc", [&] { launch_curl(c->kp, mu, t, 1, c->st); });
  timed(c, "adj_finish", [&] {
    launch_adj_finish(n3, th, c->kp.c * th * c->kp.dt, lam_E_np1, lam_B_np1, mu, t, lam_E_n, lam_B_n, c->st);
  });
  rc = launch_status(c, "relsim_field_solve_adjoint");
  if (rc) return rc;
  return solved;
}

int relsim_deposit_adjoint(relsim_ctx *c, const relsim_particles *state_n, const double *B_n, const double *E_theta,
                           const double *mu, double *lam_x, double *lam_u, double *lam_B_n) {
  if (!c) return RELSIM_EINVAL;
  if (c->p.precision != RELSIM_FP64) return fail(c, RELSIM_EINVAL, "the adjoint needs RELSIM_FP64");
  int rc = check_particles(c, state_n, false);
  if (rc) return rc;
  if (!state_n->cell || !B_n || !E_theta || !mu || !lam_x || !lam_u || !lam_B_n)
    return fail(c, RELSIM_EINVAL, "null argument");
  timed(c, "deposit_adjoint", [&] {
    launch_deposit_adjoint(c->kp, adj_inputs(state_n), (int)state_n->n, B_n, E_theta, mu, lam_x, lam_u, lam_B_n,
                           c->st);
  });
  return launch_status(c, "relsim_deposit_adjoint");
}

int relsim_timing_enable(relsim_ctx *c, int32_t on) {
  if (!c) return RELSIM_EINVAL;
  c->timing = on != 0;
  return RELSIM_OK;
}

int relsim_timing_reset(relsim_ctx *c) {
  if (!c) return RELSIM_EINVAL;
  harvest(c);
  std::fill(c->ms.begin(), c->ms.end(), 0.0);
  std::fill(c->count.begin(), c->count.end(), 0);
  return RELSIM_OK;
}

int relsim_timing_read(relsim_ctx *c, int32_t cap, char (*names)[48], double *ms, int64_t *count) {
  if (!c) return RELSIM_EINVAL;
  harvest(c);
  const int n = std::min<int>(cap, (int)c->names.size());
  for (int i = 0; i < n; ++i) {
    if (names) {
      std::strncpy(names[i], c->names[i].c_str(), 47);
      names[i][47] = 0;
    }
    if (ms) ms[i] = c->ms[i];
    if (count) count[i] = c->count[i];
  }
  return n;
}

const char *relsim_strerror(int code) {
  switch (code) {
    case RELSIM_OK: return "ok";
    case RELSIM_EINVAL: return "invalid argument";
    case RELSIM_ENOTCONVERGED: return "linear solve did not converge";
    case RELSIM_EHIP: return "HIP runtime error";
    case RELSIM_ENONFINITE: return "non-finite value";
    case RELSIM_ERANGE: return "value out of range";
    case RELSIM_EINTERNAL: return "internal consistency check failed";
    default: return "unknown error";
  }
}

const char *relsim_last_error(const relsim_ctx *c) { return c ? c->err.c_str() : "no context"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free energy diagnostic: relsim_energy without a context, its
// reduction partials in a file-scope device array instead of the caller's
// workspace.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchDoubles = size_t(1) << 19;  // 4 MiB per device
constexpr size_t kScratchFixed = 3 * (size_t)kRedBlocks + 8;  // reduction partials and the three sums
constexpr int kMaxDevices = 64;

}  // namespace

// One copy per device, held by the device until the process ends; every
// relsim_energy_noalloc call on that device uses it.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (the array's host-side name is not a device address).
int scratch_on_device(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RELSIM_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RELSIM_EHIP;
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return RELSIM_OK;
}

// out[0..3] = kinetic, electric, magnetic, total from the three sums.
__global__ void k_finish_energy(KParams kp, const double *__restrict__ sums, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double v[4];
    finish_energy(kp, sums, v);
    for (int i = 0; i < 4; ++i) out[i] = v[i];
  }
}

}  // namespace

extern "C" int relsim_energy_noalloc(const relsim_params *params, void *hip_stream, const relsim_particles *pt,
                                     const double *E, const double *B, double *out) {
  std::string msg;
  if (validate(params, msg) != RELSIM_OK) return RELSIM_EINVAL;
  if (!pt || !E || !B || !out) return RELSIM_EINVAL;
  relsim_params p = *params;
  if (p.dim == 2) p.nz = 1;
  if (pt->n < 0 || pt->n > p.max_particles) return RELSIM_EINVAL;
  if (!pt->bin_start || !records_ok(p.dim, p.precision == RELSIM_MIXED ? 4 : 8, pt->xy, pt->uw) ||
      !aligned(out, sizeof(double)))
    return RELSIM_EINVAL;
  const KParams kp = make_kparams(&p);
  const int G = choose_group(p, kp, pt->n);
  const size_t need = kScratchFixed + (size_t)kinetic_partials(kp, G);
  if (need > kScratchDoubles) return RELSIM_ERANGE;  // grid too large for the fixed scratch
  double *sc = nullptr;
  const int rc = scratch_on_device(&sc);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  // [0, 3 kRedBlocks): reduction partials; then the three sums; then the
  // per-block kinetic partials.  Every kernel writes all it reads.
  double *part = sc;
  double *res = sc + 3 * (size_t)kRedBlocks;
  double *kpart = sc + kScratchFixed;
  PartPtrs pp;
  pp.bin_start = pt->bin_start;
  pp.xy = pt->xy;
  pp.uw = pt->uw;
  pp.z = pt->z;
  enqueue_kinetic(kp, p.precision, G, pp, kpart, part, res, st);
  enqueue_field_energy(kp, E, B, part, res, st);
  hipLaunchKernelGGL(k_finish_energy, dim3(1), dim3(64), 0, st, kp, res, out);
  return hipGetLastError() == hipSuccess ? RELSIM_OK : RELSIM_EHIP;
}
