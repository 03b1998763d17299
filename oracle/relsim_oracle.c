/*
 * CPU FP64 oracle of one relativistic semi-implicit (ECsim/RelSIM-type) PIC
 * step.  TEST INFRASTRUCTURE ONLY: the tests, the package's smoke check and
 * the benchmark's CPU-baseline leg may call this; the product path never does.
 * It shares no code with the HIP library.
 *
 * What it computes (Schoeffler et al. 2025, Sec. 2, the methods paragraph: the
 * field solve is implicit, the pusher explicit, and the current is linearised
 * through per-particle mass matrices; the discrete equations are those of the
 * cited ECsim/RelSIM schemes, restated here in their standard form):
 *
 *   grid      periodic; E, J-hat and M at nodes (i, j, k)*dx; B at cell
 *             centres (i+1/2, j+1/2, k+1/2)*dx; CIC (linear) weights for both.
 *   S1        B_p  = sum_c W_c(x_p) B^n_c
 *   S2        gbar = sqrt(1 + |u^n|^2/c^2);  b = beta_s B_p / (gbar c),
 *             beta_s = q_s dt / (2 m_s);  alpha = (I - [b]x + b b^T)/(1 + b^2)
 *             where [b]x v = b x v
 *   S3        Jhat_g  = V^-1 sum_p w q W_g alpha u / gbar
 *             M_{g,g'} = V^-1 sum_p (w q beta / gbar) W_g W_g' alpha
 *   S4        [I + (c th dt)^2 C_CN C_NC + 4 pi th dt M] E_th
 *                 = E^n + c th dt C_CN B^n - 4 pi th dt Jhat
 *   S5        B^{n+1} = B^n - c dt C_NC E_th;  E^{n+1} = (E_th - (1-th) E^n)/th
 *   S6        E_p = sum_g W_g(x_p) E_th_g;  ubar = alpha (u + beta E_p);
 *             u' = 2 ubar - u;  x' = x + dt u'/gamma(u')  (periodic wrap)
 *   S7        W = sum_p w m c^2 (gamma - 1) + V/(8 pi) (sum |E|^2 + sum |B|^2)
 *
 * Energy-conserving variant (the exact relativistic case the paper's methods
 * paragraph says the standard scheme lacks): gbar = (gamma(u^n) +
 * gamma(u^{n+1}))/2 in S2, S3 and S6.  Then m c^2 (gamma^{n+1} - gamma^n) =
 * q dt E_p . ubar / gbar exactly, the work of the current S3 deposits, and the
 * step conserves W; gbar depends on u^{n+1}, so the step is a fixed point,
 * found by iterating S1-S6 (oracle.step_ec).  gbar then comes in per particle.
 *
 * The discrete curls are centred differences averaged over the transverse
 * corners, so that C_CN is the transpose of C_NC.  In 2D the z direction is
 * ignorable (d/dz = 0) and V = dx dy.
 *
 * Layouts (shared interface, not shared code): grid arrays are [3][N] with
 * node/cell (i,j,k) at i + nx (j + ny k); M is [noff][9][N] with offset index
 * sum_d (delta_d + 1) 3^d and the 3x3 block row-major.  Particle positions are
 * physical coordinates x[3][n] in [0, L).
 *
 * The nonrel flag selects the non-relativistic limit (gamma == 1, kinetic
 * energy m|u|^2/2) in which the scheme conserves energy exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t dim, nx, ny, nz;
  double dx, dy, dz, dt, c, theta;
  int32_t nonrel;
  int32_t nspecies;
  double q[8], m[8];
} ocfg;

static long nnodes(const ocfg *g) { return (long)g->nx * g->ny * (g->dim == 3 ? g->nz : 1); }
static int nz_of(const ocfg *g) { return g->dim == 3 ? g->nz : 1; }
static int noff(const ocfg *g) { return g->dim == 3 ? 27 : 9; }
static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static long lin(const ocfg *g, int i, int j, int k) {
  return (long)wrap(i, g->nx) + (long)g->nx * ((long)wrap(j, g->ny) + (long)g->ny * wrap(k, nz_of(g)));
}
static double cellvol(const ocfg *g) { return g->dx * g->dy * (g->dim == 3 ? g->dz : 1.0); }
static double spacing(const ocfg *g, int d) { return d == 0 ? g->dx : (d == 1 ? g->dy : g->dz); }
static int extent(const ocfg *g, int d) { return d == 0 ? g->nx : (d == 1 ? g->ny : g->nz); }

/* CIC stencil of one particle: 2^dim corner indices and weights.  shift = 0
 * for nodes (points i*dx), 0.5 for cell centres (points (i+1/2)*dx; the
 * centre of cell i).  Returns the number of corners. */
static int cic(const ocfg *g, const double *x, long n, long p, double shift, long idx[8], double wt[8]) {
  int base[3] = {0, 0, 0};
  double f[3] = {0, 0, 0};
  for (int d = 0; d < g->dim; ++d) {
    double s = x[d * n + p] / spacing(g, d) - shift;
    double fl = floor(s);
    base[d] = (int)fl;
    f[d] = s - fl;
  }
  int nc = 1 << g->dim;
  for (int a = 0; a < nc; ++a) {
    int o[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
    double w = 1.0;
    for (int d = 0; d < g->dim; ++d) w *= o[d] ? f[d] : 1.0 - f[d];
    idx[a] = lin(g, base[0] + o[0], base[1] + o[1], g->dim == 3 ? base[2] + o[2] : 0);
    wt[a] = w;
  }
  return nc;
}

static double gamma_of(const ocfg *g, const double u[3]) {
  if (g->nonrel) return 1.0;
  return sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / (g->c * g->c));
}

/* S2: alpha = (I - [b]x + b b^T) / (1 + |b|^2), row-major 3x3. */
void oracle_alpha(const double b[3], double al[9]) {
  double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  double inv = 1.0 / (1.0 + bb);
  /* [b]x = [[0,-bz,by],[bz,0,-bx],[-by,bx,0]] */
  double cx[9] = {0.0, -b[2], b[1], b[2], 0.0, -b[0], -b[1], b[0], 0.0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) al[3 * i + j] = ((i == j ? 1.0 : 0.0) - cx[3 * i + j] + b[i] * b[j]) * inv;
}

/* S1 (one particle): B_p gathered from cell centres. */
static void gather_centres(const ocfg *g, const double *x, long n, long p, const double *B, double out[3]) {
  long idx[8];
  double wt[8];
  long N = nnodes(g);
  int nc = cic(g, x, n, p, 0.5, idx, wt);
  out[0] = out[1] = out[2] = 0.0;
  for (int a = 0; a < nc; ++a)
    for (int k = 0; k < 3; ++k) out[k] += wt[a] * B[k * N + idx[a]];
}

static void gather_nodes(const ocfg *g, const double *x, long n, long p, const double *E, double out[3]) {
  long idx[8];
  double wt[8];
  long N = nnodes(g);
  int nc = cic(g, x, n, p, 0.0, idx, wt);
  out[0] = out[1] = out[2] = 0.0;
  for (int a = 0; a < nc; ++a)
    for (int k = 0; k < 3; ++k) out[k] += wt[a] * E[k * N + idx[a]];
}

/* S1 + S2 for one particle: alpha, gbar and beta.  gb_in, if not NULL, gives
 * gbar per particle (the energy-conserving variant: the mean of the old and
 * new Lorentz factors, from the fixed-point iteration); it is ignored in the
 * non-relativistic limit. */
static void particle_alpha(const ocfg *g, const double *x, const double *u, const int32_t *sp, long n, long p,
                           const double *B, const double *gb_in, double al[9], double *gbar, double *beta) {
  double up[3] = {u[p], u[n + p], u[2 * n + p]};
  int s = sp[p];
  double Bp[3];
  gather_centres(g, x, n, p, B, Bp);
  *gbar = (gb_in && !g->nonrel) ? gb_in[p] : gamma_of(g, up);
  *beta = g->q[s] * g->dt / (2.0 * g->m[s]);
  double b[3];
  for (int k = 0; k < 3; ++k) b[k] = *beta * Bp[k] / (*gbar * g->c);
  oracle_alpha(b, al);
}

/* S1 for all particles (diagnostic access). */
void oracle_gather_B(const ocfg *g, long n, const double *x, const double *B, double *Bp) {
  for (long p = 0; p < n; ++p) {
    double o[3];
    gather_centres(g, x, n, p, B, o);
    for (int k = 0; k < 3; ++k) Bp[k * n + p] = o[k];
  }
}

/* Node gather of a grid vector for all particles (the S6 field gather). */
void oracle_gather_E(const ocfg *g, long n, const double *x, const double *E, double *Ep) {
  for (long p = 0; p < n; ++p) {
    double o[3];
    gather_nodes(g, x, n, p, E, o);
    for (int k = 0; k < 3; ++k) Ep[k * n + p] = o[k];
  }
}

/* S1 + S2 for all particles: alpha [9][n]. */
void oracle_alphas(const ocfg *g, long n, const double *x, const double *u, const int32_t *sp, const double *B,
                   double *alpha) {
  for (long p = 0; p < n; ++p) {
    double al[9], gb, be;
    particle_alpha(g, x, u, sp, n, p, B, NULL, al, &gb, &be);
    for (int k = 0; k < 9; ++k) alpha[k * n + p] = al[k];
  }
}

/* S1-S3: Jhat [3][N] and M [noff][9][N], both overwritten. */
void oracle_deposit(const ocfg *g, long n, const double *x, const double *u, const double *w, const int32_t *sp,
                    const double *B, const double *gb_in, double *J, double *M) {
  long N = nnodes(g);
  int no = noff(g);
  double V = cellvol(g);
  memset(J, 0, sizeof(double) * 3 * N);
  memset(M, 0, sizeof(double) * (size_t)no * 9 * N);
  for (long p = 0; p < n; ++p) {
    double al[9], gb, be;
    particle_alpha(g, x, u, sp, n, p, B, gb_in, al, &gb, &be);
    int s = sp[p];
    double cJ = w[p] * g->q[s] / V;
    double cM = w[p] * g->q[s] * be / (V * gb);
    double up[3] = {u[p], u[n + p], u[2 * n + p]};
    double v[3];
    for (int i = 0; i < 3; ++i) v[i] = (al[3 * i] * up[0] + al[3 * i + 1] * up[1] + al[3 * i + 2] * up[2]) / gb;
    long idx[8];
    double wt[8];
    int nc = cic(g, x, n, p, 0.0, idx, wt);
    for (int a = 0; a < nc; ++a) {
      for (int k = 0; k < 3; ++k) J[k * N + idx[a]] += cJ * wt[a] * v[k];
      for (int b = 0; b < nc; ++b) {
        int off = 0, pw = 1;
        for (int d = 0; d < g->dim; ++d) {
          int delta = ((b >> d) & 1) - ((a >> d) & 1);
          off += (delta + 1) * pw;
          pw *= 3;
        }
        double c = cM * wt[a] * wt[b];
        for (int k = 0; k < 9; ++k) M[((long)off * 9 + k) * N + idx[a]] += c * al[k];
      }
    }
  }
}

/* S1-S3 restricted to a list of nodes (for sampled checks at large sizes):
 * Jout [3][ns], Mout [noff][9][ns] for nodes node_ids[ns].  Each sampled
 * node receives exactly the terms oracle_deposit adds into it, in the same
 * particle order.  Returns 0, -1 if the slot table cannot be allocated, or
 * -2 if a node id is out of range or listed twice (outputs then untouched). */
int oracle_deposit_nodes(const ocfg *g, long n, const double *x, const double *u, const double *w,
                         const int32_t *sp, const double *B, long ns, const long *node_ids, double *Jout,
                         double *Mout) {
  long N = nnodes(g);
  int no = noff(g);
  double V = cellvol(g);
  long *slot = (long *)malloc(sizeof(long) * (size_t)(N > 0 ? N : 1));
  if (!slot) return -1;
  for (long i = 0; i < N; ++i) slot[i] = -1;
  for (long s = 0; s < ns; ++s) {
    long id = node_ids[s];
    if (id < 0 || id >= N || slot[id] >= 0) {
      free(slot);
      return -2;
    }
    slot[id] = s;
  }
  memset(Jout, 0, sizeof(double) * 3 * ns);
  memset(Mout, 0, sizeof(double) * (size_t)no * 9 * ns);
  for (long p = 0; p < n; ++p) {
    long idx[8];
    double wt[8];
    int nc = cic(g, x, n, p, 0.0, idx, wt);
    int hit = 0;
    for (int a = 0; a < nc; ++a) hit |= slot[idx[a]] >= 0;
    if (!hit) continue;
    double al[9], gb, be;
    particle_alpha(g, x, u, sp, n, p, B, NULL, al, &gb, &be);
    int s = sp[p];
    double cJ = w[p] * g->q[s] / V;
    double cM = w[p] * g->q[s] * be / (V * gb);
    double up[3] = {u[p], u[n + p], u[2 * n + p]};
    double v[3];
    for (int i = 0; i < 3; ++i) v[i] = (al[3 * i] * up[0] + al[3 * i + 1] * up[1] + al[3 * i + 2] * up[2]) / gb;
    for (int a = 0; a < nc; ++a) {
      long sl = slot[idx[a]];
      if (sl < 0) continue;
      for (int k = 0; k < 3; ++k) Jout[k * ns + sl] += cJ * wt[a] * v[k];
      for (int b = 0; b < nc; ++b) {
        int off = 0, pw = 1;
        for (int d = 0; d < g->dim; ++d) {
          int delta = ((b >> d) & 1) - ((a >> d) & 1);
          off += (delta + 1) * pw;
          pw *= 3;
        }
        double c = cM * wt[a] * wt[b];
        for (int k = 0; k < 9; ++k) Mout[((long)off * 9 + k) * ns + sl] += c * al[k];
      }
    }
  }
  free(slot);
  return 0;
}

/* Difference along dim d, averaged over the transverse corners.
 * Nodes -> centre of cell (i,j,k):  [f(node + e_d + t) - f(node + t)] / h_d.
 * Centres -> node (i,j,k):          [g(cell - t) - g(cell - e_d - t)] / h_d,
 * t over {0,1} in every other active dimension. */
static double diff_nc(const ocfg *g, const double *f, int d, int i, int j, int k) {
  int act[3] = {1, 1, g->dim == 3};
  if (!act[d]) return 0.0;
  double acc = 0.0;
  int cnt = 0;
  for (int t = 0; t < 8; ++t) {
    int o[3] = {t & 1, (t >> 1) & 1, (t >> 2) & 1};
    int skip = 0;
    for (int e = 0; e < 3; ++e)
      if ((e == d || !act[e]) && o[e]) skip = 1;
    if (skip) continue;
    int e0[3] = {d == 0, d == 1, d == 2};
    acc += f[lin(g, i + o[0] + e0[0], j + o[1] + e0[1], k + o[2] + e0[2])] - f[lin(g, i + o[0], j + o[1], k + o[2])];
    ++cnt;
  }
  return acc / (cnt * spacing(g, d));
}

static double diff_cn(const ocfg *g, const double *f, int d, int i, int j, int k) {
  int act[3] = {1, 1, g->dim == 3};
  if (!act[d]) return 0.0;
  double acc = 0.0;
  int cnt = 0;
  for (int t = 0; t < 8; ++t) {
    int o[3] = {t & 1, (t >> 1) & 1, (t >> 2) & 1};
    int skip = 0;
    for (int e = 0; e < 3; ++e)
      if ((e == d || !act[e]) && o[e]) skip = 1;
    if (skip) continue;
    int e0[3] = {d == 0, d == 1, d == 2};
    acc += f[lin(g, i - o[0], j - o[1], k - o[2])] - f[lin(g, i - o[0] - e0[0], j - o[1] - e0[1], k - o[2] - e0[2])];
    ++cnt;
  }
  return acc / (cnt * spacing(g, d));
}

/* curl from nodes to centres (C_NC) or centres to nodes (C_CN). */
static void curl(const ocfg *g, const double *F, double *out, int to_centres) {
  long N = nnodes(g);
  const double *Fx = F, *Fy = F + N, *Fz = F + 2 * N;
  for (int k = 0; k < nz_of(g); ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        double (*D)(const ocfg *, const double *, int, int, int, int) = to_centres ? diff_nc : diff_cn;
        long c = lin(g, i, j, k);
        out[c] = D(g, Fz, 1, i, j, k) - D(g, Fy, 2, i, j, k);
        out[N + c] = D(g, Fx, 2, i, j, k) - D(g, Fz, 0, i, j, k);
        out[2 * N + c] = D(g, Fy, 0, i, j, k) - D(g, Fx, 1, i, j, k);
      }
}

void oracle_curl_nc(const ocfg *g, const double *E, double *out) { curl(g, E, out, 1); }
void oracle_curl_cn(const ocfg *g, const double *B, double *out) { curl(g, B, out, 0); }

/* (M x)_g = sum_off M[off] x_{g + delta(off)} */
void oracle_apply_M(const ocfg *g, const double *M, const double *xv, double *out) {
  long N = nnodes(g);
  int no = noff(g);
  memset(out, 0, sizeof(double) * 3 * N);
  for (int k = 0; k < nz_of(g); ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        long gi = lin(g, i, j, k);
        for (int off = 0; off < no; ++off) {
          int dx = off % 3 - 1, dy = (off / 3) % 3 - 1, dz = off / 9 - 1;
          long gj = lin(g, i + dx, j + dy, k + dz);
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) out[r * N + gi] += M[((long)off * 9 + 3 * r + c) * N + gi] * xv[c * N + gj];
        }
      }
}

/* S4 operator: A x = x + (c th dt)^2 C_CN C_NC x + 4 pi th dt M x */
void oracle_apply_A(const ocfg *g, const double *M, const double *xv, double *out) {
  long N = nnodes(g);
  double *t1 = (double *)malloc(sizeof(double) * 3 * N);
  double *t2 = (double *)malloc(sizeof(double) * 3 * N);
  double *t3 = (double *)malloc(sizeof(double) * 3 * N);
  oracle_curl_nc(g, xv, t1);
  oracle_curl_cn(g, t1, t2);
  oracle_apply_M(g, M, xv, t3);
  double a = g->c * g->theta * g->dt;
  double b = 4.0 * M_PI * g->theta * g->dt;
  for (long i = 0; i < 3 * N; ++i) out[i] = xv[i] + a * a * t2[i] + b * t3[i];
  free(t1);
  free(t2);
  free(t3);
}

/* S4 right-hand side: E^n + c th dt C_CN B^n - 4 pi th dt Jhat */
void oracle_rhs(const ocfg *g, const double *En, const double *Bn, const double *J, double *out) {
  long N = nnodes(g);
  double *t = (double *)malloc(sizeof(double) * 3 * N);
  oracle_curl_cn(g, Bn, t);
  double a = g->c * g->theta * g->dt;
  double b = 4.0 * M_PI * g->theta * g->dt;
  for (long i = 0; i < 3 * N; ++i) out[i] = En[i] + a * t[i] - b * J[i];
  free(t);
}

/* S5 */
void oracle_field_update(const ocfg *g, const double *En, const double *Bn, const double *Eth, double *Enp1,
                         double *Bnp1) {
  long N = nnodes(g);
  double *t = (double *)malloc(sizeof(double) * 3 * N);
  oracle_curl_nc(g, Eth, t);
  for (long i = 0; i < 3 * N; ++i) {
    Bnp1[i] = Bn[i] - g->c * g->dt * t[i];
    Enp1[i] = (Eth[i] - (1.0 - g->theta) * En[i]) / g->theta;
  }
  free(t);
}

/* S6 for all particles; x and u updated in place (x wrapped into [0, L)). */
void oracle_push(const ocfg *g, long n, double *x, double *u, const int32_t *sp, const double *Eth,
                 const double *Bn, const double *gb_in) {
  for (long p = 0; p < n; ++p) {
    double al[9], gb, be;
    particle_alpha(g, x, u, sp, n, p, Bn, gb_in, al, &gb, &be);
    double Ep[3];
    gather_nodes(g, x, n, p, Eth, Ep);
    double up[3] = {u[p], u[n + p], u[2 * n + p]};
    double v[3], ub[3], un[3];
    for (int k = 0; k < 3; ++k) v[k] = up[k] + be * Ep[k];
    for (int i = 0; i < 3; ++i) ub[i] = al[3 * i] * v[0] + al[3 * i + 1] * v[1] + al[3 * i + 2] * v[2];
    for (int k = 0; k < 3; ++k) un[k] = 2.0 * ub[k] - up[k];
    double gn = gamma_of(g, un);
    for (int d = 0; d < g->dim; ++d) {
      double L = extent(g, d) * spacing(g, d);
      double xn = x[d * n + p] + g->dt * un[d] / gn;
      xn = fmod(xn, L);
      if (xn < 0.0) xn += L;
      if (xn >= L) xn -= L;
      x[d * n + p] = xn;
    }
    for (int k = 0; k < 3; ++k) u[k * n + p] = un[k];
  }
}

/* Compensated running sum (Neumaier's variant of Kahan summation): the sum
 * of n terms is then correct to a few ulps plus the terms' own rounding,
 * whatever n, where a plain running sum loses up to about n ulps. */
typedef struct {
  double s, c;
} csum;

static void csum_add(csum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}

static double csum_value(const csum *a) { return a->s + a->c; }

/* S7: out = {kinetic, electric, magnetic, total}.  The kinetic energy per
 * particle is w m c^2 (gamma - 1) = w m |u|^2 / (gamma + 1) (no cancellation
 * at small |u|), or w m |u|^2 / 2 without relativity; each of the three sums
 * is compensated. */
void oracle_energy(const ocfg *g, long n, const double *u, const double *w, const int32_t *sp, const double *E,
                   const double *B, double out[4]) {
  long N = nnodes(g);
  csum ke = {0.0, 0.0}, we = {0.0, 0.0}, wb = {0.0, 0.0};
  for (long p = 0; p < n; ++p) {
    double up[3] = {u[p], u[n + p], u[2 * n + p]};
    double uu = up[0] * up[0] + up[1] * up[1] + up[2] * up[2];
    double m = g->m[sp[p]];
    if (g->nonrel)
      csum_add(&ke, 0.5 * w[p] * m * uu);
    else
      csum_add(&ke, w[p] * m * uu / (sqrt(1.0 + uu / (g->c * g->c)) + 1.0));
  }
  for (long i = 0; i < 3 * N; ++i) {
    csum_add(&we, E[i] * E[i]);
    csum_add(&wb, B[i] * B[i]);
  }
  double V = cellvol(g);
  out[0] = csum_value(&ke);
  out[1] = V / (8.0 * M_PI) * csum_value(&we);
  out[2] = V / (8.0 * M_PI) * csum_value(&wb);
  out[3] = out[0] + out[1] + out[2];
}
