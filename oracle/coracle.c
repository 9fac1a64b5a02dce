/*
 * Plain FP64 C oracle of the two-fluid active-nematic coupled step
 * (arXiv 2511.00445, Model and Numerical Simulation sections).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and
 * bench.py's cpu_baseline, never by the product path.  It shares no code with
 * the HIP library.  It runs the same algorithm and readings as the numpy oracle
 * (oracle/tfan_oracle.py), written independently as loops over sites with
 * explicit 2x2 tensor algebra, and parallelised over rows with OpenMP.
 *
 * Layout: planes [ny][nx], x fastest; populations f[9][ny][nx] per fluid,
 * stored pre-collision (after streaming).  D2Q9 order: rest, +x, +y, -x, -y,
 * +x+y, -x+y, -x-y, +x-y.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int nx, ny, n_sub;
  double rho0, tau_a, tau_p, gamma, A_ch, kappa, M, A0, gamma_ldg, K, lam, Gamma, zeta;
} oc_params;

typedef struct {
  oc_params p;
  int n;
  double *fa, *fp, *ta, *tp;  /* populations and scratch (post-collision) */
  double *phi, *qxx, *qxy;
  double *mu, *sig;           /* mu [n], stress [4][n]: xx, xy, yx, yy */
  double *ua, *up, *uc;       /* velocities [2][n] */
  double *w;                  /* velocity gradient of u_a [4][n]: W_xx, W_xy, W_yx, W_yy */
  double *phi2, *qxx2, *qxy2; /* sub-step output */
  double *mu2;
  double *pm;                 /* phi * mu at the step's start */
} oc_sim;

static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WI[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static int md(int i, int n) { return ((i % n) + n) % n; }

/* ---- 2x2 tensors: t[0]=xx t[1]=xy t[2]=yx t[3]=yy ---- */
static void mat_mul(const double* a, const double* b, double* c) {
  c[0] = a[0] * b[0] + a[1] * b[2];
  c[1] = a[0] * b[1] + a[1] * b[3];
  c[2] = a[2] * b[0] + a[3] * b[2];
  c[3] = a[2] * b[1] + a[3] * b[3];
}
static double contract(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

/* Q tensor at flat index i */
static void qtensor(const oc_sim* s, const double* qxx, const double* qxy, int i, double* q) {
  q[0] = qxx[i];
  q[1] = qxy[i];
  q[2] = qxy[i];
  q[3] = -qxx[i];
}

static double lap(const double* g, int x, int y, int nx, int ny) {
  return g[y * nx + md(x + 1, nx)] + g[y * nx + md(x - 1, nx)] + g[md(y + 1, ny) * nx + x] +
         g[md(y - 1, ny) * nx + x] - 4.0 * g[y * nx + x];
}
static double ddx(const double* g, int x, int y, int nx) {
  return 0.5 * (g[y * nx + md(x + 1, nx)] - g[y * nx + md(x - 1, nx)]);
}
static double ddy(const double* g, int x, int y, int nx, int ny) {
  return 0.5 * (g[md(y + 1, ny) * nx + x] - g[md(y - 1, ny) * nx + x]);
}

/* molecular field H = -dF/dQ + (I/2) Tr(dF/dQ), F = (A/2)TrQ^2 + (C/4)TrQ^4 + (K/2)|grad Q|^2
 * (Model, Eqs. 7-8).  A and C come from the (A0, gamma) form of the Landau-de Gennes
 * energy, (A0/2)(1 - gamma/3) TrQ^2 - (A0 gamma/3) TrQ^3 + (A0 gamma/4)(TrQ^2)^2:
 * A = A0 (1 - gamma/3) and, as TrQ^4 = (TrQ^2)^2 / 2 for a 2x2 traceless Q,
 * C = 2 A0 gamma.  The cubic term only adds a multiple of I to dF/dQ, which the
 * traceless part removes, so it is left out. */
static void molecular(const oc_sim* s, const double* qxx, const double* qxy, int x, int y, double* h) {
  const int nx = s->p.nx, ny = s->p.ny, i = y * nx + x;
  const double A = s->p.A0 * (1.0 - s->p.gamma_ldg / 3.0), C = 2.0 * s->p.A0 * s->p.gamma_ldg;
  double q[4], q2[4], q3[4], lq[4], dF[4];
  qtensor(s, qxx, qxy, i, q);
  mat_mul(q, q, q2);
  mat_mul(q2, q, q3);
  lq[0] = lap(qxx, x, y, nx, ny);
  lq[1] = lap(qxy, x, y, nx, ny);
  lq[2] = lq[1];
  lq[3] = -lq[0];
  for (int k = 0; k < 4; ++k) dF[k] = A * q[k] + C * q3[k] - s->p.K * lq[k];
  const double tr = dF[0] + dF[3];
  for (int k = 0; k < 4; ++k) h[k] = -dF[k];
  h[0] += 0.5 * tr;
  h[3] += 0.5 * tr;
}

static void feq(double rho, double ux, double uy, double* out) {
  const double uu = ux * ux + uy * uy;
  for (int k = 0; k < 9; ++k) {
    const double cu = CX[k] * ux + CY[k] * uy;
    out[k] = WI[k] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

oc_sim* oc_create(const oc_params* p) {
  oc_sim* s = (oc_sim*)calloc(1, sizeof(oc_sim));
  s->p = *p;
  s->n = p->nx * p->ny;
  const size_t n = (size_t)s->n;
  s->fa = calloc(9 * n, sizeof(double));
  s->fp = calloc(9 * n, sizeof(double));
  s->ta = calloc(9 * n, sizeof(double));
  s->tp = calloc(9 * n, sizeof(double));
  s->phi = calloc(n, sizeof(double));
  s->qxx = calloc(n, sizeof(double));
  s->qxy = calloc(n, sizeof(double));
  s->mu = calloc(n, sizeof(double));
  s->mu2 = calloc(n, sizeof(double));
  s->sig = calloc(4 * n, sizeof(double));
  s->ua = calloc(2 * n, sizeof(double));
  s->up = calloc(2 * n, sizeof(double));
  s->uc = calloc(2 * n, sizeof(double));
  s->w = calloc(4 * n, sizeof(double));
  s->phi2 = calloc(n, sizeof(double));
  s->qxx2 = calloc(n, sizeof(double));
  s->qxy2 = calloc(n, sizeof(double));
  s->pm = calloc(n, sizeof(double));
  return s;
}

void oc_destroy(oc_sim* s) {
  if (!s) return;
  double* arr[] = {s->fa, s->fp, s->ta, s->tp, s->phi, s->qxx, s->qxy, s->mu, s->mu2, s->sig,
                   s->ua, s->up, s->uc, s->w, s->phi2, s->qxx2, s->qxy2, s->pm};
  for (size_t k = 0; k < sizeof(arr) / sizeof(arr[0]); ++k) free(arr[k]);
  free(s);
}

void oc_init(oc_sim* s, const double* phi, const double* qxx, const double* qxy, const double* ua,
             const double* up) {
  const int n = s->n;
  memcpy(s->phi, phi, n * sizeof(double));
  memcpy(s->qxx, qxx, n * sizeof(double));
  memcpy(s->qxy, qxy, n * sizeof(double));
  for (int i = 0; i < n; ++i) {
    double e[9];
    feq(s->p.rho0, ua ? ua[i] : 0.0, ua ? ua[n + i] : 0.0, e);
    for (int k = 0; k < 9; ++k) s->fa[k * n + i] = e[k];
    feq(s->p.rho0, up ? up[i] : 0.0, up ? up[n + i] : 0.0, e);
    for (int k = 0; k < 9; ++k) s->fp[k * n + i] = e[k];
  }
}

/* chemical potential and full nematic stress (elastic + active) on every site */
static void potentials(oc_sim* s, const double* phi, double* mu) {
  const int nx = s->p.nx, ny = s->p.ny, n = s->n;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int i = y * nx + x;
      mu[i] = s->p.A_ch * (phi[i] * phi[i] * phi[i] - phi[i]) - s->p.kappa * lap(phi, x, y, nx, ny);
      if (mu == s->mu) s->pm[i] = phi[i] * mu[i];
    }
  (void)n;
}

static void stresses(oc_sim* s) {
  const int nx = s->p.nx, ny = s->p.ny, n = s->n;
  const double lam = s->p.lam, K = s->p.K;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int i = y * nx + x;
      double q[4], h[4], P[4], hp[4], ph[4], qh[4], hq[4], sg[4];
      qtensor(s, s->qxx, s->qxy, i, q);
      molecular(s, s->qxx, s->qxy, x, y, h);
      for (int k = 0; k < 4; ++k) P[k] = q[k];
      P[0] += 0.5;
      P[3] += 0.5;
      mat_mul(h, P, hp);
      mat_mul(P, h, ph);
      mat_mul(q, h, qh);
      mat_mul(h, q, hq);
      const double QH = contract(q, h);
      /* d_i Q_kl for i = x, y (full tensor components) */
      double dq[2][4];
      dq[0][0] = ddx(s->qxx, x, y, nx);
      dq[0][1] = ddx(s->qxy, x, y, nx);
      dq[1][0] = ddy(s->qxx, x, y, nx, ny);
      dq[1][1] = ddy(s->qxy, x, y, nx, ny);
      for (int a = 0; a < 2; ++a) {
        dq[a][2] = dq[a][1];
        dq[a][3] = -dq[a][0];
      }
      const double c1 = 0.5 * (1.0 + s->phi[i]);
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          const int k = 2 * a + b;
          const double erick = K * contract(dq[a], dq[b]);
          sg[k] = -lam * hp[k] - lam * ph[k] + 2.0 * lam * P[k] * QH - erick + qh[k] - hq[k] -
                  s->p.zeta * c1 * q[k];
        }
      for (int k = 0; k < 4; ++k) s->sig[k * n + i] = sg[k];
    }
}

/* forces, moments, implicit-drag Guo velocities and collision of both fluids */
static void collide(oc_sim* s) {
  const int nx = s->p.nx, ny = s->p.ny, n = s->n;
  const double oma = 1.0 / s->p.tau_a, omp = 1.0 / s->p.tau_p;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int i = y * nx + x;
      const double* sx = s->sig;
      /* F_a = d_j sigma_aj */
      const double Fx = ddx(sx + 0 * n, x, y, nx) + ddy(sx + 1 * n, x, y, nx, ny);
      const double Fy = ddx(sx + 2 * n, x, y, nx) + ddy(sx + 3 * n, x, y, nx, ny);
      const double ph = s->phi[i];
      const double c1 = 0.5 * (1.0 + ph), c2 = 0.5 * (1.0 - ph);
      /* capillary force mu grad(phi) - grad(phi mu), each term by central differences */
      const double chx = s->mu[i] * ddx(s->phi, x, y, nx) - ddx(s->pm, x, y, nx);
      const double chy = s->mu[i] * ddy(s->phi, x, y, nx, ny) - ddy(s->pm, x, y, nx, ny);
      const double Gax = Fx + c1 * chx, Gay = Fy + c1 * chy, Gpx = c2 * chx, Gpy = c2 * chy;
      double ra = 0, rp = 0, max_ = 0, may = 0, mpx = 0, mpy = 0;
      for (int k = 0; k < 9; ++k) {
        const double a = s->fa[k * n + i], b = s->fp[k * n + i];
        ra += a;
        rp += b;
        max_ += a * CX[k];
        may += a * CY[k];
        mpx += b * CX[k];
        mpy += b * CY[k];
      }
      /* rho_a u_a = m_a + (G_a + beta (u_p - u_a))/2, rho_p u_p = m_p + (G_p - beta (u_p - u_a))/2 */
      const double beta = s->p.gamma * c1 * c2, g = 0.5 * beta;
      const double a11 = ra + g, a12 = -g, a21 = -g, a22 = rp + g;
      const double det = a11 * a22 - a12 * a21;
      double u[2][2]; /* [fluid][component] */
      const double ba[2] = {max_ + 0.5 * Gax, may + 0.5 * Gay}, bp[2] = {mpx + 0.5 * Gpx, mpy + 0.5 * Gpy};
      for (int c = 0; c < 2; ++c) {
        u[0][c] = (ba[c] * a22 - a12 * bp[c]) / det;
        u[1][c] = (a11 * bp[c] - a21 * ba[c]) / det;
      }
      const double Fd[2] = {beta * (u[1][0] - u[0][0]), beta * (u[1][1] - u[0][1])};
      const double Fa[2] = {Gax + Fd[0], Gay + Fd[1]}, Fp[2] = {Gpx - Fd[0], Gpy - Fd[1]};
      s->ua[i] = u[0][0];
      s->ua[n + i] = u[0][1];
      s->up[i] = u[1][0];
      s->up[n + i] = u[1][1];
      s->uc[i] = c1 * u[0][0] + c2 * u[1][0];
      s->uc[n + i] = c1 * u[0][1] + c2 * u[1][1];
      for (int fl = 0; fl < 2; ++fl) {
        const double* f = fl ? s->fp : s->fa;
        double* t = fl ? s->tp : s->ta;
        const double rho = fl ? rp : ra, om = fl ? omp : oma;
        const double ux = u[fl][0], uy = u[fl][1], fx = fl ? Fp[0] : Fa[0], fy = fl ? Fp[1] : Fa[1];
        double e[9];
        feq(rho, ux, uy, e);
        for (int k = 0; k < 9; ++k) {
          const double cu = CX[k] * ux + CY[k] * uy, cf = CX[k] * fx + CY[k] * fy;
          const double src = (1.0 - 0.5 * om) * WI[k] *
                             (3.0 * (cf - (ux * fx + uy * fy)) + 9.0 * cu * cf);
          t[k * n + i] = f[k * n + i] - om * (f[k * n + i] - e[k]) + src;
        }
      }
    }
}

static void stream(oc_sim* s) {
  const int nx = s->p.nx, ny = s->p.ny, n = s->n;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x)
      for (int k = 0; k < 9; ++k) {
        const int src = md(y - CY[k], ny) * nx + md(x - CX[k], nx);
        s->fa[k * n + y * nx + x] = s->ta[k * n + src];
        s->fp[k * n + y * nx + x] = s->tp[k * n + src];
      }
}

/* one sub-step from (phi, qxx, qxy) into (phi2, qxx2, qxy2) with frozen velocities */
static void substep(oc_sim* s) {
  const int nx = s->p.nx, ny = s->p.ny, n = s->n;
  const double h = 1.0 / s->p.n_sub, lam = s->p.lam;
  potentials(s, s->phi, s->mu2);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int i = y * nx + x;
      const int e = y * nx + md(x + 1, nx), w = y * nx + md(x - 1, nx);
      const int no = md(y + 1, ny) * nx + x, so = md(y - 1, ny) * nx + x;
      /* Cahn-Hilliard */
      const double div = 0.5 * (s->phi[e] * s->uc[e] - s->phi[w] * s->uc[w]) +
                         0.5 * (s->phi[no] * s->uc[n + no] - s->phi[so] * s->uc[n + so]);
      s->phi2[i] = s->phi[i] + h * (s->p.M * lap(s->mu2, x, y, nx, ny) - div);
      /* Beris-Edwards with the full tensors */
      double q[4], H[4], W[4], E[4], O[4], P[4], A1[4], A2[4], t1[4], t2[4], R[4];
      qtensor(s, s->qxx, s->qxy, i, q);
      molecular(s, s->qxx, s->qxy, x, y, H);
      for (int k = 0; k < 4; ++k) W[k] = s->w[k * n + i];
      E[0] = W[0];
      E[3] = W[3];
      E[1] = E[2] = 0.5 * (W[1] + W[2]);
      O[0] = O[3] = 0.0;
      O[1] = 0.5 * (W[1] - W[2]);
      O[2] = -O[1];
      for (int k = 0; k < 4; ++k) {
        P[k] = q[k];
        A1[k] = lam * E[k] + O[k];
        A2[k] = lam * E[k] - O[k];
      }
      P[0] += 0.5;
      P[3] += 0.5;
      mat_mul(A1, P, t1);
      mat_mul(P, A2, t2);
      const double QW = contract(q, W);
      const double ux = s->ua[i], uy = s->ua[n + i];
      const double dqx[2] = {ddx(s->qxx, x, y, nx), ddx(s->qxy, x, y, nx)};
      const double dqy[2] = {ddy(s->qxx, x, y, nx, ny), ddy(s->qxy, x, y, nx, ny)};
      double adv[4];
      adv[0] = -(ux * dqx[0] + uy * dqy[0]);
      adv[1] = -(ux * dqx[1] + uy * dqy[1]);
      adv[2] = adv[1];
      adv[3] = -adv[0];
      for (int k = 0; k < 4; ++k) R[k] = adv[k] + t1[k] + t2[k] - 2.0 * lam * P[k] * QW + s->p.Gamma * H[k];
      s->qxx2[i] = s->qxx[i] + h * 0.5 * (R[0] - R[3]);
      s->qxy2[i] = s->qxy[i] + h * 0.5 * (R[1] + R[2]);
    }
  double* t;
  t = s->phi; s->phi = s->phi2; s->phi2 = t;
  t = s->qxx; s->qxx = s->qxx2; s->qxx2 = t;
  t = s->qxy; s->qxy = s->qxy2; s->qxy2 = t;
}

void oc_step(oc_sim* s, int nsteps) {
  const int nx = s->p.nx, ny = s->p.ny, n = s->n;
  for (int it = 0; it < nsteps; ++it) {
    potentials(s, s->phi, s->mu);
    stresses(s);
    collide(s);
    stream(s);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int i = y * nx + x;
        s->w[0 * n + i] = ddx(s->ua, x, y, nx);          /* W_xx = d_x u_x */
        s->w[1 * n + i] = ddy(s->ua, x, y, nx, ny);      /* W_xy = d_y u_x */
        s->w[2 * n + i] = ddx(s->ua + n, x, y, nx);      /* W_yx = d_x u_y */
        s->w[3 * n + i] = ddy(s->ua + n, x, y, nx, ny);  /* W_yy = d_y u_y */
      }
    for (int m = 0; m < s->p.n_sub; ++m) substep(s);
  }
}

/* fields at the current step; velocities from the step's own force evaluation */
void oc_fields(oc_sim* s, double* phi, double* qxx, double* qxy, double* ua, double* up, double* rho_a,
               double* rho_p) {
  const int n = s->n;
  potentials(s, s->phi, s->mu);
  stresses(s);
  /* collide() computes the velocities; its post-collision output is discarded */
  collide(s);
  memcpy(phi, s->phi, n * sizeof(double));
  memcpy(qxx, s->qxx, n * sizeof(double));
  memcpy(qxy, s->qxy, n * sizeof(double));
  memcpy(ua, s->ua, 2 * n * sizeof(double));
  memcpy(up, s->up, 2 * n * sizeof(double));
  for (int i = 0; i < n; ++i) {
    double a = 0, b = 0;
    for (int k = 0; k < 9; ++k) {
      a += s->fa[k * n + i];
      b += s->fp[k * n + i];
    }
    rho_a[i] = a;
    rho_p[i] = b;
  }
}

int oc_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Number of OpenMP threads of later steps (n >= 1); timing only, the results do
 * not depend on it (every row is computed by one thread, in the same order). */
void oc_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
