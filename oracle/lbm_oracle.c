/*
 * Plain FP64 CPU oracle for the D2Q9 lattice Boltzmann part of LBM-GNN
 * (Li, "LBM-GNN: Graph Neural Network Enhanced Lattice Boltzmann Method",
 * arXiv 2504.14494).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the HIP kernels are checked against.  It shares no code,
 * header, table or constant with the GPU library; only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.
 *
 * Notation follows the paper: f_i are the populations, e_i the discrete
 * velocities, w_i the weights, c_s the lattice sound speed, tau the BGK
 * relaxation time.  The paper gives only the symbols; the D2Q9 set below is
 * the textbook one (Krueger et al., cited in the paper's resolution study).
 *
 * Layout of every population array: f[i][y][x], i = 0..8, x fastest.
 * All routines are unoptimised on purpose and single-threaded by default;
 * orc_set_threads lets the BGK collision and streaming loops share their
 * independent nodes among several threads, which changes no result (each
 * node's arithmetic is the same), for the long reference runs only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static int g_threads = 1;

/* Threads the BGK collision and streaming loops may use (default 1). */
void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }

/* D2Q9: rest, 4 axis directions, 4 diagonals. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                            1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2 */

static int wrap(int a, int n) { return ((a % n) + n) % n; }

void orc_lattice(int *ex, int *ey, double *w) {
  for (int i = 0; i < 9; ++i) {
    ex[i] = EX[i];
    ey[i] = EY[i];
    w[i] = W[i];
  }
}

/* Eq. 2 (Methodology, Lattice Boltzmann Method): second-order equilibrium
 * f_i^eq = rho w_i [1 + e.u/c_s^2 + (e.u)^2/(2 c_s^4) - u.u/(2 c_s^2)]. */
void orc_equilibrium(double rho, double ux, double uy, double *feq) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    feq[i] = rho * W[i] *
             (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* Initial state on the slow manifold (textbook Chapman-Enskog expansion,
 * Krueger et al., which the paper cites; not part of the paper's method):
 * f_i = f_i^eq(rho, u) - (tau w_i rho / c_s^2) Q_i : S with
 * Q_i = e_i e_i - c_s^2 I and S the symmetric velocity gradient, taken by
 * second-order central differences on the periodic lattice.  Starting from
 * f^eq alone instead excites the non-hydrodynamic period-2 mode, which is
 * damped only by |1 - 1/tau| per step. */
void orc_init_ce(double *f, int nx, int ny, const double *rho, const double *ux,
                 const double *uy, double tau) {
  size_t plane = (size_t)nx * ny;
  double feq[9];
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t n = (size_t)y * nx + x;
      size_t xp = (size_t)y * nx + (x + 1) % nx, xm = (size_t)y * nx + (x + nx - 1) % nx;
      size_t yp = (size_t)((y + 1) % ny) * nx + x, ym = (size_t)((y + ny - 1) % ny) * nx + x;
      double dux_dx = 0.5 * (ux[xp] - ux[xm]), dux_dy = 0.5 * (ux[yp] - ux[ym]);
      double duy_dx = 0.5 * (uy[xp] - uy[xm]), duy_dy = 0.5 * (uy[yp] - uy[ym]);
      double sxx = dux_dx, syy = duy_dy, sxy = 0.5 * (dux_dy + duy_dx);
      orc_equilibrium(rho[n], ux[n], uy[n], feq);
      for (int i = 0; i < 9; ++i) {
        double qs = (EX[i] * EX[i] - CS2) * sxx + 2.0 * EX[i] * EY[i] * sxy +
                    (EY[i] * EY[i] - CS2) * syy;
        f[i * plane + n] = feq[i] - tau * W[i] * rho[n] / CS2 * qs;
      }
    }
}

/* Macroscopic moments: rho = sum_i f_i, rho u = sum_i e_i f_i. */
static void node_moments(const double *f, size_t plane, size_t n, double *rho,
                         double *ux, double *uy) {
  double r = 0, jx = 0, jy = 0;
  for (int i = 0; i < 9; ++i) {
    double v = f[i * plane + n];
    r += v;
    jx += EX[i] * v;
    jy += EY[i] * v;
  }
  *rho = r;
  *ux = jx / r;
  *uy = jy / r;
}

void orc_moments(const double *f, int nx, int ny, double *rho, double *ux,
                 double *uy) {
  size_t plane = (size_t)nx * ny;
  for (size_t n = 0; n < plane; ++n)
    node_moments(f, plane, n, &rho[n], &ux[n], &uy[n]);
}

/* Initial state: f = f^eq(rho, u) at every node. */
void orc_init_equilibrium(double *f, int nx, int ny, const double *rho,
                          const double *ux, const double *uy) {
  size_t plane = (size_t)nx * ny;
  double feq[9];
  for (size_t n = 0; n < plane; ++n) {
    orc_equilibrium(rho[n], ux[n], uy[n], feq);
    for (int i = 0; i < 9; ++i) f[i * plane + n] = feq[i];
  }
}

/* BGK collision, the right-hand side of Eq. 1:
 * f_i^* = f_i - (f_i - f_i^eq) / tau. */
void orc_collide_bgk(const double *f, double *out, int nx, int ny,
                     double tau) {
  size_t plane = (size_t)nx * ny;
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
  for (size_t n = 0; n < plane; ++n) {
    double rho, ux, uy, feq[9];
    node_moments(f, plane, n, &rho, &ux, &uy);
    orc_equilibrium(rho, ux, uy, feq);
    for (int i = 0; i < 9; ++i) {
      double v = f[i * plane + n];
      out[i * plane + n] = v - (v - feq[i]) / tau;
    }
  }
}

/* Streaming, the left-hand side of Eq. 1 with periodic wrap:
 * out_i(x + e_i) = in_i(x). */
void orc_stream(const double *in, double *out, int nx, int ny) {
  size_t plane = (size_t)nx * ny;
  for (int i = 0; i < 9; ++i)
#pragma omp parallel for num_threads(g_threads) if (g_threads > 1) schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int xd = wrap(x + EX[i], nx), yd = wrap(y + EY[i], ny);
        out[i * plane + (size_t)yd * nx + xd] =
            in[i * plane + (size_t)y * nx + x];
      }
}

/* Inverse of orc_stream: out_i(x) = in_i(x + e_i). */
void orc_unstream(const double *in, double *out, int nx, int ny) {
  size_t plane = (size_t)nx * ny;
  for (int i = 0; i < 9; ++i)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int xs = wrap(x + EX[i], nx), ys = wrap(y + EY[i], ny);
        out[i * plane + (size_t)y * nx + x] =
            in[i * plane + (size_t)ys * nx + xs];
      }
}

/* One full step of Eq. 1: collide, then stream.  `f` holds the
 * pre-collision populations at t; `out` receives those at t + 1. */
void orc_bgk_step(const double *f, double *out, int nx, int ny, double tau) {
  size_t n = (size_t)9 * nx * ny;
  double *tmp = (double *)malloc(n * sizeof(double));
  orc_collide_bgk(f, tmp, nx, ny, tau);
  orc_stream(tmp, out, nx, ny);
  free(tmp);
}

/* `steps` applications of Eq. 1, in place. */
void orc_bgk_run(double *f, int nx, int ny, double tau, int steps) {
  size_t n = (size_t)9 * nx * ny;
  double *tmp = (double *)malloc(n * sizeof(double));
  for (int s = 0; s < steps; ++s) {
    orc_collide_bgk(f, tmp, nx, ny, tau);
    orc_stream(tmp, f, nx, ny);
  }
  free(tmp);
}

/* Observables of one lattice, all in FP64.
 * tgv = {u0, kx, ky, x0, y0, nu, t} describes the decaying Taylor-Green
 * field u_x = -u0 cos(kx X) sin(ky Y), u_y = u0 (kx/ky) sin(kx X) cos(ky Y),
 * X = x - x0, Y = y - y0, scaled by exp(-nu (kx^2 + ky^2) t); pass NULL to
 * skip the error sums.
 * sums[0..7] = total mass, x- and y-momentum, kinetic energy 1/2 sum |u|^2,
 * sum |u - u_a|^2, sum |u_a|^2, smallest population, number of negative
 * populations. */
void orc_observables(const double *f, int nx, int ny, const double *tgv,
                     double *sums) {
  size_t plane = (size_t)nx * ny;
  double mass = 0, mx = 0, my = 0, ke = 0, en = 0, ed = 0, fmin = INFINITY,
         nneg = 0;
  double decay = 1.0;
  if (tgv)
    decay = exp(-tgv[5] * (tgv[1] * tgv[1] + tgv[2] * tgv[2]) * tgv[6]);
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t n = (size_t)y * nx + x;
      double rho, ux, uy;
      node_moments(f, plane, n, &rho, &ux, &uy);
      mass += rho;
      mx += rho * ux;
      my += rho * uy;
      ke += 0.5 * (ux * ux + uy * uy);
      for (int i = 0; i < 9; ++i) {
        double v = f[i * plane + n];
        if (v < fmin) fmin = v;
        if (v < 0) nneg += 1;
      }
      if (tgv) {
        double X = x - tgv[3], Y = y - tgv[4];
        double uax = -tgv[0] * cos(tgv[1] * X) * sin(tgv[2] * Y) * decay;
        double uay = tgv[0] * (tgv[1] / tgv[2]) * sin(tgv[1] * X) *
                     cos(tgv[2] * Y) * decay;
        en += (ux - uax) * (ux - uax) + (uy - uay) * (uy - uay);
        ed += uax * uax + uay * uay;
      }
    }
  sums[0] = mass;
  sums[1] = mx;
  sums[2] = my;
  sums[3] = ke;
  sums[4] = en;
  sums[5] = ed;
  sums[6] = fmin;
  sums[7] = nneg;
}

/* Fine-to-coarse restriction of a pre-collision state (training data).
 * Coarse node X sits on fine node factor*X.  From that fine node take
 * rho, u and the non-equilibrium momentum flux
 * Pi^neq = sum_i e_i e_i (f_i - f_i^eq); rebuild the coarse populations as
 * f_i = f_i^eq(rho, u) + w_i / (2 c_s^4) Q_i : Pi^neq * lambda with
 * Q_i = e_i e_i - c_s^2 I and lambda = factor * tau_c / tau_f, the first-order
 * Chapman-Enskog ratio of f^neq between lattices that share Re and Mach.
 * If `unstream` is set the result is also taken back through one coarse
 * streaming step: out_i(X) = R(f)_i(X + e_i). */
void orc_restrict(const double *ff, int nxf, int nyf, int factor,
                  double tau_f, double tau_c, int unstream, double *fc) {
  int nxc = nxf / factor, nyc = nyf / factor;
  size_t pf = (size_t)nxf * nyf, pc = (size_t)nxc * nyc;
  double lambda = factor * tau_c / tau_f;
  double *tmp = (double *)malloc(9 * pc * sizeof(double));
  double feq[9];
  for (int Y = 0; Y < nyc; ++Y)
    for (int X = 0; X < nxc; ++X) {
      size_t nf = (size_t)(factor * Y) * nxf + (size_t)factor * X;
      double rho, ux, uy;
      node_moments(ff, pf, nf, &rho, &ux, &uy);
      orc_equilibrium(rho, ux, uy, feq);
      double pxx = 0, pxy = 0, pyy = 0;
      for (int i = 0; i < 9; ++i) {
        double d = ff[i * pf + nf] - feq[i];
        pxx += EX[i] * EX[i] * d;
        pxy += EX[i] * EY[i] * d;
        pyy += EY[i] * EY[i] * d;
      }
      for (int i = 0; i < 9; ++i) {
        double qxx = EX[i] * EX[i] - CS2, qyy = EY[i] * EY[i] - CS2,
               qxy = EX[i] * EY[i];
        double qp = qxx * pxx + 2.0 * qxy * pxy + qyy * pyy;
        tmp[i * pc + (size_t)Y * nxc + X] =
            feq[i] + W[i] / (2.0 * CS2 * CS2) * qp * lambda;
      }
    }
  if (unstream)
    orc_unstream(tmp, fc, nxc, nyc);
  else
    memcpy(fc, tmp, 9 * pc * sizeof(double));
  free(tmp);
}

/* ------------------------------------------------------------------------
 * Channel flow between two resting walls (validation section, "Poiseuille
 * Flow", Eq. 5).  The paper names no wall or forcing scheme; this oracle
 * takes the textbook ones:
 *  - halfway bounce-back: the walls sit half a lattice spacing outside the
 *    first and last rows, y = -1/2 and y = ny - 1/2 (channel height H = ny);
 *    a population that would stream through a wall comes back to the node it
 *    left, reversed;
 *  - a uniform body force F = rho g along x (the driving pressure gradient G
 *    of Eq. 5 per unit mass), added with Guo's forcing: the velocity is
 *    u = (sum_i e_i f_i + F/2) / rho, f^eq is taken at that u, and the
 *    collision adds (1 - 1/(2 tau)) S_i with
 *    S_i = w_i [ (e_i - u) / c_s^2 + (e_i . u) e_i / c_s^4 ] . F.
 * The flow is periodic in x.
 * ------------------------------------------------------------------------ */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

void orc_collide_forced(const double *f, double *out, int nx, int ny,
                        double tau, double gx) {
  size_t plane = (size_t)nx * ny;
  double feq[9];
  for (size_t n = 0; n < plane; ++n) {
    double rho = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; ++i) {
      double v = f[i * plane + n];
      rho += v;
      jx += EX[i] * v;
      jy += EY[i] * v;
    }
    double fx = rho * gx, fy = 0.0;
    double ux = (jx + 0.5 * fx) / rho, uy = (jy + 0.5 * fy) / rho;
    orc_equilibrium(rho, ux, uy, feq);
    for (int i = 0; i < 9; ++i) {
      double eu = EX[i] * ux + EY[i] * uy;
      double s = W[i] * (((EX[i] - ux) * fx + (EY[i] - uy) * fy) / CS2 +
                         eu * (EX[i] * fx + EY[i] * fy) / (CS2 * CS2));
      double v = f[i * plane + n];
      out[i * plane + n] = v - (v - feq[i]) / tau + (1.0 - 0.5 / tau) * s;
    }
  }
}

/* Streaming with halfway bounce-back at the two walls, periodic in x. */
void orc_stream_channel(const double *in, double *out, int nx, int ny) {
  size_t plane = (size_t)nx * ny;
  for (int i = 0; i < 9; ++i)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        double v = in[i * plane + (size_t)y * nx + x];
        int yd = y + EY[i];
        if (yd < 0 || yd >= ny)
          out[OPP[i] * plane + (size_t)y * nx + x] = v;
        else
          out[i * plane + (size_t)yd * nx + wrap(x + EX[i], nx)] = v;
      }
}

/* `steps` channel steps (forced collision, then streaming), in place. */
void orc_channel_run(double *f, int nx, int ny, double tau, double gx,
                     int steps) {
  size_t n = (size_t)9 * nx * ny;
  double *tmp = (double *)malloc(n * sizeof(double));
  for (int s = 0; s < steps; ++s) {
    orc_collide_forced(f, tmp, nx, ny, tau, gx);
    orc_stream_channel(tmp, f, nx, ny);
  }
  free(tmp);
}
