/*
 * Plain CPU oracle for the GNN-corrected collision of LBM-GNN
 * (arXiv 2504.14494, Methodology: "Graph Neural Network Enhancement",
 * "Integration of GNN with LBM" with Eq. 3, "GNN Architecture Details",
 * "Training Methodology" with Eq. 4).
 *
 * TEST INFRASTRUCTURE ONLY: it shares no code with the HIP library and only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * The network (sizes fixed by the workload definition, not by the paper,
 * which gives none):
 *   features  x = ((f_i - w_i)_{i=0..8}, rho - 1, u_x, u_y), normalised as
 *             (x - mu) / sigma                       (12 numbers per node)
 *   encoder   e1 = GELU(W1 x + b1)      12 -> 64
 *             h0 = GELU(W2 e1 + b2)     64 -> 64
 *   rounds    r = 1..R, separate weights per round; for the 8 lattice
 *             neighbours j = n + e_d (periodic), edge feature e_d:
 *               m_d = GELU(We [h_n ; h_j ; e_d] + be)   130 -> 64
 *               a   = sum_d m_d
 *               h_n' = GELU(Wn [h_n ; a] + bn)          128 -> 64
 *   head      z = Wh h_R + bh          64 -> 10
 *             tau_adj = 0.5 + sigmoid(z_0)    (sigmoid scaled to [0.5, 1.5])
 *             delta f = s_delta * P z_{1..9}, P the orthogonal projector onto
 *             the null space of the mass and momentum moments
 *   collide   f*_i = f_i - (f_i - f_i^eq) / (tau * tau_adj) + delta f_i (Eq. 3)
 * GELU is the tanh form 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).
 *
 * Parameter blob (row-major, W[out][in]):
 *   W1[64][12] b1[64] W2[64][64] b2[64]
 *   { We[64][130] be[64] Wn[64][128] bn[64] } x R
 *   Wh[10][64] bh[10]  | mu[12] sigma[12] s_delta   (constants, not trained)
 *
 * mode 0 computes everything in FP64.  mode 1 emulates the BF16 storage of
 * the GPU path: weights, normalised features, every stored activation (after
 * GELU) and the summed message are rounded to BF16 (round to nearest even);
 * all arithmetic is still FP64.  Rounding is treated as the identity by the
 * backward pass (straight-through).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define HID 64
#define NFEAT 12
#define NOUT 10
#define EDGE_IN (2 * HID + 2)
#define NODE_IN (2 * HID)
#define MAXR 8

static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                            1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Round to the nearest value with 8 significant bits (BF16), ties to even. */
double orc_bf16_round(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  double m = frexp(x, &e); /* |m| in [0.5, 1) */
  return ldexp(nearbyint(ldexp(m, 8)), e - 8);
}

static double rnd(double x, int mode) { return mode ? orc_bf16_round(x) : x; }

static double gelu(double x) {
  const double c = sqrt(2.0 / M_PI);
  return 0.5 * x * (1.0 + tanh(c * (x + 0.044715 * x * x * x)));
}

static double gelu_grad(double x) {
  const double c = sqrt(2.0 / M_PI);
  double t = tanh(c * (x + 0.044715 * x * x * x));
  return 0.5 * (1.0 + t) +
         0.5 * x * (1.0 - t * t) * c * (1.0 + 3.0 * 0.044715 * x * x);
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

double orc_gelu(double x) { return gelu(x); }
double orc_gelu_grad(double x) { return gelu_grad(x); }

typedef struct {
  const double *W1, *b1, *W2, *b2;
  const double *We[MAXR], *be[MAXR], *Wn[MAXR], *bn[MAXR];
  const double *Wh, *bh, *mu, *sigma;
  double sdelta;
  int R;
  int act; /* 0: GELU (tanh form), 1: ReLU (the per-node network of Fig. 2) */
  /* Body force per unit mass along x (0: no force).  With a force the node
   * velocity is u = (sum_i e_i f_i + F/2) / rho (Guo), the features and f^eq
   * use it, and the collision adds (1 - 1/(2 tau tau_adj)) S_i with
   * S_i = w_i [(e_i - u)/c_s^2 + (e_i . u) e_i / c_s^4] . F, F = rho (gx, 0):
   * Guo's source at the network's effective relaxation time (the paper names
   * no forcing scheme for its network; this is the reading taken). */
  double gx;
} net_t;

static double act_fn(const net_t *n, double x) {
  return n->act ? (x > 0.0 ? x : 0.0) : gelu(x);
}

static double act_grad_fn(const net_t *n, double x) {
  return n->act ? (x > 0.0 ? 1.0 : 0.0) : gelu_grad(x);
}

/* Offsets of every tensor in the blob; the same walk sizes the gradient. */
typedef struct {
  size_t W1, b1, W2, b2, We[MAXR], be[MAXR], Wn[MAXR], bn[MAXR], Wh, bh, mu,
      sigma, sdelta, nparam, total;
} layout_t;

static layout_t layout(int R) {
  layout_t L;
  size_t o = 0;
  L.W1 = o; o += (size_t)HID * NFEAT;
  L.b1 = o; o += HID;
  L.W2 = o; o += (size_t)HID * HID;
  L.b2 = o; o += HID;
  for (int r = 0; r < R; ++r) {
    L.We[r] = o; o += (size_t)HID * EDGE_IN;
    L.be[r] = o; o += HID;
    L.Wn[r] = o; o += (size_t)HID * NODE_IN;
    L.bn[r] = o; o += HID;
  }
  L.Wh = o; o += (size_t)NOUT * HID;
  L.bh = o; o += NOUT;
  L.nparam = o;
  L.mu = o; o += NFEAT;
  L.sigma = o; o += NFEAT;
  L.sdelta = o; o += 1;
  L.total = o;
  return L;
}

size_t orc_gnn_param_count(int R) { return layout(R).nparam; }
size_t orc_gnn_blob_len(int R) { return layout(R).total; }

/* Bind the blob; in BF16 mode the weight matrices are rounded into `store`
 * (biases and constants keep full precision). */
static void bind(const double *blob, int R, int mode, double *store,
                 net_t *n) {
  layout_t L = layout(R);
  memcpy(store, blob, L.total * sizeof(double));
  if (mode) {
    size_t mats[3 + 2 * MAXR][2];
    int k = 0;
    mats[k][0] = L.W1; mats[k++][1] = (size_t)HID * NFEAT;
    mats[k][0] = L.W2; mats[k++][1] = (size_t)HID * HID;
    for (int r = 0; r < R; ++r) {
      mats[k][0] = L.We[r]; mats[k++][1] = (size_t)HID * EDGE_IN;
      mats[k][0] = L.Wn[r]; mats[k++][1] = (size_t)HID * NODE_IN;
    }
    mats[k][0] = L.Wh; mats[k++][1] = (size_t)NOUT * HID;
    for (int m = 0; m < k; ++m)
      for (size_t q = 0; q < mats[m][1]; ++q)
        store[mats[m][0] + q] = orc_bf16_round(store[mats[m][0] + q]);
  }
  n->R = R;
  n->W1 = store + L.W1; n->b1 = store + L.b1;
  n->W2 = store + L.W2; n->b2 = store + L.b2;
  for (int r = 0; r < R; ++r) {
    n->We[r] = store + L.We[r]; n->be[r] = store + L.be[r];
    n->Wn[r] = store + L.Wn[r]; n->bn[r] = store + L.bn[r];
  }
  n->Wh = store + L.Wh; n->bh = store + L.bh;
  n->mu = store + L.mu; n->sigma = store + L.sigma;
  n->sdelta = store[L.sdelta];
  n->act = 0;
  n->gx = 0.0;
}

/* out = Wm in + b, Wm row-major [nout][nin]. */
static void dense(const double *Wm, const double *b, const double *in,
                  int nin, int nout, double *out) {
  for (int o = 0; o < nout; ++o) {
    double s = b[o];
    for (int k = 0; k < nin; ++k) s += Wm[(size_t)o * nin + k] * in[k];
    out[o] = s;
  }
}

/* y += Wm^T d */
static void dense_t(const double *Wm, const double *d, int nin, int nout,
                    double *y) {
  for (int o = 0; o < nout; ++o)
    for (int k = 0; k < nin; ++k) y[k] += Wm[(size_t)o * nin + k] * d[o];
}

/* gW += d (x) in, gb += d */
static void outer_acc(double *gW, double *gb, const double *d,
                      const double *in, int nin, int nout) {
  for (int o = 0; o < nout; ++o) {
    gb[o] += d[o];
    for (int k = 0; k < nin; ++k) gW[(size_t)o * nin + k] += d[o] * in[k];
  }
}

static void moments9(const double *f9, double *rho, double *ux, double *uy) {
  double r = 0, jx = 0, jy = 0;
  for (int i = 0; i < 9; ++i) {
    r += f9[i];
    jx += EX[i] * f9[i];
    jy += EY[i] * f9[i];
  }
  *rho = r;
  *ux = jx / r;
  *uy = jy / r;
}

static void equilibrium9(double rho, double ux, double uy, double *feq) {
  const double cs2 = 1.0 / 3.0;
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    feq[i] = rho * W[i] *
             (1.0 + eu / cs2 + eu * eu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

static void features(const double *f9, const net_t *net, int mode,
                     double *x) {
  double rho, ux, uy, feat[NFEAT];
  moments9(f9, &rho, &ux, &uy);
  ux += 0.5 * net->gx;
  for (int i = 0; i < 9; ++i) feat[i] = f9[i] - W[i];
  feat[9] = rho - 1.0;
  feat[10] = ux;
  feat[11] = uy;
  for (int k = 0; k < NFEAT; ++k)
    x[k] = rnd((feat[k] - net->mu[k]) / net->sigma[k], mode);
}

static void encode(const double *x, const net_t *net, int mode, double *e1,
                   double *h0) {
  double p[HID];
  dense(net->W1, net->b1, x, NFEAT, HID, p);
  for (int c = 0; c < HID; ++c) e1[c] = rnd(act_fn(net, p[c]), mode);
  dense(net->W2, net->b2, e1, HID, HID, p);
  for (int c = 0; c < HID; ++c) h0[c] = rnd(act_fn(net, p[c]), mode);
}

/* One message-passing round for a receiver with state hn and neighbour
 * states hj[d] (d = 1..8, hj[0] unused).  Returns the summed message in
 * agg and the new state in hout. */
static void mp_node(const double *hn, const double *const hj[9],
                    const net_t *net, int r, int mode, double *agg,
                    double *hout) {
  double in[EDGE_IN], q[HID], cat[NODE_IN], p[HID];
  for (int c = 0; c < HID; ++c) agg[c] = 0.0;
  for (int d = 1; d < 9; ++d) {
    memcpy(in, hn, HID * sizeof(double));
    memcpy(in + HID, hj[d], HID * sizeof(double));
    in[2 * HID] = EX[d];
    in[2 * HID + 1] = EY[d];
    dense(net->We[r], net->be[r], in, EDGE_IN, HID, q);
    for (int c = 0; c < HID; ++c) agg[c] += act_fn(net, q[c]);
  }
  for (int c = 0; c < HID; ++c) agg[c] = rnd(agg[c], mode);
  memcpy(cat, hn, HID * sizeof(double));
  memcpy(cat + HID, agg, HID * sizeof(double));
  dense(net->Wn[r], net->bn[r], cat, NODE_IN, HID, p);
  for (int c = 0; c < HID; ++c) hout[c] = rnd(act_fn(net, p[c]), mode);
}

/* Orthogonal projector onto null(M), M = [1; e_x; e_y] (3 x 9):
 * P v = v - M^T (M M^T)^{-1} M v.  (M M^T)^{-1} is formed by cofactors. */
static void project(const double *v, double *out) {
  double M[3][9], G[3][3], Gi[3][3], mv[3], c[3];
  for (int i = 0; i < 9; ++i) {
    M[0][i] = 1.0;
    M[1][i] = EX[i];
    M[2][i] = EY[i];
  }
  for (int a = 0; a < 3; ++a) {
    mv[a] = 0;
    for (int i = 0; i < 9; ++i) mv[a] += M[a][i] * v[i];
    for (int b = 0; b < 3; ++b) {
      G[a][b] = 0;
      for (int i = 0; i < 9; ++i) G[a][b] += M[a][i] * M[b][i];
    }
  }
  double det = G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) -
               G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
               G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
  Gi[0][0] = (G[1][1] * G[2][2] - G[1][2] * G[2][1]) / det;
  Gi[0][1] = (G[0][2] * G[2][1] - G[0][1] * G[2][2]) / det;
  Gi[0][2] = (G[0][1] * G[1][2] - G[0][2] * G[1][1]) / det;
  Gi[1][0] = (G[1][2] * G[2][0] - G[1][0] * G[2][2]) / det;
  Gi[1][1] = (G[0][0] * G[2][2] - G[0][2] * G[2][0]) / det;
  Gi[1][2] = (G[0][2] * G[1][0] - G[0][0] * G[1][2]) / det;
  Gi[2][0] = (G[1][0] * G[2][1] - G[1][1] * G[2][0]) / det;
  Gi[2][1] = (G[0][1] * G[2][0] - G[0][0] * G[2][1]) / det;
  Gi[2][2] = (G[0][0] * G[1][1] - G[0][1] * G[1][0]) / det;
  for (int a = 0; a < 3; ++a) {
    c[a] = 0;
    for (int b = 0; b < 3; ++b) c[a] += Gi[a][b] * mv[b];
  }
  for (int i = 0; i < 9; ++i)
    out[i] = v[i] - (M[0][i] * c[0] + M[1][i] * c[1] + M[2][i] * c[2]);
}

void orc_project(const double *v, double *out) { project(v, out); }

/* Head and Eq. 3 at one node. */
static void head_collide(const double *f9, const double *h, double tau,
                         const net_t *net, double *z, double *fstar) {
  double rho, ux, uy, feq[9], dft[9], df[9];
  dense(net->Wh, net->bh, h, HID, NOUT, z);
  double tau_adj = 0.5 + sigmoid(z[0]);
  for (int i = 0; i < 9; ++i) dft[i] = z[1 + i];
  project(dft, df);
  moments9(f9, &rho, &ux, &uy);
  ux += 0.5 * net->gx;
  equilibrium9(rho, ux, uy, feq);
  const double cs2 = 1.0 / 3.0, fx = rho * net->gx;
  for (int i = 0; i < 9; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    double src = W[i] * ((EX[i] - ux) * fx / cs2 + eu * EX[i] * fx / (cs2 * cs2));
    fstar[i] = f9[i] - (f9[i] - feq[i]) / (tau * tau_adj) +
               net->sdelta * df[i] + (1.0 - 0.5 / (tau * tau_adj)) * src;
  }
}

static void gather9(const double *f, size_t plane, size_t n, double *f9) {
  for (int i = 0; i < 9; ++i) f9[i] = f[i * plane + n];
}

/* Activations of a whole batch, kept for the backward pass. */
typedef struct {
  int B, nx, ny, R;
  size_t N;
  double *x, *e1, *h, *agg, *z;
} acts_t;

static void acts_free(acts_t *a) {
  free(a->x);
  free(a->e1);
  free(a->h);
  free(a->agg);
  free(a->z);
}

/* Full-lattice forward over `batch` independent periodic lattices.
 * f, fstar: [batch][9][ny][nx] pre- and post-collision populations. */
static int forward(const double *f, int batch, int nx, int ny,
                   const double *tau, const net_t *net, int mode,
                   double *fstar, double *zout, acts_t *a) {
  int R = net->R;
  size_t plane = (size_t)nx * ny, N = (size_t)batch * plane;
  a->B = batch; a->nx = nx; a->ny = ny; a->R = R; a->N = N;
  a->x = (double *)malloc(N * NFEAT * sizeof(double));
  a->e1 = (double *)malloc(N * HID * sizeof(double));
  a->h = (double *)malloc((size_t)(R + 1) * N * HID * sizeof(double));
  a->agg = (double *)malloc((size_t)(R > 0 ? R : 1) * N * HID * sizeof(double));
  a->z = (double *)malloc(N * NOUT * sizeof(double));
  if (!a->x || !a->e1 || !a->h || !a->agg || !a->z) {
    acts_free(a);
    return -1;
  }
  double f9[9];
  for (int b = 0; b < batch; ++b)
    for (size_t n = 0; n < plane; ++n) {
      size_t g = (size_t)b * plane + n;
      gather9(f + (size_t)b * 9 * plane, plane, n, f9);
      features(f9, net, mode, a->x + g * NFEAT);
      encode(a->x + g * NFEAT, net, mode, a->e1 + g * HID, a->h + g * HID);
    }
  for (int r = 0; r < R; ++r) {
    const double *hin = a->h + (size_t)r * N * HID;
    double *hout = a->h + (size_t)(r + 1) * N * HID;
    for (int b = 0; b < batch; ++b)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          size_t g = (size_t)b * plane + (size_t)y * nx + x;
          const double *hj[9];
          hj[0] = NULL;
          for (int d = 1; d < 9; ++d)
            hj[d] = hin + ((size_t)b * plane +
                           (size_t)wrap(y + EY[d], ny) * nx +
                           wrap(x + EX[d], nx)) * HID;
          mp_node(hin + g * HID, hj, net, r, mode,
                  a->agg + ((size_t)r * N + g) * HID, hout + g * HID);
        }
  }
  const double *hR = a->h + (size_t)R * N * HID;
  for (int b = 0; b < batch; ++b)
    for (size_t n = 0; n < plane; ++n) {
      size_t g = (size_t)b * plane + n;
      double fs[9];
      gather9(f + (size_t)b * 9 * plane, plane, n, f9);
      head_collide(f9, hR + g * HID, tau[b], net, a->z + g * NOUT, fs);
      for (int i = 0; i < 9; ++i)
        fstar[(size_t)b * 9 * plane + i * plane + n] = fs[i];
      if (zout)
        for (int k = 0; k < NOUT; ++k) zout[g * NOUT + k] = a->z[g * NOUT + k];
    }
  return 0;
}

int orc_gnn_collide_act(const double *f, double *fstar, int batch, int nx,
                        int ny, const double *tau, const double *blob, int R,
                        int mode, int act, double *zout) {
  if (R < 0 || R > MAXR) return -1;
  double *store = (double *)malloc(layout(R).total * sizeof(double));
  net_t net;
  bind(blob, R, mode, store, &net);
  net.act = act;
  acts_t a;
  int rc = forward(f, batch, nx, ny, tau, &net, mode, fstar, zout, &a);
  if (rc == 0) acts_free(&a);
  free(store);
  return rc;
}

/* The corrected collision under a body force rho * gx along x (see net_t). */
int orc_gnn_collide_forced(const double *f, double *fstar, int batch, int nx,
                           int ny, const double *tau, const double *blob, int R,
                           int mode, int act, double gx, double *zout) {
  if (R < 0 || R > MAXR) return -1;
  double *store = (double *)malloc(layout(R).total * sizeof(double));
  net_t net;
  bind(blob, R, mode, store, &net);
  net.act = act;
  net.gx = gx;
  acts_t a;
  int rc = forward(f, batch, nx, ny, tau, &net, mode, fstar, zout, &a);
  if (rc == 0) acts_free(&a);
  free(store);
  return rc;
}

int orc_gnn_collide(const double *f, double *fstar, int batch, int nx, int ny,
                    const double *tau, const double *blob, int R, int mode,
                    double *zout) {
  if (R < 0 || R > MAXR) return -1;
  double *store = (double *)malloc(layout(R).total * sizeof(double));
  net_t net;
  bind(blob, R, mode, store, &net);
  acts_t a;
  int rc = forward(f, batch, nx, ny, tau, &net, mode, fstar, zout, &a);
  if (rc == 0) acts_free(&a);
  free(store);
  return rc;
}

/* Forward at selected nodes of one lattice, each from its own
 * (2R+1) x (2R+1) neighbourhood.  nodes[k] = y * nx + x.
 * fstar: [count][9], z: [count][10] (NULLable). */
int orc_gnn_collide_nodes(const double *f, int nx, int ny, double tau,
                          const double *blob, int R, int mode,
                          const long *nodes, int count, double *fstar,
                          double *zout) {
  if (R < 0 || R > MAXR) return -1;
  double *store = (double *)malloc(layout(R).total * sizeof(double));
  net_t net;
  bind(blob, R, mode, store, &net);
  int P = 2 * R + 1;
  size_t plane = (size_t)nx * ny;
  double *hA = (double *)malloc((size_t)P * P * HID * sizeof(double));
  double *hB = (double *)malloc((size_t)P * P * HID * sizeof(double));
  double agg[HID], f9[9], x[NFEAT], e1[HID], z[NOUT], fs[9];
  for (int k = 0; k < count; ++k) {
    int x0 = (int)(nodes[k] % nx), y0 = (int)(nodes[k] / nx);
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        size_t n = (size_t)wrap(y0 + dy, ny) * nx + wrap(x0 + dx, nx);
        gather9(f, plane, n, f9);
        features(f9, &net, mode, x);
        encode(x, &net, mode, e1, hA + ((size_t)(dy + R) * P + dx + R) * HID);
      }
    for (int r = 0; r < R; ++r) {
      int rad = R - r - 1;
      for (int dy = -rad; dy <= rad; ++dy)
        for (int dx = -rad; dx <= rad; ++dx) {
          const double *hj[9];
          hj[0] = NULL;
          for (int d = 1; d < 9; ++d)
            hj[d] = hA + ((size_t)(dy + EY[d] + R) * P + dx + EX[d] + R) * HID;
          mp_node(hA + ((size_t)(dy + R) * P + dx + R) * HID, hj, &net, r,
                  mode, agg, hB + ((size_t)(dy + R) * P + dx + R) * HID);
        }
      double *t = hA; hA = hB; hB = t;
    }
    gather9(f, plane, (size_t)y0 * nx + x0, f9);
    head_collide(f9, hA + ((size_t)R * P + R) * HID, tau, &net, z, fs);
    for (int i = 0; i < 9; ++i) fstar[(size_t)k * 9 + i] = fs[i];
    if (zout)
      for (int q = 0; q < NOUT; ++q) zout[(size_t)k * NOUT + q] = z[q];
  }
  free(hA);
  free(hB);
  free(store);
  return 0;
}

/* Gradient of a scalar loss with respect to the trainable parameters, given
 * its gradient G = dL/df* ([batch][9][ny][nx]) at the forward's output.
 * grad: [orc_gnn_param_count(R)], overwritten. */
static int backward_impl(const double *f, const double *G, int batch, int nx,
                         int ny, const double *tau, const double *blob, int R,
                         int mode, int act, double *grad);

int orc_gnn_backward(const double *f, const double *G, int batch, int nx,
                     int ny, const double *tau, const double *blob, int R,
                     int mode, double *grad) {
  return backward_impl(f, G, batch, nx, ny, tau, blob, R, mode, 0, grad);
}

int orc_gnn_backward_act(const double *f, const double *G, int batch, int nx,
                         int ny, const double *tau, const double *blob, int R,
                         int mode, int act, double *grad) {
  return backward_impl(f, G, batch, nx, ny, tau, blob, R, mode, act, grad);
}

static int backward_impl(const double *f, const double *G, int batch, int nx,
                         int ny, const double *tau, const double *blob, int R,
                         int mode, int act, double *grad) {
  if (R < 0 || R > MAXR) return -1;
  layout_t L = layout(R);
  double *store = (double *)malloc(L.total * sizeof(double));
  net_t net;
  bind(blob, R, mode, store, &net);
  net.act = act;
  size_t plane = (size_t)nx * ny, N = (size_t)batch * plane;
  double *fstar = (double *)malloc(N * 9 * sizeof(double));
  acts_t a;
  if (forward(f, batch, nx, ny, tau, &net, mode, fstar, NULL, &a) != 0) {
    free(fstar);
    free(store);
    return -1;
  }
  memset(grad, 0, L.nparam * sizeof(double));
  double *dh = (double *)calloc(N * HID, sizeof(double));
  double *dhp = (double *)calloc(N * HID, sizeof(double));
  const double *hR = a.h + (size_t)R * N * HID;

  /* Eq. 3, the projection and the head. */
  for (int b = 0; b < batch; ++b)
    for (size_t n = 0; n < plane; ++n) {
      size_t g = (size_t)b * plane + n;
      double f9[9], G9[9], Gp[9], rho, ux, uy, feq[9], dz[NOUT];
      gather9(f + (size_t)b * 9 * plane, plane, n, f9);
      gather9(G + (size_t)b * 9 * plane, plane, n, G9);
      moments9(f9, &rho, &ux, &uy);
      equilibrium9(rho, ux, uy, feq);
      const double *z = a.z + g * NOUT;
      double s = sigmoid(z[0]), tau_adj = 0.5 + s;
      double dtadj = 0.0;
      for (int i = 0; i < 9; ++i)
        dtadj += G9[i] * (f9[i] - feq[i]) / (tau[b] * tau_adj * tau_adj);
      dz[0] = dtadj * s * (1.0 - s);
      project(G9, Gp); /* P is symmetric */
      for (int i = 0; i < 9; ++i) dz[1 + i] = net.sdelta * Gp[i];
      outer_acc(grad + L.Wh, grad + L.bh, dz, hR + g * HID, HID, NOUT);
      dense_t(net.Wh, dz, HID, NOUT, dh + g * HID);
    }

  /* Rounds in reverse. dh holds dL/dh_{r+1}; dhp collects dL/dh_r. */
  for (int r = R - 1; r >= 0; --r) {
    const double *hin = a.h + (size_t)r * N * HID;
    const double *agg = a.agg + (size_t)r * N * HID;
    memset(dhp, 0, N * HID * sizeof(double));
    for (int b = 0; b < batch; ++b)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          size_t g = (size_t)b * plane + (size_t)y * nx + x;
          double cat[NODE_IN], p[HID], dp[HID], dcat[NODE_IN], in[EDGE_IN],
              q[HID], dq[HID], din[EDGE_IN];
          memcpy(cat, hin + g * HID, HID * sizeof(double));
          memcpy(cat + HID, agg + g * HID, HID * sizeof(double));
          dense(net.Wn[r], net.bn[r], cat, NODE_IN, HID, p);
          for (int c = 0; c < HID; ++c)
            dp[c] = dh[g * HID + c] * act_grad_fn(&net, p[c]);
          outer_acc(grad + L.Wn[r], grad + L.bn[r], dp, cat, NODE_IN, HID);
          memset(dcat, 0, sizeof(dcat));
          dense_t(net.Wn[r], dp, NODE_IN, HID, dcat);
          for (int c = 0; c < HID; ++c) dhp[g * HID + c] += dcat[c];
          for (int d = 1; d < 9; ++d) {
            size_t gj = (size_t)b * plane + (size_t)wrap(y + EY[d], ny) * nx +
                        wrap(x + EX[d], nx);
            memcpy(in, hin + g * HID, HID * sizeof(double));
            memcpy(in + HID, hin + gj * HID, HID * sizeof(double));
            in[2 * HID] = EX[d];
            in[2 * HID + 1] = EY[d];
            dense(net.We[r], net.be[r], in, EDGE_IN, HID, q);
            for (int c = 0; c < HID; ++c)
              dq[c] = dcat[HID + c] * act_grad_fn(&net, q[c]);
            outer_acc(grad + L.We[r], grad + L.be[r], dq, in, EDGE_IN, HID);
            memset(din, 0, sizeof(din));
            dense_t(net.We[r], dq, EDGE_IN, HID, din);
            for (int c = 0; c < HID; ++c) {
              dhp[g * HID + c] += din[c];
              dhp[gj * HID + c] += din[HID + c];
            }
          }
        }
    double *t = dh; dh = dhp; dhp = t;
  }

  /* Encoder. */
  for (size_t g = 0; g < N; ++g) {
    double p[HID], dp[HID], de1[HID];
    const double *x = a.x + g * NFEAT, *e1 = a.e1 + g * HID;
    dense(net.W2, net.b2, e1, HID, HID, p);
    for (int c = 0; c < HID; ++c) dp[c] = dh[g * HID + c] * act_grad_fn(&net, p[c]);
    outer_acc(grad + L.W2, grad + L.b2, dp, e1, HID, HID);
    memset(de1, 0, sizeof(de1));
    dense_t(net.W2, dp, HID, HID, de1);
    dense(net.W1, net.b1, x, NFEAT, HID, p);
    for (int c = 0; c < HID; ++c) dp[c] = de1[c] * act_grad_fn(&net, p[c]);
    outer_acc(grad + L.W1, grad + L.b1, dp, x, NFEAT, HID);
  }
  free(dh);
  free(dhp);
  free(fstar);
  acts_free(&a);
  free(store);
  return 0;
}

/* GNN collision with the per-step fallback rule, on one lattice.
 * The GNN result is rejected if any post-collision population is negative
 * or not finite (flag bit 1), or if the relative change of total mass
 * against mass_prev is not <= thr (flag bit 2); then the plain BGK collision
 * of the same input is returned instead.  mass_out gets the total mass of
 * what was returned. */
int orc_gnn_collide_gated(const double *f, double *out, int nx, int ny,
                          double tau, const double *blob, int R, int mode,
                          double thr, double mass_prev, unsigned *flags,
                          double *mass_out) {
  size_t plane = (size_t)nx * ny;
  int rc = orc_gnn_collide(f, out, 1, nx, ny, &tau, blob, R, mode, NULL);
  if (rc) return rc;
  unsigned fl = 0;
  double mass = 0.0;
  for (size_t k = 0; k < 9 * plane; ++k) {
    if (!(out[k] >= 0.0) || !isfinite(out[k])) fl |= 1u;
    mass += out[k];
  }
  double rel = fabs(mass - mass_prev) / mass_prev;
  if (!(rel <= thr)) fl |= 2u;
  if (fl) {
    double feq[9];
    for (size_t n = 0; n < plane; ++n) {
      double f9[9], rho, ux, uy;
      gather9(f, plane, n, f9);
      moments9(f9, &rho, &ux, &uy);
      equilibrium9(rho, ux, uy, feq);
      for (int i = 0; i < 9; ++i)
        out[i * plane + n] = f9[i] - (f9[i] - feq[i]) / tau;
    }
    mass = 0.0;
    for (size_t k = 0; k < 9 * plane; ++k) mass += out[k];
  }
  *flags = fl;
  *mass_out = mass;
  return 0;
}

/* Eq. 4 with N the number of nodes: (1/N) sum_nodes sum_i (a_i - b_i)^2.
 * a, b: [nodes][9] in any consistent order. */
double orc_mse(const double *a, const double *b, size_t nodes) {
  double s = 0.0;
  for (size_t k = 0; k < 9 * nodes; ++k) s += (a[k] - b[k]) * (a[k] - b[k]);
  return s / (double)nodes;
}

/* Eq. 4 with each node's residual r = a - b weighted by a 9 x 9 matrix Q:
 * (1/N) sum_nodes r^T Q r.  Q = identity gives orc_mse.  a, b: [nodes][9]. */
double orc_mse_weighted(const double *a, const double *b, size_t nodes, const double *q) {
  double s = 0.0;
  for (size_t n = 0; n < nodes; ++n) {
    double r[9];
    for (int i = 0; i < 9; ++i) r[i] = a[9 * n + i] - b[9 * n + i];
    for (int i = 0; i < 9; ++i)
      for (int j = 0; j < 9; ++j) s += r[i] * q[9 * i + j] * r[j];
  }
  return s / (double)nodes;
}

/* One Adam step (Kingma and Ba, Algorithm 1) with bias correction;
 * step is the 1-based step count after this update. */
void orc_adam(double *p, const double *g, double *m, double *v, size_t n,
              double lr, double beta1, double beta2, double eps, int step) {
  double c1 = 1.0 - pow(beta1, step), c2 = 1.0 - pow(beta2, step);
  for (size_t k = 0; k < n; ++k) {
    m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
    v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
    double mh = m[k] / c1, vh = v[k] / c2;
    p[k] -= lr * mh / (sqrt(vh) + eps);
  }
}
