/*
 * FP64 CPU oracle of the Gaussian rasterizer and its per-view statistics.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU baseline
 * leg of the benchmark may load this library.  It shares no code, header or
 * constant with the HIP path; both sides read the same seeded inputs.
 *
 * What it computes, step by step, in the order the method states it:
 *   camera pose      T' = Exp(xi) T, Exp the 4x4 matrix exponential (series)
 *   projection       camera point, EWA 2D covariance with the low-pass term,
 *                    conic, pixel centre, opacity-aware extents, tile rect,
 *                    view-dependent colour from real spherical harmonics
 *   compositing      per pixel, front to back over the Gaussians whose tile
 *                    rect holds the pixel's tile, in (depth, index) order:
 *                    colour and depth by alpha compositing with transmittance
 *                    T_j = prod_{m<j} (1 - alpha_m)  (depth volume rendering,
 *                    Sec. "Depth Volume Rendering" of the appendix)
 *   backward         exact derivative of the above with every threshold
 *                    decision held fixed, by suffix sums per pixel and the
 *                    chain rule written out scalar by scalar; the pose
 *                    gradient is taken through d Exp(xi)/d xi by its series
 *   statistics       footprint Omega_v(i) = pixels where Gaussian i is blended
 *                    (appendix, Sec. "Details for Lifecycle-Managed Gaussian
 *                    Mapping"), error mask M_v(u) = [||I - I^||_1 > tau_err],
 *                    kappa_v(i) = sum of M over Omega_v(i)
 *
 * Constants that the paper does not state (alpha_min, alpha_max, T_min, near
 * and far planes, low-pass term, guard band, rect margin, background) come in through
 * orc_cfg; none is hard-coded here.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC kgs_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} orc_camera;

typedef struct {
  double alpha_min, alpha_max, t_min, near_z, eps2d, guard, rect_margin, far_z;
  double bg[3];
  int32_t tile_w, tile_h;
} orc_cfg;

/* ------------------------------------------------------------------ pose */
/* se(3) hat: xi = (rho, phi); 4x4 row major. */
static void se3_hat(const double xi[6], double A[16]) {
  memset(A, 0, 16 * sizeof(double));
  A[0 * 4 + 1] = -xi[5]; A[0 * 4 + 2] = xi[4];
  A[1 * 4 + 0] = xi[5];  A[1 * 4 + 2] = -xi[3];
  A[2 * 4 + 0] = -xi[4]; A[2 * 4 + 1] = xi[3];
  A[0 * 4 + 3] = xi[0];  A[1 * 4 + 3] = xi[1]; A[2 * 4 + 3] = xi[2];
}

static void m4_mul(const double* A, const double* B, double* C) {
  double T[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += A[i * 4 + k] * B[k * 4 + j];
      T[i * 4 + j] = s;
    }
  memcpy(C, T, sizeof T);
}

#define ORC_EXP_TERMS 48

/* Exp(xi) = sum_n hat(xi)^n / n!  (the definition of the matrix exponential). */
void orc_se3_exp(const double xi[6], double T[16]) {
  double A[16], P[16];
  se3_hat(xi, A);
  memset(T, 0, 16 * sizeof(double));
  memset(P, 0, 16 * sizeof(double));
  for (int i = 0; i < 4; ++i) P[i * 5] = 1.0, T[i * 5] = 1.0;
  for (int n = 1; n < ORC_EXP_TERMS; ++n) {
    m4_mul(P, A, P);
    for (int i = 0; i < 16; ++i) P[i] /= (double)n;
    for (int i = 0; i < 16; ++i) T[i] += P[i];
  }
}

/* d Exp(hat(xi)) / d xi_k = sum_{n>=1} 1/n! sum_{m=0}^{n-1} A^m E_k A^{n-1-m},
 * with A = hat(xi) and E_k = hat(e_k). */
void orc_se3_exp_deriv(const double xi[6], int k, double D[16]) {
  double A[16], E[16], e[6] = {0, 0, 0, 0, 0, 0};
  double Ap[ORC_EXP_TERMS][16];
  e[k] = 1.0;
  se3_hat(xi, A);
  se3_hat(e, E);
  memset(Ap[0], 0, sizeof Ap[0]);
  for (int i = 0; i < 4; ++i) Ap[0][i * 5] = 1.0;
  for (int n = 1; n < ORC_EXP_TERMS; ++n) m4_mul(Ap[n - 1], A, Ap[n]);
  memset(D, 0, 16 * sizeof(double));
  double fact = 1.0;
  for (int n = 1; n < ORC_EXP_TERMS; ++n) {
    fact *= (double)n;
    double S[16];
    memset(S, 0, sizeof S);
    for (int m = 0; m < n; ++m) {
      double X[16];
      m4_mul(Ap[m], E, X);
      m4_mul(X, Ap[n - 1 - m], X);
      for (int i = 0; i < 16; ++i) S[i] += X[i];
    }
    for (int i = 0; i < 16; ++i) D[i] += S[i] / fact;
  }
}

/* Perturbed world->camera pose T' = Exp(xi) T. */
static void camera_pose(const orc_camera* cam, const double xi[6], double Rp[9], double tp[3],
                        double ctr[3]) {
  double T[16], E[16];
  memset(T, 0, sizeof T);
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) T[i * 4 + j] = cam->R[i * 3 + j];
    T[i * 4 + 3] = cam->t[i];
  }
  T[15] = 1.0;
  orc_se3_exp(xi, E);
  m4_mul(E, T, T);
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) Rp[i * 3 + j] = T[i * 4 + j];
    tp[i] = T[i * 4 + 3];
  }
  for (int j = 0; j < 3; ++j) ctr[j] = -(Rp[0 * 3 + j] * tp[0] + Rp[1 * 3 + j] * tp[1] + Rp[2 * 3 + j] * tp[2]);
}

/* ---------------------------------------------------- real spherical harmonics
 * Y_l^m with the Condon-Shortley phase, written through Cartesian polynomials:
 *   P_l^m(z) = (-1)^m (1 - z^2)^{m/2} d^m P_l / dz^m,
 *   (1 - z^2)^{m/2} cos(m phi) = Re (x + i y)^m,  ... sin(m phi) = Im (x + i y)^m
 *   Y_l^m  = sqrt2 K_l^m (-1)^m Re(x+iy)^m P_l^{(m)}(z)     (m > 0)
 *   Y_l^-m = sqrt2 K_l^m (-1)^m Im(x+iy)^m P_l^{(m)}(z)     (m > 0)
 *   Y_l^0  = K_l^0 P_l(z),  K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
 * coefficient index k = l^2 + l + m.  The gradient is that of the polynomial
 * extension; the caller projects it onto the sphere. */
static double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

static double binom(int n, int k) { return factorial(n) / (factorial(k) * factorial(n - k)); }

/* coefficients of P_l (power basis), c[j] multiplies z^j */
static void legendre_coeffs(int l, double c[8]) {
  for (int j = 0; j < 8; ++j) c[j] = 0.0;
  for (int k = 0; 2 * k <= l; ++k)
    c[l - 2 * k] = pow(-1.0, k) * binom(l, k) * binom(2 * l - 2 * k, l) / pow(2.0, l);
}

/* value of the m-th derivative of a polynomial with coefficients c */
static double poly_deriv(const double c[8], int deg, int m, double z) {
  double s = 0.0;
  for (int j = m; j <= deg; ++j) {
    double f = 1.0;
    for (int r = 0; r < m; ++r) f *= (double)(j - r);
    s += c[j] * f * pow(z, j - m);
  }
  return s;
}

/* complex power (x + i y)^m */
static void cpow_xy(double x, double y, int m, double* re, double* im) {
  double a = 1.0, b = 0.0;
  for (int r = 0; r < m; ++r) {
    double na = a * x - b * y, nb = a * y + b * x;
    a = na; b = nb;
  }
  *re = a; *im = b;
}

void orc_sh_eval(int degree, const double d[3], double* Y, double* dY /* [K][3] or NULL */) {
  const double x = d[0], y = d[1], z = d[2];
  for (int l = 0; l <= degree; ++l) {
    double c[8];
    legendre_coeffs(l, c);
    for (int m = 0; m <= l; ++m) {
      double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
      double Pm = poly_deriv(c, l, m, z), Pm1 = poly_deriv(c, l, m + 1, z);
      if (m == 0) {
        int k = l * l + l;
        Y[k] = K * Pm;
        if (dY) { dY[k * 3 + 0] = 0.0; dY[k * 3 + 1] = 0.0; dY[k * 3 + 2] = K * Pm1; }
        continue;
      }
      double re, im, re1, im1;
      cpow_xy(x, y, m, &re, &im);
      cpow_xy(x, y, m - 1, &re1, &im1);
      double s = sqrt(2.0) * K * ((m & 1) ? -1.0 : 1.0);
      int kp = l * l + l + m, kn = l * l + l - m;
      Y[kp] = s * re * Pm;
      Y[kn] = s * im * Pm;
      if (dY) {
        dY[kp * 3 + 0] = s * m * re1 * Pm;
        dY[kp * 3 + 1] = -s * m * im1 * Pm;
        dY[kp * 3 + 2] = s * re * Pm1;
        dY[kn * 3 + 0] = s * m * im1 * Pm;
        dY[kn * 3 + 1] = s * m * re1 * Pm;
        dY[kn * 3 + 2] = s * im * Pm1;
      }
    }
  }
}

/* ----------------------------------------------------------- projection */
typedef struct {
  int visible;
  double t[3];          /* camera-frame point */
  double o;             /* sigmoid(logit) */
  double qn[4];         /* unit quaternion (w, x, y, z) */
  double qnorm;
  double Rq[9], s[3];
  double covw[9], covc[9];
  double J[6];
  int clampx, clampy;   /* guard band active (0 none, -1 low, +1 high) */
  double limx, limy;    /* the bound used when clamped */
  double S2[3];         /* Sigma2D xx, xy, yy (with the low-pass term) */
  double det, conic[3];
  double mu[2];
  double depth;
  int64_t fxi, fyi, rx, ry;
  int32_t x0, x1, y0, y1;
  double dir[3], dist;
  double col[3];
  int colmask[3];
  double Y[16];
  /* diagnostics only (not used by the method): distance of the far test, of the
   * pixel centre from an integer (pixels), and of the extent before its ceil
   * from an integer (relative) -- the places where a re-evaluation in another
   * precision may take the other side of an integer decision */
  double m_far, m_cen, m_ext;
} orc_proj;

static void quat_to_rot(const double q[4], double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static int64_t floordiv64(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

#define ORC_BIG 16777216.0 /* 2^24: centre and extent limit of the rect contract */

typedef struct {
  int64_t n;
  int deg, K;
  int W, H, TW, TH, TX, TY;
  orc_cfg cfg;
  double xi[6];
  double Rp[9], tp[3], ctr[3];
  double fx, fy, cx, cy;
  const double *means, *log_scales, *quats, *logits, *sh;
  orc_proj* P;
  int64_t n_vis;
  int64_t* order;     /* visible Gaussians sorted by (fp32 depth, index) */
  int64_t* tile_off;  /* CSR over tiles */
  int64_t* tile_list;
  double *color, *depthimg, *tfinal, *margins; /* margins [4][H][W] */
  int32_t* last;
  int32_t* nblend;
} orc_view;

static void project_one(const orc_view* v, int64_t i, orc_proj* p) {
  const int64_t n = v->n;
  memset(p, 0, sizeof *p);
  p->m_cen = p->m_ext = INFINITY;
  double mu[3] = {v->means[i], v->means[n + i], v->means[2 * n + i]};
  for (int r = 0; r < 3; ++r)
    p->t[r] = v->Rp[r * 3 + 0] * mu[0] + v->Rp[r * 3 + 1] * mu[1] + v->Rp[r * 3 + 2] * mu[2] + v->tp[r];
  const double tx = p->t[0], ty = p->t[1], tz = p->t[2];
  p->m_far = fabs(tz - v->cfg.far_z) / v->cfg.far_z;
  /* near plane, and the single-level distance mask (culled at and beyond far_z) */
  if (!(tz > v->cfg.near_z) || !(tz < v->cfg.far_z)) return;
  p->o = 1.0 / (1.0 + exp(-(double)v->logits[i]));
  if (p->o < v->cfg.alpha_min) return;
  double q[4] = {v->quats[i], v->quats[n + i], v->quats[2 * n + i], v->quats[3 * n + i]};
  p->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(p->qnorm > 0.0)) return;
  for (int r = 0; r < 4; ++r) p->qn[r] = q[r] / p->qnorm;
  quat_to_rot(p->qn, p->Rq);
  for (int r = 0; r < 3; ++r) p->s[r] = exp((double)v->log_scales[r * n + i]);
  /* Sigma_w = Rq diag(s^2) Rq^T */
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += p->Rq[a * 3 + k] * p->s[k] * p->s[k] * p->Rq[b * 3 + k];
      p->covw[a * 3 + b] = acc;
    }
  /* Sigma_c = R' Sigma_w R'^T */
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += v->Rp[a * 3 + k] * p->covw[k * 3 + l] * v->Rp[b * 3 + l];
      p->covc[a * 3 + b] = acc;
    }
  /* Jacobian of the pinhole map with the guard-band clamp of x/z and y/z */
  const double hx = 0.5 * v->W / v->fx, hy = 0.5 * v->H / v->fy;
  const double mx = (0.5 * v->W - v->cx) / v->fx, my = (0.5 * v->H - v->cy) / v->fy;
  const double lox = mx - v->cfg.guard * hx, hix = mx + v->cfg.guard * hx;
  const double loy = my - v->cfg.guard * hy, hiy = my + v->cfg.guard * hy;
  double ux = tx / tz, uy = ty / tz;
  if (ux < lox) { ux = lox; p->clampx = -1; p->limx = lox; }
  else if (ux > hix) { ux = hix; p->clampx = 1; p->limx = hix; }
  if (uy < loy) { uy = loy; p->clampy = -1; p->limy = loy; }
  else if (uy > hiy) { uy = hiy; p->clampy = 1; p->limy = hiy; }
  p->J[0] = v->fx / tz; p->J[1] = 0.0; p->J[2] = -v->fx * ux / tz;
  p->J[3] = 0.0; p->J[4] = v->fy / tz; p->J[5] = -v->fy * uy / tz;
  double JS[6];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += p->J[a * 3 + k] * p->covc[k * 3 + b];
      JS[a * 3 + b] = acc;
    }
  double S00 = 0, S01 = 0, S11 = 0;
  for (int k = 0; k < 3; ++k) {
    S00 += JS[0 * 3 + k] * p->J[0 * 3 + k];
    S01 += JS[0 * 3 + k] * p->J[1 * 3 + k];
    S11 += JS[1 * 3 + k] * p->J[1 * 3 + k];
  }
  S00 += v->cfg.eps2d;
  S11 += v->cfg.eps2d;
  p->S2[0] = S00; p->S2[1] = S01; p->S2[2] = S11;
  p->det = S00 * S11 - S01 * S01;
  if (!(p->det > 0.0)) return;
  p->conic[0] = S11 / p->det;
  p->conic[1] = -S01 / p->det;
  p->conic[2] = S00 / p->det;
  p->mu[0] = v->fx * tx / tz + v->cx;
  p->mu[1] = v->fy * ty / tz + v->cy;
  if (!(fabs(p->mu[0]) < ORC_BIG && fabs(p->mu[1]) < ORC_BIG)) return;
  p->depth = tz;
  /* opacity-aware extents: alpha >= alpha_min needs q <= 2 ln(o / alpha_min),
   * and on that ellipse |dx| <= sqrt(qmax Sxx), |dy| <= sqrt(qmax Syy). */
  const double qmax = 2.0 * log(p->o / v->cfg.alpha_min);
  const double ax = sqrt(qmax * S00) * (1.0 + v->cfg.rect_margin), ay = sqrt(qmax * S11) * (1.0 + v->cfg.rect_margin);
  double ex = ceil(ax);
  double ey = ceil(ay);
  p->m_ext = fmin(fabs(ax - nearbyint(ax)) / fmax(ax, 1.0), fabs(ay - nearbyint(ay)) / fmax(ay, 1.0));
  p->m_cen = fmin(fabs(p->mu[0] - nearbyint(p->mu[0])), fabs(p->mu[1] - nearbyint(p->mu[1])));
  if (ex > ORC_BIG) ex = ORC_BIG;
  if (ey > ORC_BIG) ey = ORC_BIG;
  p->rx = (int64_t)ex;
  p->ry = (int64_t)ey;
  p->fxi = (int64_t)floor(p->mu[0]);
  p->fyi = (int64_t)floor(p->mu[1]);
  int64_t x0 = floordiv64(p->fxi - p->rx, v->TW), x1 = floordiv64(p->fxi + p->rx, v->TW) + 1;
  int64_t y0 = floordiv64(p->fyi - p->ry, v->TH), y1 = floordiv64(p->fyi + p->ry, v->TH) + 1;
  if (x0 < 0) x0 = 0;
  if (y0 < 0) y0 = 0;
  if (x1 > v->TX) x1 = v->TX;
  if (y1 > v->TY) y1 = v->TY;
  if (x0 >= x1 || y0 >= y1) return;
  p->x0 = (int32_t)x0; p->x1 = (int32_t)x1; p->y0 = (int32_t)y0; p->y1 = (int32_t)y1;
  /* colour from the view direction (Gaussian mean minus camera centre) */
  double dv[3] = {mu[0] - v->ctr[0], mu[1] - v->ctr[1], mu[2] - v->ctr[2]};
  p->dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int r = 0; r < 3; ++r) p->dir[r] = dv[r] / p->dist;
  orc_sh_eval(v->deg, p->dir, p->Y, NULL);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.0;
    for (int k = 0; k < v->K; ++k) acc += p->Y[k] * (double)v->sh[((int64_t)k * 3 + ch) * n + i];
    acc += 0.5;
    p->colmask[ch] = acc > 0.0;
    p->col[ch] = acc > 0.0 ? acc : 0.0;
  }
  p->visible = 1;
}

static const orc_view* g_sort_view;
static int cmp_depth_index(const void* a, const void* b) {
  const int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
  const float di = (float)g_sort_view->P[i].depth, dj = (float)g_sort_view->P[j].depth;
  if (di < dj) return -1;
  if (di > dj) return 1;
  return (i < j) ? -1 : (i > j);
}

/* One Gaussian evaluated at one pixel centre: q and the unclamped alpha. */
static void eval_pair(const orc_proj* p, double px, double py, double* dx, double* dy, double* q,
                      double* raw) {
  *dx = px - p->mu[0];
  *dy = py - p->mu[1];
  *q = p->conic[0] * (*dx) * (*dx) + 2.0 * p->conic[1] * (*dx) * (*dy) + p->conic[2] * (*dy) * (*dy);
  *raw = p->o * exp(-0.5 * (*q));
}

static double relmargin(double a, double b) { return fabs(a - b) / fabs(b); }

/* Relative distance of a positive z from the nearest boundary at which its
 * round-to-nearest FP32 value changes (the midpoints to the neighbouring floats). */
static double fp32_rounding_margin(double z) {
  const float f = (float)z;
  const double up = 0.5 * ((double)f + (double)nextafterf(f, INFINITY));
  const double dn = 0.5 * ((double)f + (double)nextafterf(f, 0.0f));
  return fmin(fabs(z - up), fabs(z - dn)) / z;
}

static uint32_t fp32_bits(double z) {
  const float f = (float)z;
  uint32_t b;
  memcpy(&b, &f, 4);
  return b;
}

/* Composite one pixel front to back; fills outputs and the decision margins:
 *   m[0]  min relative distance of an evaluated alpha from alpha_min
 *   m[1]  min relative distance of a candidate transmittance from T_min
 *   m[2]  min relative distance of a blended alpha from the alpha_max clamp
 *   m[3]  depth-order hazard: over consecutive contributing Gaussians (alpha >=
 *         alpha_min, up to and including the one that stops the pixel) whose
 *         FP32 depth keys are equal or one unit apart, the min relative distance
 *         of either FP64 depth from an FP32 rounding boundary (infinite if no
 *         such pair).  Only such a pair can change order when another
 *         evaluation of the same FP64 depth rounds to a neighbouring key. */
static void composite_pixel(const orc_view* v, int px, int py, double* col, double* dep, double* T_out,
                            int32_t* last, int32_t* nb, double m[4]) {
  const int tile = (py / v->TH) * v->TX + (px / v->TW);
  const double cxp = px + 0.5, cyp = py + 0.5;
  double T = 1.0, C[3] = {0, 0, 0}, D = 0.0, prevz = -1.0;
  int32_t lst = 0, cnt = 0;
  m[0] = m[1] = m[2] = m[3] = INFINITY;
  for (int64_t e = v->tile_off[tile]; e < v->tile_off[tile + 1]; ++e) {
    const orc_proj* p = &v->P[v->tile_list[e]];
    double dx, dy, q, raw;
    eval_pair(p, cxp, cyp, &dx, &dy, &q, &raw);
    double r = relmargin(raw, v->cfg.alpha_min);
    if (r < m[0]) m[0] = r;
    if (raw < v->cfg.alpha_min) continue;
    double a = raw < v->cfg.alpha_max ? raw : v->cfg.alpha_max;
    r = relmargin(raw, v->cfg.alpha_max);
    if (r < m[2]) m[2] = r;
    double Tn = T * (1.0 - a);
    if (v->cfg.t_min > 0.0) {
      r = relmargin(Tn, v->cfg.t_min);
      if (r < m[1]) m[1] = r;
    }
    if (prevz >= 0.0) {
      const uint32_t a0 = fp32_bits(prevz), a1 = fp32_bits(p->depth);
      if ((a0 > a1 ? a0 - a1 : a1 - a0) <= 1u) {
        r = fmin(fp32_rounding_margin(prevz), fp32_rounding_margin(p->depth));
        if (r < m[3]) m[3] = r;
      }
    }
    prevz = p->depth;
    if (Tn < v->cfg.t_min) break;
    for (int ch = 0; ch < 3; ++ch) C[ch] += T * a * p->col[ch];
    D += T * a * p->depth;
    T = Tn;
    lst = (int32_t)(e - v->tile_off[tile]) + 1;
    ++cnt;
  }
  for (int ch = 0; ch < 3; ++ch) col[ch] = C[ch] + T * v->cfg.bg[ch];
  *dep = D;
  *T_out = T;
  *last = lst;
  *nb = cnt;
}

orc_view* orc_view_create(int64_t n, int32_t degree, const double* means, const double* log_scales,
                          const double* quats, const double* logits, const double* sh,
                          const orc_camera* cam, const double* xi, const orc_cfg* cfg) {
  orc_view* v = (orc_view*)calloc(1, sizeof(orc_view));
  v->n = n; v->deg = degree; v->K = (degree + 1) * (degree + 1);
  v->W = cam->width; v->H = cam->height;
  v->cfg = *cfg;
  v->TW = cfg->tile_w; v->TH = cfg->tile_h;
  v->TX = (v->W + v->TW - 1) / v->TW; v->TY = (v->H + v->TH - 1) / v->TH;
  v->fx = cam->fx; v->fy = cam->fy; v->cx = cam->cx; v->cy = cam->cy;
  for (int k = 0; k < 6; ++k) v->xi[k] = xi ? xi[k] : 0.0;
  camera_pose(cam, v->xi, v->Rp, v->tp, v->ctr);
  v->means = means; v->log_scales = log_scales; v->quats = quats; v->logits = logits; v->sh = sh;
  v->P = (orc_proj*)calloc((size_t)(n > 0 ? n : 1), sizeof(orc_proj));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) project_one(v, i, &v->P[i]);
  v->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  v->n_vis = 0;
  for (int64_t i = 0; i < n; ++i)
    if (v->P[i].visible) v->order[v->n_vis++] = i;
  g_sort_view = v;
  qsort(v->order, (size_t)v->n_vis, sizeof(int64_t), cmp_depth_index);
  /* per-tile lists in (depth, index) order: a counting pass, then a fill pass */
  const int64_t ntile = (int64_t)v->TX * v->TY;
  v->tile_off = (int64_t*)calloc((size_t)ntile + 1, sizeof(int64_t));
  for (int64_t e = 0; e < v->n_vis; ++e) {
    const orc_proj* p = &v->P[v->order[e]];
    for (int ty = p->y0; ty < p->y1; ++ty)
      for (int tx = p->x0; tx < p->x1; ++tx) v->tile_off[ty * v->TX + tx + 1]++;
  }
  for (int64_t t = 0; t < ntile; ++t) v->tile_off[t + 1] += v->tile_off[t];
  v->tile_list = (int64_t*)malloc(sizeof(int64_t) * (size_t)(v->tile_off[ntile] > 0 ? v->tile_off[ntile] : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ntile);
  memcpy(fill, v->tile_off, sizeof(int64_t) * (size_t)ntile);
  for (int64_t e = 0; e < v->n_vis; ++e) {
    const int64_t gi = v->order[e];
    const orc_proj* p = &v->P[gi];
    for (int ty = p->y0; ty < p->y1; ++ty)
      for (int tx = p->x0; tx < p->x1; ++tx) v->tile_list[fill[ty * v->TX + tx]++] = gi;
  }
  free(fill);
  const int64_t npix = (int64_t)v->W * v->H;
  v->color = (double*)malloc(sizeof(double) * 3 * (size_t)npix);
  v->depthimg = (double*)malloc(sizeof(double) * (size_t)npix);
  v->tfinal = (double*)malloc(sizeof(double) * (size_t)npix);
  v->margins = (double*)malloc(sizeof(double) * 4 * (size_t)npix);
  v->last = (int32_t*)malloc(sizeof(int32_t) * (size_t)npix);
  v->nblend = (int32_t*)malloc(sizeof(int32_t) * (size_t)npix);
#pragma omp parallel for schedule(dynamic, 4)
  for (int py = 0; py < v->H; ++py)
    for (int px = 0; px < v->W; ++px) {
      const int64_t pix = (int64_t)py * v->W + px;
      double col[3], m[4];
      composite_pixel(v, px, py, col, &v->depthimg[pix], &v->tfinal[pix], &v->last[pix], &v->nblend[pix], m);
      for (int ch = 0; ch < 3; ++ch) v->color[ch * npix + pix] = col[ch];
      for (int k = 0; k < 4; ++k) v->margins[k * npix + pix] = m[k];
    }
  return v;
}

void orc_view_free(orc_view* v) {
  if (!v) return;
  free(v->P); free(v->order); free(v->tile_off); free(v->tile_list);
  free(v->color); free(v->depthimg); free(v->tfinal); free(v->margins);
  free(v->last); free(v->nblend);
  free(v);
}

int64_t orc_view_n_visible(const orc_view* v) { return v->n_vis; }
int64_t orc_view_n_pairs(const orc_view* v) { return v->tile_off[(int64_t)v->TX * v->TY]; }

void orc_view_image(const orc_view* v, double* color, double* depth, double* tfinal, int32_t* last,
                    int32_t* nblend, double* margins) {
  const int64_t npix = (int64_t)v->W * v->H;
  if (color) memcpy(color, v->color, sizeof(double) * 3 * (size_t)npix);
  if (depth) memcpy(depth, v->depthimg, sizeof(double) * (size_t)npix);
  if (tfinal) memcpy(tfinal, v->tfinal, sizeof(double) * (size_t)npix);
  if (last) memcpy(last, v->last, sizeof(int32_t) * (size_t)npix);
  if (nblend) memcpy(nblend, v->nblend, sizeof(int32_t) * (size_t)npix);
  if (margins) memcpy(margins, v->margins, sizeof(double) * 4 * (size_t)npix);
}

/* Per-Gaussian decision margins over every pixel where it is evaluated:
 * out[i][0] its own alpha vs alpha_min, out[i][1] its own alpha vs the alpha_max
 * clamp, out[i][2] the transmittance margin of the pixels where it is the
 * last blended or the terminating Gaussian. */
void orc_view_gauss_margins(const orc_view* v, double* out) {
  const int64_t n = v->n;
  for (int64_t i = 0; i < 3 * n; ++i) out[i] = INFINITY;
#pragma omp parallel
  {
    double* loc = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < 3 * n; ++i) loc[i] = INFINITY;
#pragma omp for schedule(dynamic, 4)
    for (int py = 0; py < v->H; ++py)
      for (int px = 0; px < v->W; ++px) {
        const int tile = (py / v->TH) * v->TX + (px / v->TW);
        double T = 1.0;
        int64_t lastg = -1;
        double lastm = INFINITY;
        for (int64_t e = v->tile_off[tile]; e < v->tile_off[tile + 1]; ++e) {
          const int64_t gi = v->tile_list[e];
          const orc_proj* p = &v->P[gi];
          double dx, dy, q, raw;
          eval_pair(p, px + 0.5, py + 0.5, &dx, &dy, &q, &raw);
          double r = relmargin(raw, v->cfg.alpha_min);
          if (r < loc[gi * 3]) loc[gi * 3] = r;
          if (raw < v->cfg.alpha_min) continue;
          r = relmargin(raw, v->cfg.alpha_max);
          if (r < loc[gi * 3 + 1]) loc[gi * 3 + 1] = r;
          double a = raw < v->cfg.alpha_max ? raw : v->cfg.alpha_max;
          double Tn = T * (1.0 - a);
          double rt = v->cfg.t_min > 0.0 ? relmargin(Tn, v->cfg.t_min) : INFINITY;
          if (Tn < v->cfg.t_min) {
            if (rt < loc[gi * 3 + 2]) loc[gi * 3 + 2] = rt;
            if (lastg >= 0 && rt < loc[lastg * 3 + 2]) loc[lastg * 3 + 2] = rt;
            break;
          }
          if (lastg >= 0 && lastm < loc[lastg * 3 + 2]) loc[lastg * 3 + 2] = lastm;
          lastg = gi;
          lastm = rt;
          T = Tn;
        }
      }
#pragma omp critical
    for (int64_t i = 0; i < 3 * n; ++i)
      if (loc[i] < out[i]) out[i] = loc[i];
    free(loc);
  }
}

/* Per-Gaussian projection outputs.  rec: [n][10] = mu_x, mu_y, conic a, b, c,
 * opacity, r, g, b, depth; irec: [n][8] = visible, fxi, fyi, rx, ry, x0..y1 packed
 * as x0, x1, y0, y1 in the last four; misc: [n][9] = per-Gaussian margins
 * (near plane, alpha_min cull, guard band x, guard band y, colour clamp, det,
 * far plane (relative), pixel centre from an integer, extent from an integer
 * (relative)). */
void orc_view_proj(const orc_view* v, double* rec, int64_t* irec, double* misc) {
  for (int64_t i = 0; i < v->n; ++i) {
    const orc_proj* p = &v->P[i];
    if (rec) {
      double* r = rec + i * 10;
      r[0] = p->mu[0]; r[1] = p->mu[1];
      r[2] = p->conic[0]; r[3] = p->conic[1]; r[4] = p->conic[2];
      r[5] = p->o; r[6] = p->col[0]; r[7] = p->col[1]; r[8] = p->col[2]; r[9] = p->depth;
    }
    if (irec) {
      int64_t* r = irec + i * 9;
      r[0] = p->visible; r[1] = p->fxi; r[2] = p->fyi; r[3] = p->rx; r[4] = p->ry;
      r[5] = p->x0; r[6] = p->x1; r[7] = p->y0; r[8] = p->y1;
    }
    if (misc) {
      double* r = misc + i * 9;
      const double hx = 0.5 * v->W / v->fx, hy = 0.5 * v->H / v->fy;
      const double mx = (0.5 * v->W - v->cx) / v->fx, my = (0.5 * v->H - v->cy) / v->fy;
      double ux = p->t[0] / p->t[2], uy = p->t[1] / p->t[2];
      double gx = fmin(fabs(ux - (mx - v->cfg.guard * hx)), fabs(ux - (mx + v->cfg.guard * hx)));
      double gy = fmin(fabs(uy - (my - v->cfg.guard * hy)), fabs(uy - (my + v->cfg.guard * hy)));
      double cm = INFINITY;
      for (int ch = 0; ch < 3; ++ch) {
        double raw = 0.5;
        for (int k = 0; k < v->K; ++k) raw += p->Y[k] * (double)v->sh[((int64_t)k * 3 + ch) * v->n + i];
        if (fabs(raw) < cm) cm = fabs(raw);
      }
      r[0] = fabs(p->t[2] - v->cfg.near_z);
      r[1] = relmargin(p->o, v->cfg.alpha_min);
      r[2] = gx; r[3] = gy; r[4] = cm; r[5] = p->det;
      r[6] = p->m_far; r[7] = p->m_cen; r[8] = p->m_ext;
    }
  }
}

/* The per-tile lists as (tile, gaussian) pairs in list order. */
void orc_view_pairs(const orc_view* v, int32_t* tile, int64_t* gid) {
  const int64_t ntile = (int64_t)v->TX * v->TY;
  for (int64_t t = 0; t < ntile; ++t)
    for (int64_t e = v->tile_off[t]; e < v->tile_off[t + 1]; ++e) {
      tile[e] = (int32_t)t;
      gid[e] = v->tile_list[e];
    }
}

/* -------------------------------------------------------- statistics */
/* M_v(u) = [sum_ch |I - I^| > tau_err];  Omega_v(i) = pixels where i is blended;
 * kappa_v(i) = |Omega_v(i) with M = 1|.  Also returns the mask, its margin and
 * per-pixel blended counts. */
void orc_view_stats(const orc_view* v, const float* target, double tau_err, int32_t* omega,
                    int32_t* kappa, uint8_t* mask, double* mask_margin) {
  const int64_t npix = (int64_t)v->W * v->H;
  memset(omega, 0, sizeof(int32_t) * (size_t)v->n);
  memset(kappa, 0, sizeof(int32_t) * (size_t)v->n);
#pragma omp parallel for schedule(dynamic, 4)
  for (int py = 0; py < v->H; ++py)
    for (int px = 0; px < v->W; ++px) {
      const int64_t pix = (int64_t)py * v->W + px;
      double err = 0.0;
      for (int ch = 0; ch < 3; ++ch) err += fabs((double)target[ch * npix + pix] - v->color[ch * npix + pix]);
      const int M = err > tau_err;
      if (mask) mask[pix] = (uint8_t)M;
      if (mask_margin) mask_margin[pix] = fabs(err - tau_err);
      const int tile = (py / v->TH) * v->TX + (px / v->TW);
      double T = 1.0;
      for (int64_t e = v->tile_off[tile]; e < v->tile_off[tile + 1]; ++e) {
        const int64_t gi = v->tile_list[e];
        const orc_proj* p = &v->P[gi];
        double dx, dy, q, raw;
        eval_pair(p, px + 0.5, py + 0.5, &dx, &dy, &q, &raw);
        if (raw < v->cfg.alpha_min) continue;
        double a = raw < v->cfg.alpha_max ? raw : v->cfg.alpha_max;
        double Tn = T * (1.0 - a);
        if (Tn < v->cfg.t_min) break;
#pragma omp atomic update
        omega[gi] += 1;
        if (M) {
#pragma omp atomic update
          kappa[gi] += 1;
        }
        T = Tn;
      }
    }
}

static int cmp_i64(const void* a, const void* b) {
  const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* Per-anchor footprint statistics (appendix, "Densification Score" and
 * "Pruning Score": Omega_v(i) is the set of pixels where the decoded Gaussians
 * of anchor i contribute): Gaussian g belongs to anchor anchor_of[g]; an
 * anchor's footprint is the union of its Gaussians' blended pixels, so a pixel
 * counts once for an anchor however many of its Gaussians blend there.
 * omega_a [n_anchor] += |Omega_v(a)|, kappa_a [n_anchor] += the pixels of that
 * union with ||I - I^||_1 > tau_err. */
void orc_view_anchor_stats(const orc_view* v, const int64_t* anchor_of, int64_t n_anchor, const float* target,
                           double tau_err, int64_t* omega_a, int64_t* kappa_a) {
  const int64_t npix = (int64_t)v->W * v->H;
  int64_t longest = 1;
  for (int64_t t = 0; t < (int64_t)v->TX * v->TY; ++t)
    if (v->tile_off[t + 1] - v->tile_off[t] > longest) longest = v->tile_off[t + 1] - v->tile_off[t];
#pragma omp parallel
  {
    int64_t* seen = (int64_t*)malloc(sizeof(int64_t) * (size_t)longest);
#pragma omp for schedule(dynamic, 4)
    for (int py = 0; py < v->H; ++py)
      for (int px = 0; px < v->W; ++px) {
        const int64_t pix = (int64_t)py * v->W + px;
        double err = 0.0;
        for (int ch = 0; ch < 3; ++ch) err += fabs((double)target[ch * npix + pix] - v->color[ch * npix + pix]);
        const int M = err > tau_err;
        const int tile = (py / v->TH) * v->TX + (px / v->TW);
        double T = 1.0;
        int64_t m = 0;
        for (int64_t e = v->tile_off[tile]; e < v->tile_off[tile + 1]; ++e) {
          const int64_t gi = v->tile_list[e];
          const orc_proj* p = &v->P[gi];
          double dx, dy, q, raw;
          eval_pair(p, px + 0.5, py + 0.5, &dx, &dy, &q, &raw);
          if (raw < v->cfg.alpha_min) continue;
          double a = raw < v->cfg.alpha_max ? raw : v->cfg.alpha_max;
          double Tn = T * (1.0 - a);
          if (Tn < v->cfg.t_min) break;
          seen[m++] = anchor_of[gi];
          T = Tn;
        }
        qsort(seen, (size_t)m, sizeof(int64_t), cmp_i64);
        for (int64_t k = 0; k < m; ++k) {
          if (k > 0 && seen[k] == seen[k - 1]) continue;
          const int64_t an = seen[k];
          if (an < 0 || an >= n_anchor) continue;
#pragma omp atomic update
          omega_a[an] += 1;
          if (M) {
#pragma omp atomic update
            kappa_a[an] += 1;
          }
        }
      }
    free(seen);
  }
}

/* ------------------------------------------------------------- backward */
typedef struct {
  double mu[2], conic[3], o, col[3], z;
} orc_g2;

/* Derivative of the quaternion->rotation map R(qn) with respect to qn:
 * dR[k][e] = d R_e / d qn_k. */
static void dquat_rot(const double q[4], double dR[4][9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  /* d/dw */
  double a[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  /* d/dx */
  double b[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  /* d/dy */
  double c[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  /* d/dz */
  double d[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  memcpy(dR[0], a, sizeof a); memcpy(dR[1], b, sizeof b);
  memcpy(dR[2], c, sizeof c); memcpy(dR[3], d, sizeof d);
}

/* dL/dC [3][H][W], dL/dD [H][W] (may be NULL).  Gradients are ADDED into the
 * outputs: g_means [3][n], g_logs [3][n], g_quats [4][n], g_logits [n],
 * g_sh [K][3][n], g_xi [6]; g2 (optional) receives the per-Gaussian 2D
 * gradients [n][10] (mu x, mu y, conic a, b, c, opacity, r, g, b, depth),
 * overwritten. */
void orc_view_backward(const orc_view* v, const double* dLdC, const double* dLdD, double* g_means,
                       double* g_logs, double* g_quats, double* g_logits, double* g_sh, double* g_xi,
                       double* g2out) {
  const int64_t n = v->n, npix = (int64_t)v->W * v->H;
  orc_g2* G = (orc_g2*)calloc((size_t)(n > 0 ? n : 1), sizeof(orc_g2));
#pragma omp parallel
  {
    int64_t cap = 256;
    int64_t* ids = (int64_t*)malloc(sizeof(int64_t) * cap);
    double* Ts = (double*)malloc(sizeof(double) * cap);
    double* As = (double*)malloc(sizeof(double) * cap);
    double* Qs = (double*)malloc(sizeof(double) * cap * 3); /* dx, dy, raw */
#pragma omp for schedule(dynamic, 4)
    for (int py = 0; py < v->H; ++py)
      for (int px = 0; px < v->W; ++px) {
        const int64_t pix = (int64_t)py * v->W + px;
        const int tile = (py / v->TH) * v->TX + (px / v->TW);
        /* the blended sequence of this pixel */
        int64_t K = 0;
        double T = 1.0;
        for (int64_t e = v->tile_off[tile]; e < v->tile_off[tile + 1]; ++e) {
          const int64_t gi = v->tile_list[e];
          const orc_proj* p = &v->P[gi];
          double dx, dy, q, raw;
          eval_pair(p, px + 0.5, py + 0.5, &dx, &dy, &q, &raw);
          if (raw < v->cfg.alpha_min) continue;
          double a = raw < v->cfg.alpha_max ? raw : v->cfg.alpha_max;
          double Tn = T * (1.0 - a);
          if (Tn < v->cfg.t_min) break;
          if (K == cap) {
            cap *= 2;
            ids = (int64_t*)realloc(ids, sizeof(int64_t) * cap);
            Ts = (double*)realloc(Ts, sizeof(double) * cap);
            As = (double*)realloc(As, sizeof(double) * cap);
            Qs = (double*)realloc(Qs, sizeof(double) * cap * 3);
          }
          ids[K] = gi; Ts[K] = T; As[K] = a;
          Qs[K * 3 + 0] = dx; Qs[K * 3 + 1] = dy; Qs[K * 3 + 2] = raw;
          ++K;
          T = Tn;
        }
        const double Tfin = T;
        double gC[3], gD = dLdD ? dLdD[pix] : 0.0;
        for (int ch = 0; ch < 3; ++ch) gC[ch] = dLdC[ch * npix + pix];
        /* suffix sums: colour and depth contributed behind entry k, plus the background */
        double SC[3] = {Tfin * v->cfg.bg[0], Tfin * v->cfg.bg[1], Tfin * v->cfg.bg[2]}, SD = 0.0;
        for (int64_t k = K - 1; k >= 0; --k) {
          const int64_t gi = ids[k];
          const orc_proj* p = &v->P[gi];
          const double Tk = Ts[k], a = As[k], dx = Qs[k * 3], dy = Qs[k * 3 + 1], raw = Qs[k * 3 + 2];
          double dLda = 0.0;
          for (int ch = 0; ch < 3; ++ch) dLda += gC[ch] * (Tk * p->col[ch] - SC[ch] / (1.0 - a));
          dLda += gD * (Tk * p->depth - SD / (1.0 - a));
          double dLdo = 0.0, dLdq = 0.0;
          if (raw < v->cfg.alpha_max) {
            dLdo = dLda * exp(-0.5 * (dx * dx * p->conic[0] + 2 * dx * dy * p->conic[1] + dy * dy * p->conic[2]));
            dLdq = dLda * (-0.5 * a);
          }
          orc_g2 acc;
          acc.mu[0] = dLdq * (-(2.0 * p->conic[0] * dx + 2.0 * p->conic[1] * dy));
          acc.mu[1] = dLdq * (-(2.0 * p->conic[1] * dx + 2.0 * p->conic[2] * dy));
          acc.conic[0] = dLdq * dx * dx;
          acc.conic[1] = dLdq * 2.0 * dx * dy;
          acc.conic[2] = dLdq * dy * dy;
          acc.o = dLdo;
          for (int ch = 0; ch < 3; ++ch) acc.col[ch] = gC[ch] * Tk * a;
          acc.z = gD * Tk * a;
          orc_g2* g = &G[gi];
#pragma omp atomic update
          g->mu[0] += acc.mu[0];
#pragma omp atomic update
          g->mu[1] += acc.mu[1];
#pragma omp atomic update
          g->conic[0] += acc.conic[0];
#pragma omp atomic update
          g->conic[1] += acc.conic[1];
#pragma omp atomic update
          g->conic[2] += acc.conic[2];
#pragma omp atomic update
          g->o += acc.o;
#pragma omp atomic update
          g->col[0] += acc.col[0];
#pragma omp atomic update
          g->col[1] += acc.col[1];
#pragma omp atomic update
          g->col[2] += acc.col[2];
#pragma omp atomic update
          g->z += acc.z;
          for (int ch = 0; ch < 3; ++ch) SC[ch] += Tk * a * p->col[ch];
          SD += Tk * a * p->depth;
        }
      }
    free(ids); free(Ts); free(As); free(Qs);
  }
  if (g2out)
    for (int64_t i = 0; i < n; ++i) {
      double* r = g2out + i * 10;
      r[0] = G[i].mu[0]; r[1] = G[i].mu[1];
      r[2] = G[i].conic[0]; r[3] = G[i].conic[1]; r[4] = G[i].conic[2];
      r[5] = G[i].o; r[6] = G[i].col[0]; r[7] = G[i].col[1]; r[8] = G[i].col[2]; r[9] = G[i].z;
    }

  /* chain rule to the 3D parameters; pose through dL/dR' and dL/dt' */
  double GR[9] = {0}, Gt[3] = {0};
  const int K = v->K;
  for (int64_t i = 0; i < n; ++i) {
    const orc_proj* p = &v->P[i];
    if (!p->visible) continue;
    const orc_g2* g = &G[i];
    const double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    const double fx = v->fx, fy = v->fy;
    double gt[3] = {0, 0, 0};
    /* pixel centre */
    gt[0] += g->mu[0] * fx / tz;
    gt[2] += g->mu[0] * (-fx * tx / (tz * tz));
    gt[1] += g->mu[1] * fy / tz;
    gt[2] += g->mu[1] * (-fy * ty / (tz * tz));
    /* depth */
    gt[2] += g->z;
    /* conic -> Sigma2D entries (Sxx, Sxy, Syy) */
    const double Sxx = p->S2[0], Sxy = p->S2[1], Syy = p->S2[2], det = p->det, d2 = det * det;
    const double ga = g->conic[0], gb = g->conic[1], gc = g->conic[2];
    double gSxx = ga * (-Syy * Syy / d2) + gb * (Sxy * Syy / d2) + gc * (1.0 / det - Sxx * Syy / d2);
    double gSyy = ga * (1.0 / det - Syy * Sxx / d2) + gb * (Sxy * Sxx / d2) + gc * (-Sxx * Sxx / d2);
    double gSxy = ga * (2.0 * Syy * Sxy / d2) + gb * (-1.0 / det - 2.0 * Sxy * Sxy / d2) + gc * (2.0 * Sxx * Sxy / d2);
    /* Sigma2D = J Sigma_c J^T + eps I:  G2 is the full-matrix gradient */
    const double G2[4] = {gSxx, 0.5 * gSxy, 0.5 * gSxy, gSyy};
    double GC[9], GJ[6];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) acc += p->J[r * 3 + a] * G2[r * 2 + c] * p->J[c * 3 + b];
        GC[a * 3 + b] = acc;
      }
    for (int r = 0; r < 2; ++r)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int c = 0; c < 2; ++c)
          for (int k = 0; k < 3; ++k) acc += G2[r * 2 + c] * p->J[c * 3 + k] * p->covc[k * 3 + b];
        GJ[r * 3 + b] = 2.0 * acc;
      }
    /* J(t) */
    gt[2] += GJ[0] * (-fx / (tz * tz));
    gt[2] += GJ[4] * (-fy / (tz * tz));
    if (p->clampx == 0) {
      gt[0] += GJ[2] * (-fx / (tz * tz));
      gt[2] += GJ[2] * (2.0 * fx * tx / (tz * tz * tz));
    } else {
      gt[2] += GJ[2] * (fx * p->limx / (tz * tz));
    }
    if (p->clampy == 0) {
      gt[1] += GJ[5] * (-fy / (tz * tz));
      gt[2] += GJ[5] * (2.0 * fy * ty / (tz * tz * tz));
    } else {
      gt[2] += GJ[5] * (fy * p->limy / (tz * tz));
    }
    /* Sigma_c = R' Sigma_w R'^T */
    double GW[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) acc += v->Rp[k * 3 + a] * GC[k * 3 + l] * v->Rp[l * 3 + b];
        GW[a * 3 + b] = acc;
      }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) acc += GC[a * 3 + k] * v->Rp[k * 3 + l] * p->covw[l * 3 + b];
        GR[a * 3 + b] += 2.0 * acc;
      }
    /* Sigma_w = M M^T, M = Rq diag(s) */
    double GM[9];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int b = 0; b < 3; ++b) acc += GW[a * 3 + b] * p->Rq[b * 3 + k] * p->s[k];
        GM[a * 3 + k] = 2.0 * acc;
      }
    double GRq[9];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) GRq[a * 3 + k] = GM[a * 3 + k] * p->s[k];
    for (int k = 0; k < 3; ++k) {
      double gs = 0.0;
      for (int a = 0; a < 3; ++a) gs += GM[a * 3 + k] * p->Rq[a * 3 + k];
      g_logs[k * n + i] += gs * p->s[k];
    }
    double dR[4][9], gqn[4];
    dquat_rot(p->qn, dR);
    for (int k = 0; k < 4; ++k) {
      double acc = 0.0;
      for (int e = 0; e < 9; ++e) acc += GRq[e] * dR[k][e];
      gqn[k] = acc;
    }
    double qdot = 0.0;
    for (int k = 0; k < 4; ++k) qdot += p->qn[k] * gqn[k];
    for (int k = 0; k < 4; ++k) g_quats[k * n + i] += (gqn[k] - p->qn[k] * qdot) / p->qnorm;
    /* opacity */
    g_logits[i] += g->o * p->o * (1.0 - p->o);
    /* colour: SH coefficients and the view direction */
    double Y[16], dY[48];
    orc_sh_eval(v->deg, p->dir, Y, dY);
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      if (!p->colmask[ch]) continue;
      for (int k = 0; k < K; ++k) {
        g_sh[((int64_t)k * 3 + ch) * n + i] += Y[k] * g->col[ch];
        const double c = (double)v->sh[((int64_t)k * 3 + ch) * n + i];
        for (int r = 0; r < 3; ++r) gdir[r] += g->col[ch] * c * dY[k * 3 + r];
      }
    }
    /* dir = (mu - c)/|mu - c|: d dir/d vvec = (I - dir dir^T)/|vvec| */
    double dd = gdir[0] * p->dir[0] + gdir[1] * p->dir[1] + gdir[2] * p->dir[2];
    double gvv[3];
    for (int r = 0; r < 3; ++r) gvv[r] = (gdir[r] - p->dir[r] * dd) / p->dist;
    /* t = R' mu + t' */
    for (int r = 0; r < 3; ++r) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += v->Rp[k * 3 + r] * gt[k];
      g_means[r * n + i] += acc + gvv[r];
    }
    const double mu[3] = {v->means[i], v->means[n + i], v->means[2 * n + i]};
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b) GR[a * 3 + b] += gt[a] * mu[b];
      Gt[a] += gt[a];
    }
    /* camera centre c = -R'^T t':  dL/dc = -gvv */
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        /* c_b = -sum_a R'_ab t'_a */
        GR[a * 3 + b] += (-gvv[b]) * (-v->tp[a]);
      }
    for (int a = 0; a < 3; ++a) {
      double acc = 0.0;
      for (int b = 0; b < 3; ++b) acc += v->Rp[a * 3 + b] * (-gvv[b]);
      Gt[a] += -acc;
    }
  }
  /* dL/dxi_k = < dL/dT', dExp/dxi_k T > */
  double T[16];
  memset(T, 0, sizeof T);
  {
    /* recover the unperturbed pose from T' = Exp(xi) T:  T = Exp(-xi) T' */
    double Tp[16], Ei[16], mxi[6];
    memset(Tp, 0, sizeof Tp);
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b) Tp[a * 4 + b] = v->Rp[a * 3 + b];
      Tp[a * 4 + 3] = v->tp[a];
    }
    Tp[15] = 1.0;
    for (int k = 0; k < 6; ++k) mxi[k] = -v->xi[k];
    orc_se3_exp(mxi, Ei);
    m4_mul(Ei, Tp, T);
  }
  for (int k = 0; k < 6; ++k) {
    double D[16], DT[16];
    orc_se3_exp_deriv(v->xi, k, D);
    m4_mul(D, T, DT);
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b) acc += GR[a * 3 + b] * DT[a * 4 + b];
      acc += Gt[a] * DT[a * 4 + 3];
    }
    g_xi[k] += acc;
  }
  free(G);
}

/* ------------------------------------------------ integer binning contract
 * Keys of the (tile, Gaussian) pairs of a set of projected slots, computed
 * from the integer pixel centre floor(mu), the integer extents (rx, ry) and the
 * fp32 depth bits, then sorted by (key, gaussian index).  Key layout:
 *   (view * tiles_per_view + ty * TX + tx) << 32 | depth_bits.
 * Returns the number of pairs (or -1 if cap is too small). */
typedef struct {
  uint64_t key;
  int64_t gid;
} orc_pair;

static int cmp_pair(const void* a, const void* b) {
  const orc_pair* x = (const orc_pair*)a;
  const orc_pair* y = (const orc_pair*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->gid > y->gid) - (x->gid < y->gid);
}

int64_t orc_bin_keys(int64_t n_slots, const int32_t* view, const int64_t* gid, const int64_t* fxi,
                     const int64_t* fyi, const int64_t* rx, const int64_t* ry, const uint32_t* depth_bits,
                     int32_t W, int32_t H, int32_t TW, int32_t TH, uint64_t* keys, int64_t* gids,
                     int64_t cap) {
  const int64_t TX = (W + TW - 1) / TW, TY = (H + TH - 1) / TH, per_view = TX * TY;
  int64_t np = 0;
  for (int64_t s = 0; s < n_slots; ++s) {
    int64_t x0 = floordiv64(fxi[s] - rx[s], TW), x1 = floordiv64(fxi[s] + rx[s], TW) + 1;
    int64_t y0 = floordiv64(fyi[s] - ry[s], TH), y1 = floordiv64(fyi[s] + ry[s], TH) + 1;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > TX) x1 = TX;
    if (y1 > TY) y1 = TY;
    for (int64_t ty = y0; ty < y1; ++ty)
      for (int64_t tx = x0; tx < x1; ++tx) {
        if (np >= cap) return -1;
        const uint64_t tile = (uint64_t)view[s] * (uint64_t)per_view + (uint64_t)(ty * TX + tx);
        keys[np] = (tile << 32) | (uint64_t)depth_bits[s];
        gids[np] = gid[s];
        ++np;
      }
  }
  orc_pair* tmp = (orc_pair*)malloc(sizeof(orc_pair) * (size_t)(np > 0 ? np : 1));
  for (int64_t e = 0; e < np; ++e) tmp[e].key = keys[e], tmp[e].gid = gids[e];
  qsort(tmp, (size_t)np, sizeof(orc_pair), cmp_pair);
  for (int64_t e = 0; e < np; ++e) keys[e] = tmp[e].key, gids[e] = tmp[e].gid;
  free(tmp);
  return np;
}

/* Threads of the OpenMP regions that follow (timing of the oracle on fewer cores). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
