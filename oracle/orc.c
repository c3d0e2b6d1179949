/*
 * orc.c -- FP64 CPU oracle for DeepInverse (Mousavi & Baraniuk, arXiv 1701.03891).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).  Plain loops in the order the
 * paper's definitions are written; OpenMP only splits independent images.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ Sec. 1 */
void orc_measure(const double *phi, const double *x, double *y, int B, int M, int N) {
  /* y = Phi x for every signal of the batch */
#pragma omp parallel for schedule(static)
  for (int b = 0; b < B; ++b)
    for (int m = 0; m < M; ++m) {
      double s = 0.0;
      for (int n = 0; n < N; ++n) s += phi[(long)m * N + n] * x[(long)b * N + n];
      y[(long)b * M + m] = s;
    }
}

/* Noisy measurements (Sec. 5, Table 3): y_b <- y_b + s_b e_b with s_b chosen so
 * that ||y_b||^2 / ||s_b e_b||^2 = 10^(snr_db / 10).  e is the noise draw. */
void orc_add_noise(double *y, const double *e, int B, int M, double snr_db) {
  for (int b = 0; b < B; ++b) {
    double ny = 0.0, ne = 0.0;
    for (int m = 0; m < M; ++m) {
      ny += y[(long)b * M + m] * y[(long)b * M + m];
      ne += e[(long)b * M + m] * e[(long)b * M + m];
    }
    const double s = ne > 0.0 ? sqrt(ny / ne) * pow(10.0, -snr_db / 20.0) : 0.0;
    for (int m = 0; m < M; ++m) y[(long)b * M + m] += s * e[(long)b * M + m];
  }
}

/* ------------------------------------------------------------------ Sec. 4 */
void orc_proxy(const double *wfc, const double *y, double *xt, int B, int M, int N) {
  /* fully connected layer with weights Phi^T: xt = Phi^T y */
#pragma omp parallel for schedule(static)
  for (int b = 0; b < B; ++b)
    for (int p = 0; p < N; ++p) {
      double s = 0.0;
      for (int m = 0; m < M; ++m) s += wfc[(long)p * M + m] * y[(long)b * M + m];
      xt[(long)b * N + p] = s;
    }
}

/* Eq. (1): z = (W * in) + b over the full (n1+k-1) x (n2+k-1) grid, where "*"
 * is the 2-D correlation of the filter with the input zero-padded by k-1 on
 * every side; out = S(ReLU(z)), S dropping the (k-1)/2 padding borders. */
void orc_conv_layer(const double *in, int Cin, int n1, int n2, const double *w, int Cout,
                    int k, const double *bias, int bias_full, int relu, double *zfull,
                    double *out) {
  const int f1 = n1 + k - 1, f2 = n2 + k - 1, r = (k - 1) / 2;
  for (int co = 0; co < Cout; ++co)
    for (int t1 = 0; t1 < f1; ++t1)
      for (int t2 = 0; t2 < f2; ++t2) {
        /* input pixel (i, j) = (t1 + u - (k-1), t2 + v - (k-1)); outside the image it is 0 */
        int u0 = (k - 1) - t1 > 0 ? (k - 1) - t1 : 0;
        int u1 = (n1 - 1) + (k - 1) - t1 < k - 1 ? (n1 - 1) + (k - 1) - t1 : k - 1;
        int v0 = (k - 1) - t2 > 0 ? (k - 1) - t2 : 0;
        int v1 = (n2 - 1) + (k - 1) - t2 < k - 1 ? (n2 - 1) + (k - 1) - t2 : k - 1;
        double s = 0.0;
        for (int ci = 0; ci < Cin; ++ci)
          for (int u = u0; u <= u1; ++u) {
            const double *wr = w + (((long)co * Cin + ci) * k + u) * k;
            const double *xr = in + ((long)ci * n1 + (t1 + u - (k - 1))) * n2 + (t2 - (k - 1));
            for (int v = v0; v <= v1; ++v) s += wr[v] * xr[v];
          }
        s += bias_full ? bias[((long)co * f1 + t1) * f2 + t2] : bias[co];
        if (zfull) zfull[((long)co * f1 + t1) * f2 + t2] = s;
        double a = (relu && s < 0.0) ? 0.0 : s;
        if (t1 >= r && t1 < r + n1 && t2 >= r && t2 < r + n2)
          out[((long)co * n1 + (t1 - r)) * n2 + (t2 - r)] = a;
      }
}

static long full_size(const orc_net *net, int l) {
  return (long)(net->n1 + net->k[l] - 1) * (net->n2 + net->k[l] - 1);
}

long orc_acts_per_image(const orc_net *net) {
  const long N = (long)net->n1 * net->n2;
  long s = 0;
  for (int l = 0; l <= net->L; ++l) s += net->C[l] * N;                 /* a_0 .. a_L */
  for (int l = 0; l < net->L; ++l) s += net->C[l + 1] * full_size(net, l); /* z_1 .. z_L */
  return s;
}

/* pointers into one image's activation block */
static void acts_layout(const orc_net *net, double *base, double **a, double **z) {
  const long N = (long)net->n1 * net->n2;
  double *p = base;
  for (int l = 0; l <= net->L; ++l) { a[l] = p; p += net->C[l] * N; }
  for (int l = 0; l < net->L; ++l) { z[l] = p; p += net->C[l + 1] * full_size(net, l); }
}

static void forward_one(const orc_net *net, const double *wfc, const double *const *w,
                        const double *const *b, const double *yb, double *act) {
  double *a[9], *z[8];
  acts_layout(net, act, a, z);
  const int N = net->n1 * net->n2;
  orc_proxy(wfc, yb, a[0], 1, net->M, N);   /* x~ = Phi^T y, read as an n1 x n2 image */
  for (int l = 0; l < net->L; ++l) {
    int relu = (l < net->L - 1) || net->relu_last;
    orc_conv_layer(a[l], net->C[l], net->n1, net->n2, w[l], net->C[l + 1], net->k[l], b[l],
                   net->bias_full, relu, z[l], a[l + 1]);
  }
}

void orc_forward(const orc_net *net, const double *wfc, const double *const *w,
                 const double *const *b, const double *y, int B, double *xhat, double *acts) {
  const long per = orc_acts_per_image(net);
  const int N = net->n1 * net->n2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int bi = 0; bi < B; ++bi) {
    double *act = acts ? acts + per * bi : (double *)malloc(sizeof(double) * per);
    forward_one(net, wfc, w, b, y + (long)bi * net->M, act);
    double *a[9], *z[8];
    acts_layout(net, act, a, z);
    memcpy(xhat + (long)bi * N, a[net->L], sizeof(double) * N);
    if (!acts) free(act);
  }
}

/* ------------------------------------------- reduced-precision operands (BF16, FP8) */
/* Rounding to a binary floating-point format, from its definition: p significand bits
 * (the leading one included), normal numbers from 2^emin up (below that the spacing
 * stays 2^(emin - p + 1): the subnormals), largest finite value maxv.  The result is the
 * nearest representable value; a tie goes to the one with an even last significand
 * bit.  With sat, magnitudes from maxv up give +-maxv (the clamp that precedes a
 * saturating conversion); without it a value that rounds past maxv becomes +-inf. */
static double round_format(double v, int p, int emin, double maxv, int sat) {
  if (v == 0.0 || v != v) return v;
  double a = fabs(v);
  if (sat && a >= maxv) return copysign(maxv, v);
  int e;
  frexp(a, &e);                /* a = f 2^e with f in [0.5, 1): leading bit 2^(e-1) */
  int E = e - 1 < emin ? emin : e - 1;
  double q = ldexp(1.0, E - p + 1);      /* spacing of representable values at a */
  double n = a / q;                      /* exact: q is a power of two */
  double fl = floor(n), d = n - fl;
  if (d > 0.5 || (d == 0.5 && fmod(fl, 2.0) != 0.0)) fl += 1.0;
  double r = fl * q;
  if (r > maxv) r = sat ? maxv : INFINITY;
  return copysign(r, v);
}

/* spacing of the format's values at magnitude |v| (the unit in the last place) */
static double ulp_format(double v, int p, int emin) {
  double a = fabs(v);
  int e;
  if (a == 0.0) return ldexp(1.0, emin - p + 1);
  frexp(a, &e);
  int E = e - 1 < emin ? emin : e - 1;
  return ldexp(1.0, E - p + 1);
}

/* BF16: 8 significand bits, the exponent range of FP32.  OCP FP8 e4m3 ("fn"): 4
 * significand bits, normals from 2^-6, largest finite value 1.75 * 2^8 = 448. */
#define BF16_MAX (255.0 * 1.329227995784916e+36)   /* (2 - 2^-7) 2^127 = 255 * 2^120 */
double orc_round(double v, int fmt) {
  if (fmt == ORC_Q_BF16) return round_format(v, 8, -126, BF16_MAX, 0);
  if (fmt == ORC_Q_E4M3) return round_format(v, 4, -6, 448.0, 1);
  return v;
}

static double q_value(double v, orc_q q) {
  return q.fmt == ORC_Q_NONE ? v : orc_round(v / q.scale, q.fmt) * q.scale;
}

/* variance of the rounding error of v under q, modelled as uniform over one spacing:
 * (scale * ulp(v / scale))^2 / 12 */
static double q_var(double v, orc_q q) {
  if (q.fmt == ORC_Q_NONE) return 0.0;
  double u = q.fmt == ORC_Q_BF16 ? ulp_format(v / q.scale, 8, -126) : ulp_format(v / q.scale, 4, -6);
  u *= q.scale;
  return u * u / 12.0;
}

void orc_quantize(const double *x, double *out, long n, int fmt, double scale) {
  orc_q q = {fmt, scale};
  for (long i = 0; i < n; ++i) out[i] = q_value(x[i], q);
}

/* Variance of the error of an FP32 running sum of n terms, per unit of sum of
 * squared terms: step t adds an error of variance at most ulp(S_t)^2 / 12 with
 * ulp(S_t) <= 2^-23 |S_t|, and a sum of terms of random sign has E[S_t^2] =
 * (t/n) sum_k term_k^2, so the n steps add (n / 24) 2^-46 sum_k term_k^2. */
static double acc_var_coeff(int acc_fp32, long n) {
  return acc_fp32 ? (double)n / 24.0 * ldexp(1.0, -46) : 0.0;
}

/* One image of the reduced-precision forward pass, and (var != NULL) the variance
 * of each output pixel's error against the exact network, propagated linearly:
 * a rounding error passes through a layer like a small input change (weights
 * squared, ReLU passing it where the unit is active), and errors are taken as
 * independent with the variances of q_var and acc_var_coeff.  wfc2, w2[l] hold the
 * squared rounded weights and wfcc, wc[l] the per-product variances of the weight
 * rounding plus the accumulation step (both read only when var != NULL). */
static void forward_one_q(const orc_net *net, const double *wfcq, const double *wfc2,
                          const double *wfcc, const double *const *wq, const double *const *w2,
                          const double *const *wc, const double *const *b,
                          const double *yb, const orc_quant *qs, double *act, double *var) {
  const int N = net->n1 * net->n2, M = net->M, n1 = net->n1, n2 = net->n2;
  double *a[9], *z[8];
  acts_layout(net, act, a, z);
  double *yq = (double *)malloc(sizeof(double) * M);
  for (int m = 0; m < M; ++m) yq[m] = q_value(yb[m], qs->y);
  orc_proxy(wfcq, yq, a[0], 1, M, N);
  int cmax = 1;
  for (int l = 0; l <= net->L; ++l) cmax = net->C[l] > cmax ? net->C[l] : cmax;
  double *V = NULL, *Vn = NULL, *t1 = NULL, *t2 = NULL, *sq = NULL, *zero = NULL;
  if (var) {
    V = (double *)malloc(sizeof(double) * cmax * N);
    Vn = (double *)malloc(sizeof(double) * cmax * N);
    t1 = (double *)malloc(sizeof(double) * cmax * N);
    t2 = (double *)malloc(sizeof(double) * cmax * N);
    sq = (double *)malloc(sizeof(double) * cmax * N);
    zero = (double *)calloc((size_t)cmax, sizeof(double));
    /* proxy: rounding of y (through W^2), of W_fc (times y^2), of the sum, of x~ */
    double *vy = (double *)malloc(sizeof(double) * M), *y2 = (double *)malloc(sizeof(double) * M);
    for (int m = 0; m < M; ++m) { vy[m] = q_var(yb[m], qs->y); y2[m] = yq[m] * yq[m]; }
    orc_proxy(wfc2, vy, t1, 1, M, N);
    orc_proxy(wfcc, y2, t2, 1, M, N);
    for (int p = 0; p < N; ++p) V[p] = t1[p] + t2[p];
    free(vy); free(y2);
  }
  for (int p = 0; p < N; ++p) {
    double v = q_value(a[0][p], qs->xt);
    if (var) V[p] += q_var(a[0][p], qs->xt);
    a[0][p] = v;
  }
  for (int l = 0; l < net->L; ++l) {
    const int relu = (l < net->L - 1) || net->relu_last;
    const int Cin = net->C[l], Cout = net->C[l + 1], k = net->k[l];
    const long no = (long)Cout * N;
    orc_conv_layer(a[l], Cin, n1, n2, wq[l], Cout, k, b[l], net->bias_full, relu, z[l], a[l + 1]);
    if (var) {
      /* Vz = W^2 * V + (var(W) + c W^2) * a^2 */
      for (long i = 0; i < (long)Cin * N; ++i) sq[i] = a[l][i] * a[l][i];
      orc_conv_layer(V, Cin, n1, n2, w2[l], Cout, k, zero, 0, 0, NULL, t1);
      orc_conv_layer(sq, Cin, n1, n2, wc[l], Cout, k, zero, 0, 0, NULL, t2);
      for (long i = 0; i < no; ++i) Vn[i] = (relu && !(a[l + 1][i] > 0.0)) ? 0.0 : t1[i] + t2[i];
    }
    for (long i = 0; i < no; ++i) {
      double v = q_value(a[l + 1][i], qs->a[l]);
      if (var) Vn[i] += q_var(a[l + 1][i], qs->a[l]);
      a[l + 1][i] = v;
    }
    if (var) { double *t = V; V = Vn; Vn = t; }
  }
  if (var) {
    memcpy(var, V, sizeof(double) * N);
    free(V); free(Vn); free(t1); free(t2); free(sq); free(zero);
  }
  free(yq);
}

void orc_forward_q(const orc_net *net, const double *wfc, const double *const *w,
                   const double *const *b, const double *y, int B, const orc_quant *qs,
                   double *xhat, double *sigma) {
  const int N = net->n1 * net->n2, M = net->M, L = net->L;
  const long per = orc_acts_per_image(net);
  /* rounded weights and, for the error model, their squares W^2 and the variances
   * var(W) + c W^2 of each product's weight rounding and accumulation step (c from
   * acc_var_coeff for the layer's number of terms) */
  const long nfc = (long)N * M;
  double *wfcq = (double *)malloc(sizeof(double) * nfc);
  double *wfc2 = sigma ? (double *)malloc(sizeof(double) * nfc) : NULL;
  double *wfcc = sigma ? (double *)malloc(sizeof(double) * nfc) : NULL;
  const double cfc = acc_var_coeff(qs->acc_fp32, M);
  for (long i = 0; i < nfc; ++i) {
    wfcq[i] = q_value(wfc[i], qs->wfc);
    if (sigma) { wfc2[i] = wfcq[i] * wfcq[i]; wfcc[i] = q_var(wfc[i], qs->wfc) + cfc * wfc2[i]; }
  }
  double *wq[8], *w2[8], *wc[8];
  for (int l = 0; l < L; ++l) {
    const long nw = (long)net->C[l + 1] * net->C[l] * net->k[l] * net->k[l];
    const double ca = acc_var_coeff(qs->acc_fp32, (long)net->C[l] * net->k[l] * net->k[l] + 1);
    wq[l] = (double *)malloc(sizeof(double) * nw);
    w2[l] = sigma ? (double *)malloc(sizeof(double) * nw) : NULL;
    wc[l] = sigma ? (double *)malloc(sizeof(double) * nw) : NULL;
    for (long i = 0; i < nw; ++i) {
      wq[l][i] = q_value(w[l][i], qs->w[l]);
      if (sigma) { w2[l][i] = wq[l][i] * wq[l][i]; wc[l][i] = q_var(w[l][i], qs->w[l]) + ca * w2[l][i]; }
    }
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int bi = 0; bi < B; ++bi) {
    double *act = (double *)malloc(sizeof(double) * per);
    double *var = sigma ? (double *)malloc(sizeof(double) * N) : NULL;
    forward_one_q(net, wfcq, wfc2, wfcc, (const double *const *)wq, (const double *const *)w2,
                  (const double *const *)wc, b, y + (long)bi * M, qs, act, var);
    double *a[9], *z[8];
    acts_layout(net, act, a, z);
    memcpy(xhat + (long)bi * N, a[L], sizeof(double) * N);
    if (sigma)
      for (int p = 0; p < N; ++p) sigma[(long)bi * N + p] = sqrt(var[p]);
    free(var);
    free(act);
  }
  for (int l = 0; l < L; ++l) { free(wq[l]); free(w2[l]); free(wc[l]); }
  free(wfcq);
  free(wfc2);
  free(wfcc);
}

/* ------------------------------------------------------------- Sec. 4 loss */
double orc_loss(const double *xhat, const double *x, int B, int N, double *g) {
  double L = 0.0;
  for (int b = 0; b < B; ++b) {
    double s = 0.0;
    for (int p = 0; p < N; ++p) {
      double d = xhat[(long)b * N + p] - x[(long)b * N + p];
      s += d * d;
      if (g) g[(long)b * N + p] = 2.0 * d / B;
    }
    L += s;
  }
  return L / B;
}

static long nparams_w(const orc_net *net, int l) {
  return (long)net->C[l + 1] * net->C[l] * net->k[l] * net->k[l];
}
static long nparams_b(const orc_net *net, int l) {
  return net->bias_full ? net->C[l + 1] * full_size(net, l) : net->C[l + 1];
}

/* Backpropagation of L through Eq. (1) for one image: accumulates into gw, gb,
 * optionally gwfc, and writes gyb.  g_out = dL/dxhat for this image. */
static void backward_one(const orc_net *net, const double *wfc, const double *const *w,
                         const double *yb, const double *act, const double *g_out,
                         double *const *gw, double *const *gb, double *gyb, double *gwfc) {
  const int n1 = net->n1, n2 = net->n2, N = n1 * n2;
  double *a[9], *z[8];
  acts_layout(net, (double *)act, a, z);
  double *ga = (double *)malloc(sizeof(double) * N * net->C[net->L]);
  memcpy(ga, g_out, sizeof(double) * N * net->C[net->L]);
  for (int l = net->L - 1; l >= 0; --l) {
    const int k = net->k[l], f1 = n1 + k - 1, f2 = n2 + k - 1, r = (k - 1) / 2;
    const int Cin = net->C[l], Cout = net->C[l + 1];
    const int relu = (l < net->L - 1) || net->relu_last;
    /* dL/dz on the full grid: the crop S passes gradient only to its window,
     * ReLU passes it where z > 0 (ReLU'(0) = 0) */
    double *gz = (double *)calloc((size_t)Cout * f1 * f2, sizeof(double));
    for (int co = 0; co < Cout; ++co)
      for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j) {
          long t = ((long)co * f1 + i + r) * f2 + j + r;
          double gv = ga[((long)co * n1 + i) * n2 + j];
          gz[t] = (relu && !(z[l][t] > 0.0)) ? 0.0 : gv;
        }
    /* bias */
    for (int co = 0; co < Cout; ++co)
      for (int t1 = 0; t1 < f1; ++t1)
        for (int t2 = 0; t2 < f2; ++t2) {
          double gv = gz[((long)co * f1 + t1) * f2 + t2];
          if (net->bias_full) gb[l][((long)co * f1 + t1) * f2 + t2] += gv;
          else gb[l][co] += gv;
        }
    /* weights: dz[co][t1][t2]/dw[co][ci][u][v] = in(ci, t1+u-(k-1), t2+v-(k-1)) */
    for (int co = 0; co < Cout; ++co)
      for (int ci = 0; ci < Cin; ++ci)
        for (int u = 0; u < k; ++u)
          for (int v = 0; v < k; ++v) {
            double s = 0.0;
            for (int t1 = 0; t1 < f1; ++t1) {
              int i = t1 + u - (k - 1);
              if (i < 0 || i >= n1) continue;
              for (int t2 = 0; t2 < f2; ++t2) {
                int j = t2 + v - (k - 1);
                if (j < 0 || j >= n2) continue;
                s += gz[((long)co * f1 + t1) * f2 + t2] * a[l][((long)ci * n1 + i) * n2 + j];
              }
            }
            gw[l][(((long)co * Cin + ci) * k + u) * k + v] += s;
          }
    /* input of the layer: every z[co][t1][t2] it feeds, through w[co][ci][u][v] */
    double *gin = (double *)calloc((size_t)Cin * N, sizeof(double));
    for (int ci = 0; ci < Cin; ++ci)
      for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j) {
          double s = 0.0;
          for (int co = 0; co < Cout; ++co)
            for (int u = 0; u < k; ++u)
              for (int v = 0; v < k; ++v) {
                int t1 = i + (k - 1) - u, t2 = j + (k - 1) - v;
                s += gz[((long)co * f1 + t1) * f2 + t2] *
                     w[l][(((long)co * Cin + ci) * k + u) * k + v];
              }
          gin[((long)ci * n1 + i) * n2 + j] = s;
        }
    free(gz);
    free(ga);
    ga = gin;
  }
  /* fully connected layer: xt = wfc y */
  const int M = net->M;
  if (gyb)
    for (int m = 0; m < M; ++m) {
      double s = 0.0;
      for (int p = 0; p < N; ++p) s += wfc[(long)p * M + m] * ga[p];
      gyb[m] = s;
    }
  if (gwfc)
    for (int p = 0; p < N; ++p)
      for (int m = 0; m < M; ++m) gwfc[(long)p * M + m] += ga[p] * yb[m];
  free(ga);
}

/* Sum of per-image gradient blocks in image order (deterministic). */
static void sum_private(const orc_net *net, const double *priv, long np, long nfc, int B,
                        double *const *gw, double *const *gb, double *gwfc) {
  const int L = net->L;
  for (int l = 0; l < L; ++l) {
    memset(gw[l], 0, sizeof(double) * nparams_w(net, l));
    memset(gb[l], 0, sizeof(double) * nparams_b(net, l));
  }
  if (gwfc) memset(gwfc, 0, sizeof(double) * nfc);
  for (int bi = 0; bi < B; ++bi) {
    const double *pg = priv + (long)bi * (np + nfc);
    for (int l = 0; l < L; ++l) {
      for (long q = 0; q < nparams_w(net, l); ++q) gw[l][q] += *pg++;
      for (long q = 0; q < nparams_b(net, l); ++q) gb[l][q] += *pg++;
    }
    if (gwfc)
      for (long q = 0; q < nfc; ++q) gwfc[q] += pg[q];
  }
}

static long nparams_all(const orc_net *net) {
  long np = 0;
  for (int l = 0; l < net->L; ++l) np += nparams_w(net, l) + nparams_b(net, l);
  return np;
}

static void split_private(const orc_net *net, double *pg, double **gwl, double **gbl, double **fc) {
  for (int l = 0; l < net->L; ++l) {
    gwl[l] = pg; pg += nparams_w(net, l);
    gbl[l] = pg; pg += nparams_b(net, l);
  }
  *fc = pg;
}

double orc_backward(const orc_net *net, const double *wfc, const double *const *w,
                    const double *const *b, const double *y, const double *x, int B,
                    double *const *gw, double *const *gb, double *gy, double *gwfc) {
  const int N = net->n1 * net->n2, M = net->M, L = net->L;
  const long per = orc_acts_per_image(net);
  const long np = nparams_all(net);
  const long nfc = gwfc ? (long)N * M : 0;
  /* one private gradient block per image, summed afterwards in image order */
  double *priv = (double *)calloc((size_t)B * (np + nfc), sizeof(double));
  double *sse = (double *)calloc((size_t)B, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int bi = 0; bi < B; ++bi) {
    double *act = (double *)malloc(sizeof(double) * per);
    forward_one(net, wfc, w, b, y + (long)bi * M, act);
    double *a[9], *z[8];
    acts_layout(net, act, a, z);
    double *g = (double *)malloc(sizeof(double) * N);
    double s = 0.0;
    for (int p = 0; p < N; ++p) {
      double d = a[L][p] - x[(long)bi * N + p];
      s += d * d;
      g[p] = 2.0 * d / B;     /* dL/dxhat with L = (1/B) sum_b ||xhat_b - x_b||^2 */
    }
    sse[bi] = s;
    double *gwl[8], *gbl[8], *fc;
    split_private(net, priv + (long)bi * (np + nfc), gwl, gbl, &fc);
    backward_one(net, wfc, w, y + (long)bi * M, act, g, gwl, gbl,
                 gy ? gy + (long)bi * M : NULL, gwfc ? fc : NULL);
    free(g);
    free(act);
  }
  sum_private(net, priv, np, nfc, B, gw, gb, gwfc);
  double loss = 0.0;
  for (int bi = 0; bi < B; ++bi) loss += sse[bi];
  free(priv);
  free(sse);
  return loss / B;
}

void orc_backward_acts(const orc_net *net, const double *wfc, const double *const *w,
                       const double *y, const double *acts, const double *g_out, int B,
                       double *const *gw, double *const *gb, double *gy, double *gwfc) {
  const int N = net->n1 * net->n2, M = net->M, L = net->L;
  const long per = orc_acts_per_image(net);
  long given = 0;
  for (int l = 0; l <= L; ++l) given += (long)net->C[l] * N;
  const long np = nparams_all(net);
  const long nfc = gwfc ? (long)N * M : 0;
  double *priv = (double *)calloc((size_t)B * (np + nfc), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
  for (int bi = 0; bi < B; ++bi) {
    /* activation block of backward_one: a_0..a_L as given; z_l = a_l inside the crop
     * window (a > 0 exactly where z > 0 for a ReLU layer), 0 on the borders, which
     * receive no gradient */
    double *act = (double *)calloc((size_t)per, sizeof(double));
    double *a[9], *z[8];
    acts_layout(net, act, a, z);
    memcpy(a[0], acts + (long)bi * given, sizeof(double) * given);
    for (int l = 0; l < L; ++l) {
      const int k = net->k[l], f2 = net->n2 + k - 1, r = (k - 1) / 2, f1 = net->n1 + k - 1;
      for (int c = 0; c < net->C[l + 1]; ++c)
        for (int i = 0; i < net->n1; ++i)
          for (int j = 0; j < net->n2; ++j)
            z[l][((long)c * f1 + i + r) * f2 + j + r] = a[l + 1][((long)c * net->n1 + i) * net->n2 + j];
    }
    double *gwl[8], *gbl[8], *fc;
    split_private(net, priv + (long)bi * (np + nfc), gwl, gbl, &fc);
    backward_one(net, wfc, w, y + (long)bi * M, act, g_out + (long)bi * N * net->C[L], gwl, gbl,
                 gy ? gy + (long)bi * M : NULL, gwfc ? fc : NULL);
    free(act);
  }
  sum_private(net, priv, np, nfc, B, gw, gb, gwfc);
  free(priv);
}

/* ------------------------------------------------------ Adam (Kingma & Ba) */
void orc_adam(double *theta, const double *g, double *m, double *v, long n, long t,
              double lr, double beta1, double beta2, double eps) {
  const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
  for (long q = 0; q < n; ++q) {
    m[q] = beta1 * m[q] + (1.0 - beta1) * g[q];
    v[q] = beta2 * v[q] + (1.0 - beta2) * g[q] * g[q];
    double mh = m[q] / c1, vh = v[q] / c2;
    theta[q] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ----------------------------------------------------------- Sec. 5 metrics */
double orc_psnr(const double *xhat, const double *x, int N) {
  double peak = x[0], mse = 0.0;
  for (int p = 0; p < N; ++p) {
    if (x[p] > peak) peak = x[p];
    double d = xhat[p] - x[p];
    mse += d * d;
  }
  mse /= N;
  return 10.0 * log10(peak * peak / mse);
}

double orc_relerr(const double *a, const double *ref, int N) {
  double num = 0.0, den = 0.0;
  for (int p = 0; p < N; ++p) {
    double d = a[p] - ref[p];
    num += d * d;
    den += ref[p] * ref[p];
  }
  return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

int orc_success(const double *xhat, const double *x, int N, double thr) {
  double num = 0.0, den = 0.0;
  for (int p = 0; p < N; ++p) {
    double d = xhat[p] - x[p];
    num += d * d;
    den += x[p] * x[p];
  }
  return num / den <= thr;
}

/* --------------------------------------------- classical reference: ISTA-DCT */
void orc_dct_matrix(int n, double *C) {
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < n; ++k) {
    double a = k == 0 ? sqrt(1.0 / n) : sqrt(2.0 / n);
    for (int i = 0; i < n; ++i) C[(long)k * n + i] = a * cos(pi * (2 * i + 1) * k / (2.0 * n));
  }
}

double orc_spectral_norm(const double *phi, int M, int N, int iters) {
  double *v = (double *)malloc(sizeof(double) * N), *u = (double *)malloc(sizeof(double) * M);
  for (int n = 0; n < N; ++n) v[n] = 1.0 / sqrt((double)N) * (1.0 + 0.01 * (n % 7));
  double sigma = 0.0;
  for (int it = 0; it < iters; ++it) {
    for (int m = 0; m < M; ++m) {
      double s = 0.0;
      for (int n = 0; n < N; ++n) s += phi[(long)m * N + n] * v[n];
      u[m] = s;
    }
    double nu = 0.0;
    for (int n = 0; n < N; ++n) {
      double s = 0.0;
      for (int m = 0; m < M; ++m) s += phi[(long)m * N + n] * u[m];
      v[n] = s;
      nu += s * s;
    }
    nu = sqrt(nu);
    sigma = sqrt(nu);      /* ||Phi^T Phi v|| -> sigma^2 for unit v */
    for (int n = 0; n < N; ++n) v[n] /= nu;
  }
  free(v);
  free(u);
  return sigma;
}

/* X = C1^T S C2 (inverse 2-D DCT) */
static void idct2(const double *C1, const double *C2, int n1, int n2, const double *S,
                  double *X, double *tmp) {
  for (int a = 0; a < n1; ++a)   /* tmp = S C2 : [n1][n2] */
    for (int j = 0; j < n2; ++j) {
      double s = 0.0;
      for (int q = 0; q < n2; ++q) s += S[a * n2 + q] * C2[q * n2 + j];
      tmp[a * n2 + j] = s;
    }
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n2; ++j) {
      double s = 0.0;
      for (int a = 0; a < n1; ++a) s += C1[a * n1 + i] * tmp[a * n2 + j];
      X[i * n2 + j] = s;
    }
}

/* S = C1 X C2^T (forward 2-D DCT) */
static void dct2(const double *C1, const double *C2, int n1, int n2, const double *X,
                 double *S, double *tmp) {
  for (int i = 0; i < n1; ++i)   /* tmp = X C2^T */
    for (int b = 0; b < n2; ++b) {
      double s = 0.0;
      for (int j = 0; j < n2; ++j) s += X[i * n2 + j] * C2[b * n2 + j];
      tmp[i * n2 + b] = s;
    }
  for (int a = 0; a < n1; ++a)
    for (int b = 0; b < n2; ++b) {
      double s = 0.0;
      for (int i = 0; i < n1; ++i) s += C1[a * n1 + i] * tmp[i * n2 + b];
      S[a * n2 + b] = s;
    }
}

/* Cholesky solve of the SPD system G z = h (n x n), in place. Returns 0 on success. */
static int chol_solve(double *G, double *h, int n) {
  for (int j = 0; j < n; ++j) {
    double d = G[j * n + j];
    for (int q = 0; q < j; ++q) d -= G[j * n + q] * G[j * n + q];
    if (!(d > 0.0)) return -1;
    d = sqrt(d);
    G[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = G[i * n + j];
      for (int q = 0; q < j; ++q) s -= G[i * n + q] * G[j * n + q];
      G[i * n + j] = s / d;
    }
  }
  for (int i = 0; i < n; ++i) {      /* L w = h */
    double s = h[i];
    for (int q = 0; q < i; ++q) s -= G[i * n + q] * h[q];
    h[i] = s / G[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) { /* L^T z = w */
    double s = h[i];
    for (int q = i + 1; q < n; ++q) s -= G[q * n + i] * h[q];
    h[i] = s / G[i * n + i];
  }
  return 0;
}

/* Least-squares debias of one ISTA result on its support {|s_j| > 1e-6 max|s|}
 * (in place on s, when the support has at most M elements and its Gram matrix is
 * positive definite), then the image x = Psi s.  Returns the support size. */
static int ista_debias(const double *phi, const double *y, int M, int n1, int n2, const double *C1,
                       const double *C2, double *s, double *x) {
  const int N = n1 * n2;
  double *img = (double *)malloc(sizeof(double) * N), *tmp = (double *)malloc(sizeof(double) * N);
  double smax = 0.0;
  for (int n = 0; n < N; ++n) smax = fabs(s[n]) > smax ? fabs(s[n]) : smax;
  int *sup = (int *)malloc(sizeof(int) * N);
  int ns = 0;
  for (int n = 0; n < N; ++n)
    if (smax > 0.0 && fabs(s[n]) > 1e-6 * smax) sup[ns++] = n;
  if (ns > 0 && ns <= M) {
    double *AS = (double *)malloc(sizeof(double) * (long)M * ns);
    double *G = (double *)malloc(sizeof(double) * (long)ns * ns);
    double *h = (double *)malloc(sizeof(double) * ns);
    double *e = (double *)calloc((size_t)N, sizeof(double));
    for (int q = 0; q < ns; ++q) {                     /* column q of A: Phi idct2(e_q) */
      e[sup[q]] = 1.0;
      idct2(C1, C2, n1, n2, e, img, tmp);
      e[sup[q]] = 0.0;
      for (int m = 0; m < M; ++m) {
        double acc = 0.0;
        for (int n = 0; n < N; ++n) acc += phi[(long)m * N + n] * img[n];
        AS[(long)m * ns + q] = acc;
      }
    }
    for (int a = 0; a < ns; ++a) {
      for (int c = 0; c < ns; ++c) {
        double acc = 0.0;
        for (int m = 0; m < M; ++m) acc += AS[(long)m * ns + a] * AS[(long)m * ns + c];
        G[a * ns + c] = acc;
      }
      double acc = 0.0;
      for (int m = 0; m < M; ++m) acc += AS[(long)m * ns + a] * y[m];
      h[a] = acc;
    }
    if (chol_solve(G, h, ns) == 0) {
      memset(s, 0, sizeof(double) * N);
      for (int q = 0; q < ns; ++q) s[sup[q]] = h[q];
    }
    free(AS); free(G); free(h); free(e);
  }
  idct2(C1, C2, n1, n2, s, x, tmp);
  free(sup); free(img); free(tmp);
  return ns;
}

/* ISTA on B measurement vectors at once.  Every image goes through exactly the
 * steps (and the order of every sum) of a single-image run; the images share only
 * the passes over Phi: the residual r_b = y_b - Phi Psi s_b and the back-projection
 * Phi^T r_b are computed for all b while a row of Phi is at hand, each sum still
 * over ascending m or n.  Y [B][M]; S, X [B][n1 n2]; supp [B] (nullable) receives
 * the debias support sizes. */
void orc_ista_dct_batch(const double *phi, const double *Y, int B, int M, int n1, int n2, int stages,
                        int iters, double decay, double *S, double *X, int *supp) {
  const int N = n1 * n2;
  const int NB = 64;                                    /* columns of Phi per thread block */
  double *C1 = (double *)malloc(sizeof(double) * n1 * n1);
  double *C2 = (double *)malloc(sizeof(double) * n2 * n2);
  orc_dct_matrix(n1, C1);
  orc_dct_matrix(n2, C2);
  double *imgT = (double *)malloc(sizeof(double) * (long)N * B);   /* [N][B] */
  double *backT = (double *)malloc(sizeof(double) * (long)N * B);  /* [N][B] */
  double *resT = (double *)malloc(sizeof(double) * (long)M * B);   /* [M][B] */
  double *work = (double *)malloc(sizeof(double) * (long)3 * N * B);  /* per image: img, grad, tmp */
  double *lam = (double *)malloc(sizeof(double) * B);
  /* A = Phi Psi has the same spectral norm as Phi (Psi orthonormal) */
  const double sig = orc_spectral_norm(phi, M, N, 300);
  const double tau = 0.99 / (sig * sig);
  /* back-projection Phi^T v for every image: backT[n][b] = sum over ascending m */
#define ISTA_BACK(V)                                                                   \
  do {                                                                                 \
    _Pragma("omp parallel for schedule(static)")                                      \
    for (int n0 = 0; n0 < N; n0 += NB) {                                               \
      const int n1e = n0 + NB < N ? n0 + NB : N;                                       \
      for (long q = (long)n0 * B; q < (long)n1e * B; ++q) backT[q] = 0.0;              \
      for (int m = 0; m < M; ++m)                                                      \
        for (int n = n0; n < n1e; ++n) {                                               \
          const double f = phi[(long)m * N + n];                                       \
          for (int b = 0; b < B; ++b) backT[(long)n * B + b] += f * (V);               \
        }                                                                              \
    }                                                                                  \
  } while (0)
  /* lam_0 = 0.5 ||A^T y||_inf per image */
  ISTA_BACK(Y[(long)b * M + m]);
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < B; ++b) {
    double *img = work + (long)b * 3 * N, *grad = img + N, *tmp = grad + N;
    for (int n = 0; n < N; ++n) img[n] = backT[(long)n * B + b];
    dct2(C1, C2, n1, n2, img, grad, tmp);
    double l = 0.0;
    for (int n = 0; n < N; ++n) l = fabs(grad[n]) > l ? fabs(grad[n]) : l;
    lam[b] = 0.5 * l;
  }
  memset(S, 0, sizeof(double) * (long)N * B);
  for (int st = 0; st < stages; ++st) {
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(dynamic, 1)
      for (int b = 0; b < B; ++b) {                      /* image of the current coefficients */
        double *img = work + (long)b * 3 * N, *tmp = img + 2 * N;
        idct2(C1, C2, n1, n2, S + (long)b * N, img, tmp);
        for (int n = 0; n < N; ++n) imgT[(long)n * B + b] = img[n];
      }
#pragma omp parallel for schedule(static)
      for (int m = 0; m < M; ++m) {                      /* r = y - A s */
        double acc[256];
        for (int b0 = 0; b0 < B; b0 += 256) {
          const int bn = B - b0 < 256 ? B - b0 : 256;
          for (int b = 0; b < bn; ++b) acc[b] = 0.0;
          for (int n = 0; n < N; ++n) {
            const double f = phi[(long)m * N + n];
            const double *im = imgT + (long)n * B + b0;
            for (int b = 0; b < bn; ++b) acc[b] += f * im[b];
          }
          for (int b = 0; b < bn; ++b) resT[(long)m * B + b0 + b] = Y[(long)(b0 + b) * M + m] - acc[b];
        }
      }
      ISTA_BACK(resT[(long)m * B + b]);                  /* A^T r (before the DCT) */
#pragma omp parallel for schedule(dynamic, 1)
      for (int b = 0; b < B; ++b) {
        double *img = work + (long)b * 3 * N, *grad = img + N, *tmp = grad + N;
        double *s = S + (long)b * N;
        for (int n = 0; n < N; ++n) img[n] = backT[(long)n * B + b];
        dct2(C1, C2, n1, n2, img, grad, tmp);
        const double thr = lam[b] * tau;
        for (int n = 0; n < N; ++n) {                    /* soft thresholding */
          double v = s[n] + tau * grad[n];
          s[n] = v > thr ? v - thr : (v < -thr ? v + thr : 0.0);
        }
      }
    }
    for (int b = 0; b < B; ++b) lam[b] *= decay;
  }
#undef ISTA_BACK
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < B; ++b) {
    int ns = ista_debias(phi, Y + (long)b * M, M, n1, n2, C1, C2, S + (long)b * N, X + (long)b * N);
    if (supp) supp[b] = ns;
  }
  free(C1); free(C2); free(imgT); free(backT); free(resT); free(work); free(lam);
}

int orc_ista_dct(const double *phi, const double *y, int M, int n1, int n2, int stages,
                 int iters, double decay, double *s, double *x) {
  int ns = 0;
  orc_ista_dct_batch(phi, y, 1, M, n1, n2, stages, iters, decay, s, x, &ns);
  return ns;
}
