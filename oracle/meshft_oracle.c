/*
 * FP64 CPU oracle for the Fourier transform of a triangle mesh and its
 * vertex gradient.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
 * the benchmark's CPU-baseline leg call it; the product never does.  It shares
 * no code with the GPU library.
 *
 * Notation follows the paper (Sec. 4): triangle T = (v1, v2, v3), phases
 * y_p = v_p . xi, edges e_p = v_{p-1} - v_{p+1} (indices mod 3), area A_T,
 * normal N_T, edge normals w_p = e_p x N_T.
 *
 *  - Triangle transform, Eq. 7-8:  u_T(xi) = 2 A_T f_T(xi),
 *      f_T = sum_p exp(-i y_p) / ((e_{p-}.xi)(e_{p+}.xi))
 *    which is the second divided difference of exp at the nodes z_p = -i y_p
 *    (the function g of Eq. 11 taken at the vertex projections with the
 *    exponent sign of Eq. 8).
 *  - Gradient of f_T, Eq. 10:  df_T/dv_p = xi * B_p with B_p the printed
 *    five-term bracket; equivalently B_p = -i DD4(z1, z2, z3, z_p).
 *  - When two phases nearly coincide (Sec. 4.1.3) the closed forms lose
 *    accuracy; the oracle then evaluates the divided difference from its
 *    exact definition as the corner entry of exp of a bidiagonal matrix
 *    (Opitz' theorem), computed by scaling and squaring.
 *  - Surface density, Eq. 5-6 (normalised by |Lambda| in the Python layer).
 *  - Several surfaces or materials (Sec. 3.3: a weighted sum of densities;
 *    cell-cell interfaces as double membranes): every triangle carries a
 *    density weight w_T (1 when no weights are given) that multiplies its
 *    contribution; the surface normalisation becomes sum_T w_T A_T, and for
 *    the indicator density w_T is the density jump across the triangle.
 *  - Indicator density: by the divergence theorem
 *      chi(xi) = (i/|xi|^2) sum_T (xi . n_T) f_T(xi),  n_T = (v2-v1)x(v3-v1),
 *    and chi(0) = enclosed volume.  Its vertex gradient is the boundary
 *    shape derivative: d chi / d v_p |_T = n_T DD4(z1,z2,z3,z_p).
 *
 * All arithmetic is double precision; loops are plain, one frequency at a
 * time; OpenMP only splits independent frequencies across threads.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Gap below which the closed forms hand over to the matrix definition.
 * Eq. 8 loses about eps/gap^2 and Eq. 10 about eps/gap^3 in relative terms;
 * at these thresholds both stay below 1e-11. */
#define GAP3 1e-2
#define GAP4 5e-2
#define MAXN 5

/* ---- divided differences of exp via Opitz' theorem -------------------- */
/* DD[x_0..x_{n-1}] exp = (exp(Z))_{0,n-1},  Z = diag(x) + superdiagonal ones. */
static void matmul(int n, cplx A[MAXN][MAXN], cplx B[MAXN][MAXN], cplx C[MAXN][MAXN]) {
  cplx T[MAXN][MAXN];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cplx s = 0;
      for (int k = 0; k < n; ++k) s += A[i][k] * B[k][j];
      T[i][j] = s;
    }
  memcpy(C, T, sizeof(T));
}

static cplx dd_exp_matrix(const cplx* x, int n) {
  cplx mean = 0;
  for (int i = 0; i < n; ++i) mean += x[i];
  mean /= n;
  /* exp(Z) = exp(mean) exp(Z - mean I): the shift keeps the matrix small. */
  double norm = 1.0;
  for (int i = 0; i < n; ++i) {
    double a = cabs(x[i] - mean) + 1.0;
    if (a > norm) norm = a;
  }
  int s = 0;
  while (norm / ldexp(1.0, s) > 0.25) ++s;
  double scale = ldexp(1.0, -s);
  cplx A[MAXN][MAXN], E[MAXN][MAXN], P[MAXN][MAXN];
  memset(A, 0, sizeof(A));
  for (int i = 0; i < n; ++i) {
    A[i][i] = (x[i] - mean) * scale;
    if (i + 1 < n) A[i][i + 1] = scale;
  }
  /* Taylor series of exp(A), ||A|| <= 1/4: 24 terms reach 1e-30. */
  memset(E, 0, sizeof(E));
  memset(P, 0, sizeof(P));
  for (int i = 0; i < n; ++i) E[i][i] = P[i][i] = 1.0;
  for (int k = 1; k <= 24; ++k) {
    matmul(n, P, A, P);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) P[i][j] /= k;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) E[i][j] += P[i][j];
  }
  for (int k = 0; k < s; ++k) matmul(n, E, E, E);
  return cexp(mean) * E[0][n - 1];
}

/* Exported for the tests: divided difference of exp at n <= 5 complex nodes. */
void oracle_dd_exp(const double* nodes_re_im, int n, double* out_re_im) {
  cplx x[MAXN];
  for (int i = 0; i < n; ++i) x[i] = nodes_re_im[2 * i] + I * nodes_re_im[2 * i + 1];
  cplx r = dd_exp_matrix(x, n);
  out_re_im[0] = creal(r);
  out_re_im[1] = cimag(r);
}

static double min_gap3(const double y[3]) {
  double a = fabs(y[0] - y[1]), b = fabs(y[1] - y[2]), c = fabs(y[2] - y[0]);
  double m = a < b ? a : b;
  return m < c ? m : c;
}

/* f_T of Eq. 8 from the three vertex phases y_p = v_p . xi. */
static cplx tri_f(const double y[3]) {
  if (min_gap3(y) >= GAP3) {
    cplx f = 0;
    for (int p = 0; p < 3; ++p) {
      int pm = (p + 2) % 3, pp = (p + 1) % 3;
      double em = y[pp] - y[p];   /* e_{p-} . xi = y_{p+1} - y_p */
      double ep = y[p] - y[pm];   /* e_{p+} . xi = y_p - y_{p-1} */
      f += cexp(-I * y[p]) / (em * ep);
    }
    return f;
  }
  cplx z[3] = {-I * y[0], -I * y[1], -I * y[2]};
  return dd_exp_matrix(z, 3);
}

/* B_p of Eq. 10 (df_T/dv_p = xi B_p) for p = 0, 1, 2. */
static void tri_dfdv(const double y[3], cplx B[3]) {
  if (min_gap3(y) >= GAP4) {
    for (int p = 0; p < 3; ++p) {
      int pm = (p + 2) % 3, pp = (p + 1) % 3;
      double em = y[pp] - y[p];   /* e_{p-} . xi */
      double ep = y[p] - y[pm];   /* e_{p+} . xi */
      double e0 = y[pm] - y[pp];  /* e_p . xi = y_{p-1} - y_{p+1} */
      cplx Ep = cexp(-I * y[p]), Epp = cexp(-I * y[pp]), Epm = cexp(-I * y[pm]);
      B[p] = Epp / (em * em * e0) - Epm / (e0 * ep * ep) - I * Ep / (em * ep)
           + Ep / (em * em * ep) - Ep / (em * ep * ep);
    }
    return;
  }
  for (int p = 0; p < 3; ++p) {
    cplx z[4] = {-I * y[0], -I * y[1], -I * y[2], -I * y[p]};
    B[p] = -I * dd_exp_matrix(z, 4);
  }
}

static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

typedef struct {
  double v[3][3];   /* vertices */
  double n[3];      /* (v2-v1)x(v3-v1) = 2 A_T N_T */
  double twoA;      /* 2 A_T */
  double w[3][3];   /* w_p = e_p x N_T (zero for a zero-area triangle) */
  double wt;        /* density weight of the triangle */
} tri_geom;

static void build_geom(const double* V, const int* F, int t, tri_geom* g) {
  for (int p = 0; p < 3; ++p)
    for (int j = 0; j < 3; ++j) g->v[p][j] = V[3 * F[3 * t + p] + j];
  double a[3], b[3];
  for (int j = 0; j < 3; ++j) { a[j] = g->v[1][j] - g->v[0][j]; b[j] = g->v[2][j] - g->v[0][j]; }
  cross3(a, b, g->n);
  g->twoA = sqrt(dot3(g->n, g->n));
  double N[3] = {0, 0, 0};
  if (g->twoA > 0)
    for (int j = 0; j < 3; ++j) N[j] = g->n[j] / g->twoA;
  for (int p = 0; p < 3; ++p) {
    int pm = (p + 2) % 3, pp = (p + 1) % 3;
    double e[3];
    for (int j = 0; j < 3; ++j) e[j] = g->v[pm][j] - g->v[pp][j];
    cross3(e, N, g->w[p]);
  }
}

static void phases(const tri_geom* g, const double xi[3], double y[3]) {
  for (int p = 0; p < 3; ++p) y[p] = dot3(g->v[p], xi);
}

/* Mesh transform at nk frequencies.
 * mode 0 (indicator):  chi(xi) (enclosed volume at xi = 0).
 * mode 1 (surface):    sum_T u_T(xi) = sum_T 2 A_T f_T  (not yet divided by |Lambda|).
 * Each triangle's term is multiplied by tri_w[t] (tri_w NULL: by 1).
 * V: [nv][3] positions relative to the grid origin; F: [nt][3]; xi: [nk][3]. */
void oracle_mesh_ft(int mode, const double* V, int nv, const int* F, int nt, const double* tri_w,
                    const double* xi, int nk, double* out_re_im) {
  (void)nv;
  tri_geom* G = (tri_geom*)malloc(sizeof(tri_geom) * (size_t)(nt > 0 ? nt : 1));
  for (int t = 0; t < nt; ++t) {
    build_geom(V, F, t, &G[t]);
    G[t].wt = tri_w ? tri_w[t] : 1.0;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int k = 0; k < nk; ++k) {
    const double* x = xi + 3 * k;
    double q2 = dot3(x, x);
    cplx s = 0;
    if (mode == 0 && q2 == 0.0) {
      for (int t = 0; t < nt; ++t) s += G[t].wt * dot3(G[t].v[0], G[t].n) / 6.0;
    } else {
      for (int t = 0; t < nt; ++t) {
        double y[3];
        phases(&G[t], x, y);
        cplx f = tri_f(y);
        s += G[t].wt * (mode == 0 ? dot3(x, G[t].n) : G[t].twoA) * f;
      }
      if (mode == 0) s *= I / q2;
    }
    out_re_im[2 * k] = creal(s);
    out_re_im[2 * k + 1] = cimag(s);
  }
  free(G);
}

/* Vertex gradient of L = sum_k Re[ W_k * u(xi_k) ] where u is
 *   mode 0: chi(xi);   mode 1: the normalised surface transform of Eq. 5;
 *   mode 2: the unnormalised surface transform sum_T 2 A_T f_T (Eq. 9 alone,
 *           the triangle terms of Eq. 6 without the 1/|Lambda| factor and
 *           without the normalisation term).
 * For mode 1 the normalisation term of Eq. 6 needs u at every xi_k, which the
 * routine evaluates itself.  With density weights (tri_w, NULL for 1) the
 * transforms are the weighted sums of oracle_mesh_ft and mode 1 divides by
 * sum_T w_T A_T.  dV: [nv][3], overwritten. */
void oracle_mesh_ft_vjp(int mode, const double* V, int nv, const int* F, int nt, const double* tri_w,
                        const double* xi, const double* W_re_im, int nk, double* dV) {
  tri_geom* G = (tri_geom*)malloc(sizeof(tri_geom) * (size_t)(nt > 0 ? nt : 1));
  double area = 0;
  for (int t = 0; t < nt; ++t) {
    build_geom(V, F, t, &G[t]);
    G[t].wt = tri_w ? tri_w[t] : 1.0;
    area += G[t].wt * 0.5 * G[t].twoA;
  }
  memset(dV, 0, sizeof(double) * 3 * (size_t)nv);
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  double* acc = (double*)calloc((size_t)nthreads * 3 * (size_t)nv, sizeof(double));
  cplx* fbuf = (cplx*)malloc(sizeof(cplx) * (size_t)nthreads * (size_t)(nt > 0 ? nt : 1));
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* a = acc + (size_t)tid * 3 * nv;
    cplx* fT = fbuf + (size_t)tid * nt;
#pragma omp for schedule(dynamic, 16)
    for (int k = 0; k < nk; ++k) {
      const double* x = xi + 3 * k;
      cplx W = W_re_im[2 * k] + I * W_re_im[2 * k + 1];
      if (mode == 0) {
        for (int t = 0; t < nt; ++t) {
          double y[3];
          cplx B[3];
          phases(&G[t], x, y);
          tri_dfdv(y, B);
          for (int p = 0; p < 3; ++p) {
            /* DD4_p = i B_p ;  d chi / d v_p = n_T DD4_p */
            double r = G[t].wt * creal(W * (I * B[p]));
            int v = F[3 * t + p];
            for (int j = 0; j < 3; ++j) a[3 * v + j] += r * G[t].n[j];
          }
        }
      } else if (mode == 2) {
        /* Eq. 9: du_T/dv_p = -f_T w_p + 2 A_T df_T/dv_p, summed over the triangles. */
        for (int t = 0; t < nt; ++t) {
          double y[3];
          cplx B[3];
          phases(&G[t], x, y);
          const cplx f = tri_f(y);
          tri_dfdv(y, B);
          for (int p = 0; p < 3; ++p) {
            int v = F[3 * t + p];
            for (int j = 0; j < 3; ++j) {
              cplx duT = -f * G[t].w[p][j] + G[t].twoA * x[j] * B[p];
              a[3 * v + j] += G[t].wt * creal(W * duT);
            }
          }
        }
      } else {
        /* Eq. 6: du/dv = (1/|L|) ( sum_T du_T/dv - u sum_T dA_T/dv ),
         * Eq. 9: du_T/dv_p = -f_T w_p + 2 A_T df_T/dv_p,  dA_T/dv_p = -w_p/2. */
        cplx u = 0;
        for (int t = 0; t < nt; ++t) {
          double y[3];
          phases(&G[t], x, y);
          fT[t] = tri_f(y);
          u += G[t].wt * G[t].twoA * fT[t];
        }
        u /= area;
        for (int t = 0; t < nt; ++t) {
          double y[3];
          cplx B[3];
          phases(&G[t], x, y);
          tri_dfdv(y, B);
          for (int p = 0; p < 3; ++p) {
            int v = F[3 * t + p];
            for (int j = 0; j < 3; ++j) {
              cplx duT = -fT[t] * G[t].w[p][j] + G[t].twoA * x[j] * B[p];
              cplx dA = -0.5 * G[t].w[p][j];
              a[3 * v + j] += G[t].wt * creal(W * (duT - u * dA)) / area;
            }
          }
        }
      }
    }
  }
  for (int tid = 0; tid < nthreads; ++tid)
    for (int i = 0; i < 3 * nv; ++i) dV[i] += acc[(size_t)tid * 3 * nv + i];
  free(acc);
  free(fbuf);
  free(G);
}

/* Indicator transform by an independent decomposition (for the checks):
 * the region is the union of signed cones from a point c to every face, and
 * the transform of the tetrahedron (c, v1, v2, v3) is
 *   det[v1-c, v2-c, v3-c] * DD4(z_c, z_1, z_2, z_3)  (Hermite-Genocchi),
 * evaluated here by the matrix definition for every frequency. */
void oracle_cone_volume_ft(const double* V, int nv, const int* F, int nt, const double* c,
                           const double* xi, int nk, double* out_re_im) {
  (void)nv;
#pragma omp parallel for schedule(dynamic, 16)
  for (int k = 0; k < nk; ++k) {
    const double* x = xi + 3 * k;
    cplx s = 0;
    for (int t = 0; t < nt; ++t) {
      double d[3][3];
      for (int p = 0; p < 3; ++p)
        for (int j = 0; j < 3; ++j) d[p][j] = V[3 * F[3 * t + p] + j] - c[j];
      double cr[3];
      cross3(d[1], d[2], cr);
      double det = dot3(d[0], cr);
      cplx z[4] = {0, -I * dot3(d[0], x), -I * dot3(d[1], x), -I * dot3(d[2], x)};
      s += det * dd_exp_matrix(z, 4);
    }
    s *= cexp(-I * dot3(c, x));
    out_re_im[2 * k] = creal(s);
    out_re_im[2 * k + 1] = cimag(s);
  }
}

/* Single-triangle entry points for the checks: f_T and B_p from three phases. */
void oracle_tri_f(const double* y, double* out_re_im) {
  cplx f = tri_f(y);
  out_re_im[0] = creal(f);
  out_re_im[1] = cimag(f);
}

void oracle_tri_dfdv(const double* y, double* out_re_im) {
  cplx B[3];
  tri_dfdv(y, B);
  for (int p = 0; p < 3; ++p) {
    out_re_im[2 * p] = creal(B[p]);
    out_re_im[2 * p + 1] = cimag(B[p]);
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of later parallel regions (for timing the oracle on fewer cores). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
