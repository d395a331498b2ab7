/* Host sanitizer harness of the FP64 oracle (oracle/meshft_oracle.c), built
 * with it alone under -fsanitize=address,undefined by
 * tests/test_sanitize_cpu.py.  Calls every exported routine on small inputs
 * (near-coincident and repeated phases, the axis-aligned box whose edges make
 * every degenerate branch fire, a mesh without triangles, weights, the
 * origin frequency) and checks the results against closed forms the oracle's
 * own tests pin: the box transform is a product of sincs and its value at
 * xi = 0 the volume; the cone decomposition equals the divergence form.
 * Exit status 0 iff every check holds. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_dd_exp(const double* nodes_re_im, int n, double* out_re_im);
void oracle_tri_f(const double* y, double* out_re_im);
void oracle_tri_dfdv(const double* y, double* out_re_im);
void oracle_mesh_ft(int mode, const double* V, int nv, const int* F, int nt, const double* tri_w,
                    const double* xi, int nk, double* out_re_im);
void oracle_mesh_ft_vjp(int mode, const double* V, int nv, const int* F, int nt, const double* tri_w,
                        const double* xi, const double* W_re_im, int nk, double* dV);
void oracle_cone_volume_ft(const double* V, int nv, const int* F, int nt, const double* c,
                           const double* xi, int nk, double* out_re_im);
void oracle_set_num_threads(int n);

static int g_fail = 0;
#define EXPECT(c)                                                          \
  do {                                                                     \
    if (!(c)) {                                                            \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                            \
    }                                                                      \
  } while (0)

static int finite_all(const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i])) return 0;
  return 1;
}

static double sinc(double x) { return fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : sin(x) / x; }

/* box [a, b] as 12 triangles, outward orientation */
static void box_mesh(const double a[3], const double b[3], double V[24], int F[36]) {
  for (int c = 0; c < 8; ++c) {
    V[3 * c] = (c & 1) ? b[0] : a[0];
    V[3 * c + 1] = (c & 2) ? b[1] : a[1];
    V[3 * c + 2] = (c & 4) ? b[2] : a[2];
  }
  static const int f[36] = {0, 2, 3, 0, 3, 1, 4, 5, 7, 4, 7, 6, 0, 1, 5, 0, 5, 4,
                            2, 6, 7, 2, 7, 3, 0, 4, 6, 0, 6, 2, 1, 3, 7, 1, 7, 5};
  for (int i = 0; i < 36; ++i) F[i] = f[i];
}

static void test_divided_differences(void) {
  /* repeated and nearly repeated imaginary nodes: DD of exp, n = 1..5 */
  double gaps[] = {1.0, 1e-1, 1e-3, 1e-6, 1e-12, 0.0};
  for (int n = 1; n <= 5; ++n)
    for (int gi = 0; gi < 6; ++gi) {
      double nodes[10], out[2];
      for (int k = 0; k < n; ++k) {
        nodes[2 * k] = 0.0;
        nodes[2 * k + 1] = -(0.7 + gaps[gi] * k);
      }
      oracle_dd_exp(nodes, n, out);
      EXPECT(finite_all(out, 2));
      /* |DD_{n-1}| of exp on the imaginary axis is at most 1/(n-1)! */
      double fact = 1.0;
      for (int k = 2; k < n; ++k) fact *= k;
      EXPECT(hypot(out[0], out[1]) <= 1.0 / fact + 1e-12);
    }
  /* f_T and its derivatives across the switch to the matrix definition */
  double ys[][3] = {{0.1, 2.0, -1.3}, {0.5, 0.5 + 1e-9, 0.5 - 1e-9}, {3.0, 3.0, 3.0}, {0.0, 0.0, 7.0},
                    {100.0, -100.0, 0.01}, {1e-3, 2e-3, 3e-3}};
  for (int i = 0; i < 6; ++i) {
    double f[2], B[6];
    oracle_tri_f(ys[i], f);
    oracle_tri_dfdv(ys[i], B);
    EXPECT(finite_all(f, 2) && finite_all(B, 6));
    EXPECT(hypot(f[0], f[1]) <= 0.5 + 1e-12);
  }
  {
    /* all three phases equal: f = e^{-i y} / 2 */
    double y[3] = {3.0, 3.0, 3.0}, f[2];
    oracle_tri_f(y, f);
    EXPECT(fabs(f[0] - 0.5 * cos(3.0)) < 1e-14 && fabs(f[1] + 0.5 * sin(3.0)) < 1e-14);
  }
}

static void test_box(void) {
  const double a[3] = {0.3, -0.2, 0.1}, b[3] = {1.5, 0.9, 2.2};
  double V[24];
  int F[36];
  box_mesh(a, b, V, F);
  enum { NK = 7 };
  /* frequencies on the coordinate planes and axes make the edge phases coincide */
  const double xi[3 * NK] = {0, 0, 0, 1.3, 0, 0, 0, -2.1, 0, 0, 0, 0.7, 1.1, 0.4, 0, 0.3, -0.8, 2.5, 40.0, 0, 0};
  double out[2 * NK], cone[2 * NK];
  oracle_mesh_ft(0, V, 8, F, 12, NULL, xi, NK, out);
  const double c[3] = {0.2, 0.1, 0.4};
  oracle_cone_volume_ft(V, 8, F, 12, c, xi, NK, cone);
  for (int k = 0; k < NK; ++k) {
    const double* x = xi + 3 * k;
    double complex want = 1.0;
    double ph = 0.0;
    for (int j = 0; j < 3; ++j) {
      const double L = b[j] - a[j];
      want *= L * sinc(0.5 * x[j] * L);
      ph += x[j] * 0.5 * (a[j] + b[j]);
    }
    want *= cexp(-I * ph);
    EXPECT(cabs(out[2 * k] + I * out[2 * k + 1] - want) < 1e-12 * (1.0 + cabs(want)));
    EXPECT(cabs(cone[2 * k] + I * cone[2 * k + 1] - want) < 1e-12 * (1.0 + cabs(want)));
  }
  /* weights of 1 change nothing; surface mode at xi = 0 is the area */
  double w[12], outw[2 * NK], surf[2];
  for (int t = 0; t < 12; ++t) w[t] = 1.0;
  oracle_mesh_ft(0, V, 8, F, 12, w, xi, NK, outw);
  for (int i = 0; i < 2 * NK; ++i) EXPECT(outw[i] == out[i]);
  oracle_mesh_ft(1, V, 8, F, 12, NULL, xi, 1, surf);
  const double L0 = b[0] - a[0], L1 = b[1] - a[1], L2 = b[2] - a[2];
  EXPECT(fabs(surf[0] - 2.0 * (L0 * L1 + L1 * L2 + L0 * L2)) < 1e-12 && fabs(surf[1]) < 1e-12);
  /* gradients in all modes, the origin frequency included */
  double W[2 * NK], dV[24];
  for (int k = 0; k < NK; ++k) {
    W[2 * k] = 0.3 + 0.1 * k;
    W[2 * k + 1] = -0.2 + 0.05 * k;
  }
  for (int mode = 0; mode <= 2; ++mode) {
    oracle_mesh_ft_vjp(mode, V, 8, F, 12, NULL, xi, W, NK, dV);
    EXPECT(finite_all(dV, 24));
    oracle_mesh_ft_vjp(mode, V, 8, F, 12, w, xi, W, NK, dV);
    EXPECT(finite_all(dV, 24));
  }
}

static void test_degenerate_meshes(void) {
  double V[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 1, 1, 0};
  const double xi[6] = {0.5, -0.3, 0.2, 0, 0, 0};
  const double W[4] = {1.0, 0.5, -0.25, 2.0};
  double out[4], dV[12];
  /* no triangles */
  oracle_mesh_ft(1, V, 4, NULL, 0, NULL, xi, 2, out);
  EXPECT(out[0] == 0.0 && out[1] == 0.0 && out[2] == 0.0 && out[3] == 0.0);
  oracle_mesh_ft_vjp(0, V, 4, NULL, 0, NULL, xi, W, 2, dV);
  for (int i = 0; i < 12; ++i) EXPECT(dV[i] == 0.0);
  /* zero-area triangles: a repeated vertex and three collinear points */
  const int F[6] = {0, 1, 1, 0, 1, 3};
  V[9] = 2.0;
  V[10] = 0.0;
  oracle_mesh_ft(1, V, 4, F, 2, NULL, xi, 2, out);
  EXPECT(finite_all(out, 4));
  EXPECT(fabs(out[0]) < 1e-15 && fabs(out[1]) < 1e-15);
  oracle_mesh_ft_vjp(2, V, 4, F, 2, NULL, xi, W, 2, dV);
  EXPECT(finite_all(dV, 12));
  /* no frequencies */
  oracle_mesh_ft(0, V, 4, F, 2, NULL, xi, 0, out);
  oracle_mesh_ft_vjp(0, V, 4, F, 2, NULL, xi, W, 0, dV);
  for (int i = 0; i < 12; ++i) EXPECT(dV[i] == 0.0);
}

int main(void) {
  oracle_set_num_threads(2);
  test_divided_differences();
  test_box();
  test_degenerate_meshes();
  if (g_fail) {
    fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  printf("oracle harness: all checks passed\n");
  return 0;
}
