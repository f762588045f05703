// Coefficients of the 6- and 7-product schemes (Section 2.1).
//
// 6 products: x_1..x_8 of (eq:cosm8), in closed form with sqrt(36681), and the
// rational z_0..z_8 of the sine (Algorithm6sA). They are evaluated here in
// 80-bit long double and rounded once to float64.
// 7 products: a_{i,j} of (Coefs7cA) and z_0..z_11 of (Coefs7sA), printed to
// 20 digits; the literals below are parsed with correct rounding.
#pragma once

#include <math.h>

namespace sc {

struct Coeffs {
  double x[9];      // x[1..8]
  double z6[9];     // z[0..8]
  double a[4][5];   // a[i][j], i = 0..3, j = 1..4
  double z7[12];    // z[0..11]
};

inline Coeffs make_coeffs() {
  Coeffs c{};
  const long double r = sqrtl(36681.0L);
  c.x[1] = (double)(7.0L / 500.0L);
  c.x[2] = (double)(-7.0L / 60000.0L);
  c.x[3] = (double)((-1533.0L + 7.0L * r) / 2500.0L);
  c.x[4] = (double)(-5.0L * (124581.0L + 391.0L * r) / 10594584.0L);
  c.x[5] = (double)(9775.0L / 10594584.0L);
  c.x[6] = (double)(-5.0L * (1001.0L + r) / 508540032.0L);
  c.x[7] = (double)(3125.0L / 889945056.0L);
  c.x[8] = (double)((1549211.0L + 3246.0L * r) / 63063000.0L);
  c.z6[0] = (double)(8887.0L / 4794.0L);
  c.z6[1] = (double)(-1897.0L / 3196.0L);
  c.z6[2] = (double)(25259.0L / 575280.0L);
  c.z6[3] = (double)(-965093875.0L / 9674368704.0L);
  c.z6[4] = (double)(-4093.0L / 4794.0L);
  c.z6[5] = (double)(25698275.0L / 29023106112.0L);
  c.z6[6] = (double)(-3907675.0L / 348277273344.0L);
  c.z6[7] = (double)(11865625.0L / 3656911370112.0L);
  c.z6[8] = (double)(25.0L / 308756448.0L);
  // a[i][j]: coefficient of A_{2i} in C_j
  c.a[0][1] = 0.0;
  c.a[1][1] = 0.0;
  c.a[2][1] = 0.02264979811206039519;
  c.a[3][1] = -0.00013110924142135755;
  c.a[0][2] = 0.55751443809990408029;
  c.a[1][2] = -0.61577924683458386455;
  c.a[2][2] = 0.00747198841446687051;
  c.a[3][2] = -0.00003362444420476012;
  c.a[0][3] = 0.75936877868464999248;
  c.a[1][3] = -0.01560333979813817129;
  c.a[2][3] = 0.00010936989591908396;
  c.a[3][3] = -1.03893360877457159499e-6;
  c.a[0][4] = 0.0;
  c.a[1][4] = -0.039649968743474473091;
  c.a[2][4] = 0.000155490073503821463;
  c.a[3][4] = -1.126739663071170022488e-6;
  c.z7[0] = 0.10090808375109885598;
  c.z7[1] = -0.07668753546445299316;
  c.z7[2] = 0.00084924846993243257;
  c.z7[3] = -0.00001220406904464391;
  c.z7[4] = 0.98499703159318860027;
  c.z7[5] = -0.84925233648155398756;
  c.z7[6] = 1.0;
  c.z7[7] = 0.00095544138280925799;
  c.z7[8] = 4.56337109377154270633e-6;
  c.z7[9] = 2.73461259403000427141e-8;
  c.z7[10] = 0.00048550288474842477;
  c.z7[11] = -4.15891109384923342531e-7;
  return c;
}

inline const Coeffs& coeffs() {
  static const Coeffs c = make_coeffs();
  return c;
}

}  // namespace sc
