// Host-side setup of the demag kernel: cell-averaged tensor in FP64 and its
// spectrum on the zero-padded grid (real, stored on one octant in FP32).
//
// Tensor of two uniformly magnetised cuboids averaged over the target cell:
//   N_ab(R) = 1/(4 pi V) Int_{[-d,d]^3} prod_c (d_c - |s_c|) K_ab(R + s) ds,
//   K_ab(r) = (delta_ab r^2 - 3 r_a r_b) / r^5,
// evaluated in closed form (Newell, Williams & Dunlop 1993, the f and g
// functions with a 27-point second difference) below 6 cells of distance
// and by Gauss-Legendre quadrature of the integral (two panels per axis,
// 6 / 4 / 3 points per panel below 12 / below 40 / beyond, in cells) above.
#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "mm_host.h"

namespace mmh {

namespace {

inline double ratio(double num, double den) { return den != 0.0 ? num / den : 0.0; }

// Newell f (even in every argument)
double nf(double x, double y, double z) {
  x = std::fabs(x);
  y = std::fabs(y);
  z = std::fabs(z);
  const double xx = x * x, yy = y * y, zz = z * z;
  const double r = std::sqrt(xx + yy + zz);
  double s = (2.0 * xx - yy - zz) * r / 6.0;
  s += 0.5 * y * (zz - xx) * std::asinh(ratio(y, std::sqrt(xx + zz)));
  s += 0.5 * z * (yy - xx) * std::asinh(ratio(z, std::sqrt(xx + yy)));
  s -= x * y * z * std::atan(ratio(y * z, x * r));
  return s;
}

// Newell g (odd in x and y, even in z)
double ng(double x, double y, double z) {
  const double sgn = (x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0)) * (y > 0 ? 1.0 : (y < 0 ? -1.0 : 0.0));
  if (sgn == 0.0) return 0.0;
  x = std::fabs(x);
  y = std::fabs(y);
  z = std::fabs(z);
  const double xx = x * x, yy = y * y, zz = z * z;
  const double r = std::sqrt(xx + yy + zz);
  double s = -x * y * r / 3.0;
  s += x * y * z * std::asinh(ratio(z, std::sqrt(xx + yy)));
  s += y / 6.0 * (3.0 * zz - yy) * std::asinh(ratio(x, std::sqrt(yy + zz)));
  s += x / 6.0 * (3.0 * zz - xx) * std::asinh(ratio(y, std::sqrt(xx + zz)));
  s -= zz * z / 6.0 * std::atan(ratio(x * y, z * r));
  s -= z * yy / 2.0 * std::atan(ratio(x * z, y * r));
  s -= z * xx / 2.0 * std::atan(ratio(y * z, x * r));
  return sgn * s;
}

template <class F>
double second_diff(F fn, double X, double Y, double Z, double dx, double dy, double dz) {
  static const double w[3] = {-1.0, 2.0, -1.0};
  double acc = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        acc += w[i] * w[j] * w[k] * fn(X + (i - 1) * dx, Y + (j - 1) * dy, Z + (k - 1) * dz);
  return acc / (4.0 * M_PI * dx * dy * dz);
}

void exact(double X, double Y, double Z, double dx, double dy, double dz, double* o) {
  o[0] = second_diff(nf, X, Y, Z, dx, dy, dz);
  o[1] = second_diff(nf, Y, X, Z, dy, dx, dz);
  o[2] = second_diff(nf, Z, Y, X, dz, dy, dx);
  o[3] = second_diff(ng, X, Y, Z, dx, dy, dz);
  o[4] = second_diff(ng, X, Z, Y, dx, dz, dy);
  o[5] = second_diff(ng, Y, Z, X, dy, dz, dx);
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

struct HatRule {
  std::vector<double> s, w;   // nodes on [-d, d] and weights including (d - |s|)
};

HatRule hat_rule(double d, int n) {
  std::vector<double> x, w;
  legendre(n, x, w);
  HatRule r;
  for (int side = -1; side <= 1; side += 2)
    for (int i = 0; i < n; ++i) {
      const double s = 0.5 * d * (x[i] + 1.0);
      r.s.push_back(side * s);
      r.w.push_back(0.5 * d * w[i] * (d - s));
    }
  return r;
}

void far(double X, double Y, double Z, const HatRule& hx, const HatRule& hy, const HatRule& hz,
         double V, double* o) {
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (size_t a = 0; a < hx.s.size(); ++a) {
    const double rx = X + hx.s[a];
    for (size_t b = 0; b < hy.s.size(); ++b) {
      const double ry = Y + hy.s[b];
      const double wab = hx.w[a] * hy.w[b];
      for (size_t c = 0; c < hz.s.size(); ++c) {
        const double rz = Z + hz.s[c];
        const double r2 = rx * rx + ry * ry + rz * rz;
        const double q = wab * hz.w[c] / (r2 * r2 * std::sqrt(r2));
        acc[0] += q * (r2 - 3.0 * rx * rx);
        acc[1] += q * (r2 - 3.0 * ry * ry);
        acc[2] += q * (r2 - 3.0 * rz * rz);
        acc[3] -= q * 3.0 * rx * ry;
        acc[4] -= q * 3.0 * rx * rz;
        acc[5] -= q * 3.0 * ry * rz;
      }
    }
  }
  const double sc = 1.0 / (4.0 * M_PI * V);
  for (int i = 0; i < 6; ++i) o[i] = acc[i] * sc;
}

struct TensorEval {
  double dx, dy, dz, dmax, V;
  HatRule r6[3], r4[3], r3[3];
  TensorEval(double dx_, double dy_, double dz_) : dx(dx_), dy(dy_), dz(dz_) {
    dmax = std::max(dx, std::max(dy, dz));
    V = dx * dy * dz;
    const double d[3] = {dx, dy, dz};
    for (int a = 0; a < 3; ++a) {
      r6[a] = hat_rule(d[a], 6);
      r4[a] = hat_rule(d[a], 4);
      r3[a] = hat_rule(d[a], 3);
    }
  }
  void operator()(double X, double Y, double Z, double* o) const {
    const double rc = std::sqrt(X * X + Y * Y + Z * Z) / dmax;
    if (rc < 6.0) exact(X, Y, Z, dx, dy, dz, o);
    else if (rc < 12.0) far(X, Y, Z, r6[0], r6[1], r6[2], V, o);
    else if (rc < 40.0) far(X, Y, Z, r4[0], r4[1], r4[2], V, o);
    else far(X, Y, Z, r3[0], r3[1], r3[2], V, o);
  }
};

// in-place radix-2 complex FFT (forward), power-of-two n, stride s
void fft1d(std::complex<double>* a, int n, int s, std::vector<std::complex<double>>& tmp,
           const std::vector<std::complex<double>>& tw, int twlen) {
  if (n <= 1) return;
  tmp.resize(n);
  for (int i = 0; i < n; ++i) tmp[i] = a[(size_t)i * s];
  // bit reversal
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(tmp[i], tmp[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const int step = twlen / len;
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < len / 2; ++k) {
        const std::complex<double> w = tw[(size_t)k * step];
        const std::complex<double> u = tmp[i + k], v = tmp[i + k + len / 2] * w;
        tmp[i + k] = u + v;
        tmp[i + k + len / 2] = u - v;
      }
  }
  for (int i = 0; i < n; ++i) a[(size_t)i * s] = tmp[i];
}

}  // namespace

void demag_tensor(double X, double Y, double Z, double dx, double dy, double dz, double* out6) {
  TensorEval ev(dx, dy, dz);
  ev(X, Y, Z, out6);
}

int padded(int n) {
  if (n == 1) return 1;
  int p = 1;
  while (p < 2 * n) p *= 2;
  return p;
}

// Octant kernel spectrum: out[Px/2+1][6][Pz/2+1][Py/2+1] (float), kx-major so that
// one kx plane of all six components is contiguous.
void kernel_spectrum(int nx, int ny, int nz, double dx, double dy, double dz, std::vector<float>& out) {
  const int px = padded(nx), py = padded(ny), pz = padded(nz);
  const int hx = px / 2 + 1, hy = py / 2 + 1, hz = pz / 2 + 1;
  const int kxn = (px == 1) ? 1 : hx, kyn = (py == 1) ? 1 : hy, kzn = (pz == 1) ? 1 : hz;
  // tensor on the non-negative octant of displacements
  std::vector<double> oct((size_t)6 * nx * ny * nz);
  {
    TensorEval ev(dx, dy, dz);
    const size_t total = (size_t)nx * ny * nz;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth; ++t)
      pool.emplace_back([&, t]() {
        double o[6];
        for (size_t q = t; q < total; q += nth) {
          const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((size_t)nx * ny));
          ev(i * dx, j * dy, k * dz, o);
          for (int c = 0; c < 6; ++c) oct[(size_t)c * total + q] = o[c];
        }
      });
    for (auto& th : pool) th.join();
  }
  // mirror to the padded grid with exact parity and transform each component
  const size_t np = (size_t)px * py * pz;
  std::vector<std::complex<double>> tw(1024);
  for (int m = 0; m < 1024; ++m) tw[m] = std::polar(1.0, -2.0 * M_PI * m / 1024.0);
  out.assign((size_t)6 * kzn * kyn * kxn, 0.0f);
  // parity of each component in (x, y, z): +1 even, -1 odd
  static const int par[6][3] = {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}, {-1, -1, 1}, {-1, 1, -1}, {1, -1, -1}};
  std::vector<std::complex<double>> buf(np);
  for (int c = 0; c < 6; ++c) {
    std::fill(buf.begin(), buf.end(), std::complex<double>(0.0, 0.0));
    for (int k = -(nz - 1); k < nz; ++k)
      for (int j = -(ny - 1); j < ny; ++j)
        for (int i = -(nx - 1); i < nx; ++i) {
          const int ai = std::abs(i), aj = std::abs(j), ak = std::abs(k);
          double v = oct[(size_t)c * nx * ny * nz + ((size_t)ak * ny + aj) * nx + ai];
          if (i < 0) v *= par[c][0];
          if (j < 0) v *= par[c][1];
          if (k < 0) v *= par[c][2];
          const int ii = (i + px) % px, jj = (j + py) % py, kk = (k + pz) % pz;
          buf[((size_t)kk * py + jj) * px + ii] = v;
        }
    std::vector<std::complex<double>> tmp;
    for (int k = 0; k < pz; ++k)
      for (int j = 0; j < py; ++j) fft1d(&buf[((size_t)k * py + j) * px], px, 1, tmp, tw, 1024);
    for (int k = 0; k < pz; ++k)
      for (int i = 0; i < px; ++i) fft1d(&buf[(size_t)k * py * px + i], py, px, tmp, tw, 1024);
    for (int j = 0; j < py; ++j)
      for (int i = 0; i < px; ++i) fft1d(&buf[(size_t)j * px + i], pz, px * py, tmp, tw, 1024);
    for (int k = 0; k < kzn; ++k)
      for (int j = 0; j < kyn; ++j)
        for (int i = 0; i < kxn; ++i)
          out[(((size_t)i * 6 + c) * kzn + k) * kyn + j] =
              (float)buf[((size_t)k * py + j) * px + i].real();
  }
}

}  // namespace mmh
