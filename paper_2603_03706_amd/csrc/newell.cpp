// Host-side setup of the demag kernel: cell-averaged tensor in FP64 and its
// spectrum on the zero-padded grid (real, stored on one octant in FP32).
//
// Tensor of two uniformly magnetised cuboids averaged over the target cell:
//   N_ab(R) = 1/(4 pi V) Int_{[-d,d]^3} prod_c (d_c - |s_c|) K_ab(R + s) ds,
//   K_ab(r) = (delta_ab r^2 - 3 r_a r_b) / r^5.
// Below |R| = 10 max(d) it is the closed form of Newell, Williams & Dunlop
// (1993): the second difference over 27 points of their f and g functions,
// evaluated in 80-bit long double, since the difference cancels about
// (|R| / min d)^6 of the magnitude of its terms.  From 10 cells on, the
// averaged kernel is expanded about R: with s distributed as the normalised
// weight prod_c (d_c - |s_c|) / d_c^2 (independent triangles on [-d_c, d_c]),
//   N_ab(R) = V / (4 pi) E[K_ab(R + s)],
// and, with e = R/|R|, sigma = s/|R|, u = e + sigma, t = 2 e.sigma + |sigma|^2,
//   K_ab(R + s) = |R|^-3 (delta_ab (1 + t) - 3 u_a u_b) (1 + t)^(-5/2),
// taken as a power series in sigma truncated at total degree 10, whose
// expectation uses the triangle's moments E[s^2m] = 2 d^2m / ((2m+1)(2m+2))
// (odd ones vanish).
// Truncation error ~ (max d / |R|)^12.  Against a 60-digit evaluation of the
// closed form this is within 1e-12 relative for cells of aspect ratio up to
// 5:3 (the loss of the long-double closed form below the switch grows with
// the aspect ratio).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <thread>
#include <vector>

#include "mm_host.h"

namespace mmh {

namespace {

using LD = long double;

inline LD ratio(LD num, LD den) { return den != 0 ? num / den : 0; }

// Newell f (even in every argument)
LD nf(LD x, LD y, LD z) {
  x = std::fabs(x);
  y = std::fabs(y);
  z = std::fabs(z);
  const LD xx = x * x, yy = y * y, zz = z * z, r = std::sqrt(xx + yy + zz);
  LD v = (2 * xx - yy - zz) * r / 6;
  if (y > 0) v += y * (zz - xx) / 2 * std::asinh(ratio(y, std::sqrt(xx + zz)));
  if (z > 0) v += z * (yy - xx) / 2 * std::asinh(ratio(z, std::sqrt(xx + yy)));
  if (x > 0) v -= x * y * z * std::atan(ratio(y * z, x * r));
  return v;
}

// Newell g (odd in x and y, even in z)
LD ng(LD x, LD y, LD z) {
  const int sgn = ((x > 0) - (x < 0)) * ((y > 0) - (y < 0));
  if (sgn == 0) return 0;
  x = std::fabs(x);
  y = std::fabs(y);
  z = std::fabs(z);
  const LD xx = x * x, yy = y * y, zz = z * z, r = std::sqrt(xx + yy + zz);
  LD v = -x * y * r / 3;
  v += x * y * z * std::asinh(ratio(z, std::sqrt(xx + yy)));
  v += y * (3 * zz - yy) / 6 * std::asinh(ratio(x, std::sqrt(yy + zz)));
  v += x * (3 * zz - xx) / 6 * std::asinh(ratio(y, std::sqrt(xx + zz)));
  if (z > 0) {
    v -= zz * z / 6 * std::atan(ratio(x * y, z * r));
    v -= z * yy / 2 * std::atan(ratio(x * z, y * r));
    v -= z * xx / 2 * std::atan(ratio(y * z, x * r));
  }
  return sgn * v;
}

// weights (-1, 2, -1) along each axis over the 27 neighbouring arguments, / (4 pi V)
template <class F>
double second_diff(F fn, LD X, LD Y, LD Z, LD a, LD b, LD c) {
  static const LD w[3] = {-1, 2, -1};
  LD acc = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) acc += w[i] * w[j] * w[k] * fn(X + (i - 1) * a, Y + (j - 1) * b, Z + (k - 1) * c);
  return (double)(acc / (4 * 3.141592653589793238462643383279502884L * a * b * c));
}

void closed_form(double X, double Y, double Z, double dx, double dy, double dz, double* o) {
  o[0] = second_diff(nf, X, Y, Z, dx, dy, dz);
  o[1] = second_diff(nf, Y, X, Z, dy, dx, dz);
  o[2] = second_diff(nf, Z, Y, X, dz, dy, dx);
  o[3] = second_diff(ng, X, Y, Z, dx, dy, dz);
  o[4] = second_diff(ng, X, Z, Y, dx, dz, dy);
  o[5] = second_diff(ng, Y, Z, X, dy, dz, dx);
}

// Truncated power series in (s_x, s_y, s_z) of total degree <= kDeg;
// c[i][j][k] is the coefficient of s_x^i s_y^j s_z^k.
constexpr int kDeg = 10;
struct Series {
  double c[kDeg + 1][kDeg + 1][kDeg + 1];
  Series() { std::memset(c, 0, sizeof(c)); }
};

void expansion(double X, double Y, double Z, double dx, double dy, double dz, double* o) {
  const double R = std::sqrt(X * X + Y * Y + Z * Z);
  const double e[3] = {X / R, Y / R, Z / R}, h[3] = {dx / R, dy / R, dz / R};
  // t = 2 e.s + |s|^2 (s in units of |R|): r^2 = |R|^2 (1 + t)
  static const int tp[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}};
  const double tc[6] = {2 * e[0], 2 * e[1], 2 * e[2], 1.0, 1.0, 1.0};
  // P = (1 + t)^(-5/2) = sum_k C(-5/2, k) t^k
  Series P, tk;
  P.c[0][0][0] = 1;
  tk.c[0][0][0] = 1;
  double bin = 1;
  for (int k = 1; k <= kDeg; ++k) {
    Series nx;
    for (int i = 0; i <= kDeg; ++i)
      for (int j = 0; i + j <= kDeg; ++j)
        for (int l = 0; i + j + l <= kDeg; ++l) {
          const double v = tk.c[i][j][l];
          if (v == 0) continue;
          for (int m = 0; m < 6; ++m) {
            const int a = i + tp[m][0], b = j + tp[m][1], c = l + tp[m][2];
            if (a + b + c <= kDeg) nx.c[a][b][c] += v * tc[m];
          }
        }
    tk = nx;
    bin *= (-2.5 - (k - 1)) / k;
    for (int i = 0; i <= kDeg; ++i)
      for (int j = 0; i + j <= kDeg; ++j)
        for (int l = 0; i + j + l <= kDeg; ++l) P.c[i][j][l] += bin * tk.c[i][j][l];
  }
  // moments of the triangle weight per axis (odd ones are zero)
  double mom[3][kDeg + 1];
  for (int a = 0; a < 3; ++a)
    for (int n = 0; n <= kDeg; ++n) mom[a][n] = (n & 1) ? 0.0 : 2.0 * std::pow(h[a], n) / ((n + 1.0) * (n + 2.0));
  // |R|^3 K_ab(R + s) = (delta_ab (1 + t) - 3 u_a u_b) P,  u = e + s
  static const int ca[6] = {0, 1, 2, 0, 0, 1}, cb[6] = {0, 1, 2, 1, 2, 2};
  for (int m = 0; m < 6; ++m) {
    const int a = ca[m], b = cb[m];
    // the prefactor as a list of (exponents, coefficient), at most ten terms
    int qe[12][3];
    double qc[12];
    int nq = 0;
    auto add = [&](int i, int j, int k, double v) {
      for (int q = 0; q < nq; ++q)
        if (qe[q][0] == i && qe[q][1] == j && qe[q][2] == k) {
          qc[q] += v;
          return;
        }
      qe[nq][0] = i, qe[nq][1] = j, qe[nq][2] = k, qc[nq] = v, ++nq;
    };
    if (a == b) {
      add(0, 0, 0, 1.0);
      for (int q = 0; q < 6; ++q) add(tp[q][0], tp[q][1], tp[q][2], tc[q]);
    }
    int ua[3] = {0, 0, 0}, ub[3] = {0, 0, 0};
    ua[a] = 1;
    ub[b] = 1;
    add(0, 0, 0, -3 * e[a] * e[b]);
    add(ub[0], ub[1], ub[2], -3 * e[a]);
    add(ua[0], ua[1], ua[2], -3 * e[b]);
    add(ua[0] + ub[0], ua[1] + ub[1], ua[2] + ub[2], -3.0);
    // expectation: only terms whose exponent on every axis is even survive
    double acc = 0;
    for (int q = 0; q < nq; ++q) {
      const int i0 = qe[q][0], j0 = qe[q][1], k0 = qe[q][2];
      for (int p = i0 & 1; i0 + p + j0 + k0 <= kDeg; p += 2)
        for (int r = j0 & 1; i0 + p + j0 + r + k0 <= kDeg; r += 2)
          for (int s = k0 & 1; i0 + p + j0 + r + k0 + s <= kDeg; s += 2)
            acc += qc[q] * P.c[p][r][s] * mom[0][i0 + p] * mom[1][j0 + r] * mom[2][k0 + s];
    }
    o[m] = acc * dx * dy * dz / (4.0 * M_PI * R * R * R);
  }
}

void tensor_at(double X, double Y, double Z, double dx, double dy, double dz, double* o) {
  const double rc = std::sqrt(X * X + Y * Y + Z * Z) / std::max(dx, std::max(dy, dz));
  if (rc < 10.0) closed_form(X, Y, Z, dx, dy, dz, o);
  else expansion(X, Y, Z, dx, dy, dz, o);
}

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
  tensor_at(X, Y, Z, dx, dy, dz, out6);
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
    const size_t total = (size_t)nx * ny * nz;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth; ++t)
      pool.emplace_back([&, t]() {
        double o[6];
        for (size_t q = t; q < total; q += nth) {
          const int i = (int)(q % nx), j = (int)((q / nx) % ny), k = (int)(q / ((size_t)nx * ny));
          tensor_at(i * dx, j * dy, k * dz, dx, dy, dz, o);
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
