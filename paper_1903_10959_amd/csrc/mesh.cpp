// Host-side construction of the GLL spectral-element tables (Sec. 2.4).
#include "mesh.hpp"

#include <algorithm>
#include <cmath>

namespace chfsi {

namespace {

// Legendre values P_{k}(x) for k = 0..kmax by Bonnet's recurrence.
void legendre_all(int kmax, double x, std::vector<double> &P) {
  P.assign(kmax + 1, 0.0);
  P[0] = 1.0;
  if (kmax >= 1) P[1] = x;
  for (int k = 1; k < kmax; ++k) P[k + 1] = ((2.0 * k + 1.0) * x * P[k] - k * P[k - 1]) / (k + 1.0);
}

}  // namespace

// GLL nodes are the zeros of (1 - x^2) P_p'(x), which is proportional to
// P_{p-1}(x) - P_{p+1}(x).  Newton's method on f = P_{p+1} - P_{p-1} uses
// f' = (2p+1) P_p.  Weights: 2 / (p (p+1) P_p(x)^2).
void gll_rule(int p, std::vector<double> &xi, std::vector<double> &w) {
  const double pi = 3.14159265358979323846;
  xi.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  std::vector<double> P;
  for (int k = 1; k < p; ++k) {
    double x = -std::cos(pi * k / p);
    for (int it = 0; it < 100; ++it) {
      legendre_all(p + 1, x, P);
      double f = P[p + 1] - P[p - 1];
      double df = (2.0 * p + 1.0) * P[p];
      double dx = f / df;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    xi[k] = x;
  }
  xi[0] = -1.0;
  xi[p] = 1.0;
  // symmetrise (the rule is symmetric about 0; removes last-bit asymmetry)
  for (int k = 0; k <= p / 2; ++k) {
    double s = 0.5 * (xi[p - k] - xi[k]);
    xi[k] = -s;
    xi[p - k] = s;
  }
  if (p % 2 == 0) xi[p / 2] = 0.0;
  for (int k = 0; k <= p; ++k) {
    legendre_all(p, xi[k], P);
    w[k] = 2.0 / (p * (p + 1.0) * P[p] * P[p]);
  }
}

void sym_eigvals(std::vector<double> a, int n, std::vector<double> &out) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double v = a[(size_t)i * n + j] * a[(size_t)i * n + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot) break;
    for (int pi = 0; pi < n - 1; ++pi)
      for (int qi = pi + 1; qi < n; ++qi) {
        double apq = a[(size_t)pi * n + qi];
        if (apq == 0.0) continue;
        double app = a[(size_t)pi * n + pi], aqq = a[(size_t)qi * n + qi];
        double tau = (aqq - app) / (2.0 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double akp = a[(size_t)k * n + pi], akq = a[(size_t)k * n + qi];
          a[(size_t)k * n + pi] = c * akp - s * akq;
          a[(size_t)k * n + qi] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double apk = a[(size_t)pi * n + k], aqk = a[(size_t)qi * n + k];
          a[(size_t)pi * n + k] = c * apk - s * aqk;
          a[(size_t)qi * n + k] = s * apk + c * aqk;
        }
      }
  }
  out.resize(n);
  for (int i = 0; i < n; ++i) out[i] = a[(size_t)i * n + i];
  std::sort(out.begin(), out.end());
}

std::string build_mesh(double L, int n_el, int p, MeshTables &m, bool periodic) {
  if (!(L > 0) || n_el < 1 || p < 1 || p > 12) return "set_mesh: need L > 0, n_el >= 1, 1 <= p <= 12";
  if ((int64_t)n_el * p < 2) return "set_mesh: n_el*p must be >= 2 (at least one interior node)";
  if ((int64_t)n_el * p - 1 > 2000) return "set_mesh: mesh too large";
  if (periodic && (n_el < 2 || n_el % 2)) return "set_mesh_periodic: n_el must be even and >= 2";
  m = MeshTables();
  m.periodic = periodic;
  m.L = L;
  m.n_el = n_el;
  m.p = p;
  m.q = p + 1;
  m.h = L / n_el;
  m.n = periodic ? n_el * p : n_el * p - 1;
  m.n_loc = m.q * m.q * m.q;
  m.np = (m.n_loc + 15) / 16 * 16;
  m.n_dof = (int64_t)m.n * m.n * m.n;
  m.n_cells = (int64_t)n_el * n_el * n_el;
  const int q = m.q;
  gll_rule(p, m.xi, m.w);

  // D[qq][a] = l_a'(xi_qq): P_p(xi_qq) / (P_p(xi_a) (xi_qq - xi_a)) off the
  // diagonal; -p(p+1)/4 and +p(p+1)/4 at the two ends; 0 elsewhere on the diagonal.
  std::vector<double> Pp(q), P;
  for (int k = 0; k < q; ++k) {
    legendre_all(p, m.xi[k], P);
    Pp[k] = P[p];
  }
  m.D.assign((size_t)q * q, 0.0);
  for (int i = 0; i < q; ++i)
    for (int a = 0; a < q; ++a) {
      double v;
      if (i != a) v = Pp[i] / (Pp[a] * (m.xi[i] - m.xi[a]));
      else if (i == 0) v = -p * (p + 1.0) / 4.0;
      else if (i == p) v = p * (p + 1.0) / 4.0;
      else v = 0.0;
      m.D[(size_t)i * q + a] = v;
    }
  // K1 = D^T W D
  m.K1.assign((size_t)q * q, 0.0);
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) {
      double s = 0;
      for (int i = 0; i < q; ++i) s += m.w[i] * m.D[(size_t)i * q + a] * m.D[(size_t)i * q + b];
      m.K1[(size_t)a * q + b] = s;
    }
  // cell stiffness 1/2 (h/2) [K1 (x) W (x) W + W (x) K1 (x) W + W (x) W (x) K1],
  // local node l = a + q b + q^2 c.
  const int nl = m.n_loc;
  m.kcell.assign((size_t)nl * nl, 0.0);
  const double f = 0.5 * (m.h / 2.0);
  for (int c = 0; c < q; ++c)
    for (int b = 0; b < q; ++b)
      for (int a = 0; a < q; ++a) {
        int l = a + q * b + q * q * c;
        for (int c2 = 0; c2 < q; ++c2)
          for (int b2 = 0; b2 < q; ++b2)
            for (int a2 = 0; a2 < q; ++a2) {
              int l2 = a2 + q * b2 + q * q * c2;
              double v = 0;
              if (b == b2 && c == c2) v += m.K1[(size_t)a * q + a2] * m.w[b] * m.w[c];
              if (a == a2 && c == c2) v += m.w[a] * m.K1[(size_t)b * q + b2] * m.w[c];
              if (a == a2 && b == b2) v += m.w[a] * m.w[b] * m.K1[(size_t)c * q + c2];
              m.kcell[(size_t)l * nl + l2] = f * v;
            }
      }

  // cell -> dof map, colours, GLL mass
  const int n = m.n;
  m.cmap.assign((size_t)m.n_cells * nl, -1);
  m.colors.assign((size_t)m.n_cells, 0);
  m.mass.assign((size_t)m.n_dof, 0.0);
  const double jac = (m.h / 2.0) * (m.h / 2.0) * (m.h / 2.0);
  const int edge = n_el * p;
  for (int ez = 0; ez < n_el; ++ez)
    for (int ey = 0; ey < n_el; ++ey)
      for (int ex = 0; ex < n_el; ++ex) {
        int64_t e = ex + (int64_t)n_el * (ey + (int64_t)n_el * ez);
        m.colors[e] = (uint8_t)((ex & 1) | ((ey & 1) << 1) | ((ez & 1) << 2));
        for (int c = 0; c < q; ++c)
          for (int b = 0; b < q; ++b)
            for (int a = 0; a < q; ++a) {
              int I = ex * p + a, J = ey * p + b, K = ez * p + c;
              int l = a + q * b + q * q * c;
              int64_t d;
              if (periodic) {
                d = (int64_t)(I % edge) + (int64_t)n * ((J % edge) + (int64_t)n * (K % edge));
              } else {
                if (I == 0 || J == 0 || K == 0 || I == edge || J == edge || K == edge) continue;
                d = (int64_t)(I - 1) + (int64_t)n * ((J - 1) + (int64_t)n * (K - 1));
              }
              m.cmap[(size_t)e * nl + l] = (int32_t)d;
              m.mass[d] += jac * m.w[a] * m.w[b] * m.w[c];
            }
      }
  m.cell_order.resize((size_t)m.n_cells);
  int pos = 0;
  for (int col = 0; col < 8; ++col) {
    m.color_offset[col] = pos;
    for (int64_t e = 0; e < m.n_cells; ++e)
      if (m.colors[e] == col) m.cell_order[pos++] = (int32_t)e;
  }
  m.color_offset[8] = pos;

  // first-derivative cell matrices of the k-point operator (periodic only):
  // G_x[(a,b,c), (a2,b2,c2)] = (h/2)^2 w_a w_b w_c D[a][a2] delta_b,b2 delta_c,c2
  // and the same along y and z; the GLL rule is exact for this integrand's
  // degree (2p - 1) in the derivative direction.
  if (periodic) {
    const double s2 = (m.h / 2.0) * (m.h / 2.0);
    for (int dd = 0; dd < 3; ++dd) m.gcell[dd].assign((size_t)nl * nl, 0.0);
    for (int c = 0; c < q; ++c)
      for (int b = 0; b < q; ++b)
        for (int a = 0; a < q; ++a) {
          const int l = a + q * b + q * q * c;
          const double wl = s2 * m.w[a] * m.w[b] * m.w[c];
          for (int t = 0; t < q; ++t) {
            m.gcell[0][(size_t)l * nl + (t + q * b + q * q * c)] = wl * m.D[(size_t)a * q + t];
            m.gcell[1][(size_t)l * nl + (a + q * t + q * q * c)] = wl * m.D[(size_t)b * q + t];
            m.gcell[2][(size_t)l * nl + (a + q * b + q * q * t)] = wl * m.D[(size_t)c * q + t];
          }
        }
  }

  // 1D operator A = 1/2 M1^-1/2 K1D M1^-1/2 on the n interior nodes, for the
  // spectral upper bound; n <= 2000 keeps the host Jacobi affordable only for
  // small n, so beyond 400 nodes a Gershgorin bound (still rigorous) is used.
  {
    // assembled over the n_el p + 1 nodes of the line (periodic: indices
    // wrapped onto n_el p nodes), then restricted to the n unknowns
    const int n1 = periodic ? edge : edge + 1, off = periodic ? 0 : 1;
    std::vector<double> K1D((size_t)n1 * n1, 0.0), M1(n1, 0.0);
    for (int e = 0; e < n_el; ++e)
      for (int a = 0; a < q; ++a) {
        const int ia = (e * p + a) % n1;
        M1[ia] += (m.h / 2.0) * m.w[a];
        for (int b = 0; b < q; ++b)
          K1D[(size_t)ia * n1 + (e * p + b) % n1] += (2.0 / m.h) * m.K1[(size_t)a * q + b];
      }
    std::vector<double> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        A[(size_t)i * n + j] =
            0.5 * K1D[(size_t)(i + off) * n1 + (j + off)] / std::sqrt(M1[i + off] * M1[j + off]);
    if (n <= 400) {
      std::vector<double> ev;
      sym_eigvals(A, n, ev);
      // pad by a few ulps of the spectral radius so the bound stays rigorous
      m.lam1d_max = ev[n - 1] * (1.0 + 64 * 2.220446049250313e-16);
    } else {
      double g = 0;
      for (int i = 0; i < n; ++i) {
        double r = 0;
        for (int j = 0; j < n; ++j) r += std::fabs(A[(size_t)i * n + j]);
        g = std::max(g, r);
      }
      m.lam1d_max = g;
    }
  }
  return "";
}

double bloch_1d_max(const MeshTables &m, double k) {
  const int q = m.q, p = m.p, n = m.n_el * p;
  std::vector<double> K1D((size_t)n * n, 0.0), C1D((size_t)n * n, 0.0), M1(n, 0.0);
  for (int e = 0; e < m.n_el; ++e)
    for (int a = 0; a < q; ++a) {
      const int ia = (e * p + a) % n;
      M1[ia] += (m.h / 2.0) * m.w[a];
      for (int b = 0; b < q; ++b) {
        const int ib = (e * p + b) % n;
        K1D[(size_t)ia * n + ib] += (2.0 / m.h) * m.K1[(size_t)a * q + b];
        C1D[(size_t)ia * n + ib] += m.w[a] * m.D[(size_t)a * q + b];   // int phi_a phi_b'
      }
    }
  // A = Re + i Im, Re = m^-1/2 (K1D/2 + k^2 m/2) m^-1/2, Im = -k m^-1/2 C1D m^-1/2
  std::vector<double> re((size_t)n * n), im((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double s = 1.0 / std::sqrt(M1[i] * M1[j]);
      re[(size_t)i * n + j] = s * (0.5 * K1D[(size_t)i * n + j] + (i == j ? 0.5 * k * k * M1[i] : 0.0));
      im[(size_t)i * n + j] = -k * s * C1D[(size_t)i * n + j];
    }
  if (n <= 200) {
    // the real symmetric form [[Re, -Im], [Im, Re]] carries every eigenvalue of A twice
    const int n2 = 2 * n;
    std::vector<double> E((size_t)n2 * n2);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        E[(size_t)i * n2 + j] = re[(size_t)i * n + j];
        E[(size_t)i * n2 + n + j] = -im[(size_t)i * n + j];
        E[(size_t)(n + i) * n2 + j] = im[(size_t)i * n + j];
        E[(size_t)(n + i) * n2 + n + j] = re[(size_t)i * n + j];
      }
    std::vector<double> ev;
    sym_eigvals(E, n2, ev);
    return ev[n2 - 1] * (1.0 + 64 * 2.220446049250313e-16);
  }
  double g = 0;
  for (int i = 0; i < n; ++i) {
    double r = 0;
    for (int j = 0; j < n; ++j) r += std::hypot(re[(size_t)i * n + j], im[(size_t)i * n + j]);
    g = std::max(g, r);
  }
  return g;
}

void dof_coords(const MeshTables &m, double *xyz) {
  std::vector<double> x1(m.n);
  const int I0 = m.periodic ? 0 : 1;   // periodic unknowns start at the node x = 0
  for (int i = 0; i < m.n; ++i) {
    const int I = i + I0, ex = I / m.p, a = I % m.p;
    x1[i] = ex * m.h + (1.0 + m.xi[a]) * m.h / 2.0;
  }
  for (int K = 0; K < m.n; ++K)
    for (int J = 0; J < m.n; ++J)
      for (int I = 0; I < m.n; ++I) {
        int64_t d = I + (int64_t)m.n * (J + (int64_t)m.n * K);
        xyz[3 * d + 0] = x1[I];
        xyz[3 * d + 1] = x1[J];
        xyz[3 * d + 2] = x1[K];
      }
}

}  // namespace chfsi
