// Dense contraction of the channel site tensors into the full Fock-space
// Hamiltonian (tiny systems only).  Test support for the host-side operator
// factorization: it lets the CPU test-suite compare the factorized
// Hamiltonian with an independent construction.  Not used by any compute path.
#include <cmath>
#include <vector>

#include "qc_mpo.hpp"

namespace dmrg {

namespace {
struct Dense {
  int n = 0;
  std::vector<double> a;
  Dense() = default;
  explicit Dense(int n_) : n(n_), a(size_t(n_) * n_, 0.0) {}
  double& at(int i, int j) { return a[size_t(i) * n + j]; }
  double at(int i, int j) const { return a[size_t(i) * n + j]; }
};

int nparticles_dense(int idx, int nsites) {
  int c = 0;
  for (int s = 0; s < nsites; ++s) {
    int v = (idx >> (2 * s)) & 3;
    c += (v & 1) + (v >> 1);
  }
  return c;
}

// dense dot matrix of string sid; for width 2 re-indexed to n1 + 4 n2
std::vector<double> dot_matrix(const DotString& ds, int width) {
  int d = 1 << (2 * width);
  std::vector<double> m(size_t(d) * d, 0.0);
  auto perm = [&](int n) { return width == 1 ? n : (n / 4) + 4 * (n % 4); };
  for (size_t k = 0; k < ds.val.size(); ++k) m[size_t(perm(ds.bra[k])) * d + perm(ds.ket[k])] += ds.val[k];
  return m;
}

int dot_particles(int n, int width) {
  int c = 0;
  for (int s = 0; s < width; ++s) {
    int v = (n >> (2 * s)) & 3;
    c += (v & 1) + (v >> 1);
  }
  return c;
}
}  // namespace

// Left-to-right contraction: Lop_{b+w}[w'] = sum (Lop_b[w] P^{p(y)}) (x) y.
// Basis index of the dense space: sum_i n_i 4^i (site 0 least significant).
int debug_mpo_dense_left(QCHamiltonian& H, int wide_bond, double* out) {
  const int L = H.L();
  std::vector<Dense> env(1, Dense(1));
  env[0].at(0, 0) = 1.0;  // bond 0: channel ID_H, identity on the empty block
  int b = 0, nsites = 0;
  while (b < L) {
    int width = (b == wide_bond) ? 2 : 1;
    const SiteOp& W = H.site_op(b, width, H.mode_left(b), H.mode_left(b + width));
    const BondChannels& B1 = H.left_channels(b + width);
    int d = 1 << (2 * width);
    int n0 = env.empty() ? 1 : env[0].n;
    std::vector<Dense> nxt(B1.ch.size(), Dense(n0 * d));
    for (const WEntry& e : W.e) {
      const DotString& ds = H.dot_string(width, e.sid);
      std::vector<double> y = dot_matrix(ds, width);
      const Dense& X = env[e.src];
      Dense& Y = nxt[e.dst];
      for (int i = 0; i < n0; ++i)
        for (int j = 0; j < n0; ++j) {
          double x = X.at(i, j);
          if (x == 0.0) continue;
          double sg = (ds.parity && (nparticles_dense(j, nsites) & 1)) ? -1.0 : 1.0;
          for (int p = 0; p < d; ++p)
            for (int q = 0; q < d; ++q) {
              double v = y[size_t(p) * d + q];
              if (v != 0.0) Y.at(i + n0 * p, j + n0 * q) += e.c * sg * x * v;
            }
        }
    }
    env.swap(nxt);
    b += width;
    nsites += width;
  }
  const BondChannels& BL = H.left_channels(L);
  int w = BL.find(chan_key(CH_H_ID, -1, -1));
  const Dense& R = env[w];
  for (size_t k = 0; k < R.a.size(); ++k) out[k] = R.a[k];
  return 0;
}

// Right-to-left contraction: Rop_b[w] = sum (y P_D^{p(Z)}) (x) Rop_{b+w}[w'].
int debug_mpo_dense_right(QCHamiltonian& H, int wide_bond, double* out) {
  const int L = H.L();
  std::vector<Dense> env(1, Dense(1));
  env[0].at(0, 0) = 1.0;  // bond L: channel H_ID, identity on the empty block
  int b = L;
  while (b > 0) {
    int width = (wide_bond >= 0 && b - 2 == wide_bond) ? 2 : 1;
    int b0 = b - width;
    const SiteOp& W = H.site_op(b0, width, H.mode_right(b0), H.mode_right(b));
    const BondChannels& B0 = H.right_channels(b0);
    const BondChannels& B1 = H.right_channels(b);
    int d = 1 << (2 * width);
    int n0 = env[0].n;
    std::vector<Dense> nxt(B0.ch.size(), Dense(n0 * d));
    for (const WEntry& e : W.e) {
      const DotString& ds = H.dot_string(width, e.sid);
      std::vector<double> y = dot_matrix(ds, width);
      const Dense& Z = env[e.dst];
      int pz = B1.ch[e.dst].parity;
      Dense& Y = nxt[e.src];
      for (int p = 0; p < d; ++p)
        for (int q = 0; q < d; ++q) {
          double v = y[size_t(p) * d + q];
          if (v == 0.0) continue;
          double sg = (pz && (dot_particles(q, width) & 1)) ? -1.0 : 1.0;
          for (int i = 0; i < n0; ++i)
            for (int j = 0; j < n0; ++j) {
              double z = Z.at(i, j);
              if (z != 0.0) Y.at(p + d * i, q + d * j) += e.c * sg * v * z;
            }
        }
    }
    env.swap(nxt);
    b = b0;
  }
  const BondChannels& B0 = H.right_channels(0);
  int w = B0.find(chan_key(CH_ID_H, -1, -1));
  const Dense& R = env[w];
  for (size_t k = 0; k < R.a.size(); ++k) out[k] = R.a[k];
  return 0;
}

}  // namespace dmrg
