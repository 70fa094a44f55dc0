// Host-side FP64 finite-element assembly of the diffusion operator of the
// monodomain equation (paper Sec. 2, eq. 2b-c) and its device layouts.
//
// K_ij = sum_e int_e grad N_i . D_e grad N_j,  m_i = sum_e int_e N_i
// (row-sum lumping of the consistent mass, which is what makes the
// forward-Euler diffusion substep explicit and what eq. 3's m_ii refers to).
// Q1 isoparametric elements with 2^dim Gauss points, and P1 simplices
// (triangles, tetrahedra) with one point at the centroid (their gradients
// are constant, so the rule is exact).  Per-node conductivity
// scales the off-diagonal entries by (sigma_i + sigma_j)/2 and the diagonal
// is reset to minus the off-diagonal row sum, so K stays symmetric with zero
// row sums.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>

#include "mono_internal.h"

namespace mono {
namespace {

// Reference coordinate (+1/-1) of element node a along axis k for the node
// orderings declared in mono.h (quad counter-clockwise, hex = two quads).
inline double ref_sign(int a, int k) {
  const int q = a & 3;
  if (k == 0) return (q == 1 || q == 2) ? 1.0 : -1.0;
  if (k == 1) return (q >= 2) ? 1.0 : -1.0;
  return (a >= 4) ? 1.0 : -1.0;
}

struct RefTables {
  int dim, nen, nq;
  double w[8];            // quadrature weight of point q
  double N[8][8];         // [q][a]
  double dN[8][8][3];     // [q][a][k] = dN_a/dxi_k at Gauss point q
};

// P1 simplex on the unit reference simplex: N_0 = 1 - sum xi, N_a = xi_a;
// one point at the centroid with the reference volume 1/dim! as weight.
RefTables make_simplex_tables(int dim) {
  RefTables t{};
  t.dim = dim;
  t.nen = dim + 1;
  t.nq = 1;
  t.w[0] = dim == 2 ? 0.5 : 1.0 / 6.0;
  for (int a = 0; a < t.nen; ++a) {
    t.N[0][a] = 1.0 / (dim + 1);
    for (int k = 0; k < dim; ++k) t.dN[0][a][k] = a == 0 ? -1.0 : (a - 1 == k ? 1.0 : 0.0);
  }
  return t;
}

RefTables make_tables(int dim) {
  RefTables t{};
  t.dim = dim;
  t.nen = 1 << dim;
  t.nq = 1 << dim;
  const double gp = 1.0 / std::sqrt(3.0);
  for (int q = 0; q < t.nq; ++q) {
    t.w[q] = 1.0;
    double xi[3] = {0, 0, 0};
    // Gauss point q takes the sign pattern of element node q
    for (int k = 0; k < dim; ++k) xi[k] = gp * ref_sign(q, k);
    for (int a = 0; a < t.nen; ++a) {
      double lin[3];
      for (int k = 0; k < dim; ++k) lin[k] = 0.5 * (1.0 + ref_sign(a, k) * xi[k]);
      double prod = 1.0;
      for (int k = 0; k < dim; ++k) prod *= lin[k];
      t.N[q][a] = prod;
      for (int k = 0; k < dim; ++k) {
        double g = 0.5 * ref_sign(a, k);
        for (int m = 0; m < dim; ++m)
          if (m != k) g *= lin[m];
        t.dN[q][a][k] = g;
      }
    }
  }
  return t;
}

// Solve J X = B for X (dim x nen) by Gaussian elimination with partial
// pivoting; returns det J.
double solve_small(int dim, double J[3][3], double B[3][8], int nen) {
  double det = 1.0;
  for (int c = 0; c < dim; ++c) {
    int piv = c;
    for (int r = c + 1; r < dim; ++r)
      if (std::fabs(J[r][c]) > std::fabs(J[piv][c])) piv = r;
    if (piv != c) {
      for (int k = 0; k < dim; ++k) std::swap(J[c][k], J[piv][k]);
      for (int k = 0; k < nen; ++k) std::swap(B[c][k], B[piv][k]);
      det = -det;
    }
    const double d = J[c][c];
    det *= d;
    if (d == 0.0) return 0.0;
    for (int r = c + 1; r < dim; ++r) {
      const double f = J[r][c] / d;
      for (int k = c; k < dim; ++k) J[r][k] -= f * J[c][k];
      for (int k = 0; k < nen; ++k) B[r][k] -= f * B[c][k];
    }
  }
  for (int c = dim - 1; c >= 0; --c) {
    for (int k = 0; k < nen; ++k) {
      double s = B[c][k];
      for (int m = c + 1; m < dim; ++m) s -= J[c][m] * B[m][k];
      B[c][k] = s / J[c][c];
    }
  }
  return det;
}

}  // namespace

int assemble_fe(const mono_mesh_desc* d, HostCSR& K, std::string& err) {
  const int dim = d->dim;
  const int64_t n = d->n_nodes, ne = d->n_elems;
  const bool simplex = dim >= 2 && d->etype == dim + 1;
  const int nen = simplex ? dim + 1 : 1 << dim;
  if (!d->xyz || !d->conn || !d->D_elem) {
    err = "mesh arrays must not be NULL";
    return MONO_EINVAL;
  }
  // node -> element incidence (CSR)
  std::vector<int64_t> n2e_ptr(n + 1, 0);
  for (int64_t e = 0; e < ne; ++e)
    for (int a = 0; a < nen; ++a) {
      const int32_t g = d->conn[e * nen + a];
      if (g < 0 || g >= n) {
        err = "element " + std::to_string(e) + " references node out of range";
        return MONO_EINVAL;
      }
      n2e_ptr[g + 1]++;
    }
  for (int64_t i = 0; i < n; ++i) n2e_ptr[i + 1] += n2e_ptr[i];
  std::vector<int64_t> n2e(n2e_ptr[n]);
  {
    std::vector<int64_t> fill(n2e_ptr.begin(), n2e_ptr.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
      for (int a = 0; a < nen; ++a) n2e[fill[d->conn[e * nen + a]]++] = e;
  }
  // sparsity: row i couples to every node of every element touching i
  K.n = n;
  K.rp.assign(n + 1, 0);
  {
    std::vector<int32_t> cand;
    cand.reserve(64);
    std::vector<int32_t> cols;
    cols.reserve((size_t)n * (dim == 3 ? 27 : (dim == 2 ? 9 : 3)));
    for (int64_t i = 0; i < n; ++i) {
      cand.clear();
      cand.push_back((int32_t)i);
      for (int64_t p = n2e_ptr[i]; p < n2e_ptr[i + 1]; ++p) {
        const int64_t e = n2e[p];
        for (int a = 0; a < nen; ++a) cand.push_back(d->conn[e * nen + a]);
      }
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      cols.insert(cols.end(), cand.begin(), cand.end());
      K.rp[i + 1] = (int64_t)cols.size();
    }
    K.col.swap(cols);
  }
  K.val.assign(K.col.size(), 0.0);
  K.mass.assign(n, 0.0);

  const RefTables t = simplex ? make_simplex_tables(dim) : make_tables(dim);
  for (int64_t e = 0; e < ne; ++e) {
    const int32_t* en = d->conn + e * nen;
    const double* D = d->D_elem + e * dim * dim;
    double Ke[8][8] = {{0}};
    double me[8] = {0};
    for (int q = 0; q < t.nq; ++q) {
      // Jacobian from coordinates relative to the element's first node (the
      // shape-function derivatives sum to zero, so J is unchanged): elements
      // of the same shape then give bitwise the same matrices wherever they
      // sit, which lets the stencil rows of structured meshes repeat exactly.
      double J[3][3] = {{0}};
      for (int k = 0; k < dim; ++k)
        for (int c = 0; c < dim; ++c) {
          const double x0 = d->xyz[(int64_t)en[0] * dim + c];
          double s = 0.0;
          for (int a = 1; a < nen; ++a)
            s += t.dN[q][a][k] * (d->xyz[(int64_t)en[a] * dim + c] - x0);
          J[k][c] = s;
        }
      double B[3][8];
      for (int k = 0; k < dim; ++k)
        for (int a = 0; a < nen; ++a) B[k][a] = t.dN[q][a][k];
      const double jac = solve_small(dim, J, B, nen);   // B <- J^-1 dN (physical gradients)
      if (!(jac > 0.0)) {
        err = "element " + std::to_string(e) + " has a non-positive Jacobian";
        return MONO_EINVAL;
      }
      const double det = jac * t.w[q];
      // DB = D * B
      double DB[3][8];
      for (int k = 0; k < dim; ++k)
        for (int a = 0; a < nen; ++a) {
          double s = 0.0;
          for (int c = 0; c < dim; ++c) s += D[k * dim + c] * B[c][a];
          DB[k][a] = s;
        }
      for (int a = 0; a < nen; ++a) {
        me[a] += det * t.N[q][a];
        for (int b = 0; b < nen; ++b) {
          double s = 0.0;
          for (int k = 0; k < dim; ++k) s += B[k][a] * DB[k][b];
          Ke[a][b] += det * s;
        }
      }
    }
    for (int a = 0; a < nen; ++a) {
      const int64_t i = en[a];
      K.mass[i] += me[a];
      const int32_t* rb = K.col.data() + K.rp[i];
      const int32_t* re = K.col.data() + K.rp[i + 1];
      for (int b = 0; b < nen; ++b) {
        const int32_t* p = std::lower_bound(rb, re, en[b]);
        K.val[p - K.col.data()] += Ke[a][b];
      }
    }
  }
  if (d->sigma_node) {
    for (int64_t i = 0; i < n; ++i) {
      if (!(d->sigma_node[i] > 0.0) || !std::isfinite(d->sigma_node[i])) {
        err = "sigma_node must be positive and finite";
        return MONO_EINVAL;
      }
    }
    for (int64_t i = 0; i < n; ++i) {
      double off = 0.0;
      int64_t pd = -1;
      for (int64_t p = K.rp[i]; p < K.rp[i + 1]; ++p) {
        const int32_t j = K.col[p];
        if (j == i) {
          pd = p;
          continue;
        }
        K.val[p] *= 0.5 * (d->sigma_node[i] + d->sigma_node[j]);
        off += K.val[p];
      }
      K.val[pd] = -off;
    }
  }
  return MONO_OK;
}

void build_ell(const HostCSR& K, int64_t Np, EllHost& out) {
  int w = 0;
  for (int64_t i = 0; i < K.n; ++i) w = std::max<int>(w, (int)(K.rp[i + 1] - K.rp[i] - 1));
  out.width = w;
  out.col.assign((size_t)w * Np, 0);
  out.val.assign((size_t)w * Np, 0.0);
  for (int64_t i = 0; i < Np; ++i)
    for (int s = 0; s < w; ++s) out.col[(size_t)s * Np + i] = (int32_t)std::min<int64_t>(i, K.n - 1);
  for (int64_t i = 0; i < K.n; ++i) {
    int s = 0;
    for (int64_t p = K.rp[i]; p < K.rp[i + 1]; ++p) {
      if (K.col[p] == i) continue;
      out.col[(size_t)s * Np + i] = K.col[p];
      out.val[(size_t)s * Np + i] = -K.val[p] / K.mass[i];
      ++s;
    }
  }
}

bool build_stencil(const HostCSR& K, const std::vector<int64_t>& inst_off, int64_t Np,
                   StencilHost& out) {
  const int ni = (int)inst_off.size() - 1;
  std::vector<std::vector<int32_t>> offs(ni);
  int P = 0;
  for (int q = 0; q < ni; ++q) {
    std::vector<int32_t>& o = offs[q];
    for (int64_t i = inst_off[q]; i < inst_off[q + 1]; ++i)
      for (int64_t p = K.rp[i]; p < K.rp[i + 1]; ++p) {
        const int64_t dj = (int64_t)K.col[p] - i;
        if (dj <= 0) continue;
        if (std::find(o.begin(), o.end(), (int32_t)dj) == o.end()) {
          o.push_back((int32_t)dj);
          if ((int)o.size() > kMaxOffsets) return false;
        }
      }
    std::sort(o.begin(), o.end());
    P = std::max<int>(P, (int)o.size());
  }
  P = std::max(P, 1);
  out.P = P;
  out.off.assign((size_t)ni * P, 0);
  out.e.assign((size_t)P * Np, 0.0);
  out.minv.assign(Np, 0.0);
  for (int q = 0; q < ni; ++q)
    for (size_t p = 0; p < offs[q].size(); ++p) out.off[(size_t)q * P + p] = offs[q][p];
  for (int q = 0; q < ni; ++q) {
    const std::vector<int32_t>& o = offs[q];
    for (int64_t i = inst_off[q]; i < inst_off[q + 1]; ++i) {
      out.minv[i] = 1.0 / K.mass[i];
      for (int64_t p = K.rp[i]; p < K.rp[i + 1]; ++p) {
        const int64_t dj = (int64_t)K.col[p] - i;
        if (dj <= 0) continue;
        const size_t slot = std::lower_bound(o.begin(), o.end(), (int32_t)dj) - o.begin();
        out.e[slot * Np + i] = -K.val[p];
      }
    }
  }
  return true;
}

bool build_row_classes(const StencilHost& sh, int64_t n, int64_t Np, bool fp32,
                       int max_classes, RowClasses& out) {
  if ((int64_t)sh.off.size() != (int64_t)sh.P) return false;   // one instance only
  const int P = sh.P;
  const int tw = (2 * P + 1 + 1) & ~1;
  std::unordered_map<std::string, int> ids;
  std::vector<uint16_t> cls(Np, 0);
  std::vector<double> table;
  std::vector<double> row(tw);
  std::string key(tw * sizeof(double), '\0');
  const int64_t cap = std::min<int64_t>(max_classes, std::max<int64_t>(Np / 8, 1));
  for (int64_t i = 0; i < Np; ++i) {
    std::fill(row.begin(), row.end(), 0.0);
    for (int p = 0; p < P; ++p) {
      const int64_t jb = i - sh.off[p];
      row[p] = sh.e[(size_t)p * Np + i];
      row[P + p] = (jb >= 0 && i < n) ? sh.e[(size_t)p * Np + jb] : 0.0;
    }
    row[2 * P] = sh.minv[i];
    if (fp32)
      for (double& v : row) v = (double)(float)v;
    std::memcpy(&key[0], row.data(), key.size());
    auto it = ids.find(key);
    if (it == ids.end()) {
      const int id = (int)ids.size();
      if (id >= cap) return false;
      ids.emplace(key, id);
      table.insert(table.end(), row.begin(), row.end());
      cls[i] = (uint16_t)id;
    } else {
      cls[i] = (uint16_t)it->second;
    }
  }
  out.tw = tw;
  out.n_classes = (int)ids.size();
  out.cls.swap(cls);
  out.table.swap(table);
  return true;
}

}  // namespace mono
