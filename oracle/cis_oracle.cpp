// Plain CPU oracle of one implicit iteration of the conservative implicit scheme
// for steady diatomic (Rykov) flow on unstructured physical and velocity meshes
// (arXiv 2303.10846, Sec. 2-3).
//
// TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
// checked against; it shares no code with the library.  Only the test suite,
// the package smoke check and the benchmark's CPU-baseline leg may build, load
// or call it.  The product path never does.
//
// Style: plain sequential loops in the order of the paper's algorithm
// (Sec. 3.5, Steps 1-7), FP64 throughout.  Loops over independent cells,
// faces or velocity ranges carry OpenMP pragmas; no arithmetic is fused,
// blocked or reordered beyond what the equations state.  Every routine is a
// template on the scalar type S (double or std::complex<double>) so the same
// code yields a complex-step derivative; branches (upwind side, limiter
// min/max, |.|) are taken on real parts.
//
// Readings of points the paper leaves open are marked "reading:" where they
// are used.

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using std::exp;
using std::pow;
using std::sqrt;

using cplx = std::complex<double>;
inline double re(double x) { return x; }
inline double re(const cplx& z) { return z.real(); }
template <class S> inline S absr(const S& x) { return re(x) < 0.0 ? S(-x) : x; }
template <class S> inline S sq(const S& x) { return x * x; }

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Constants (passed from Python as flat double arrays)
// ---------------------------------------------------------------------------
enum GasIdx { G_R, G_GAMMA, G_Z, G_DELTA, G_OMEGA0, G_OMEGA1, G_MUREF, G_OMEGAV, G_TREF, G_CS, G_COUNT };
enum NumIdx { N_CFL, N_INVDT, N_CFLIMP, N_LIMK, N_LIMITER, N_NMACRO, N_NMICRO, N_SNAP, N_EXACTJVP, N_COUNT };

struct Gas {
  double R, gamma, Z, delta, omega0, omega1, mu_ref, omega_v, T_ref, C_s;
  explicit Gas(const double* g)
      : R(g[G_R]), gamma(g[G_GAMMA]), Z(g[G_Z]), delta(g[G_DELTA]), omega0(g[G_OMEGA0]),
        omega1(g[G_OMEGA1]), mu_ref(g[G_MUREF]), omega_v(g[G_OMEGAV]), T_ref(g[G_TREF]), C_s(g[G_CS]) {}
};

struct Num {
  double cfl, inv_dt, cfl_imp, lim_K, snap;
  int limiter, n_macro, n_micro, exact_jvp;
  explicit Num(const double* n)
      : cfl(n[N_CFL]), inv_dt(n[N_INVDT]), cfl_imp(n[N_CFLIMP]), lim_K(n[N_LIMK]), snap(n[N_SNAP]),
        limiter(int(n[N_LIMITER])), n_macro(int(n[N_NMACRO])), n_micro(int(n[N_NMICRO])),
        exact_jvp(int(n[N_EXACTJVP])) {}
};

enum BcKind { BC_WALL = 1, BC_FARFIELD = 2 };

template <class S> struct Bc {
  int tag = 0, kind = 0;
  S rho = 1.0, U[3] = {0.0, 0.0, 0.0}, T = 1.0;
};

// ---------------------------------------------------------------------------
// Geometry of the physical mesh and the DVS (Sec. 3.1: V_i, A_ij, n_ij; Sec. 3.3: x_ij)
// ---------------------------------------------------------------------------
struct Geom {
  int64_t nc = 0, nf = 0, nv = 0;
  std::vector<double> V, xc, h, dt;  // cells
  int mf = 4;                        // face slots per cell (4 when every cell is a tetrahedron, else 6)
  std::vector<int> nfc;              // faces of each cell
  std::vector<int64_t> cf;           // [nc][mf] faces of each cell (-1 past nfc)
  std::vector<int64_t> fo, fn;       // owner, neighbour (-1 on the boundary)
  std::vector<int> ftag;             // boundary tag (0 interior)
  std::vector<double> A, n, xf, s, dl;
  std::vector<double> Minv;  // least-squares normal matrix inverse per cell, [nc][9]
  std::vector<double> u, w;  // DVS points and weights
  std::vector<double> umag;
  double umax = 0.0;
};

inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

inline bool inv3(const double* M, double* I) {
  double c00 = M[4] * M[8] - M[5] * M[7], c01 = M[5] * M[6] - M[3] * M[8], c02 = M[3] * M[7] - M[4] * M[6];
  double det = M[0] * c00 + M[1] * c01 + M[2] * c02;
  if (!(std::fabs(det) > 0.0)) return false;
  double id = 1.0 / det;
  I[0] = c00 * id;
  I[1] = (M[2] * M[7] - M[1] * M[8]) * id;
  I[2] = (M[1] * M[5] - M[2] * M[4]) * id;
  I[3] = c01 * id;
  I[4] = (M[0] * M[8] - M[2] * M[6]) * id;
  I[5] = (M[2] * M[3] - M[0] * M[5]) * id;
  I[6] = c02 * id;
  I[7] = (M[1] * M[6] - M[0] * M[7]) * id;
  I[8] = (M[0] * M[4] - M[1] * M[3]) * id;
  return true;
}

// Local faces of the cell kinds (by node count): tetrahedron (the face opposite local vertex a), pyramid
// (base quad 0-3, apex 4), prism (triangles 0-2 and 3-5) and hexahedron (quads 0-3 and 4-7); quads in cyclic
// order.
struct LocalFaces {
  int n;
  int size[6];
  int node[6][4];
};
const LocalFaces* local_faces(int kind) {
  static const LocalFaces tet = {4, {3, 3, 3, 3}, {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}}};
  static const LocalFaces pyr = {5, {4, 3, 3, 3, 3}, {{0, 1, 2, 3}, {0, 1, 4}, {1, 2, 4}, {2, 3, 4}, {3, 0, 4}}};
  static const LocalFaces pri = {5, {3, 3, 4, 4, 4}, {{0, 1, 2}, {3, 4, 5}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}}};
  static const LocalFaces hex = {6, {4, 4, 4, 4, 4, 4},
                                 {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}}};
  switch (kind) {
    case 4: return &tet;
    case 5: return &pyr;
    case 6: return &pri;
    case 8: return &hex;
    default: return nullptr;
  }
}

using FaceKey = std::array<int32_t, 4>;  // sorted node ids, -1 in the last place for a triangle
FaceKey face_key(const int32_t* nodes, int n) {
  FaceKey k = {nodes[0], nodes[1], nodes[2], n == 4 ? nodes[3] : -1};
  std::sort(k.begin(), k.begin() + n);
  return k;
}

// Vector area and centroid of a face with nodes p[0..n-1] in cyclic order (n = 3 or 4).  A quad need not be
// planar: its vector area is half the cross product of its diagonals (the vector area of the closed polygon,
// so every closed cell has sum_f A n = 0 exactly), and its centroid the average of the centroids of the four
// triangles it makes with its node average, weighted by their areas along the face normal.
void face_geometry(const double* const* p, int n, double* S, double* xf) {
  if (n == 3) {
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
      e1[k] = p[1][k] - p[0][k];
      e2[k] = p[2][k] - p[0][k];
    }
    cross3(e1, e2, S);
    for (int k = 0; k < 3; ++k) {
      S[k] *= 0.5;
      xf[k] = (p[0][k] + p[1][k] + p[2][k]) / 3.0;
    }
    return;
  }
  double d1[3], d2[3], m[3];
  for (int k = 0; k < 3; ++k) {
    d1[k] = p[2][k] - p[0][k];
    d2[k] = p[3][k] - p[1][k];
    m[k] = 0.25 * (p[0][k] + p[1][k] + p[2][k] + p[3][k]);
  }
  cross3(d1, d2, S);
  for (int k = 0; k < 3; ++k) S[k] *= 0.5;
  const double len = std::sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
  double wsum = 0.0, acc[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const double* a = p[q];
    const double* b = p[(q + 1) % 4];
    double e1[3], e2[3], t[3];
    for (int k = 0; k < 3; ++k) {
      e1[k] = b[k] - a[k];
      e2[k] = m[k] - a[k];
    }
    cross3(e1, e2, t);
    const double wq = 0.5 * (t[0] * S[0] + t[1] * S[1] + t[2] * S[2]) / len;
    wsum += wq;
    for (int k = 0; k < 3; ++k) acc[k] += wq * (a[k] + b[k] + m[k]) / 3.0;
  }
  for (int k = 0; k < 3; ++k) xf[k] = acc[k] / wsum;
}

// Geometry of the physical mesh.  cells [nc][8] node ids (unused places ignored), kinds [nc] = node count
// (4 tetrahedron, 5 pyramid, 6 prism, 8 hexahedron); bface [nb][4] boundary faces (-1 in the last place for a
// triangle) with tags btag.
int build_geom(Geom& g, const double* xyz, int64_t nn, const int32_t* cells, const int32_t* kinds, int64_t nc,
               const int32_t* bface, const int32_t* btag, int64_t nb, const double* u, const double* w, int64_t nv,
               double cfl) {
  g.nc = nc;
  g.nv = nv;
  g.V.assign(nc, 0.0);
  g.xc.assign(3 * nc, 0.0);
  g.mf = 4;
  for (int64_t i = 0; i < nc; ++i) {
    const LocalFaces* lf = local_faces(kinds[i]);
    if (!lf) return -2;
    g.mf = std::max(g.mf, lf->n);
    for (int a = 0; a < kinds[i]; ++a)
      if (cells[8 * i + a] < 0 || cells[8 * i + a] >= nn) return -2;
  }
  g.nfc.assign(nc, 0);
  for (int64_t i = 0; i < nc; ++i) {
    const int32_t* cn = cells + 8 * i;
    const int kind = kinds[i];
    const LocalFaces* lf = local_faces(kind);
    g.nfc[i] = lf->n;
    if (kind == 4) {
      // tetrahedron: volume |det| / 6, centroid the mean of the vertices
      const double* p[4];
      for (int a = 0; a < 4; ++a) p[a] = xyz + 3 * cn[a];
      double d1[3], d2[3], d3[3], c[3];
      for (int k = 0; k < 3; ++k) {
        d1[k] = p[1][k] - p[0][k];
        d2[k] = p[2][k] - p[0][k];
        d3[k] = p[3][k] - p[0][k];
      }
      cross3(d2, d3, c);
      double vol = std::fabs(d1[0] * c[0] + d1[1] * c[1] + d1[2] * c[2]) / 6.0;
      if (!(vol > 0.0)) return -2;
      g.V[i] = vol;
      for (int k = 0; k < 3; ++k) g.xc[3 * i + k] = 0.25 * (p[0][k] + p[1][k] + p[2][k] + p[3][k]);
      continue;
    }
    // other kinds: tetrahedra from the node average p0 to the triangles of every face (a quad fanned about its
    // node average); volume the sum of theirs, centroid their volume-weighted centroids
    double p0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < kind; ++a)
      for (int k = 0; k < 3; ++k) p0[k] += xyz[3 * cn[a] + k] / kind;
    double vol = 0.0, acc[3] = {0.0, 0.0, 0.0};
    for (int fa = 0; fa < lf->n; ++fa) {
      const int n = lf->size[fa];
      const double* p[4];
      for (int q = 0; q < n; ++q) p[q] = xyz + 3 * cn[lf->node[fa][q]];
      double m[3] = {0.0, 0.0, 0.0};
      for (int q = 0; q < n; ++q)
        for (int k = 0; k < 3; ++k) m[k] += p[q][k] / n;
      const int ntri = n == 3 ? 1 : 4;
      double vs[4], cs[4][3], vface = 0.0;
      for (int t = 0; t < ntri; ++t) {
        const double* a = n == 3 ? p[0] : p[t];
        const double* b = n == 3 ? p[1] : p[(t + 1) % 4];
        const double* c = n == 3 ? p[2] : m;
        double e1[3], e2[3], e3[3], x[3];
        for (int k = 0; k < 3; ++k) {
          e1[k] = b[k] - a[k];
          e2[k] = c[k] - a[k];
          e3[k] = p0[k] - a[k];
        }
        cross3(e1, e2, x);
        vs[t] = -(x[0] * e3[0] + x[1] * e3[1] + x[2] * e3[2]) / 6.0;
        for (int k = 0; k < 3; ++k) cs[t][k] = 0.25 * (a[k] + b[k] + c[k] + p0[k]);
        vface += vs[t];
      }
      const double sg = vface >= 0.0 ? 1.0 : -1.0;  // orientation of the local node order
      for (int t = 0; t < ntri; ++t) {
        if (!(sg * vs[t] > 0.0)) return -2;  // folded or degenerate cell
        vol += sg * vs[t];
        for (int k = 0; k < 3; ++k) acc[k] += sg * vs[t] * cs[t][k];
      }
    }
    g.V[i] = vol;
    for (int k = 0; k < 3; ++k) g.xc[3 * i + k] = acc[k] / vol;
  }
  // faces, matched by their sorted node ids
  std::map<FaceKey, std::pair<int64_t, int>> seen;
  std::vector<std::array<int32_t, 4>> fnodes;  // the nodes of every face in cyclic order (-1: triangle)
  g.cf.assign((size_t)g.mf * nc, -1);
  auto cyc = [&](int64_t i, int a) {
    const LocalFaces* lf = local_faces(kinds[i]);
    std::array<int32_t, 4> v = {-1, -1, -1, -1};
    for (int q = 0; q < lf->size[a]; ++q) v[q] = cells[8 * i + lf->node[a][q]];
    return v;
  };
  for (int64_t i = 0; i < nc; ++i) {
    const LocalFaces* lf = local_faces(kinds[i]);
    for (int a = 0; a < lf->n; ++a) {
      std::array<int32_t, 4> v = cyc(i, a);
      FaceKey key = face_key(v.data(), lf->size[a]);
      auto it = seen.find(key);
      if (it == seen.end()) {
        seen[key] = {i, a};
      } else {
        if (it->second.first < 0) return -2;  // third use of a face
        int64_t f = (int64_t)g.fo.size();
        g.fo.push_back(it->second.first);
        g.fn.push_back(i);
        g.ftag.push_back(0);
        fnodes.push_back(cyc(it->second.first, it->second.second));
        g.cf[(size_t)g.mf * it->second.first + it->second.second] = f;
        g.cf[(size_t)g.mf * i + a] = f;
        it->second.first = -1;
      }
    }
  }
  std::map<FaceKey, int32_t> btags;
  for (int64_t b = 0; b < nb; ++b) {
    const int n = bface[4 * b + 3] < 0 ? 3 : 4;
    btags[face_key(bface + 4 * b, n)] = btag[b];
  }
  for (auto& kv : seen) {
    if (kv.second.first < 0) continue;
    auto bt = btags.find(kv.first);
    if (bt == btags.end()) return -2;  // open face without a boundary tag
    int64_t f = (int64_t)g.fo.size();
    g.fo.push_back(kv.second.first);
    g.fn.push_back(-1);
    g.ftag.push_back(bt->second);
    fnodes.push_back(cyc(kv.second.first, kv.second.second));
    g.cf[(size_t)g.mf * kv.second.first + kv.second.second] = f;
  }
  g.nf = (int64_t)g.fo.size();
  g.A.assign(g.nf, 0.0);
  g.n.assign(3 * g.nf, 0.0);
  g.xf.assign(3 * g.nf, 0.0);
  for (int64_t f = 0; f < g.nf; ++f) {
    const int n = fnodes[f][3] < 0 ? 3 : 4;
    const double* p[4];
    for (int q = 0; q < n; ++q) p[q] = xyz + 3 * fnodes[f][q];
    double nn3[3];
    face_geometry(p, n, nn3, &g.xf[3 * f]);
    for (int k = 0; k < 3; ++k) nn3[k] *= 2.0;  // twice the vector area, as the triangle's cross product
    double len = std::sqrt(nn3[0] * nn3[0] + nn3[1] * nn3[1] + nn3[2] * nn3[2]);
    // n points out of the owner cell (from cell i to cell j, Sec. 3.1)
    const double* xo = &g.xc[3 * g.fo[f]];
    double dot = 0.0;
    for (int k = 0; k < 3; ++k) dot += nn3[k] * (g.xf[3 * f + k] - xo[k]);
    double sgn = dot >= 0.0 ? 1.0 : -1.0;
    g.A[f] = 0.5 * len;
    for (int k = 0; k < 3; ++k) g.n[3 * f + k] = sgn * nn3[k] / len;
    // reading: an interior face takes the orientation whose first normal component beyond 1e-9
    // is positive; i is the cell n points out of.  The "x_j otherwise" tie rule of Eq. 46 then does
    // not depend on how the cells are numbered.
    if (g.fn[f] >= 0) {
      int d0 = 0;
      while (d0 < 2 && std::fabs(g.n[3 * f + d0]) <= 1e-9) ++d0;
      if (g.n[3 * f + d0] < 0.0) {
        for (int k = 0; k < 3; ++k) g.n[3 * f + k] = -g.n[3 * f + k];
        std::swap(g.fo[f], g.fn[f]);
      }
    }
  }
  // closure check: sum_f A n = 0 per cell
  for (int64_t i = 0; i < nc; ++i) {
    double acc[3] = {0, 0, 0}, asum = 0.0;
    for (int a = 0; a < g.nfc[i]; ++a) {
      int64_t f = g.cf[(size_t)g.mf * i + a];
      double sg = (g.fo[f] == i) ? 1.0 : -1.0;
      for (int k = 0; k < 3; ++k) acc[k] += sg * g.A[f] * g.n[3 * f + k];
      asum += g.A[f];
    }
    if (std::sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]) > 1e-10 * asum) return -2;
  }
  g.u.assign(u, u + 3 * nv);
  g.w.assign(w, w + nv);
  g.umag.assign(nv, 0.0);
  g.umax = 0.0;
  for (int64_t k = 0; k < nv; ++k) {
    if (!(w[k] > 0.0)) return -3;
    g.umag[k] = std::sqrt(u[3 * k] * u[3 * k] + u[3 * k + 1] * u[3 * k + 1] + u[3 * k + 2] * u[3 * k + 2]);
    g.umax = std::max(g.umax, g.umag[k]);
  }
  // reading: h_i = 6 V_i / sum_f A_f, dt_i = CFL h_i / max_k |u_k|; s_ij = min(dt_i, dt_j) (Eq. 45);
  // a boundary face uses dt of its cell.  Delta l_ij = |x_i - x_j| (Eq. 41), 2|x_f - x_i| on the boundary.
  g.h.assign(nc, 0.0);
  g.dt.assign(nc, 0.0);
  for (int64_t i = 0; i < nc; ++i) {
    double asum = 0.0;
    for (int a = 0; a < g.nfc[i]; ++a) asum += g.A[g.cf[(size_t)g.mf * i + a]];
    g.h[i] = 6.0 * g.V[i] / asum;
    g.dt[i] = cfl * g.h[i] / g.umax;
  }
  g.s.assign(g.nf, 0.0);
  g.dl.assign(g.nf, 0.0);
  for (int64_t f = 0; f < g.nf; ++f) {
    int64_t i = g.fo[f], j = g.fn[f];
    double d2 = 0.0;
    if (j >= 0) {
      g.s[f] = std::min(g.dt[i], g.dt[j]);
      for (int k = 0; k < 3; ++k) d2 += sq(g.xc[3 * i + k] - g.xc[3 * j + k]);
      g.dl[f] = std::sqrt(d2);
    } else {
      g.s[f] = g.dt[i];
      for (int k = 0; k < 3; ++k) d2 += sq(g.xf[3 * f + k] - g.xc[3 * i + k]);
      g.dl[f] = 2.0 * std::sqrt(d2);
    }
  }
  // reading: unweighted least squares over the face neighbours; a boundary face enters with
  // d = x_f - x_i and a zero difference.
  g.Minv.assign(9 * nc, 0.0);
  for (int64_t i = 0; i < nc; ++i) {
    double M[9] = {0};
    for (int a = 0; a < g.nfc[i]; ++a) {
      int64_t f = g.cf[(size_t)g.mf * i + a];
      int64_t j = (g.fo[f] == i) ? g.fn[f] : g.fo[f];
      double d[3];
      for (int k = 0; k < 3; ++k) d[k] = (j >= 0 ? g.xc[3 * j + k] : g.xf[3 * f + k]) - g.xc[3 * i + k];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] += d[r] * d[c];
    }
    if (!inv3(M, &g.Minv[9 * i])) return -2;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Sec. 2: macroscopic variables, temperatures, viscosity, relaxation time
// ---------------------------------------------------------------------------
template <class S> struct Prim {
  S rho, U[3], T, Ttr, Trot;
};

// Eqs. 1-5 with K_tr = 3, K_rot = 2:
//   rho E = 1/2 rho |U|^2 + 5/2 rho R T,  rho E_rot = rho R T_rot,
//   rho E - rho E_rot = 1/2 rho |U|^2 + 3/2 rho R T_tr.
template <class S> Prim<S> primitives(const S* W, const Gas& g) {
  Prim<S> p;
  p.rho = W[0];
  for (int k = 0; k < 3; ++k) p.U[k] = W[1 + k] / W[0];
  S ke = 0.5 * W[0] * (sq(p.U[0]) + sq(p.U[1]) + sq(p.U[2]));
  p.T = (2.0 / 5.0) * (W[4] - ke) / (W[0] * g.R);
  p.Trot = W[5] / (W[0] * g.R);
  p.Ttr = (2.0 / 3.0) * (W[4] - ke - W[5]) / (W[0] * g.R);
  return p;
}

// Eq. 13 (VHS): mu = mu_ref (T_tr / T_ref)^omega;  Eq. 14 (Sutherland, when C_s > 0):
// mu = mu_ref (T_tr / T_ref)^(3/2) (T_ref + C_s) / (T_tr + C_s);  tau = mu(T_tr) / p_tr (text after Eq. 12)
template <class S> S viscosity(const S& Ttr, const Gas& g) {
  if (g.C_s > 0.0) return g.mu_ref * pow(Ttr / g.T_ref, 1.5) * (g.T_ref + g.C_s) / (Ttr + g.C_s);
  return g.mu_ref * pow(Ttr / g.T_ref, g.omega_v);
}
template <class S> S relax_time(const Prim<S>& p, const Gas& g) {
  return viscosity(p.Ttr, g) / (p.rho * g.R * p.Ttr);
}

// Eq. 23: Maxwellian g^eq(u; rho, U, T)
template <class S> S maxwellian(const double* u, const S& rho, const S* U, const S& T, const Gas& g) {
  S c2 = sq(u[0] - U[0]) + sq(u[1] - U[1]) + sq(u[2] - U[2]);
  return rho * pow(2.0 * kPi * g.R * T, -1.5) * exp(-c2 / (2.0 * g.R * T));
}

// Eqs. 17-22: reduced Rykov equilibria at one velocity.
// reading: the p_2 of Eq. 12 is p = rho R T, as in Eqs. 20 and 22.
template <class S>
void rykov_equilibrium(const Prim<S>& p, const S* qtr, const S* qrot, const double* u, const Gas& g, S& Gs, S& Rs,
                       S* parts = nullptr) {
  const double R = g.R;
  S c[3] = {u[0] - p.U[0], u[1] - p.U[1], u[2] - p.U[2]};
  S c2 = sq(c[0]) + sq(c[1]) + sq(c[2]);
  S cqt = c[0] * qtr[0] + c[1] * qtr[1] + c[2] * qtr[2];
  S cqr = c[0] * qrot[0] + c[1] * qrot[1] + c[2] * qrot[2];
  S ptr = p.rho * R * p.Ttr, prot = p.rho * R * p.Trot, pp = p.rho * R * p.T;
  S geq_tr = maxwellian(u, p.rho, p.U, p.Ttr, g);
  S geq_T = maxwellian(u, p.rho, p.U, p.T, g);
  // Eq. 19
  S Gtr = geq_tr * (1.0 + cqt / (15.0 * R * p.Ttr * ptr) * (c2 / (R * p.Ttr) - 5.0));
  // Eq. 20
  S Grot = geq_T * (1.0 + g.omega0 * cqt / (15.0 * R * p.T * pp) * (c2 / (R * p.T) - 5.0));
  // Eq. 21
  S Rtr = R * p.Trot * (Gtr + (1.0 - g.delta) * cqr / (R * p.Ttr * prot) * geq_tr);
  // Eq. 22
  S Rrot = R * p.T * (Grot + g.omega1 * (1.0 - g.delta) * cqr / (R * p.T * pp) * geq_T);
  // Eqs. 17-18
  Gs = (1.0 - 1.0 / g.Z) * Gtr + Grot / g.Z;
  Rs = (1.0 - 1.0 / g.Z) * Rtr + Rrot / g.Z;
  if (parts) {
    parts[0] = Gtr;
    parts[1] = Grot;
    parts[2] = Rtr;
    parts[3] = Rrot;
  }
}

// Venkatakrishnan's limiter function of one face (the published method the paper cites for Eq. 46):
// d2 = grad(phi) . (x_f - x_i) is the unlimited change towards the face, d1 the room to the stencil's
// extremum on that side, eps2 the smoothing constant;
//   psi = [(d1^2 + eps2) d2 + 2 d2^2 d1] / [d2 (d1^2 + 2 d2^2 + d1 d2 + eps2)],  psi = 1 when d2 = 0.
template <class S> S venkat_psi(const S& d1, const S& d2, const S& eps2) {
  if (re(d2) == 0.0) return S(1.0);
  return ((sq(d1) + eps2) * d2 + 2.0 * sq(d2) * d1) / (d2 * (sq(d1) + 2.0 * sq(d2) + d1 * d2 + eps2));
}

// u.n with the tie rule: |u.n| <= snap |u| counts as 0 (reading: u.n = 0 is not "> 0", so the
// upwind cell is x_j, Eq. 46, and the boundary ghost side is used).
inline double u_dot_n(const Geom& g, int64_t k, const double* n, double snap) {
  const double* u = &g.u[3 * k];
  double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
  if (std::fabs(un) <= snap * g.umag[k]) un = 0.0;
  return un;
}

// Face macroscopic state after the collision coupling (Eqs. 47-52)
template <class S> struct FaceState {
  Prim<S> prim;
  S tau, q[6];
  S rho, rhoU[3], rhoE, sumR, Erot;
};

// Steps 2(b)-(d) on one interior face: from the reconstructed phi_bar (Eq. 46) to the face
// distribution of Eq. 45.  Gbar/Rbar/Gf/Rf are length-nv arrays over the DVS.
template <class S>
void face_collision(int64_t nv, const double* u, const double* w, const S* Gbar, const S* Rbar, double s,
                    const Gas& g, S* Gf, S* Rf, FaceState<S>& fs) {
  const double R = g.R, Z = g.Z;
  // Eqs. 47-49 and sum_k w R_bar
  S rho = 0.0, m[3] = {0.0, 0.0, 0.0}, E = 0.0, Er = 0.0;
  for (int64_t k = 0; k < nv; ++k) {
    const double* uk = u + 3 * k;
    double u2 = uk[0] * uk[0] + uk[1] * uk[1] + uk[2] * uk[2];
    rho += w[k] * Gbar[k];
    for (int d = 0; d < 3; ++d) m[d] += w[k] * uk[d] * Gbar[k];
    E += w[k] * (0.5 * u2 * Gbar[k] + Rbar[k]);
    Er += w[k] * Rbar[k];
  }
  S U[3] = {m[0] / rho, m[1] / rho, m[2] / rho};
  S ke = 0.5 * rho * (sq(U[0]) + sq(U[1]) + sq(U[2]));
  S T = (2.0 / 5.0) * (E - ke) / (rho * R);
  // reading: tau at the face from the translational temperature of phi_bar's own moments
  S Ttr_bar = (2.0 / 3.0) * (E - ke - Er) / (rho * R);
  S tau = viscosity(Ttr_bar, g) / (rho * R * Ttr_bar);
  // Eq. 50
  S Erot = (Z * tau * Er + s * rho * R * T) / (Z * tau + s);
  Prim<S> p;
  p.rho = rho;
  for (int d = 0; d < 3; ++d) p.U[d] = U[d];
  p.T = T;
  p.Trot = Erot / (rho * R);
  p.Ttr = (2.0 / 3.0) * (E - ke - Erot) / (rho * R);
  // Eqs. 51-52, c = u - U at the face
  S sq3[3] = {0.0, 0.0, 0.0}, sr[3] = {0.0, 0.0, 0.0};
  for (int64_t k = 0; k < nv; ++k) {
    const double* uk = u + 3 * k;
    S c[3] = {uk[0] - U[0], uk[1] - U[1], uk[2] - U[2]};
    S c2 = sq(c[0]) + sq(c[1]) + sq(c[2]);
    for (int d = 0; d < 3; ++d) {
      sq3[d] += w[k] * c[d] * c2 * Gbar[k];
      sr[d] += w[k] * c[d] * Rbar[k];
    }
  }
  S den_tr = tau + s - (s / 3.0) * (1.0 - 1.0 / Z + g.omega0 / Z);
  S den_rot = tau + s - s * (1.0 - g.delta) * (1.0 - 1.0 / Z + g.omega1 / Z);
  S q[6];
  for (int d = 0; d < 3; ++d) {
    q[d] = tau * 0.5 * sq3[d] / den_tr;
    q[3 + d] = tau * sr[d] / den_rot;
  }
  // Step 2(c)-(d): phi* at the face, then Eq. 45
  for (int64_t k = 0; k < nv; ++k) {
    S Gs, Rs;
    rykov_equilibrium(p, q, q + 3, u + 3 * k, g, Gs, Rs);
    Gf[k] = (tau * Gbar[k] + s * Gs) / (tau + s);
    Rf[k] = (tau * Rbar[k] + s * Rs) / (tau + s);
  }
  fs.prim = p;
  fs.tau = tau;
  for (int d = 0; d < 6; ++d) fs.q[d] = q[d];
  fs.rho = rho;
  for (int d = 0; d < 3; ++d) fs.rhoU[d] = m[d];
  fs.rhoE = E;
  fs.sumR = Er;
  fs.Erot = Erot;
}

// Euler flux with the rotational-energy row (Eq. 40), p = rho R T
template <class S> void euler_flux(const S* W, const double* n, const Gas& g, S* out) {
  Prim<S> p = primitives(W, g);
  S pr = p.rho * g.R * p.T;
  S Un = p.U[0] * n[0] + p.U[1] * n[1] + p.U[2] * n[2];
  out[0] = W[0] * Un;
  for (int d = 0; d < 3; ++d) out[1 + d] = W[1 + d] * Un + pr * n[d];
  out[4] = (W[4] + pr) * Un;
  out[5] = W[5] * Un;
}

// Exact Jacobian-vector product of the Euler flux (test mode for Eq. 42)
template <class S> void euler_flux_jvp(const S* W, const S* dW, const double* n, const Gas& g, S* out) {
  S rho = W[0];
  S U[3] = {W[1] / rho, W[2] / rho, W[3] / rho};
  S dU[3];
  for (int d = 0; d < 3; ++d) dU[d] = (dW[1 + d] - U[d] * dW[0]) / rho;
  S U2 = sq(U[0]) + sq(U[1]) + sq(U[2]);
  // p = (2/5)(rho E - 1/2 rho |U|^2) is rho R T with 5 internal degrees of freedom
  S pr = (2.0 / 5.0) * (W[4] - 0.5 * rho * U2);
  S dp = (2.0 / 5.0) * (dW[4] - (U[0] * dW[1] + U[1] * dW[2] + U[2] * dW[3]) + 0.5 * U2 * dW[0]);
  S Un = U[0] * n[0] + U[1] * n[1] + U[2] * n[2];
  S dUn = dU[0] * n[0] + dU[1] * n[1] + dU[2] * n[2];
  out[0] = dW[1] * n[0] + dW[2] * n[1] + dW[3] * n[2];
  for (int d = 0; d < 3; ++d) out[1 + d] = dW[1 + d] * Un + W[1 + d] * dUn + dp * n[d];
  out[4] = (dW[4] + dp) * Un + (W[4] + pr) * dUn;
  out[5] = dW[5] * Un + W[5] * dUn;
}

// ---------------------------------------------------------------------------
// The solver state and one implicit iteration (Sec. 3.5)
// ---------------------------------------------------------------------------
template <class S> struct Solver {
  const Geom& geo;
  Gas gas;
  Num num;
  std::vector<Bc<S>> bcs;
  int64_t nc, nf, nv;
  std::vector<S> G, R, W, q;  // state: phi [nc][nv]; W, q [nc][6]
  // stage outputs of the last pass
  std::vector<S> gradG, gradR;  // L * grad(phi), [nc][nv][3]
  std::vector<double> LfG, LfR; // limiter = 3: frozen limiter values, [nc][nv]
  bool capture = false;         // store the limiter values of the next reconstruction into LfG, LfR
  std::vector<S> ffG, ffR;      // face flux A (u.n) phi_f, [nf][nv]
  std::vector<S> ffmac;         // face macro flux A sum_k w (u.n) Phi phi_f, [nf][6]
  std::vector<S> Qface;         // A sum_k w (u.n)(|u|^2/2 G_f + R_f) on boundary faces, [nf]
  std::vector<S> FG, FR;        // micro flux per cell (Eq. 31), [nc][nv]
  std::vector<S> Fmac;          // macro flux per cell (Eq. 37), [nc][6]
  std::vector<S> dW, Wt, tau_t; // macro prediction (Eq. 43)
  std::vector<S> Gs, Rs;        // predicted equilibrium [nc][nv]
  std::vector<S> ResG, ResR, dG, dR;
  S res[6];

  Solver(const Geom& g, const double* gas_, const double* num_, const double* bc, int nbc)
      : geo(g), gas(gas_), num(num_), nc(g.nc), nf(g.nf), nv(g.nv) {
    for (int b = 0; b < nbc; ++b) {
      Bc<S> x;
      x.tag = int(bc[7 * b]);
      x.kind = int(bc[7 * b + 1]);
      x.rho = bc[7 * b + 2];
      for (int d = 0; d < 3; ++d) x.U[d] = bc[7 * b + 3 + d];
      x.T = bc[7 * b + 6];
      bcs.push_back(x);
    }
    size_t P = size_t(nc) * nv;
    G.assign(P, 0.0);
    R.assign(P, 0.0);
    W.assign(6 * nc, 0.0);
    q.assign(6 * nc, 0.0);
    for (auto& r : res) r = 0.0;
  }

  // Implicit time step of Eqs. 29 and 34 (one per cell, shared by both equations).
  // reading: 1/dt_i = inv_dt + max_k |u_k| / (CFL_imp h_i); CFL_imp = 0 drops the second term.
  double inv_dt_cell(int64_t i) const {
    double v = num.inv_dt;
    if (num.cfl_imp > 0.0) v += geo.umax / (num.cfl_imp * geo.h[i]);
    return v;
  }

  const Bc<S>* bc_of(int tag) const {
    for (auto& b : bcs)
      if (b.tag == tag) return &b;
    return nullptr;
  }

  // Step 1: equilibrium initial field, phi = phi*(W0, q = 0)
  void init_equilibrium(const double* W0, bool per_cell) {
    for (int64_t i = 0; i < nc; ++i) {
      const double* w0 = per_cell ? W0 + 6 * i : W0;
      for (int d = 0; d < 6; ++d) W[6 * i + d] = w0[d];
      for (int d = 0; d < 6; ++d) q[6 * i + d] = 0.0;
      Prim<S> p = primitives(&W[6 * i], gas);
      S z[3] = {0.0, 0.0, 0.0};
      for (int64_t k = 0; k < nv; ++k)
        rykov_equilibrium(p, z, z, &geo.u[3 * k], gas, G[size_t(i) * nv + k], R[size_t(i) * nv + k]);
    }
  }

  // Eq. 46 gradient: least squares + Venkatakrishnan limiter; stores L * grad(phi)
  void reconstruct_gradients() {
    size_t P = size_t(nc) * nv;
    gradG.assign(3 * P, 0.0);
    gradR.assign(3 * P, 0.0);
    if (capture) {
      LfG.assign(P, 1.0);
      LfR.assign(P, 1.0);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nc; ++i) {
      for (int which = 0; which < 2; ++which) {
        const std::vector<S>& phi = which == 0 ? G : R;
        std::vector<S>& out = which == 0 ? gradG : gradR;
        std::vector<double>& Lf = which == 0 ? LfG : LfR;
        const int lim = capture ? 1 : num.limiter;
        const double* Mi = &geo.Minv[9 * i];
        double kh3 = std::pow(num.lim_K * geo.h[i], 3.0);
        for (int64_t k = 0; k < nv; ++k) {
          S pi = phi[size_t(i) * nv + k];
          S b[3] = {0.0, 0.0, 0.0};
          S pmax = pi, pmin = pi;
          for (int a = 0; a < geo.nfc[i]; ++a) {
            int64_t f = geo.cf[(size_t)geo.mf * i + a];
            int64_t j = (geo.fo[f] == i) ? geo.fn[f] : geo.fo[f];
            if (j < 0) continue;
            S pj = phi[size_t(j) * nv + k];
            for (int d = 0; d < 3; ++d) b[d] += (geo.xc[3 * j + d] - geo.xc[3 * i + d]) * (pj - pi);
            if (re(pj) > re(pmax)) pmax = pj;
            if (re(pj) < re(pmin)) pmin = pj;
          }
          S gr[3];
          for (int r = 0; r < 3; ++r) gr[r] = Mi[3 * r] * b[0] + Mi[3 * r + 1] * b[1] + Mi[3 * r + 2] * b[2];
          S L = 1.0;
          // reading: eps^2 = (K h)^3 applied to phi scaled by its largest magnitude on the stencil,
          // i.e. eps^2 = (K h)^3 max(|phi_max|, |phi_min|)^2 (distribution values are far from O(1))
          // eps^2 is a function of phi: it carries the derivative of max(|phi_max|, |phi_min|)^2
          S scale = std::fabs(re(pmax)) >= std::fabs(re(pmin)) ? pmax : pmin;
          S eps2 = kh3 * scale * scale;
          if (lim == 3) {
            // frozen values (limiter freezing): a constant of every derivative
            L = S(Lf[size_t(i) * nv + k]);
          } else if (lim) {
            for (int a = 0; a < geo.nfc[i]; ++a) {
              int64_t f = geo.cf[(size_t)geo.mf * i + a];
              S d2 = 0.0;
              for (int d = 0; d < 3; ++d) d2 += gr[d] * (geo.xf[3 * f + d] - geo.xc[3 * i + d]);
              S d1 = re(d2) > 0.0 ? S(pmax - pi) : S(pmin - pi);
              S psi = venkat_psi(d1, d2, eps2);
              if (re(psi) < re(L)) L = psi;  // reading: L = min(1, min_f psi_f)
            }
            // limiter = 2: the same L in the iteration, held fixed in derivatives (frozen limiter), so a
            // complex step carries none of it
            if (lim == 2) L = S(re(L));
            // limiter = 4 (monotone freezing): the smaller of this value and the stored one, stored back
            if (lim == 4 && Lf[size_t(i) * nv + k] < re(L)) L = S(Lf[size_t(i) * nv + k]);
            if (lim == 4) L = S(re(L));
            if (capture || lim == 4) Lf[size_t(i) * nv + k] = re(L);
          }
          for (int d = 0; d < 3; ++d) out[3 * (size_t(i) * nv + k) + d] = L * gr[d];
        }
      }
    }
  }

  // Eq. 46: phi at x_f - u_k s from the cell c
  S recon(const std::vector<S>& phi, const std::vector<S>& grad, int64_t c, int64_t f, int64_t k, double s) const {
    const double* u = &geo.u[3 * k];
    S v = phi[size_t(c) * nv + k];
    for (int d = 0; d < 3; ++d)
      v += (geo.xf[3 * f + d] - u[d] * s - geo.xc[3 * c + d]) * grad[3 * (size_t(c) * nv + k) + d];
    return v;
  }

  // Steps 2-3: face distributions, micro flux (Eq. 31) and macro flux (Eq. 37)
  void face_pass() {
    size_t FP = size_t(nf) * nv;
    ffG.assign(FP, 0.0);
    ffR.assign(FP, 0.0);
    ffmac.assign(6 * nf, 0.0);
    Qface.assign(nf, 0.0);
#pragma omp parallel
    {
      std::vector<S> Gb(nv), Rb(nv), Gf(nv), Rf(nv);
#pragma omp for schedule(dynamic, 8)
      for (int64_t f = 0; f < nf; ++f) {
        const double* n = &geo.n[3 * f];
        const int64_t i = geo.fo[f], j = geo.fn[f];
        const double s = geo.s[f];
        if (j >= 0) {
          // Step 2(a): upwind reconstruction, x_c = x_i if u.n > 0 else x_j
          for (int64_t k = 0; k < nv; ++k) {
            double un = u_dot_n(geo, k, n, num.snap);
            int64_t c = un > 0.0 ? i : j;
            Gb[k] = recon(G, gradG, c, f, k, s);
            Rb[k] = recon(R, gradR, c, f, k, s);
          }
          FaceState<S> fs;
          face_collision(nv, geo.u.data(), geo.w.data(), Gb.data(), Rb.data(), s, gas, Gf.data(), Rf.data(), fs);
        } else {
          // Boundary face (reading): outgoing u.n > 0 carries phi_bar of the cell; incoming
          // u.n <= 0 carries the ghost: wall = Maxwellian at (U_w, T_w) with R = R T_w G and rho_w from
          // zero net mass flux; far field = free-stream Maxwellian.  No collision coupling.
          const Bc<S>* bc = bc_of(geo.ftag[f]);
          S out_mass = 0.0, in_mass = 0.0;
          S one = 1.0;
          for (int64_t k = 0; k < nv; ++k) {
            double un = u_dot_n(geo, k, n, num.snap);
            if (un > 0.0) {
              Gb[k] = recon(G, gradG, i, f, k, s);
              Rb[k] = recon(R, gradR, i, f, k, s);
              out_mass += geo.w[k] * un * Gb[k];
            } else if (bc->kind == BC_WALL) {
              in_mass += geo.w[k] * (-un) * maxwellian(&geo.u[3 * k], one, bc->U, bc->T, gas);
            }
          }
          S rho_w = bc->kind == BC_WALL ? S(out_mass / in_mass) : S(0.0);
          for (int64_t k = 0; k < nv; ++k) {
            double un = u_dot_n(geo, k, n, num.snap);
            if (un > 0.0) {
              Gf[k] = Gb[k];
              Rf[k] = Rb[k];
            } else if (bc->kind == BC_WALL) {
              Gf[k] = maxwellian(&geo.u[3 * k], rho_w, bc->U, bc->T, gas);
              Rf[k] = gas.R * bc->T * Gf[k];
            } else {
              Gf[k] = maxwellian(&geo.u[3 * k], bc->rho, bc->U, bc->T, gas);
              Rf[k] = gas.R * bc->T * Gf[k];
            }
          }
        }
        // Eq. 31 summand and Eq. 37 summand of this face
        S mac[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        S qw = 0.0;
        for (int64_t k = 0; k < nv; ++k) {
          const double* u = &geo.u[3 * k];
          double un = u_dot_n(geo, k, n, num.snap);
          double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
          ffG[size_t(f) * nv + k] = geo.A[f] * un * Gf[k];
          ffR[size_t(f) * nv + k] = geo.A[f] * un * Rf[k];
          double wun = geo.w[k] * un;
          mac[0] += wun * Gf[k];
          for (int d = 0; d < 3; ++d) mac[1 + d] += wun * u[d] * Gf[k];
          mac[4] += wun * (0.5 * u2 * Gf[k] + Rf[k]);
          mac[5] += wun * Rf[k];
          qw += wun * (0.5 * u2 * Gf[k] + Rf[k]);  // Eq. 72 numerator
        }
        for (int d = 0; d < 6; ++d) ffmac[6 * f + d] = geo.A[f] * mac[d];
        Qface[f] = j >= 0 ? S(0.0) : S(geo.A[f] * qw);
      }
    }
    // Eq. 31 and Eq. 37: per-cell sums over the faces of the cell
    size_t P = size_t(nc) * nv;
    FG.assign(P, 0.0);
    FR.assign(P, 0.0);
    Fmac.assign(6 * nc, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) {
      for (int a = 0; a < geo.nfc[i]; ++a) {
        int64_t f = geo.cf[(size_t)geo.mf * i + a];
        double sg = geo.fo[f] == i ? 1.0 : -1.0;  // n_ij points out of cell i
        for (int64_t k = 0; k < nv; ++k) {
          FG[size_t(i) * nv + k] += sg * ffG[size_t(f) * nv + k] / geo.V[i];
          FR[size_t(i) * nv + k] += sg * ffR[size_t(f) * nv + k] / geo.V[i];
        }
        for (int d = 0; d < 6; ++d) Fmac[6 * i + d] += sg * ffmac[6 * f + d] / geo.V[i];
      }
    }
  }

  // Step 4: implicit macroscopic prediction (Eqs. 38-43), PR-SGS with n_macro forward+backward sweeps.
  void macro_predict() {
    std::vector<Prim<S>> pr(nc);
    std::vector<S> tau(nc), mu(nc);
    for (int64_t i = 0; i < nc; ++i) {
      pr[i] = primitives(&W[6 * i], gas);
      tau[i] = relax_time(pr[i], gas);
    }
    // spectral radius r_ij (Eq. 41); reading: face state = arithmetic mean of the two cells'
    // rho, U, T, T_tr (a boundary face takes its cell's state); a = sqrt(gamma R T); mu = mu(T_tr).
    std::vector<S> rf(nf);
    for (int64_t f = 0; f < nf; ++f) {
      int64_t i = geo.fo[f], j = geo.fn[f];
      const Prim<S>& a = pr[i];
      const Prim<S>& b = j >= 0 ? pr[j] : pr[i];
      S rho = 0.5 * (a.rho + b.rho), T = 0.5 * (a.T + b.T), Ttr = 0.5 * (a.Ttr + b.Ttr);
      S Un = 0.0;
      for (int d = 0; d < 3; ++d) Un += 0.5 * (a.U[d] + b.U[d]) * geo.n[3 * f + d];
      S snd = sqrt(gas.gamma * gas.R * T);
      rf[f] = absr(Un) + snd + 2.0 * viscosity(Ttr, gas) / (rho * geo.dl[f]);
    }
    // Eq. 43: diagonal D_i and right-hand side Res_i.
    // reading: the source uses the lagged rho R T and tau of W^n; D_i sums r over every face of i.
    std::vector<S> D(nc), Res(6 * nc);
    for (int64_t i = 0; i < nc; ++i) {
      S acc = 0.0;
      for (int a = 0; a < geo.nfc[i]; ++a) {
        int64_t f = geo.cf[(size_t)geo.mf * i + a];
        acc += 0.5 * geo.A[f] / geo.V[i] * rf[f];
      }
      D[i] = inv_dt_cell(i) + acc;
      for (int d = 0; d < 6; ++d) Res[6 * i + d] = -Fmac[6 * i + d];
      Res[6 * i + 5] += (pr[i].rho * gas.R * pr[i].T - W[6 * i + 5]) / (gas.Z * tau[i]);
    }
    dW.assign(6 * nc, 0.0);
    auto relax = [&](int64_t i) {
      S acc[6];
      for (int d = 0; d < 6; ++d) acc[d] = Res[6 * i + d];
      for (int a = 0; a < geo.nfc[i]; ++a) {
        int64_t f = geo.cf[(size_t)geo.mf * i + a];
        int64_t j = (geo.fo[f] == i) ? geo.fn[f] : geo.fo[f];
        if (j < 0) continue;  // no increment across a boundary face
        double sg = geo.fo[f] == i ? 1.0 : -1.0;
        double n[3] = {sg * geo.n[3 * f], sg * geo.n[3 * f + 1], sg * geo.n[3 * f + 2]};
        S dG[6];
        if (num.exact_jvp) {
          euler_flux_jvp(&W[6 * j], &dW[6 * j], n, gas, dG);
        } else {
          // reading: dG/dW dW evaluated as G(W + dW) - G(W) (matrix-free)
          S Wp[6], G1[6], G0[6];
          for (int d = 0; d < 6; ++d) Wp[d] = W[6 * j + d] + dW[6 * j + d];
          euler_flux(Wp, n, gas, G1);
          euler_flux(&W[6 * j], n, gas, G0);
          for (int d = 0; d < 6; ++d) dG[d] = G1[d] - G0[d];
        }
        for (int d = 0; d < 6; ++d) acc[d] -= 0.5 * geo.A[f] / geo.V[i] * (dG[d] - rf[f] * dW[6 * j + d]);
      }
      for (int d = 0; d < 5; ++d) dW[6 * i + d] = acc[d] / D[i];
      dW[6 * i + 5] = acc[5] / (D[i] + 1.0 / (gas.Z * tau[i]));
    };
    for (int it = 0; it < num.n_macro; ++it) {
      for (int64_t i = 0; i < nc; ++i) relax(i);
      for (int64_t i = nc - 1; i >= 0; --i) relax(i);
    }
    Wt.assign(6 * nc, 0.0);
    for (size_t x = 0; x < Wt.size(); ++x) Wt[x] = W[x] + dW[x];
  }

  // Step 4 (second half) and the right-hand side of Eq. 33:
  // predicted equilibrium from W~ with q~ = q^n (reading), and Res = (phi~* - phi)/tau~ - F.
  void micro_residual() {
    size_t P = size_t(nc) * nv;
    Gs.assign(P, 0.0);
    Rs.assign(P, 0.0);
    ResG.assign(P, 0.0);
    ResR.assign(P, 0.0);
    tau_t.assign(nc, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) {
      Prim<S> p = primitives(&Wt[6 * i], gas);
      S tt = relax_time(p, gas);
      tau_t[i] = tt;
      for (int64_t k = 0; k < nv; ++k) {
        size_t x = size_t(i) * nv + k;
        rykov_equilibrium(p, &q[6 * i], &q[6 * i + 3], &geo.u[3 * k], gas, Gs[x], Rs[x]);
        ResG[x] = (Gs[x] - G[x]) / tt - FG[x];
        ResR[x] = (Rs[x] - R[x]) / tt - FR[x];
      }
    }
  }

  // Step 5: PR-SGS on Eq. 33 with the first-order upwind face increment of Eq. 32.
  void micro_sweeps() {
    size_t P = size_t(nc) * nv;
    dG.assign(P, 0.0);
    dR.assign(P, 0.0);
#pragma omp parallel
    {
#ifdef _OPENMP
      int tid = omp_get_thread_num();
      int nth = omp_get_num_threads();
#else
      int tid = 0, nth = 1;
#endif
      // each thread owns a contiguous range of velocities; the systems of different k are independent
      int64_t k0 = nv * tid / nth, k1 = nv * (tid + 1) / nth;
      auto relax = [&](int64_t i) {
        for (int64_t k = k0; k < k1; ++k) {
          S diag = inv_dt_cell(i) + 1.0 / tau_t[i];
          S accG = ResG[size_t(i) * nv + k], accR = ResR[size_t(i) * nv + k];
          for (int a = 0; a < geo.nfc[i]; ++a) {
            int64_t f = geo.cf[(size_t)geo.mf * i + a];
            double sg = geo.fo[f] == i ? 1.0 : -1.0;
            double n[3] = {sg * geo.n[3 * f], sg * geo.n[3 * f + 1], sg * geo.n[3 * f + 2]};
            double un = u_dot_n(geo, k, n, num.snap);
            double av = geo.A[f] / geo.V[i];
            diag += av * std::max(un, 0.0);  // D_i,k of Eq. 33
            int64_t j = (geo.fo[f] == i) ? geo.fn[f] : geo.fo[f];
            if (j < 0) continue;  // boundary increments are zero
            accG -= av * std::min(un, 0.0) * dG[size_t(j) * nv + k];  // D_j,k of Eq. 33
            accR -= av * std::min(un, 0.0) * dR[size_t(j) * nv + k];
          }
          dG[size_t(i) * nv + k] = accG / diag;
          dR[size_t(i) * nv + k] = accR / diag;
        }
      };
      for (int it = 0; it < num.n_micro; ++it) {
        for (int64_t i = 0; i < nc; ++i) relax(i);
        for (int64_t i = nc - 1; i >= 0; --i) relax(i);
      }
    }
  }

  // Step 6: phi^{n+1} = phi^n + dphi and the integral error compensation (Eqs. 62-67),
  // c = u - U~ (reading).  Step 7 residual: mean |W^{n+1} - W^n| over cells per component (reading).
  void update() {
    std::vector<S> Wn(6 * nc), qn(6 * nc);
    const double Z = gas.Z;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) {
      Prim<S> p = primitives(&Wt[6 * i], gas);
      S s[12];
      for (auto& x : s) x = 0.0;
      for (int64_t k = 0; k < nv; ++k) {
        size_t x = size_t(i) * nv + k;
        G[x] += dG[x];
        R[x] += dR[x];
        const double* u = &geo.u[3 * k];
        double wk = geo.w[k];
        double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        S gd = G[x] - Gs[x], rd = R[x] - Rs[x];
        S c[3] = {u[0] - p.U[0], u[1] - p.U[1], u[2] - p.U[2]};
        S c2 = sq(c[0]) + sq(c[1]) + sq(c[2]);
        s[0] += wk * gd;
        for (int d = 0; d < 3; ++d) s[1 + d] += wk * u[d] * gd;
        s[4] += wk * (0.5 * u2 * gd + rd);
        s[5] += wk * rd;
        for (int d = 0; d < 3; ++d) {
          s[6 + d] += wk * 0.5 * c[d] * c2 * gd;
          s[9 + d] += wk * c[d] * rd;
        }
      }
      const S* wt = &Wt[6 * i];
      Wn[6 * i + 0] = s[0] + wt[0];                                                  // Eq. 62
      for (int d = 0; d < 3; ++d) Wn[6 * i + 1 + d] = s[1 + d] + wt[1 + d];          // Eq. 63
      Wn[6 * i + 4] = s[4] + wt[4];                                                  // Eq. 64
      Wn[6 * i + 5] = s[5] + p.rho * gas.R * ((1.0 - 1.0 / Z) * p.Trot + p.T / Z);  // Eq. 65, K_rot/2 = 1
      for (int d = 0; d < 3; ++d) {
        qn[6 * i + d] = s[6 + d] + q[6 * i + d] * (1.0 / 3.0) * (1.0 - (1.0 - gas.omega0) / Z);           // Eq. 66
        qn[6 * i + 3 + d] = s[9 + d] + q[6 * i + 3 + d] * (1.0 - gas.delta) * (1.0 - (1.0 - gas.omega1) / Z);  // Eq. 67
      }
    }
    for (int d = 0; d < 6; ++d) res[d] = 0.0;
    for (int64_t i = 0; i < nc; ++i)
      for (int d = 0; d < 6; ++d) res[d] += absr(S(Wn[6 * i + d] - W[6 * i + d]));
    for (int d = 0; d < 6; ++d) res[d] /= double(nc);
    W.swap(Wn);
    q.swap(qn);
  }

  void explicit_pass() {
    reconstruct_gradients();
    face_pass();
  }

  void iterate() {
    explicit_pass();   // Steps 2-3
    macro_predict();   // Step 4
    micro_residual();  // Step 4-5
    micro_sweeps();    // Step 5
    update();          // Step 6
  }

  S wall_heat_flux(int tag) const {
    S acc = 0.0;
    for (int64_t f = 0; f < nf; ++f)
      if (geo.fn[f] < 0 && geo.ftag[f] == tag) acc += Qface[f];
    return acc;
  }

  // Steady residual of the fixed point of Steps 2-6 (reading: the adjoint's residual, not in the paper).
  // With W~ = W and q~ = q, a fixed point of the iteration satisfies
  //   R_phi = (phi*(W, q) - phi)/tau(W) - F(phi)                    (right-hand side of Eq. 33)
  //   R_W   = W - [sum_k w Phi (phi - phi*(W, q)) + M(W)]           (Eqs. 62-65 at W^{n+1} = W^n)
  //   R_q   = q - [1/2 sum w c|c|^2 (G - G*) + a0 q_tr ; sum w c (R - R*) + a1 q_rot]   (Eqs. 66-67)
  // where M(W) holds the analytic moments of phi*(W, q).
  void steady_residual(std::vector<S>& rG, std::vector<S>& rR, std::vector<S>& rW, std::vector<S>& rq) {
    explicit_pass();
    size_t P = size_t(nc) * nv;
    rG.assign(P, 0.0);
    rR.assign(P, 0.0);
    rW.assign(6 * nc, 0.0);
    rq.assign(6 * nc, 0.0);
    const double Z = gas.Z;
    for (int64_t i = 0; i < nc; ++i) {
      Prim<S> p = primitives(&W[6 * i], gas);
      S tau = relax_time(p, gas);
      S s[12];
      for (auto& x : s) x = 0.0;
      for (int64_t k = 0; k < nv; ++k) {
        size_t x = size_t(i) * nv + k;
        S Gs, Rs;
        rykov_equilibrium(p, &q[6 * i], &q[6 * i + 3], &geo.u[3 * k], gas, Gs, Rs);
        rG[x] = (Gs - G[x]) / tau - FG[x];
        rR[x] = (Rs - R[x]) / tau - FR[x];
        const double* u = &geo.u[3 * k];
        double wk = geo.w[k];
        double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        S gd = G[x] - Gs, rd = R[x] - Rs;
        S c[3] = {u[0] - p.U[0], u[1] - p.U[1], u[2] - p.U[2]};
        S c2 = sq(c[0]) + sq(c[1]) + sq(c[2]);
        s[0] += wk * gd;
        for (int d = 0; d < 3; ++d) s[1 + d] += wk * u[d] * gd;
        s[4] += wk * (0.5 * u2 * gd + rd);
        s[5] += wk * rd;
        for (int d = 0; d < 3; ++d) {
          s[6 + d] += wk * 0.5 * c[d] * c2 * gd;
          s[9 + d] += wk * c[d] * rd;
        }
      }
      const S* w = &W[6 * i];
      for (int d = 0; d < 5; ++d) rW[6 * i + d] = w[d] - (s[d] + w[d]);
      rW[6 * i + 5] = w[5] - (s[5] + p.rho * gas.R * ((1.0 - 1.0 / Z) * p.Trot + p.T / Z));
      for (int d = 0; d < 3; ++d) {
        rq[6 * i + d] = q[6 * i + d] - (s[6 + d] + q[6 * i + d] * (1.0 / 3.0) * (1.0 - (1.0 - gas.omega0) / Z));
        rq[6 * i + 3 + d] =
            q[6 * i + 3 + d] - (s[9 + d] + q[6 * i + 3 + d] * (1.0 - gas.delta) * (1.0 - (1.0 - gas.omega1) / Z));
      }
    }
  }
};

struct Handle {
  const Geom* geo;
  Solver<double>* sol;
};

template <class S> void copy_out(const std::vector<S>& v, double* out) {
  for (size_t x = 0; x < v.size(); ++x) out[x] = re(v[x]);
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface used by the Python wrapper (tests only)
// ---------------------------------------------------------------------------
extern "C" {

// cells [nc][8] node ids with kinds [nc] (4 tetrahedron, 5 pyramid, 6 prism, 8 hexahedron); bface [nb][4]
// boundary faces (-1 in the last place for a triangle) with tags btag.
void* orc_geom_create(const double* xyz, int64_t nn, const int32_t* cells, const int32_t* kinds, int64_t nc,
                      const int32_t* bface, const int32_t* btag, int64_t nb, const double* u, const double* w,
                      int64_t nv, double cfl, int32_t* status) {
  Geom* g = new Geom();
  int st = build_geom(*g, xyz, nn, cells, kinds, nc, bface, btag, nb, u, w, nv, cfl);
  if (status) *status = st;
  if (st != 0) {
    delete g;
    return nullptr;
  }
  return g;
}

void orc_geom_destroy(void* g) { delete static_cast<Geom*>(g); }

// OpenMP thread count of the oracle's parallel loops (n <= 0 leaves it); returns the count now in force.
int32_t orc_threads(int32_t n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

// counts: nc, nf, n_interior, nv, face slots per cell
void orc_geom_counts(void* gp, int64_t* out) {
  Geom* g = static_cast<Geom*>(gp);
  int64_t ni = 0;
  for (auto j : g->fn) ni += (j >= 0);
  out[0] = g->nc;
  out[1] = g->nf;
  out[2] = ni;
  out[3] = g->nv;
  out[4] = g->mf;
}

void orc_geom_arrays(void* gp, double* V, double* xc, double* h, double* dt, int64_t* cf, int64_t* fo, int64_t* fn,
                     int32_t* ftag, double* A, double* n, double* xf, double* s) {
  Geom* g = static_cast<Geom*>(gp);
  std::copy(g->V.begin(), g->V.end(), V);
  std::copy(g->xc.begin(), g->xc.end(), xc);
  std::copy(g->h.begin(), g->h.end(), h);
  std::copy(g->dt.begin(), g->dt.end(), dt);
  std::copy(g->cf.begin(), g->cf.end(), cf);
  std::copy(g->fo.begin(), g->fo.end(), fo);
  std::copy(g->fn.begin(), g->fn.end(), fn);
  std::copy(g->ftag.begin(), g->ftag.end(), ftag);
  std::copy(g->A.begin(), g->A.end(), A);
  std::copy(g->n.begin(), g->n.end(), n);
  std::copy(g->xf.begin(), g->xf.end(), xf);
  std::copy(g->s.begin(), g->s.end(), s);
}

void* orc_solver_create(void* gp, const double* gas, const double* num, const double* bc, int32_t nbc) {
  Geom* g = static_cast<Geom*>(gp);
  return new Solver<double>(*g, gas, num, bc, nbc);
}

void orc_solver_destroy(void* s) { delete static_cast<Solver<double>*>(s); }

void orc_init_equilibrium(void* sp, const double* W0, int32_t per_cell) {
  static_cast<Solver<double>*>(sp)->init_equilibrium(W0, per_cell != 0);
}

void orc_set_state(void* sp, const double* G, const double* R, const double* W, const double* q) {
  auto* s = static_cast<Solver<double>*>(sp);
  size_t P = size_t(s->nc) * s->nv;
  std::copy(G, G + P, s->G.begin());
  std::copy(R, R + P, s->R.begin());
  std::copy(W, W + 6 * s->nc, s->W.begin());
  std::copy(q, q + 6 * s->nc, s->q.begin());
}

void orc_get_state(void* sp, double* G, double* R, double* W, double* q) {
  auto* s = static_cast<Solver<double>*>(sp);
  if (G) copy_out(s->G, G);
  if (R) copy_out(s->R, R);
  if (W) copy_out(s->W, W);
  if (q) copy_out(s->q, q);
}

int32_t orc_iterate(void* sp, int32_t n, double* res_hist) {
  auto* s = static_cast<Solver<double>*>(sp);
  for (int it = 0; it < n; ++it) {
    s->iterate();
    if (res_hist)
      for (int d = 0; d < 6; ++d) res_hist[6 * it + d] = s->res[d];
    for (int d = 0; d < 6; ++d)
      if (!std::isfinite(s->res[d])) return -5;
  }
  return 0;
}

// Limiter freezing: store the limiter values (limiter 1's) of the current state; limiter = 3 then uses them.
void orc_freeze_limiter(void* sp) {
  auto* s = static_cast<Solver<double>*>(sp);
  s->capture = true;
  s->reconstruct_gradients();
  s->capture = false;
}

// Replace the numerics constants (e.g. the implicit time step between iterations)
void orc_set_num(void* sp, const double* num) { static_cast<Solver<double>*>(sp)->num = Num(num); }

void orc_explicit(void* sp) { static_cast<Solver<double>*>(sp)->explicit_pass(); }

// Stage arrays of the last pass: 0 FG, 1 FR, 2 Fmac, 3 dW, 4 ResG, 5 ResR, 6 dG, 7 dR,
// 8 gradG, 9 gradR, 10 Gs, 11 Rs, 12 Qface, 13 Wt, 14 ffG, 15 ffR, 16 ffmac, 17 tau_t
int64_t orc_stage(void* sp, int32_t which, double* out) {
  auto* s = static_cast<Solver<double>*>(sp);
  const std::vector<double>* v = nullptr;
  switch (which) {
    case 0: v = &s->FG; break;
    case 1: v = &s->FR; break;
    case 2: v = &s->Fmac; break;
    case 3: v = &s->dW; break;
    case 4: v = &s->ResG; break;
    case 5: v = &s->ResR; break;
    case 6: v = &s->dG; break;
    case 7: v = &s->dR; break;
    case 8: v = &s->gradG; break;
    case 9: v = &s->gradR; break;
    case 10: v = &s->Gs; break;
    case 11: v = &s->Rs; break;
    case 12: v = &s->Qface; break;
    case 13: v = &s->Wt; break;
    case 14: v = &s->ffG; break;
    case 15: v = &s->ffR; break;
    case 16: v = &s->ffmac; break;
    case 17: v = &s->tau_t; break;
    default: return -1;
  }
  if (out) copy_out(*v, out);
  return (int64_t)v->size();
}

double orc_wall_heat_flux(void* sp, int32_t tag) {
  auto* s = static_cast<Solver<double>*>(sp);
  s->explicit_pass();
  return s->wall_heat_flux(tag);
}

// Complex-step derivative of the wall heat flux after n_iter iterations from the current state,
// with respect to p = 0: T_w of the wall tag, 1: rho_inf, 2: |U_inf| of the far-field tag.
int32_t orc_cs_gradient(void* sp, int32_t param, int32_t wall_tag, int32_t ff_tag, double hstep, int32_t n_iter,
                        double* dJ, double* J) {
  auto* s = static_cast<Solver<double>*>(sp);
  std::vector<double> bcflat;
  for (auto& b : s->bcs) {
    bcflat.push_back(b.tag);
    bcflat.push_back(b.kind);
    bcflat.push_back(b.rho);
    for (int d = 0; d < 3; ++d) bcflat.push_back(b.U[d]);
    bcflat.push_back(b.T);
  }
  double gas[G_COUNT] = {s->gas.R,      s->gas.gamma,  s->gas.Z,       s->gas.delta, s->gas.omega0,
                         s->gas.omega1, s->gas.mu_ref, s->gas.omega_v, s->gas.T_ref, s->gas.C_s};
  double num[N_COUNT] = {s->num.cfl, s->num.inv_dt, s->num.cfl_imp, s->num.lim_K, double(s->num.limiter),
                         double(s->num.n_macro), double(s->num.n_micro), s->num.snap, double(s->num.exact_jvp)};
  Solver<cplx> c(s->geo, gas, num, bcflat.data(), int(s->bcs.size()));
  for (auto& b : c.bcs) {
    if (param == 0 && b.tag == wall_tag) b.T += cplx(0.0, hstep);
    if (param == 1 && b.tag == ff_tag) b.rho += cplx(0.0, hstep);
    if (param == 2 && b.tag == ff_tag) {
      double m = std::sqrt(sq(b.U[0].real()) + sq(b.U[1].real()) + sq(b.U[2].real()));
      for (int d = 0; d < 3; ++d) b.U[d] *= (m + cplx(0.0, hstep)) / m;
    }
  }
  c.LfG = s->LfG;
  c.LfR = s->LfR;
  for (size_t x = 0; x < c.G.size(); ++x) {
    c.G[x] = s->G[x];
    c.R[x] = s->R[x];
  }
  for (size_t x = 0; x < c.W.size(); ++x) {
    c.W[x] = s->W[x];
    c.q[x] = s->q[x];
  }
  for (int it = 0; it < n_iter; ++it) c.iterate();
  c.explicit_pass();
  cplx Jc = c.wall_heat_flux(wall_tag);
  *dJ = Jc.imag() / hstep;
  if (J) *J = Jc.real();
  return 0;
}

// Steady residual at the current state (reading of the adjoint's residual, see steady_residual) and
// J = wall heat flux of `wall_tag`.
void orc_steady_residual(void* sp, int32_t wall_tag, double* rG, double* rR, double* rW, double* rq, double* J) {
  auto* s = static_cast<Solver<double>*>(sp);
  std::vector<double> a, b, c, d;
  s->steady_residual(a, b, c, d);
  copy_out(a, rG);
  copy_out(b, rR);
  copy_out(c, rW);
  copy_out(d, rq);
  if (J) *J = s->wall_heat_flux(wall_tag);
}

// Complex-step directional derivative of the steady residual and of J at the current state along
// (uG, uR, uW, uq) in the state and up = (dT_w, drho_inf, d|U_inf|) in the parameters.
void orc_steady_residual_jvp(void* sp, int32_t wall_tag, int32_t ff_tag, const double* uG, const double* uR,
                             const double* uW, const double* uq, const double* up, double hstep, double* jG,
                             double* jR, double* jW, double* jq, double* jJ) {
  auto* s = static_cast<Solver<double>*>(sp);
  std::vector<double> bcflat;
  for (auto& b : s->bcs) {
    bcflat.push_back(b.tag);
    bcflat.push_back(b.kind);
    bcflat.push_back(b.rho);
    for (int d = 0; d < 3; ++d) bcflat.push_back(b.U[d]);
    bcflat.push_back(b.T);
  }
  double gas[G_COUNT] = {s->gas.R,      s->gas.gamma,  s->gas.Z,       s->gas.delta, s->gas.omega0,
                         s->gas.omega1, s->gas.mu_ref, s->gas.omega_v, s->gas.T_ref, s->gas.C_s};
  double num[N_COUNT] = {s->num.cfl, s->num.inv_dt, s->num.cfl_imp, s->num.lim_K, double(s->num.limiter),
                         double(s->num.n_macro), double(s->num.n_micro), s->num.snap, double(s->num.exact_jvp)};
  Solver<cplx> c(s->geo, gas, num, bcflat.data(), int(s->bcs.size()));
  const cplx ih(0.0, hstep);
  for (auto& b : c.bcs) {
    if (b.tag == wall_tag) b.T += ih * up[0];
    if (b.tag == ff_tag) {
      b.rho += ih * up[1];
      double m = std::sqrt(sq(b.U[0].real()) + sq(b.U[1].real()) + sq(b.U[2].real()));
      for (int d = 0; d < 3; ++d) b.U[d] *= (m + ih * up[2]) / m;
    }
  }
  c.LfG = s->LfG;
  c.LfR = s->LfR;
  for (size_t x = 0; x < c.G.size(); ++x) {
    c.G[x] = s->G[x] + ih * uG[x];
    c.R[x] = s->R[x] + ih * uR[x];
  }
  for (size_t x = 0; x < c.W.size(); ++x) {
    c.W[x] = s->W[x] + ih * uW[x];
    c.q[x] = s->q[x] + ih * uq[x];
  }
  std::vector<cplx> a, b, cc, d;
  c.steady_residual(a, b, cc, d);
  for (size_t x = 0; x < a.size(); ++x) {
    jG[x] = a[x].imag() / hstep;
    jR[x] = b[x].imag() / hstep;
  }
  for (size_t x = 0; x < cc.size(); ++x) {
    jW[x] = cc[x].imag() / hstep;
    jq[x] = d[x].imag() / hstep;
  }
  if (jJ) *jJ = c.wall_heat_flux(wall_tag).imag() / hstep;
}

// Rykov equilibrium at nv velocities for prim = (rho, U0, U1, U2, T, T_tr, T_rot) and q = (q_tr, q_rot).
void orc_equilibrium(const double* prim, const double* qv, const double* u, int64_t nv, const double* gas,
                     double* G, double* R, double* parts) {
  Gas g(gas);
  Prim<double> p;
  p.rho = prim[0];
  for (int d = 0; d < 3; ++d) p.U[d] = prim[1 + d];
  p.T = prim[4];
  p.Ttr = prim[5];
  p.Trot = prim[6];
  for (int64_t k = 0; k < nv; ++k) {
    double pt[4];
    rykov_equilibrium(p, qv, qv + 3, u + 3 * k, g, G[k], R[k], pt);
    if (parts)
      for (int a = 0; a < 4; ++a) parts[a * nv + k] = pt[a];
  }
}

// One interior face: phi_bar -> phi_f (Eqs. 45, 47-52).  macro = (rho, U0..2, T, T_tr, T_rot, tau,
// q_tr0..2, q_rot0..2, sumR, Erot)
void orc_face_collision(int64_t nv, const double* u, const double* w, const double* Gbar, const double* Rbar,
                        double s, const double* gas, double* Gf, double* Rf, double* macro) {
  Gas g(gas);
  FaceState<double> fs;
  face_collision(nv, u, w, Gbar, Rbar, s, g, Gf, Rf, fs);
  macro[0] = fs.prim.rho;
  for (int d = 0; d < 3; ++d) macro[1 + d] = fs.prim.U[d];
  macro[4] = fs.prim.T;
  macro[5] = fs.prim.Ttr;
  macro[6] = fs.prim.Trot;
  macro[7] = fs.tau;
  for (int d = 0; d < 6; ++d) macro[8 + d] = fs.q[d];
  macro[14] = fs.sumR;
  macro[15] = fs.Erot;
}

// Venkatakrishnan's function of one face (the function the limiter of Eq. 46 takes the minimum of)
double orc_venkat_psi(double d1, double d2, double eps2) { return venkat_psi(d1, d2, eps2); }

// Euler flux and its matrix-free / exact increments for a single state (pins of Eq. 40, 42)
void orc_euler_flux(const double* W, const double* n, const double* gas, double* out) {
  Gas g(gas);
  euler_flux(W, n, g, out);
}
void orc_euler_flux_jvp(const double* W, const double* dW, const double* n, const double* gas, double* out) {
  Gas g(gas);
  euler_flux_jvp(W, dW, n, g, out);
}

}  // extern "C"
