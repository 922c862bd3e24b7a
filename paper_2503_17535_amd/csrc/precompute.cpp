// Host precompute of the HPS discretization (see precompute.hpp).
#include "precompute.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>

namespace hps {

int n_terms(int d) { return d == 2 ? 6 : 10; }

// ---------------------------------------------------------------------------
// merge geometry
// ---------------------------------------------------------------------------
static MergeGeom make_geom(int d) {
  MergeGeom g;
  g.d = d;
  g.nchild = 1 << d;
  g.nfaces = 2 * d;
  g.sub_per_face = 1 << (d - 1);
  if (d == 2) {
    // sides S, E, N, W
    const FaceDesc f[4] = {{1, 0, {0, -1}}, {0, 1, {1, -1}}, {1, 1, {0, -1}}, {0, 0, {1, -1}}};
    for (int i = 0; i < 4; ++i) g.faces[i] = f[i];
    const int off[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};   // a b c d = SW SE NE NW
    for (int c = 0; c < 4; ++c) { g.child_off[c][0] = off[c][0]; g.child_off[c][1] = off[c][1]; g.child_off[c][2] = 0; }
    // interfaces 5, 7, 6, 8 of the 2D merge (a|b, c|d, b|c, d|a): 5 and 7
    // share no child, so D's leading 2 x 2 interface blocks are block diagonal
    const int it[4][4] = {{0, 1, 1, 3}, {2, 3, 3, 1}, {1, 2, 2, 0}, {3, 0, 0, 2}};
    g.schur_p = 1;
    g.nint = 4;
    for (int i = 0; i < 4; ++i) for (int k = 0; k < 4; ++k) g.iface[i][k] = it[i][k];
  } else {
    // faces x-, x+, y-, y+, z-, z+ with tangential axes (y,z), (x,z), (x,y)
    const FaceDesc f[6] = {{0, 0, {1, 2}}, {0, 1, {1, 2}}, {1, 0, {0, 2}},
                           {1, 1, {0, 2}}, {2, 0, {0, 1}}, {2, 1, {0, 1}}};
    for (int i = 0; i < 6; ++i) g.faces[i] = f[i];
    const int off[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                           {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
    for (int c = 0; c < 8; ++c) for (int a = 0; a < 3; ++a) g.child_off[c][a] = off[c][a];
    // interfaces 9..20 of the 3D merge: the lower ring (a..d), the upper
    // ring (e..h), then the four horizontal ones; the two rings share no
    // child, so D's leading 8 x 8 interface blocks are block diagonal
    g.schur_p = 4;
    const int it[12][4] = {{0, 1, 1, 0}, {1, 3, 2, 2}, {2, 0, 3, 1}, {3, 2, 0, 3},
                           {4, 1, 5, 0}, {5, 3, 6, 2}, {6, 0, 7, 1}, {7, 2, 4, 3},
                           {0, 5, 4, 4}, {1, 5, 5, 4}, {2, 5, 6, 4}, {3, 5, 7, 4}};
    g.nint = 12;
    for (int i = 0; i < 12; ++i) for (int k = 0; k < 4; ++k) g.iface[i][k] = it[i][k];
  }
  // quadrant order of sub-faces: (lo,lo), (hi,lo), (hi,hi), (lo,hi)
  const int quad[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
  for (int c = 0; c < 8; ++c)
    for (int f = 0; f < 6; ++f) g.group_of[c][f] = -1;
  int grp = 0;
  for (int F = 0; F < g.nfaces; ++F) {
    const FaceDesc& fd = g.faces[F];
    for (int k = 0; k < g.sub_per_face; ++k) {
      int found = -1;
      for (int c = 0; c < g.nchild; ++c) {
        if (g.child_off[c][fd.axis] != fd.side) continue;
        bool ok = true;
        if (d == 2) ok = g.child_off[c][fd.tang[0]] == k;
        else ok = g.child_off[c][fd.tang[0]] == quad[k][0] && g.child_off[c][fd.tang[1]] == quad[k][1];
        if (ok) { found = c; break; }
      }
      g.group_child[grp] = found;
      g.group_face[grp] = F;
      g.group_of[found][F] = grp;
      ++grp;
    }
  }
  for (int c = 0; c < g.nchild; ++c) {
    int ne = 0;
    for (int F = 0; F < g.nfaces; ++F)
      if (g.child_off[c][g.faces[F].axis] == g.faces[F].side) g.ext_face[c][ne++] = F;
    for (int i = 0; i < 12; ++i) g.face_on_iface[c][i] = -1;
    int ni = 0;
    for (int i = 0; i < g.nint; ++i) {
      if (g.iface[i][0] == c) { g.face_on_iface[c][i] = g.iface[i][1]; g.int_list[c][ni++] = i; }
      if (g.iface[i][2] == c) { g.face_on_iface[c][i] = g.iface[i][3]; g.int_list[c][ni++] = i; }
    }
  }
  return g;
}

const MergeGeom& merge_geom(int d) {
  static const MergeGeom g2 = make_geom(2);
  static const MergeGeom g3 = make_geom(3);
  return d == 2 ? g2 : g3;
}

// ---------------------------------------------------------------------------
// 1D pieces
// ---------------------------------------------------------------------------
static void gauss_legendre_newton(int q, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration on the Legendre polynomial P_q from the asymptotic
  // initial guesses cos(pi (k + 3/4) / (q + 1/2)); weights 2 / ((1-x^2) P_q'^2).
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int k = 0; k < q; ++k) {
    double t = std::cos(M_PI * (k + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int j = 1; j < q; ++j) {
        double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      if (q == 0) p1 = 1.0;
      // p1 = P_q(t), p0 = P_{q-1}(t)
      dp = q * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = t;
    for (int j = 1; j < q; ++j) {
      double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
      p0 = p1;
      p1 = p2;
    }
    dp = q * (t * p1 - p0) / (t * t - 1.0);
    x[k] = t;
    w[k] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  std::vector<int> ord(q);
  for (int k = 0; k < q; ++k) ord[k] = k;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(q), ws(q);
  for (int k = 0; k < q; ++k) { xs[k] = x[ord[k]]; ws[k] = w[ord[k]]; }
  x.swap(xs);
  w.swap(ws);
}

// Barycentric weights by their product formula.
static std::vector<double> bary(const std::vector<double>& x) {
  const int n = (int)x.size();
  std::vector<double> w(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) w[j] /= (x[j] - x[k]);
  return w;
}

// Row-major (ny x nx) interpolation matrix from nodes x to targets y.
static std::vector<double> interp(const std::vector<double>& x, const std::vector<double>& y) {
  const int nx = (int)x.size(), ny = (int)y.size();
  std::vector<double> w = bary(x), M((size_t)nx * ny, 0.0);
  for (int i = 0; i < ny; ++i) {
    int hit = -1;
    for (int j = 0; j < nx; ++j)
      if (std::fabs(y[i] - x[j]) < 1e-15) hit = j;
    if (hit >= 0) { M[(size_t)i * nx + hit] = 1.0; continue; }
    double s = 0.0;
    for (int j = 0; j < nx; ++j) s += w[j] / (y[i] - x[j]);
    for (int j = 0; j < nx; ++j) M[(size_t)i * nx + j] = (w[j] / (y[i] - x[j])) / s;
  }
  return M;
}

// ---------------------------------------------------------------------------
// leaf operators
// ---------------------------------------------------------------------------
static LeafOps make_leaf_ops(int d, int p) {
  LeafOps o;
  o.d = d;
  o.p = p;
  o.q = p - 2;
  const int q = o.q;
  o.npts = d == 2 ? p * p : p * p * p;
  o.cheb.resize(p);
  const int N = p - 1;
  for (int j = 0; j < p; ++j) o.cheb[j] = -std::cos(M_PI * j / N);
  if (p % 2 == 1) o.cheb[p / 2] = 0.0;
  gauss_legendre_newton(q, o.gl, o.glw);
  // Chebyshev differentiation matrix, closed form
  //   D_ij = (c_i / c_j) (-1)^(i+j) / (x_i - x_j),  c_0 = c_N = 2, else 1,
  // with the diagonal from the zero row sums.
  o.D.assign((size_t)p * p, 0.0);
  for (int i = 0; i < p; ++i) {
    double ci = (i == 0 || i == N) ? 2.0 : 1.0, rs = 0.0;
    for (int j = 0; j < p; ++j) {
      if (i == j) continue;
      double cj = (j == 0 || j == N) ? 2.0 : 1.0;
      double v = (ci / cj) * (((i + j) % 2) ? -1.0 : 1.0) / (o.cheb[i] - o.cheb[j]);
      o.D[(size_t)i * p + j] = v;
      rs += v;
    }
    o.D[(size_t)i * p + i] = -rs;
  }
  o.G2C = interp(o.gl, o.cheb);
  o.C2G = interp(o.cheb, o.gl);
  // index sets
  auto coord = [&](int pt, int a) { return a == 0 ? pt % p : (a == 1 ? (pt / p) % p : pt / (p * p)); };
  o.pos_i.assign(o.npts, -1);
  o.pos_e.assign(o.npts, -1);
  for (int pt = 0; pt < o.npts; ++pt) {
    bool inner = true;
    for (int a = 0; a < d; ++a) {
      int c = coord(pt, a);
      if (c == 0 || c == p - 1) inner = false;
    }
    if (inner) { o.pos_i[pt] = (int)o.Ii.size(); o.Ii.push_back(pt); }
    else { o.pos_e[pt] = (int)o.Ie.size(); o.Ie.push_back(pt); }
  }
  o.n_i = (int)o.Ii.size();
  o.n_e = (int)o.Ie.size();
  o.n_face = d == 2 ? q : q * q;
  o.n_b = 2 * d * o.n_face;
  const MergeGeom& g = merge_geom(d);
  // Chebyshev points of each face in tensor order of its tangential coords
  o.face_cheb.assign(2 * d, {});
  for (int f = 0; f < 2 * d; ++f) {
    const FaceDesc& fd = g.faces[f];
    const int fixed = fd.side ? p - 1 : 0;
    const int n1 = p, n2 = d == 2 ? 1 : p;
    for (int t2 = 0; t2 < n2; ++t2)
      for (int t1 = 0; t1 < n1; ++t1) {
        int c[3] = {0, 0, 0};
        c[fd.axis] = fixed;
        c[fd.tang[0]] = t1;
        if (d == 3) c[fd.tang[1]] = t2;
        o.face_cheb[f].push_back(c[0] + p * c[1] + p * p * c[2]);
      }
  }
  // P with corner / edge averaging
  const int nf = o.n_face, npf = d == 2 ? p : p * p;
  o.P.assign((size_t)o.n_e * o.n_b, 0.0);
  std::vector<int> cnt(o.n_e, 0);
  for (int f = 0; f < 2 * d; ++f) {
    for (int t = 0; t < npf; ++t) {
      const int pt = o.face_cheb[f][t];
      const int row = o.pos_e[pt];
      cnt[row]++;
      const int t1 = t % p, t2 = t / p;
      for (int s = 0; s < nf; ++s) {
        const int s1 = s % q, s2 = s / q;
        double v = o.G2C[(size_t)t1 * q + s1];
        if (d == 3) v *= o.G2C[(size_t)t2 * q + s2];
        o.P[(size_t)row * o.n_b + f * nf + s] += v;
      }
    }
  }
  for (int r = 0; r < o.n_e; ++r)
    for (int c = 0; c < o.n_b; ++c) o.P[(size_t)r * o.n_b + c] /= cnt[r];
  // Q: normal derivative (sign = outward) at the face's Chebyshev points,
  // then Chebyshev -> Gauss interpolation on the face.
  o.Qref.assign((size_t)o.n_b * o.npts, 0.0);
  std::vector<double> Nf((size_t)npf * o.npts);
  for (int f = 0; f < 2 * d; ++f) {
    const FaceDesc& fd = g.faces[f];
    const double sign = fd.side ? 1.0 : -1.0;
    std::fill(Nf.begin(), Nf.end(), 0.0);
    for (int t = 0; t < npf; ++t) {
      const int pt = o.face_cheb[f][t];
      const int ca = coord(pt, fd.axis);
      for (int m = 0; m < p; ++m) {
        // point with coordinate `axis` replaced by m
        int c[3] = {coord(pt, 0), coord(pt, 1), d == 3 ? coord(pt, 2) : 0};
        c[fd.axis] = m;
        const int col = c[0] + p * c[1] + p * p * c[2];
        Nf[(size_t)t * o.npts + col] += sign * o.D[(size_t)ca * p + m];
      }
    }
    for (int s = 0; s < nf; ++s) {
      const int s1 = s % q, s2 = s / q;
      for (int t = 0; t < npf; ++t) {
        const int t1 = t % p, t2 = t / p;
        double w = o.C2G[(size_t)s1 * p + t1];
        if (d == 3) w *= o.C2G[(size_t)s2 * p + t2];
        if (w == 0.0) continue;
        for (int col = 0; col < o.npts; ++col)
          o.Qref[(size_t)(f * nf + s) * o.npts + col] += w * Nf[(size_t)t * o.npts + col];
      }
    }
  }
  return o;
}

const LeafOps& leaf_ops(int d, int p) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, LeafOps*> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(d, p);
  auto it = cache.find(key);
  if (it != cache.end()) return *it->second;
  LeafOps* o = new LeafOps(make_leaf_ops(d, p));
  cache[key] = o;
  return *o;
}

// Entry (pt_r, pt_c) of the term-t operator on a cell of half-width r.
// Term order: 2D xx, xy, yy, x, y, 0;  3D xx, yy, zz, xy, xz, yz, x, y, z, 0.
static inline double term_entry(const LeafOps& o, const std::vector<double>& D2, int t,
                                double r, int pr, int pc) {
  const int p = o.p, d = o.d;
  int cr[3] = {pr % p, (pr / p) % p, d == 3 ? pr / (p * p) : 0};
  int cc[3] = {pc % p, (pc / p) % p, d == 3 ? pc / (p * p) : 0};
  int kind, a = 0, b = 0;  // kind 0 = second derivative aa, 1 = mixed ab, 2 = first a, 3 = identity
  if (d == 2) {
    const int K[6] = {0, 1, 0, 2, 2, 3}, A[6] = {0, 0, 1, 0, 1, 0}, B[6] = {0, 1, 0, 0, 0, 0};
    kind = K[t]; a = A[t]; b = B[t];
  } else {
    const int K[10] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 3};
    const int A[10] = {0, 1, 2, 0, 0, 1, 0, 1, 2, 0}, B[10] = {0, 0, 0, 1, 2, 2, 0, 0, 0, 0};
    kind = K[t]; a = A[t]; b = B[t];
  }
  auto same_except = [&](int e1, int e2) {
    for (int k = 0; k < d; ++k)
      if (k != e1 && k != e2 && cr[k] != cc[k]) return false;
    return true;
  };
  switch (kind) {
    case 0:
      if (!same_except(a, a)) return 0.0;
      return D2[(size_t)cr[a] * p + cc[a]] / (r * r);
    case 1:
      if (!same_except(a, b)) return 0.0;
      return o.D[(size_t)cr[a] * p + cc[a]] * o.D[(size_t)cr[b] * p + cc[b]] / (r * r);
    case 2:
      if (!same_except(a, a)) return 0.0;
      return o.D[(size_t)cr[a] * p + cc[a]] / r;
    default:
      return pr == pc ? 1.0 : 0.0;
  }
}

void term_block(const LeafOps& o, int t, double r, const std::vector<int>& rows,
                const std::vector<int>& cols, std::vector<double>& out) {
  const int p = o.p;
  std::vector<double> D2((size_t)p * p, 0.0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += o.D[(size_t)i * p + k] * o.D[(size_t)k * p + j];
      D2[(size_t)i * p + j] = s;
    }
  out.assign(rows.size() * cols.size(), 0.0);
  for (size_t i = 0; i < rows.size(); ++i)
    for (size_t j = 0; j < cols.size(); ++j)
      out[i * cols.size() + j] = term_entry(o, D2, t, r, rows[i], cols[j]);
}

// ---------------------------------------------------------------------------
// points
// ---------------------------------------------------------------------------
static void leaf_corner(int d, int depth, double lo, double hi, long long leaf, double* corner) {
  const MergeGeom& g = merge_geom(d);
  const int nc = 1 << d;
  std::vector<int> digits(depth);
  for (int l = depth - 1; l >= 0; --l) { digits[l] = (int)(leaf % nc); leaf /= nc; }
  double size = hi - lo;
  for (int a = 0; a < d; ++a) corner[a] = lo;
  for (int l = 0; l < depth; ++l) {
    size *= 0.5;
    for (int a = 0; a < d; ++a) corner[a] += size * g.child_off[digits[l]][a];
  }
}

void leaf_points(int d, int depth, double lo, double hi, int p, double* xyz) {
  const LeafOps& o = leaf_ops(d, p);
  const long long nl = 1LL << (d * depth);
  const double r = (hi - lo) / 2.0 / (double)(1LL << depth);
  for (long long l = 0; l < nl; ++l) {
    double corner[3];
    leaf_corner(d, depth, lo, hi, l, corner);
    for (int pt = 0; pt < o.npts; ++pt) {
      int c[3] = {pt % p, (pt / p) % p, pt / (p * p)};
      for (int a = 0; a < d; ++a)
        xyz[((size_t)l * o.npts + pt) * d + a] = corner[a] + (o.cheb[c[a]] + 1.0) * r;
    }
  }
}

long long n_root_bdry(int d, int depth, int p) {
  const long long q = p - 2;
  if (d == 2) return 4LL * q * (1LL << depth);
  return 6LL * q * q * (1LL << (2 * depth));
}

void boundary_points(int d, int depth, double lo, double hi, int p, double* xyz) {
  const LeafOps& o = leaf_ops(d, p);
  const MergeGeom& g = merge_geom(d);
  const int q = o.q;
  const double w = (hi - lo) / (double)(1LL << depth);  // panel width
  const int quad[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
  size_t k = 0;
  const long long npanel = 1LL << ((d - 1) * depth);
  for (int F = 0; F < 2 * d; ++F) {
    const FaceDesc& fd = g.faces[F];
    for (long long pan = 0; pan < npanel; ++pan) {
      // hierarchical panel index -> panel position on the face
      long long i1 = 0, i2 = 0, rem = pan;
      std::vector<int> digits(depth);
      const int base = d == 2 ? 2 : 4;
      for (int l = depth - 1; l >= 0; --l) { digits[l] = (int)(rem % base); rem /= base; }
      for (int l = 0; l < depth; ++l) {
        if (d == 2) { i1 = 2 * i1 + digits[l]; }
        else { i1 = 2 * i1 + quad[digits[l]][0]; i2 = 2 * i2 + quad[digits[l]][1]; }
      }
      const int ns2 = d == 2 ? 1 : q;
      for (int s2 = 0; s2 < ns2; ++s2)
        for (int s1 = 0; s1 < q; ++s1) {
          double pt[3];
          pt[fd.axis] = fd.side ? hi : lo;
          pt[fd.tang[0]] = lo + w * (i1 + 0.5 * (o.gl[s1] + 1.0));
          if (d == 3) pt[fd.tang[1]] = lo + w * (i2 + 0.5 * (o.gl[s2] + 1.0));
          for (int a = 0; a < d; ++a) xyz[k * d + a] = pt[a];
          ++k;
        }
    }
  }
}

// ---------------------------------------------------------------------------
// interpolation at scattered points: containing leaf + tensor barycentric
// weights on its Chebyshev grid
// ---------------------------------------------------------------------------
static long long cell_leaf(int d, int depth, const long long* cell) {
  const MergeGeom& g = merge_geom(d);
  long long leaf = 0;
  for (int l = 0; l < depth; ++l) {
    const int sh = depth - 1 - l;
    int digit = 0;
    for (int c = 0; c < (1 << d); ++c) {
      bool ok = true;
      for (int a = 0; a < d; ++a) ok = ok && g.child_off[c][a] == (int)((cell[a] >> sh) & 1);
      if (ok) { digit = c; break; }
    }
    leaf = leaf * (1 << d) + digit;
  }
  return leaf;
}

int interp_weights(int d, int depth, double lo, double hi, int p, const double* x, long long m, long long* leaf,
                   double* w) {
  const LeafOps& o = leaf_ops(d, p);
  const long long ncell = 1LL << depth;
  const double h = (hi - lo) / (double)ncell, r = h / 2.0, tol = 1e-14;
  for (long long k = 0; k < m; ++k) {
    const double* xk = x + k * d;
    long long c0[3];
    for (int a = 0; a < d; ++a) {
      if (!(xk[a] >= lo - tol && xk[a] <= hi + tol)) return -1;
      c0[a] = std::min(ncell - 1, std::max(0LL, (long long)std::floor((xk[a] - lo) / h)));
    }
    // lowest-index leaf among the (up to 3^d) nearby cells that contain x
    long long best = -1, bestcell[3] = {0, 0, 0};
    const int nn = d == 2 ? 9 : 27;
    for (int t = 0; t < nn; ++t) {
      long long cell[3] = {0, 0, 0};
      bool ok = true;
      int tt = t;
      for (int a = 0; a < d; ++a) {
        cell[a] = c0[a] + (tt % 3) - 1;
        tt /= 3;
        if (cell[a] < 0 || cell[a] >= ncell) { ok = false; break; }
        const double clo = lo + (double)cell[a] * h;
        if (xk[a] < clo - tol || xk[a] > clo + h + tol) { ok = false; break; }
      }
      if (!ok) continue;
      const long long lf = cell_leaf(d, depth, cell);
      if (best < 0 || lf < best) {
        best = lf;
        for (int a = 0; a < d; ++a) bestcell[a] = cell[a];
      }
    }
    if (best < 0) return -1;
    leaf[k] = best;
    std::vector<double> w1[3];
    for (int a = 0; a < d; ++a) {
      double ref = (xk[a] - (lo + (double)bestcell[a] * h)) / r - 1.0;
      ref = std::min(1.0, std::max(-1.0, ref));
      w1[a] = interp(o.cheb, std::vector<double>{ref});
    }
    double* wk = w + k * (long long)o.npts;
    for (int pt = 0; pt < o.npts; ++pt) {
      const int c[3] = {pt % p, (pt / p) % p, pt / (p * p)};
      double v = 1.0;
      for (int a = 0; a < d; ++a) v *= w1[a][c[a]];
      wk[pt] = v;
    }
  }
  return 0;
}

void leaf_face_tables(int depth, int p, std::vector<int>& nbr, std::vector<long long>& bidx) {
  const MergeGeom& g = merge_geom(2);
  const long long nl = 1LL << (2 * depth), ncell = 1LL << depth;
  const int q = p - 2;
  nbr.assign(nl * 4, -1);
  bidx.assign(nl * 4, -1);
  std::vector<long long> cx(nl), cy(nl);
  std::vector<long long> at((size_t)ncell * ncell);
  for (long long l = 0; l < nl; ++l) {
    long long x = 0, y = 0, rem = l;
    std::vector<int> digits(depth);
    for (int k = depth - 1; k >= 0; --k) { digits[k] = (int)(rem % 4); rem /= 4; }
    for (int k = 0; k < depth; ++k) {
      x = 2 * x + g.child_off[digits[k]][0];
      y = 2 * y + g.child_off[digits[k]][1];
    }
    cx[l] = x;
    cy[l] = y;
    at[(size_t)(y * ncell + x)] = l;
  }
  const int opposite[4] = {2, 3, 0, 1};
  for (long long l = 0; l < nl; ++l)
    for (int f = 0; f < 4; ++f) {
      const FaceDesc& fd = g.faces[f];
      long long c[2] = {cx[l], cy[l]};
      c[fd.axis] += fd.side ? 1 : -1;
      if (c[fd.axis] < 0 || c[fd.axis] >= ncell) {
        const long long t = fd.axis == 0 ? cy[l] : cx[l];  // panel position along the face
        bidx[l * 4 + f] = ((long long)f * ncell + t) * q;
      } else {
        nbr[l * 4 + f] = (int)(at[(size_t)(c[1] * ncell + c[0])] * 4 + opposite[f]);
      }
    }
}

}  // namespace hps
