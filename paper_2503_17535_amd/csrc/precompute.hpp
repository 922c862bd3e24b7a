// Host-side (fp64) precomputation of the HPS leaf discretization and of the
// index tables that drive the merge and solve kernels.
//
// Discretization (Section 3.1; Appendix A.1 in 2D, Appendix C.1 in 3D):
//   * p Chebyshev-Lobatto points per leaf side (tensor grid, p^d points),
//   * q = p-2 Gauss-Legendre points per leaf side / q^2 per leaf face,
//   * P  (n_e x n_b): Gauss boundary data -> exterior Chebyshev points, by
//     barycentric Lagrange interpolation per face; corner (2D) and edge/corner
//     (3D) points average the faces they lie on,
//   * Q  (n_b x p^d): outward normal derivative at each face's Chebyshev
//     points followed by Chebyshev -> Gauss interpolation on that face.
// Layout conventions (identical to those the library's point queries expose):
//   point index ix + p*iy (+ p^2*iz), nodes ascending; faces x-,x+,y-,y+,z-,z+
//   (2D sides S,E,N,W); Gauss points of a face in tensor order of its
//   tangential coordinates (first fastest); a parent face is the
//   concatenation of its child faces in quadrant order (lo,lo),(hi,lo),
//   (hi,hi),(lo,hi).
#pragma once
#include <cstdint>
#include <vector>

namespace hps {

struct FaceDesc {
  int axis;     // normal axis
  int side;     // 0 = lo, 1 = hi
  int tang[2];  // tangential axes (tang[1] = -1 in 2D)
};

// Geometry of a 2^d-to-1 merge.
struct MergeGeom {
  int d = 2;
  int nchild = 4;       // 2^d
  int nfaces = 4;       // 2d
  int nint = 4;         // interior interfaces (4 in 2D, 12 in 3D)
  int sub_per_face = 2; // child faces per parent face (2^(d-1))
  FaceDesc faces[6];
  int child_off[8][3];
  // interface i: (child c1, face f1) | (child c2, face f2)
  int iface[12][4];
  // parent boundary groups, in parent order: group g -> (child, face)
  int group_child[24], group_face[24];
  // child c: its exterior faces (face order) and touched interfaces (increasing)
  int ext_face[8][3], int_list[8][3];
  int face_on_iface[8][12];  // face of child c on interface i, or -1
  // interfaces [0, schur_p) and [schur_p, 2 schur_p) share no child (the
  // D blocks between them are zero); the rest follow
  int schur_p = 0;
  int group_of[8][6];        // parent group of (child, exterior face), or -1
};
const MergeGeom& merge_geom(int d);

// Leaf operators for a given (d, p) on the reference cell [-1,1]^d.
struct LeafOps {
  int d = 2, p = 0, q = 0, npts = 0, n_i = 0, n_e = 0, n_b = 0, n_face = 0;
  std::vector<double> cheb, gl, glw;   // nodes / Gauss nodes / Gauss weights
  std::vector<double> D;               // p x p, row-major, d/dx on [-1,1]
  std::vector<double> G2C, C2G;        // p x q, q x p (row-major)
  std::vector<int> Ii, Ie;             // interior / exterior point lists (ascending)
  std::vector<int> pos_i, pos_e;       // point -> position in Ii / Ie (or -1)
  std::vector<std::vector<int>> face_cheb;  // per face: its Chebyshev points
  std::vector<double> P;               // n_e x n_b, row-major
  std::vector<double> Qref;            // n_b x npts, row-major (reference cell)
};
const LeafOps& leaf_ops(int d, int p);  // cached

// Dense operator of a coefficient term t on a cell of half-width r, restricted
// to rows `rows` and columns `cols` of the point grid; row-major result.
void term_block(const LeafOps& ops, int t, double r, const std::vector<int>& rows,
                const std::vector<int>& cols, std::vector<double>& out);

int n_terms(int d);

// Gauss points of the domain boundary / leaf points (see hps.h).
void leaf_points(int d, int depth, double lo, double hi, int p, double* xyz);
void boundary_points(int d, int depth, double lo, double hi, int p, double* xyz);
long long n_root_bdry(int d, int depth, int p);

// 2D leaf adjacency: nbr[leaf*4 + f] = neighbour leaf * 4 + its face across
// face f, or -1 on the domain boundary; bidx[leaf*4 + f] = offset of face f's
// Gauss points in the root boundary order, or -1 for an interior face.
void leaf_face_tables(int depth, int p, std::vector<int>& nbr, std::vector<long long>& bidx);

// Containing leaf and tensor barycentric weights of m scattered points (see
// hps_interp_weights); returns -1 if a point lies outside the domain.
int interp_weights(int d, int depth, double lo, double hi, int p, const double* x, long long m, long long* leaf,
                   double* w);

}  // namespace hps
