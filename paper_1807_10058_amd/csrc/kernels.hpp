// Device code of the radix-2x2x2 FCC cosine transform (Sec. IV-B, eq.
// FastAlgorithm) for gfx950.
//
// Data layout.  One volume is an n^3 array in lexicographic order.  The
// transform runs in place level by level on this index space: at level L a
// node J in [0,2^L)^3 owns the strided sub-lattice J + 2^L * a, a in [0, nl)^3,
// nl = n >> L, holding its coefficient vector in the basis b_nl.  The node's
// children are its 2x2x2 cosets: child i owns J + 2^L i + 2^(L+1) k, and its
// skew parameter is ((r,s,t) + J + 2^L i) / 2^(L+1) (eq. BaseCaseA3AlgebraLevel).
// After the last level every node is a single point and position j holds the
// value at the zero theta_j, so the permutation P_n of eq. PermutationStep...
// costs nothing.
//
// One thread owns one 2x2x2 cube of one node: (J, abc), abc in [0, nl/2)^3.
//   forward : y(def) = row (def,abc) of B_nl(c) applied to the node (gather),
//             z = DCT_2(phi) y, stored at the cube's 8 positions;
//   inverse : y = DCT_2(phi)^{-1} z on the cube, then a second pass gathers
//             x(kappa) = row kappa of C_nl(c) applied to y.
// DCT_2(phi)[i, def] = T_def((phi + i)/2) = (H_8 A(phi))[i, def], with
// H_8[i, mu] = (-1)^(i.mu) and A(phi)[mu, def] = (1/24) sum_{g: g def = mu mod 2}
// exp(i pi (g def).phi).  A is block diagonal over the classes of {0,1}^3 mod W:
// {000}, {001,011,100,110}, {010,101,111}.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fcc {

template <typename R>
struct cx {
  R x, y;
};
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cdiv(cx<R> a, cx<R> b) {
  R d = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
template <typename R>
__device__ __forceinline__ R cabs2(cx<R> a) { return a.x * a.x + a.y * a.y; }

// ---- element access (real or interleaved complex, float or double) ----------
template <typename T, typename R>
struct IO;
template <typename R>
struct IO<float, R> {
  static __device__ __forceinline__ cx<R> ld(const float* p, long long i) { return {R(p[i]), R(0)}; }
  static __device__ __forceinline__ void st(float* p, long long i, cx<R> v) { p[i] = float(v.x); }
};
template <typename R>
struct IO<double, R> {
  static __device__ __forceinline__ cx<R> ld(const double* p, long long i) { return {R(p[i]), R(0)}; }
  static __device__ __forceinline__ void st(double* p, long long i, cx<R> v) { p[i] = double(v.x); }
};
template <typename R>
struct IO<float2, R> {
  static __device__ __forceinline__ cx<R> ld(const float2* p, long long i) {
    float2 v = p[i];
    return {R(v.x), R(v.y)};
  }
  static __device__ __forceinline__ void st(float2* p, long long i, cx<R> v) { p[i] = make_float2(float(v.x), float(v.y)); }
};
template <typename R>
struct IO<double2, R> {
  static __device__ __forceinline__ cx<R> ld(const double2* p, long long i) {
    double2 v = p[i];
    return {R(v.x), R(v.y)};
  }
  static __device__ __forceinline__ void st(double2* p, long long i, cx<R> v) { p[i] = make_double2(double(v.x), double(v.y)); }
};

template <typename R2, typename R>
struct IO<cx<R2>, R> {
  static __device__ __forceinline__ cx<R> ld(const cx<R2>* p, long long i) {
    cx<R2> v = p[i];
    return {R(v.x), R(v.y)};
  }
  static __device__ __forceinline__ void st(cx<R2>* p, long long i, cx<R> v) { p[i] = {R2(v.x), R2(v.y)}; }
};

// Coefficient polynomials use the monomials {1, c3, c1, c2, c1 c3} of
// c = (sigma, tau, rho) of the node, in that order.
constexpr int kNumMono = 5;

// Order of a node's m^3 cubes in the sliced tables and in the thread map of
// the gather passes: tiles of 2^la x 2^lb x 2^lc cubes in lexicographic tile
// order, lexicographic inside a tile.  (0,0,0) is the plain order (a*m+b)*m+c.
struct CubeOrder {
  int la, lb, lc;
};
__host__ __device__ __forceinline__ void cube_abc(int q, int lgm, CubeOrder o, int a[3]) {
  const int li = o.la + o.lb + o.lc;
  const int inner = q & ((1 << li) - 1), tile = q >> li;
  const int ntc = lgm - o.lc, ntb = lgm - o.lb;
  a[2] = ((tile & ((1 << ntc) - 1)) << o.lc) | (inner & ((1 << o.lc) - 1));
  a[1] = (((tile >> ntc) & ((1 << ntb) - 1)) << o.lb) | ((inner >> o.lc) & ((1 << o.lb) - 1));
  a[0] = ((tile >> (ntc + ntb)) << o.la) | (inner >> (o.lb + o.lc));
}

// Fields of a packed table entry (node sizes up to 256).
__device__ __forceinline__ int ent_x(uint32_t e) { return int(e >> 24); }
__device__ __forceinline__ int ent_y(uint32_t e) { return int((e >> 16) & 255u); }
__device__ __forceinline__ int ent_z(uint32_t e) { return int((e >> 8) & 255u); }
__device__ __forceinline__ int ent_pid(uint32_t e) { return int(e & 255u); }

// Device view of the basis-change tables of one node size, sliced for the
// wavefronts that read them: the rows of S consecutive cubes form a slice; for
// each def (or i) the slice stores max-length entries interleaved cube by cube
// (entry e of the slice's cube j at start + e * S + j), padded with entries of
// coefficient zero.  S = 64 / 8^L at levels 0 and 1 (one slice per
// wavefront), S = 1 below (every lane of a wavefront reads the same row).
struct DevSide {
  const int* start;     // per (slice * 8 + f)
  const int* len;       // per (slice * 8 + f)
  const uint32_t* ent;  // (x << 24) | (y << 16) | (z << 8) | p: node-local source (x,y,z), polynomial p
  CubeOrder order;      // cube order of the slices
  const int* perm;      // S > 1: groups of 4 slices in block order (see GatherMap::cluster), else nullptr
};
struct DevLevel {
  DevSide b, c;        // forward B_nl, inverse C_nl
  const double* poly;  // npoly * kNumMono, constant polynomials first
  int npoly;
  int nconst;          // ids below nconst are constants
  int S;               // cubes per slice
};

// Thread map of a gather pass.  xcd: the blocks that the hardware deals
// round-robin to the 8 XCDs are renumbered so that each XCD works through one
// contiguous range of rows.  f_inner: the 8 rows f of one table slice are
// consecutive (otherwise f is the slowest index).  lg: log2 of the node group
// (levels >= 2): all rows of 2^lg consecutive nodes run before the next group;
// 3L means one group of all 8^L nodes.
// balance (levels with long rows): row f is summed by K_f = 2^kf adjacent
// lanes, each over a contiguous part of the row, then combined with lane
// shuffles.  Within a node group the threads run f by f in the order forder
// (decreasing K_f, which keeps every row's lanes aligned), lane k fastest,
// then cube, then node; off[i] is the first thread of the i-th f in the
// group and off[8] the group's thread count.
// cluster (levels 0 and 1): the threads run groups of 4 consecutive slices
// of one f, the 8 f of the same group one after the other, and the groups in
// the order DevSide::perm, which keeps the cubes of a block of B (or C)
// together: they read the same sources, so with xcd these stay in one XCD's L2.
struct GatherMap {
  int xcd, f_inner, lg;
  int balance, cluster;
  unsigned char kf[8], forder[8];
  long long off[9];
};

// Orbit-block form of the basis change (orbit_level.hpp).
// One orbit kind on the device.
// Every array offset below is a multiple of 16 bytes, and every array is
// padded to a multiple of 16 bytes, so blocks copy them with 16-byte loads.
struct DevOrbitKind {
  int nc;             // cubes of the orbit
  int off_w;          // wmat: 9 nc entries, the matrices G[w_j] of the cube slots (row-major)
  // sides: [0] B, [1] C, [2] B^T, [3] C^T (the transposed transform's factors;
  // B^T has C's layout and C^T has B's: rows are indexed by the other side's slots)
  int off_perm[4];    // i16: 8 ceil(nc/8) cube slots in wavefront order (-1: idle lane)
  int off_rowptr[4];  // u16: 40 nc + 1 segment starts, relative to off_ent
  int off_ent[4];     // u32: entries (slot << 16) | (k & 0xffff), coefficient k / 144
  int nent[4];
};
// Templates and representatives of one node size.  Each row of B (C) is split
// by the monomials {1, c3, c1, c2, c1 c3} of the node's coefficient
// polynomials: segment (row, q) lists the sources whose coefficient has a
// nonzero q-th monomial coefficient k / 144 (k a 16-bit integer: every
// coefficient is a multiple of 1/144), so a row is
// (1/144) sum_q mono_q(node) * (sum over segment q of k_e x_e).
struct DevOrbitLevel {
  const DevOrbitKind* kinds;
  const int16_t* perm;
  const uint16_t* rowptr;
  const uint32_t* ent;
  const int8_t* wmat;
  const uint32_t* reps;  // representatives p0 packed (x << 20) | (y << 10) | z
  // one block's orbits per chunk, {kind, first representative, count, log2 U}
  // with U the units of a block of that kind; [0] for blocks of one node
  // (level 0, K = U orbits), [1] for blocks of 8 nodes (K = U / 8)
  const int4* chunks[2];
  int nchunk[2];
  int lgm;               // log2 m
};

// Where the volumes of one launch live: one volume at `one` (arr == nullptr)
// or one pointer per volume in the device array `arr`.
struct VolPtrs {
  void* const* arr;
  void* one;
};
__device__ __forceinline__ void* vol_ptr(const VolPtrs& p, long long v) { return p.arr ? p.arr[v] : p.one; }
struct VolSet {
  VolPtrs in, out;
};

}  // namespace fcc
