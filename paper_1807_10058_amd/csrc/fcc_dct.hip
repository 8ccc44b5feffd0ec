// MI355X (gfx950) implementation of the C ABI in include/fcc_dct.h: the
// radix-2x2x2 fast FCC cosine transform of Sec. IV-B (eq. FastAlgorithm) and
// its inverse, one launch per level (two for the inverse), FP64 or FP32
// stages.  Layout and per-thread work are described in kernels.hpp.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "asp_tables.hpp"
#include "fcc_dct.h"
#include "fold_plan.hpp"
#include "kernels.hpp"
#include "orbit_blocks.hpp"
#include "orbits.inc"
#include "plan.hpp"

namespace fcc {


// ---------------------------------------------------------------------------
// Per-node constants
// ---------------------------------------------------------------------------

// The half phases h_d = exp(i pi phi_d) of node J at level L (phi = ((r,s,t) +
// J) / 2^L): the phase table hph holds h_d for every J_d of the level.
// Positive powers only: Q[d][k] = h_d^(k+1), k = 0..2; negative powers are
// conjugates (|h_d| = 1).  Indices are compile-time constants at every use.
template <typename R>
__device__ __forceinline__ void node_pos_powers(const double2* __restrict__ hph, int L, const int J[3], cx<R> Q[3][3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double2 hv = hph[(d << L) + J[d]];
    Q[d][0] = {R(hv.x), R(hv.y)};
    Q[d][1] = Q[d][0] * Q[d][0];
    Q[d][2] = Q[d][1] * Q[d][0];
  }
}
template <typename R>
__device__ __forceinline__ cx<R> qpow(const cx<R> Q[3][3], int d, int l) {
  if (l == 0) return {R(1), R(0)};
  return l > 0 ? Q[d][l - 1] : conj(Q[d][-l - 1]);
}
template <typename R>
__device__ __forceinline__ cx<R> qphase(const cx<R> Q[3][3], int l0, int l1, int l2) {
  cx<R> v = qpow(Q, 0, l0);
  if (l1 != 0) v = v * qpow(Q, 1, l1);
  if (l2 != 0) v = v * qpow(Q, 2, l2);
  return v;
}

// t = A(phi) y accumulated term by term (A is never materialised):
// t[mu] = sum over orbit terms (f, lambda) with lambda = mu mod 2 of w e^{i pi lambda.phi} y[f].
template <typename R>
__device__ __forceinline__ void apply_A(const cx<R> Q[3][3], const cx<R> y[8], cx<R> t[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) t[i] = {R(0), R(0)};
#define FCC_APPLY_A(f, l0, l1, l2, w)                                               \
  {                                                                                 \
    constexpr int mu_ = (((l0) & 1) << 2) | (((l1) & 1) << 1) | ((l2) & 1);        \
    t[mu_] = t[mu_] + (R(w) * qphase(Q, (l0), (l1), (l2))) * y[f];                 \
  }
  FCC_DCT2_TERMS(FCC_APPLY_A)
#undef FCC_APPLY_A
}

// c = (sigma, tau, rho)(phi) = (T_100, T_010, T_001)(phi) and the five
// monomials of the coefficient polynomials, in the fixed order
// {1, c3, c1, c2, c1 c3} (the only ones the derivation produces).  Each c_d is
// an orbit sum of exp(2 pi i k.phi) = prod_d g_d^(k_d) with g_d = h_d^2 and
// k_d in {-1, 0, 1} (the c-terms), so a node needs a few complex products.
template <typename R, int l>
__device__ __forceinline__ cx<R> gpow(cx<R> g) {
  if constexpr (l > 0)
    return g;
  else
    return conj(g);
}
template <typename R, int l0, int l1, int l2>
__device__ __forceinline__ cx<R> gphase(const cx<R> g[3]) {
  if constexpr (l0 != 0) {
    cx<R> v = gpow<R, l0>(g[0]);
    if constexpr (l1 != 0) v = v * gpow<R, l1>(g[1]);
    if constexpr (l2 != 0) v = v * gpow<R, l2>(g[2]);
    return v;
  } else if constexpr (l1 != 0) {
    cx<R> v = gpow<R, l1>(g[1]);
    if constexpr (l2 != 0) v = v * gpow<R, l2>(g[2]);
    return v;
  } else if constexpr (l2 != 0) {
    return gpow<R, l2>(g[2]);
  } else {
    return cx<R>{R(1), R(0)};
  }
}
template <typename R>
__device__ __forceinline__ void node_mono(const double2* __restrict__ hph, int L, const int J[3],
                                          cx<R> mono[kNumMono]) {
  cx<R> g[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double2 hv = hph[(d << L) + J[d]];
    const cx<R> h{R(hv.x), R(hv.y)};
    g[d] = h * h;
  }
  cx<R> c[3] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
#define FCC_ADD_C(d, l0, l1, l2, w) c[d] = c[d] + R(w) * gphase<R, (l0), (l1), (l2)>(g);
  FCC_C_TERMS(FCC_ADD_C)
#undef FCC_ADD_C
  mono[0] = {R(1), R(0)};
  mono[1] = c[2];
  mono[2] = c[0];
  mono[3] = c[1];
  mono[4] = c[0] * c[2];
}

// Index of mu / def inside its block of A (class 1: {1,3,4,6}, class 2: {2,5,7}).
__host__ __device__ constexpr int blk_pos(int f) {
  // f: 0 1 2 3 4 5 6 7
  // ->  0 0 0 1 2 1 3 2
  return (0x23121000 >> (4 * f)) & 0xF;
}
__host__ __device__ constexpr int blk_class(int f) {
  // f: 0 1 2 3 4 5 6 7 -> 0 1 2 1 1 2 1 2
  return (0x21211210 >> (4 * f)) & 0xF;
}

// One block of A(phi): class CLS = 1 gives a4 (K = 4, classes {1,3,4,6}),
// CLS = 2 gives a3 (K = 3, {2,5,7}); A[0][0] = 1.
template <typename R, int CLS, int K>
__device__ __forceinline__ void build_A_block(const cx<R> Q[3][3], cx<R> a[K][K]) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) a[i][j] = {R(0), R(0)};
#define FCC_ADD_A(f, l0, l1, l2, w)                                                   \
  if constexpr ((f) != 0 && blk_class(f) == CLS) {                                    \
    constexpr int mu_ = (((l0) & 1) << 2) | (((l1) & 1) << 1) | ((l2) & 1);           \
    a[blk_pos(mu_)][blk_pos(f)] = a[blk_pos(mu_)][blk_pos(f)] + R(w) * qphase(Q, (l0), (l1), (l2)); \
  }
  FCC_DCT2_TERMS(FCC_ADD_A)
#undef FCC_ADD_A
}
template <typename R>
__device__ __forceinline__ void build_A(const cx<R> Q[3][3], cx<R> a4[4][4], cx<R> a3[3][3]) {
  build_A_block<R, 1, 4>(Q, a4);
  build_A_block<R, 2, 3>(Q, a3);
}

// In-place 8-point Walsh-Hadamard transform: z[i] = sum_mu (-1)^(i.mu) t[mu].
template <typename R>
__device__ __forceinline__ void hadamard8(cx<R> t[8]) {
#pragma unroll
  for (int s = 1; s < 8; s <<= 1)
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (!(i & s)) {
        cx<R> a = t[i], b = t[i | s];
        t[i] = a + b;
        t[i | s] = a - b;
      }
}

// Solve M v = b in place (Gaussian elimination, partial pivoting), small K.
// One real division per pivot: its reciprocal conj(p) / |p|^2 serves the
// elimination factors of its column and the back substitution.
template <typename R, int K>
__device__ __forceinline__ void solve_small(cx<R> M[K][K], cx<R> b[K]) {
  cx<R> ip[K];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    int piv = c;
    R best = cabs2(M[c][c]);
#pragma unroll
    for (int r = c + 1; r < K; ++r) {
      R v = cabs2(M[r][c]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
#pragma unroll
    for (int r = c + 1; r < K; ++r)
      if (r == piv) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          cx<R> tmp = M[c][j];
          M[c][j] = M[r][j];
          M[r][j] = tmp;
        }
        cx<R> tb = b[c];
        b[c] = b[r];
        b[r] = tb;
      }
    const R rd = R(1) / cabs2(M[c][c]);
    ip[c] = {M[c][c].x * rd, -M[c][c].y * rd};
#pragma unroll
    for (int r = c + 1; r < K; ++r) {
      cx<R> f = M[r][c] * ip[c];
#pragma unroll
      for (int j = c + 1; j < K; ++j) M[r][j] = M[r][j] - f * M[c][j];
      b[r] = b[r] - f * b[c];
    }
  }
#pragma unroll
  for (int c = K - 1; c >= 0; --c) {
    cx<R> s = b[c];
#pragma unroll
    for (int j = c + 1; j < K; ++j) s = s - M[c][j] * b[j];
    b[c] = s * ip[c];
  }
}

struct CubeIdx {
  int J[3], a[3];
};
// Thread t -> (node J, cube abc): the 8^L nodes of level L vary fastest, so
// from level 2 on a whole wavefront works on one cube position of 64 nodes
// (one table row, loads of adjacent nodes' elements); at levels 0 and 1 a
// wavefront covers one table slice.
__device__ __forceinline__ CubeIdx cube_of(long long t, int n, int L, int* cube) {
  const int mask = (1 << L) - 1;
  const int jf = int(t & ((1LL << (3 * L)) - 1));
  const long long c = t >> (3 * L);
  const int m = (n >> L) >> 1;
  CubeIdx ci;
  ci.J[0] = jf >> (2 * L);
  ci.J[1] = (jf >> L) & mask;
  ci.J[2] = jf & mask;
  ci.a[0] = int(c / ((long long)m * m));
  ci.a[1] = int((c / m) % m);
  ci.a[2] = int(c % m);
  *cube = int(c);
  return ci;
}
__device__ __forceinline__ long long gpos(int n, int L, const int J[3], int kx, int ky, int kz) {
  return ((long long)(J[0] + (kx << L)) * n + (J[1] + (ky << L))) * n + (J[2] + (kz << L));
}

// Coefficient of one table entry: polynomials are sorted so that ids below
// lv.nconst are constants (86% of all entries), read with one load.
template <typename R>
__device__ __forceinline__ cx<R> poly_value(const double* poly, int nconst, int pid, const cx<R> mono[kNumMono]) {
  const double* pc = poly + pid * kNumMono;
  if (pid < nconst) return {R(pc[0]), R(0)};
  cx<R> v = R(pc[0]) * mono[0];
#pragma unroll
  for (int q = 1; q < kNumMono; ++q) v = v + R(pc[q]) * mono[q];
  return v;
}

// The level's coefficient polynomials, copied to LDS by the whole block.
constexpr int kMaxPoly = 256;
__device__ __forceinline__ void load_polys(const DevLevel& lv, double* sp) {
  for (int i = threadIdx.x; i < lv.npoly * kNumMono; i += blockDim.x) sp[i] = lv.poly[i];
  __syncthreads();
}

// Gather sum_e coef(pid_e) in[J + 2^L src_e] over one sliced row, in entry
// order.  Software pipelined in chunks of 8: the table entries of chunk c+1
// are loaded while the data of chunk c is in flight, so a row of len entries
// costs about len/8 dependent memory round trips.  row_begin issues the row's
// first table loads (kernels call it before the barrier that publishes the
// polynomials in LDS, so the two overlap); row_finish does the rest.
constexpr int kChunk = 8;
struct RowCursor {
  int e0, len;
  uint32_t e8[kChunk];
};
__device__ __forceinline__ void row_begin(const DevSide& sd, int S, int r, int j, RowCursor& rc, int k = 0,
                                          int kf = 0) {
  const int len = sd.len[r];
  // part k of 2^kf: a contiguous range of the row's entries
  const int per = (len + (1 << kf) - 1) >> kf;
  const int eb = min(len, k * per);
  rc.e0 = sd.start[r] + j + eb * S;
  rc.len = min(len, eb + per) - eb;
  if (rc.len <= 0) return;
#pragma unroll
  for (int u = 0; u < kChunk; ++u) {
    const int e = min(u, rc.len - 1);  // past the row's end: repeat its last entry, unused
    rc.e8[u] = sd.ent[rc.e0 + e * S];
  }
}
// Sum of the parts of a row over its 2^kf adjacent lanes (every lane gets it).
template <typename R>
__device__ __forceinline__ cx<R> combine_parts(cx<R> v, int kf) {
  if (kf >= 1) v = v + cx<R>{__shfl_xor(v.x, 1), __shfl_xor(v.y, 1)};
  if (kf >= 2) v = v + cx<R>{__shfl_xor(v.x, 2), __shfl_xor(v.y, 2)};
  return v;
}
template <typename R, typename TI>
__device__ __forceinline__ cx<R> row_finish(const TI* __restrict__ in, int n, int L, const int J[3], const DevSide& sd,
                                            int S, RowCursor& rc, const double* sp, int nconst,
                                            const cx<R> mono[kNumMono]) {
  cx<R> acc{R(0), R(0)};
  const int len = rc.len, e0 = rc.e0;
  for (int c = 0; c < len; c += kChunk) {
    cx<R> v8[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      v8[u] = IO<TI, R>::ld(in, gpos(n, L, J, ent_x(rc.e8[u]), ent_y(rc.e8[u]), ent_z(rc.e8[u])));
    uint32_t en[kChunk];
    const bool more = c + kChunk < len;
    if (more) {
#pragma unroll
      for (int u = 0; u < kChunk; ++u) en[u] = sd.ent[e0 + min(c + kChunk + u, len - 1) * S];
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      if (c + u < len) acc = acc + poly_value(sp, nconst, ent_pid(rc.e8[u]), mono) * v8[u];
    if (more) {
#pragma unroll
      for (int u = 0; u < kChunk; ++u) rc.e8[u] = en[u];
    }
  }
  return acc;
}

// Gather of a row that is the same on every lane of the wavefront (levels >= 2
// with one cube per slice and at least 64 consecutive nodes per group: lanes
// differ only in the node).  The row index is made provably uniform, so the
// table entries and the polynomial coefficients are read through the scalar
// cache and no LDS copy of the polynomials is needed.  Same entry order as
// row_finish.
template <typename R, typename TI>
__device__ __forceinline__ cx<R> row_uniform(const TI* __restrict__ in, int n, int L, const int J[3],
                                             const DevSide& sd, int r, const double* __restrict__ poly, int nconst,
                                             const cx<R> mono[kNumMono]) {
  r = __builtin_amdgcn_readfirstlane(r);
  const int e0 = __builtin_amdgcn_readfirstlane(sd.start[r]);
  const int len = __builtin_amdgcn_readfirstlane(sd.len[r]);
  cx<R> acc{R(0), R(0)};
  for (int c = 0; c < len; c += kChunk) {
    uint32_t e8[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) e8[u] = __builtin_amdgcn_readfirstlane(sd.ent[e0 + min(c + u, len - 1)]);
    cx<R> v8[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) v8[u] = IO<TI, R>::ld(in, gpos(n, L, J, ent_x(e8[u]), ent_y(e8[u]), ent_z(e8[u])));
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      if (c + u < len) acc = acc + poly_value(poly, nconst, ent_pid(e8[u]), mono) * v8[u];
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Per-node constants of one level, precomputed in FP64 at plan time for the
// levels with few nodes (every cube of such a node reuses them).
// (A's blocks are stored, not their inverses: the inverse pass solves with
// partial pivoting per cube, which stays accurate where A is ill conditioned;
// applying a precomputed inverse raised the n = 256 round-trip error 1e4-fold.)
struct NodeConst {
  double2 a4[16], a3[9];  // blocks of A(phi)
};
constexpr long long kNodeTableMax = 1 << 18;  // levels with at most this many nodes get a table (126 MB)

__global__ void k_node_table(NodeConst* out, int L, const double2* __restrict__ hph) {
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= (1LL << (3 * L))) return;
  const int mask = (1 << L) - 1;
  const int J[3] = {int(node >> (2 * L)), int((node >> L) & mask), int(node & mask)};
  cx<double> Q[3][3];
  node_pos_powers(hph, L, J, Q);
  cx<double> a4[4][4], a3[3][3];
  build_A(Q, a4, a3);
  NodeConst& nc = out[node];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) nc.a4[4 * i + j] = make_double2(a4[i][j].x, a4[i][j].y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) nc.a3[3 * i + j] = make_double2(a3[i][j].x, a3[i][j].y);
}

template <typename R>
__device__ __forceinline__ cx<R> ldc(const double2& v) {
  return {R(v.x), R(v.y)};
}

// Thread t (within one volume) -> one row of the level's gather: node J (the
// 8^L nodes vary fastest), then cube (in the side's cube order) and f.  With
// f outermost, a wavefront at level 0 (1) covers the 64 (8) cubes of one table
// slice for one f; with f_inner the 8 f of a slice follow each other.  From
// level 2 on a wavefront covers 64 nodes of one row.
struct RowIdx {
  int J[3], a[3], cube, f;
};
__device__ __forceinline__ RowIdx row_of(long long t, int n, int L, CubeOrder ord, int S, GatherMap gm,
                                         const int* perm = nullptr) {
  const int mask = (1 << L) - 1;
  const int lgm = __ffs(n) - 2 - L;  // log2 of m = n / 2^(L+1)
  // node within its group fastest, then the row, then the group
  const int lg = gm.lg;
  const long long rows = 8LL << (3 * lgm);
  const long long hi = t >> lg;
  const long long grp = hi / rows, rest = hi - grp * rows;
  const int jf = int((grp << lg) | (t & ((1LL << lg) - 1)));
  RowIdx r;
  if (gm.cluster) {
    // unit q = (block of 4 slices, f, slice within the block); 64 lanes each
    const long long q = rest / S;
    r.f = int((q >> 2) & 7);
    r.cube = (perm[q >> 5] * 4 + int(q & 3)) * S + int(rest - q * S);
  } else if (gm.f_inner) {
    const long long sf = rest / S;  // slice * 8 + f
    r.f = int(sf & 7);
    r.cube = int((sf >> 3) * S + (rest - sf * S));
  } else {
    r.f = int(rest >> (3 * lgm));
    r.cube = int(rest & ((1LL << (3 * lgm)) - 1));
  }
  r.J[0] = jf >> (2 * L);
  r.J[1] = (jf >> L) & mask;
  r.J[2] = jf & mask;
  cube_abc(r.cube, lgm, ord, r.a);
  return r;
}

// Balanced map (GatherMap::balance): thread t of one volume -> (row, lane k
// of the row's K = 2^kf lanes).
struct RowPart {
  RowIdx r;
  int k, kf;
};
__device__ __forceinline__ RowPart row_part_of(long long t, int n, int L, CubeOrder ord, const GatherMap& gm) {
  const int mask = (1 << L) - 1;
  const int lgm = __ffs(n) - 2 - L;
  const long long per = gm.off[8];
  const long long grp = t / per;
  const long long r0 = t - grp * per;
  int i = 0;
#pragma unroll
  for (int q = 1; q < 8; ++q) i += r0 >= gm.off[q] ? 1 : 0;
  RowPart rp;
  rp.r.f = gm.forder[i];
  rp.kf = gm.kf[i];
  const long long v = r0 - gm.off[i];
  rp.k = int(v & ((1 << rp.kf) - 1));
  const long long w = v >> rp.kf;  // cube, then node within the group
  rp.r.cube = int(w >> gm.lg);
  const int jf = int((grp << gm.lg) | (w & ((1LL << gm.lg) - 1)));
  rp.r.J[0] = jf >> (2 * L);
  rp.r.J[1] = (jf >> L) & mask;
  rp.r.J[2] = jf & mask;
  cube_abc(rp.r.cube, lgm, ord, rp.r.a);
  return rp;
}

// Block index of a gather launch (GatherMap::xcd: blocks i, i+8, i+16, ... run
// on one XCD and get one contiguous range).
// xcd = 2: runs of 16 consecutive blocks per XCD instead (blocks past the last
// whole group of 8 x 16 keep their number).
__device__ __forceinline__ long long gather_block(int xcd) {
  if (!xcd) return blockIdx.x;
  const unsigned nb = gridDim.x, i = blockIdx.x, x = i & 7u, l = i >> 3;
  if (xcd == 2) {
    const unsigned whole = nb / 128u * 128u;
    if (i >= whole) return i;
    return (long long)(l >> 4) * 128 + x * 16 + (l & 15u);
  }
  const unsigned per = nb >> 3, rem = nb & 7u;
  return (long long)x * per + min(x, rem) + l;
}

template <typename R>
__device__ __forceinline__ void load_mono(const NodeConst*, const double2* __restrict__ hph, int L, const int J[3],
                                          cx<R> mono[kNumMono]) {
  node_mono(hph, L, J, mono);
}

// Forward level L, first pass: y(def, abc) = row (def,abc) of B_nl(c) applied to
// the node, one thread per row, stored at node-local position def + 2 abc.
template <typename R, typename TI, bool kUni>
__global__ __launch_bounds__(256) void k_fwd_gather(VolSet vs, int nvol, int n, int L, DevLevel lv,
                                                    const double2* __restrict__ hph, const NodeConst* nodes, GatherMap gm) {
  if constexpr (kUni) {
    // wave-uniform rows (see row_uniform): no LDS, no barrier
    const long long N = (long long)n * n * n;
    const long long tg = gather_block(gm.xcd) * blockDim.x + threadIdx.x;
    if (tg >= N * nvol) return;
    const long long vol = tg / N, t = tg - vol * N;
    const RowIdx ri = row_of(t, n, L, lv.b.order, 1, gm);
    cx<R> mono[kNumMono];
    load_mono(nodes, hph, L, ri.J, mono);
    const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, vol));
    cx<R>* __restrict__ out = static_cast<cx<R>*>(vol_ptr(vs.out, vol));
    const cx<R> y = row_uniform<R, TI>(in, n, L, ri.J, lv.b, ri.cube * 8 + ri.f, lv.poly, lv.nconst, mono);
    out[gpos(n, L, ri.J, ((ri.f >> 2) & 1) + 2 * ri.a[0], ((ri.f >> 1) & 1) + 2 * ri.a[1], (ri.f & 1) + 2 * ri.a[2])] = y;
    return;
  }
  __shared__ double sp[kMaxPoly * kNumMono];
  const long long N = gm.balance ? gm.off[8] * ((1LL << (3 * L)) >> gm.lg) : (long long)n * n * n;  // threads per volume
  const long long tg = gather_block(gm.xcd) * blockDim.x + threadIdx.x;
  const bool active = tg < N * nvol;
  const long long vol = active ? tg / N : 0, t = tg - vol * N;
  RowIdx ri{};
  RowCursor rc{};
  cx<R> mono[kNumMono];
  int k = 0, kf = 0;
  if (active) {
    if (gm.balance) {
      const RowPart rp = row_part_of(t, n, L, lv.b.order, gm);
      ri = rp.r, k = rp.k, kf = rp.kf;
    } else {
      ri = row_of(t, n, L, lv.b.order, lv.S, gm, lv.b.perm);
    }
    const int slice = ri.cube / lv.S;
    row_begin(lv.b, lv.S, slice * 8 + ri.f, ri.cube - slice * lv.S, rc, k, kf);
    load_mono(nodes, hph, L, ri.J, mono);
  }
  load_polys(lv, sp);
  if (!active) return;
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, vol));
  cx<R>* __restrict__ out = static_cast<cx<R>*>(vol_ptr(vs.out, vol));
  cx<R> y = row_finish<R, TI>(in, n, L, ri.J, lv.b, lv.S, rc, sp, lv.nconst, mono);
  if (gm.balance) y = combine_parts(y, kf);
  if (k == 0)
    out[gpos(n, L, ri.J, ((ri.f >> 2) & 1) + 2 * ri.a[0], ((ri.f >> 1) & 1) + 2 * ri.a[1], (ri.f & 1) + 2 * ri.a[2])] = y;
}

// Forward level L in one pass.  Lane f of an aligned group of 8 lanes gathers
// row (f, abc) of B_nl for one cube; the group then applies DCT_2 = H_8 A(phi)
// to the cube's 8 values with lane shuffles (A is block diagonal: each lane
// combines at most 4 values of its class; H_8 is a 3-stage butterfly) and
// lane i stores output i at node-local position i + 2 abc.
struct CubeUnit {
  int J[3], a[3], cube;
};
// unit u = one (node, cube): node within its group fastest, then the cube (in
// the table's cube order), then the group
__device__ __forceinline__ CubeUnit unit_of(long long u, int n, int L, CubeOrder ord, int lg) {
  const int mask = (1 << L) - 1;
  const int lgm = __ffs(n) - 2 - L;
  const long long hi = u >> lg;
  const long long grp = hi >> (3 * lgm);
  CubeUnit c;
  c.cube = int(hi & ((1LL << (3 * lgm)) - 1));
  const int jf = int((grp << lg) | (u & ((1LL << lg) - 1)));
  c.J[0] = jf >> (2 * L);
  c.J[1] = (jf >> L) & mask;
  c.J[2] = jf & mask;
  cube_abc(c.cube, lgm, ord, c.a);
  return c;
}
template <typename R>
__device__ __forceinline__ cx<R> shfl8(cx<R> v, int src) {
  return {__shfl(v.x, src, 8), __shfl(v.y, src, 8)};
}
template <typename R>
__device__ __forceinline__ cx<R> shfl_xor8(cx<R> v, int m) {
  return {__shfl_xor(v.x, m, 8), __shfl_xor(v.y, m, 8)};
}
// z_i = sum_mu (-1)^(i.mu) w_mu over the 8 lanes of a group (lane = index)
template <typename R>
__device__ __forceinline__ cx<R> hadamard8_lanes(cx<R> w, int f) {
#pragma unroll
  for (int s = 1; s < 8; s <<= 1) {
    const cx<R> o = shfl_xor8(w, s);
    w = (f & s) ? o - w : w + o;
  }
  return w;
}
// (A y)_f on the lanes of a group; y is this lane's row value.  kTable: the
// level has a node table (A's blocks precomputed); otherwise every lane forms
// A y for the whole cube (a separate instantiation: it needs many registers).
template <typename R, bool kTable>
__device__ __forceinline__ cx<R> apply_A_lanes(const NodeConst* nodes, const double2* __restrict__ hph, int L,
                                               const int J[3], int f, cx<R> y) {
  if constexpr (kTable) {
    const NodeConst& nc = nodes[((long long)J[0] << (2 * L)) | ((long long)J[1] << L) | J[2]];
    // classes {0}, {1,3,4,6} (rows of the 4x4 block), {2,5,7} (3x3 block)
    const bool c4 = (0x5Au >> f) & 1u, c3 = (0xA4u >> f) & 1u;
    const int pos = int((0x23121000u >> (4 * f)) & 0xFu);      // row within the class
    const unsigned src = c4 ? 0x6431u : (c3 ? 0x0752u : 0u);  // source lanes, one nibble each
    cx<R> w{R(0), R(0)};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const cx<R> v = shfl8(y, int((src >> (4 * j)) & 0xFu));
      cx<R> a{R(0), R(0)};
      if (c4)
        a = ldc<R>(nc.a4[4 * pos + j]);
      else if (c3 && j < 3)
        a = ldc<R>(nc.a3[3 * pos + j]);
      else if (!c4 && !c3 && j == 0)
        a = cx<R>{R(1), R(0)};
      w = w + a * v;
    }
    return w;
  } else {
    cx<R> ys[8], tt[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) ys[i] = shfl8(y, i);
    cx<R> Q[3][3];
    node_pos_powers(hph, L, J, Q);
    apply_A(Q, ys, tt);
    cx<R> w = tt[0];
#pragma unroll
    for (int i = 1; i < 8; ++i) w = (f == i) ? tt[i] : w;
    return w;
  }
}

template <typename R, typename TI, typename TO, bool kTable>
__global__ __launch_bounds__(256) void k_fwd_level(VolSet vs, int nvol, int n, int L, DevLevel lv,
                                                   const double2* __restrict__ hph, const NodeConst* nodes,
                                                   GatherMap gm) {
  __shared__ double sp[kMaxPoly * kNumMono];
  const long long N = (long long)n * n * n;
  const long long tg = gather_block(gm.xcd) * blockDim.x + threadIdx.x;
  const bool active = tg < N * nvol;  // whole groups of 8 lanes: N is a multiple of 8
  const long long vol = active ? tg / N : 0, t = tg - vol * N;
  const int f = int(t & 7);
  CubeUnit cu{};
  RowCursor rc{};
  cx<R> mono[kNumMono];
  if (active) {
    cu = unit_of(t >> 3, n, L, lv.b.order, gm.lg);
    const int slice = cu.cube / lv.S;
    row_begin(lv.b, lv.S, slice * 8 + f, cu.cube - slice * lv.S, rc);
    load_mono(nodes, hph, L, cu.J, mono);
  }
  load_polys(lv, sp);
  if (!active) return;
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, vol));
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, vol));
  const cx<R> y = row_finish<R, TI>(in, n, L, cu.J, lv.b, lv.S, rc, sp, lv.nconst, mono);
  const cx<R> z = hadamard8_lanes(apply_A_lanes<R, kTable>(nodes, hph, L, cu.J, f, y), f);
  IO<TO, R>::st(out, gpos(n, L, cu.J, ((f >> 2) & 1) + 2 * cu.a[0], ((f >> 1) & 1) + 2 * cu.a[1], (f & 1) + 2 * cu.a[2]),
                z);
}

// y <- DCT_2(phi) y = H_8 A(phi) y for the 8 values of one cube of node J at
// level L (nodes: the level's node table, or null to form A from the phases).
// (direct: `nodes` points at node J's own entry, e.g. a copy in LDS.)
template <typename R>
__device__ __forceinline__ void dct2_apply(const NodeConst* nodes, const double2* __restrict__ hph, int L,
                                           const int J[3], cx<R> y[8], bool direct = false) {
  cx<R> tt[8];
  const int c4[4] = {1, 3, 4, 6}, c3[3] = {2, 5, 7};
  if (nodes) {
    const NodeConst& nc = direct ? nodes[0] : nodes[((long long)J[0] << (2 * L)) | ((long long)J[1] << L) | J[2]];
    tt[0] = y[0];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cx<R> s{R(0), R(0)};
#pragma unroll
      for (int j = 0; j < 4; ++j) s = s + ldc<R>(nc.a4[4 * i + j]) * y[c4[j]];
      tt[c4[i]] = s;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cx<R> s{R(0), R(0)};
#pragma unroll
      for (int j = 0; j < 3; ++j) s = s + ldc<R>(nc.a3[3 * i + j]) * y[c3[j]];
      tt[c3[i]] = s;
    }
  } else {
    cx<R> Q[3][3];
    node_pos_powers(hph, L, J, Q);
    apply_A(Q, y, tt);
  }
  hadamard8(tt);
#pragma unroll
  for (int i = 0; i < 8; ++i) y[i] = tt[i];
}

// Forward level L, second pass: z = DCT_2(phi) y = H_8 A(phi) y on every cube
// (may run in place when TO is the stage type).
template <typename R, typename TO>
__global__ __launch_bounds__(256) void k_fwd_dct2(VolSet vs, int nvol, int n, int L, const double2* __restrict__ hph,
                                                  const NodeConst* nodes) {
  const long long h = n >> 1, cubes = h * h * h;
  const long long tg = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tg >= cubes * nvol) return;
  const long long vol = tg / cubes, t = tg - vol * cubes;
  const cx<R>* in = static_cast<const cx<R>*>(vol_ptr(vs.in, vol));
  TO* out = static_cast<TO*>(vol_ptr(vs.out, vol));
  int cube;
  CubeIdx ci = cube_of(t, n, L, &cube);
  cx<R> y[8];
  long long pos[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    pos[i] = gpos(n, L, ci.J, ((i >> 2) & 1) + 2 * ci.a[0], ((i >> 1) & 1) + 2 * ci.a[1], (i & 1) + 2 * ci.a[2]);
    y[i] = in[pos[i]];
  }
  dct2_apply(nodes, hph, L, ci.J, y);
#pragma unroll
  for (int i = 0; i < 8; ++i) IO<TO, R>::st(out, pos[i], y[i]);
}

// The DCT_2 pass of level L = D - 2 (node size 4) and the whole last level in
// one launch.  Lane c of an aligned group of 8 owns cube c of a level-L node J
// and applies its DCT_2; output i of cube c is value c of child i (node
// J + 2^L i, a single cube).  The group exchanges the values through LDS, and
// lane i applies child i's DCT_2 and stores its 8 outputs.  The arithmetic is
// that of the two separate passes, in the same order.
template <typename R, typename TO>
__global__ __launch_bounds__(256) void k_fwd_dct2_last2(VolSet vs, int nvol, int n, int L,
                                                        const double2* __restrict__ hph0, const NodeConst* nodes0,
                                                        const double2* __restrict__ hph1, const NodeConst* nodes1) {
  extern __shared__ unsigned char xch_raw[];
  cx<R>* xch = reinterpret_cast<cx<R>*>(xch_raw);  // blockDim.x * 9 values (rows of 8, padded)
  const long long h = n >> 1, cubes = h * h * h;     // 8 cubes per level-L node
  const long long tg = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = tg < cubes * nvol;             // whole groups of 8: cubes is a multiple of 8
  const long long vol = active ? tg / cubes : 0, t = tg - vol * cubes;
  const int mask = (1 << L) - 1;
  const int jf = int(t >> 3), c = int(t & 7);
  const int J[3] = {jf >> (2 * L), (jf >> L) & mask, jf & mask};
  cx<R> y[8];
  if (active) {
    const cx<R>* in = static_cast<const cx<R>*>(vol_ptr(vs.in, vol));
#pragma unroll
    for (int f = 0; f < 8; ++f)
      y[f] = in[gpos(n, L, J, ((f >> 2) & 1) + 2 * ((c >> 2) & 1), ((f >> 1) & 1) + 2 * ((c >> 1) & 1),
                     (f & 1) + 2 * (c & 1))];
    dct2_apply(nodes0, hph0, L, J, y);
#pragma unroll
    for (int i = 0; i < 8; ++i) xch[threadIdx.x * 9 + i] = y[i];
  }
  __syncthreads();
  if (!active) return;
  const int base = int(threadIdx.x) & ~7;
#pragma unroll
  for (int f = 0; f < 8; ++f) y[f] = xch[(base + f) * 9 + c];
  // child c of node J at level L + 1
  const int Jc[3] = {J[0] + (((c >> 2) & 1) << L), J[1] + (((c >> 1) & 1) << L), J[2] + ((c & 1) << L)};
  dct2_apply(nodes1, hph1, L + 1, Jc, y);
  TO* out = static_cast<TO*>(vol_ptr(vs.out, vol));
#pragma unroll
  for (int i = 0; i < 8; ++i) IO<TO, R>::st(out, gpos(n, L + 1, Jc, (i >> 2) & 1, (i >> 1) & 1, i & 1), y[i]);
}

// z <- DCT_2(phi)^{-1} z = A(phi)^{-1} H_8 z / 8 for the 8 values of one cube of
// node J at level L (4x4 and 3x3 solves with partial pivoting).
template <typename R>
__device__ __forceinline__ void idct2_apply(const NodeConst* nodes, const double2* __restrict__ hph, int L,
                                            const int J[3], cx<R> z[8], bool direct = false) {
  hadamard8(z);
  const int c4[4] = {1, 3, 4, 6}, c3[3] = {2, 5, 7};
  const NodeConst* nc =
      nodes ? (direct ? nodes : nodes + (((long long)J[0] << (2 * L)) | ((long long)J[1] << L) | J[2])) : nullptr;
  cx<R> Q[3][3];
  if (!nc) node_pos_powers(hph, L, J, Q);
  // the two blocks one after the other: only one block's matrix is live
  {
    cx<R> a4[4][4], b4[4];
    if (nc) {
#pragma unroll
      for (int i = 0; i < 16; ++i) a4[i / 4][i % 4] = ldc<R>(nc->a4[i]);
    } else {
      build_A_block<R, 1, 4>(Q, a4);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) b4[i] = R(0.125) * z[c4[i]];
    solve_small<R, 4>(a4, b4);
#pragma unroll
    for (int i = 0; i < 4; ++i) z[c4[i]] = b4[i];
  }
  {
    cx<R> a3[3][3], b3[3];
    if (nc) {
#pragma unroll
      for (int i = 0; i < 9; ++i) a3[i / 3][i % 3] = ldc<R>(nc->a3[i]);
    } else {
      build_A_block<R, 2, 3>(Q, a3);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) b3[i] = R(0.125) * z[c3[i]];
    solve_small<R, 3>(a3, b3);
#pragma unroll
    for (int i = 0; i < 3; ++i) z[c3[i]] = b3[i];
  }
  z[0] = R(0.125) * z[0];
}

// Dense DCT_2(phi) = H_8 A(phi) and its inverse A(phi)^{-1} H_8 / 8 of every
// node of one level, for the orbit-block launches: column-major 8 x 8 FP64
// complex, D[f * 8 + i] = DCT_2[i][f] and Dinv[i * 8 + f] = DCT_2^{-1}[f][i]
// (the column a cube's value f, or i, multiplies).  The inverse columns are
// the solves of A (partial pivoting) for the unit vectors e_i.
struct OrbitNode {
  double2 D[64];
  double2 Dinv[64];
};
__global__ void k_orbit_nodes(OrbitNode* out, int L, const double2* __restrict__ hph) {
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= (1LL << (3 * L))) return;
  const int mask = (1 << L) - 1;
  const int J[3] = {int(node >> (2 * L)), int((node >> L) & mask), int(node & mask)};
  cx<double> Q[3][3];
  node_pos_powers(hph, L, J, Q);
  OrbitNode& on = out[node];
  for (int f = 0; f < 8; ++f) {
    cx<double> y[8], t[8];
    for (int k = 0; k < 8; ++k) y[k] = {k == f ? 1.0 : 0.0, 0.0};
    apply_A(Q, y, t);
    hadamard8(t);
    for (int i = 0; i < 8; ++i) on.D[f * 8 + i] = make_double2(t[i].x, t[i].y);
  }
  for (int i = 0; i < 8; ++i) {
    cx<double> z[8];
    for (int k = 0; k < 8; ++k) z[k] = {k == i ? 1.0 : 0.0, 0.0};
    idct2_apply<double>(nullptr, hph, L, J, z, false);
    for (int f = 0; f < 8; ++f) on.Dinv[i * 8 + f] = make_double2(z[f].x, z[f].y);
  }
}

// The last level of the transposed transform (node size 2, B_2 = C_2 = I),
// one thread per node J at level L = D - 1 (its 8 points J + 2^L i):
//   forward (kInv false): y = DCT_2(phi)^T z = A(phi)^T H_8 z,
//   inverse (kInv true) : y = DCT_2(phi)^{-T} z = H_8 A(phi)^{-T} z / 8 (solves with A^T).
template <typename R, typename TI, typename TO, bool kInv>
__global__ __launch_bounds__(256) void k_tr_last(VolSet vs, int nvol, int n, int L, const double2* __restrict__ hph) {
  const long long nodes = 1LL << (3 * L);
  const long long tg = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tg >= nodes * nvol) return;
  const long long vol = tg / nodes, node = tg - vol * nodes;
  const int mask = (1 << L) - 1;
  const int J[3] = {int(node >> (2 * L)), int((node >> L) & mask), int(node & mask)};
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, vol));
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, vol));
  cx<R> z[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) z[i] = IO<TI, R>::ld(in, gpos(n, L, J, (i >> 2) & 1, (i >> 1) & 1, i & 1));
  cx<R> Q[3][3], a4[4][4], a3[3][3];
  node_pos_powers(hph, L, J, Q);
  build_A(Q, a4, a3);
  const int c4[4] = {1, 3, 4, 6}, c3[3] = {2, 5, 7};
  cx<R> y[8];
  if constexpr (!kInv) {
    hadamard8(z);
    y[0] = z[0];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cx<R> acc{R(0), R(0)};
#pragma unroll
      for (int i = 0; i < 4; ++i) acc = acc + a4[i][j] * z[c4[i]];
      y[c4[j]] = acc;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<R> acc{R(0), R(0)};
#pragma unroll
      for (int i = 0; i < 3; ++i) acc = acc + a3[i][j] * z[c3[i]];
      y[c3[j]] = acc;
    }
  } else {
    cx<R> t4[4][4], t3[3][3], b4[4], b3[3];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      b4[i] = z[c4[i]];
#pragma unroll
      for (int j = 0; j < 4; ++j) t4[i][j] = a4[j][i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      b3[i] = z[c3[i]];
#pragma unroll
      for (int j = 0; j < 3; ++j) t3[i][j] = a3[j][i];
    }
    solve_small<R, 4>(t4, b4);
    solve_small<R, 3>(t3, b3);
    y[0] = z[0];
#pragma unroll
    for (int i = 0; i < 4; ++i) y[c4[i]] = b4[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) y[c3[i]] = b3[i];
    hadamard8(y);
#pragma unroll
    for (int i = 0; i < 8; ++i) y[i] = R(0.125) * y[i];
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) IO<TO, R>::st(out, gpos(n, L, J, (i >> 2) & 1, (i >> 1) & 1, i & 1), y[i]);
}

// Hermitian packing of the spectrum of real input: the sample points pair up
// as iota' = (c - g^T iota) mod n with X[iota'] = conj X[iota] (g in W fixed
// by the skew, Sec. III realness of T); slot[iota] = k >= 0 for the k-th
// representative (iota <= iota' in flat order), -(k + 1) for the partner of
// representative k.
template <typename T>
__global__ __launch_bounds__(256) void k_hpack(const T* __restrict__ full, T* __restrict__ packed,
                                               const int* __restrict__ slot, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int k = slot[i];
  if (k >= 0) packed[k] = full[i];
}
template <typename T>
__global__ __launch_bounds__(256) void k_hunpack(const T* __restrict__ packed, T* __restrict__ full,
                                                 const int* __restrict__ slot, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int k = slot[i];
  T v = packed[k >= 0 ? k : -k - 1];
  if (k < 0) v.y = -v.y;
  full[i] = v;
}

// Inverse level L, first pass: y = DCT_2(phi)^{-1} z = A(phi)^{-1} H_8 z / 8 on every cube.
template <typename R, typename TI>
__global__ __launch_bounds__(256) void k_inv_dct2(VolSet vs, int nvol, int n, int L, const double2* __restrict__ hph,
                                                  const NodeConst* nodes) {
  const long long h = n >> 1, cubes = h * h * h;
  const long long tg = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tg >= cubes * nvol) return;
  const long long vol = tg / cubes, t = tg - vol * cubes;
  // may run in place (in == out): each thread reads and writes only its own cube
  const TI* in = static_cast<const TI*>(vol_ptr(vs.in, vol));
  cx<R>* out = static_cast<cx<R>*>(vol_ptr(vs.out, vol));
  int cube;
  CubeIdx ci = cube_of(t, n, L, &cube);
  cx<R> z[8];
  long long pos[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    pos[i] = gpos(n, L, ci.J, ((i >> 2) & 1) + 2 * ci.a[0], ((i >> 1) & 1) + 2 * ci.a[1], (i & 1) + 2 * ci.a[2]);
    z[i] = IO<TI, R>::ld(in, pos[i]);
  }
  idct2_apply(nodes, hph, L, ci.J, z);
#pragma unroll
  for (int i = 0; i < 8; ++i) out[pos[i]] = z[i];
}

// The whole last level (node size 2) and the DCT_2^{-1} pass of level
// L = D - 2 in one launch, the mirror of k_fwd_dct2_last2: lane i of an
// aligned group of 8 inverts child i (node J + 2^L i) of a level-L node J; its
// value f is output i of cube f of J.  After an exchange through LDS, lane c
// inverts cube c of J and stores its 8 values (stage type).
constexpr int kLast2cEnt = 512, kLast2cPoly = 128;  // bounds of the C_4 table held in LDS
// kC: the basis change C_4 of level L follows in the same launch.  The node's
// 64 cube values y(def + 2 abc) go to a second LDS area (cube abc's 8 values
// in a row of 9, a node's rows 73 values apart); the thread (cube abc, node)
// of the node-fastest order forms that node's 8 outputs x(f + 2 abc) from the
// level's row table (one cube per slice, copied to LDS) and writes them to
// out, the stage buffer of level L.
template <typename R, typename TI, bool kC = false>
__global__ __launch_bounds__(256) void k_inv_dct2_last2(VolSet vs, int nvol, int n, int L,
                                                        const double2* __restrict__ hph0, const NodeConst* nodes0,
                                                        const double2* __restrict__ hph1, const NodeConst* nodes1,
                                                        DevLevel lv = DevLevel{}, int nent4 = 0) {
  extern __shared__ unsigned char xch_raw[];
  cx<R>* xch = reinterpret_cast<cx<R>*>(xch_raw);  // blockDim.x * 9 values (rows of 8, padded); kC: twice
  // kC: the level's C_4 table (64 rows) and polynomials, copied to LDS here
  // and published by the first barrier
  __shared__ struct {
    int start[kC ? 64 : 1], len[kC ? 64 : 1];
    uint32_t ent[kC ? kLast2cEnt : 1];
    double poly[kC ? kLast2cPoly * kNumMono : 1];
  } t4;
  if constexpr (kC) {
    for (int i = threadIdx.x; i < 64; i += blockDim.x) t4.start[i] = lv.c.start[i], t4.len[i] = lv.c.len[i];
    for (int i = threadIdx.x; i < nent4; i += blockDim.x) t4.ent[i] = lv.c.ent[i];
    for (int i = threadIdx.x; i < lv.npoly * kNumMono; i += blockDim.x) t4.poly[i] = lv.poly[i];
  }
  const long long h = n >> 1, cubes = h * h * h;     // 8 cubes per level-L node
  const long long tg = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = tg < cubes * nvol;             // whole groups of 8: cubes is a multiple of 8
  const long long vol = active ? tg / cubes : 0, t = tg - vol * cubes;
  const int mask = (1 << L) - 1;
  const int jf = int(t >> 3), c = int(t & 7);
  const int J[3] = {jf >> (2 * L), (jf >> L) & mask, jf & mask};
  cx<R> z[8];
  if (active) {
    const TI* in = static_cast<const TI*>(vol_ptr(vs.in, vol));
    // child c of node J at level L + 1
    const int Jc[3] = {J[0] + (((c >> 2) & 1) << L), J[1] + (((c >> 1) & 1) << L), J[2] + ((c & 1) << L)};
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = IO<TI, R>::ld(in, gpos(n, L + 1, Jc, (i >> 2) & 1, (i >> 1) & 1, i & 1));
    idct2_apply(nodes1, hph1, L + 1, Jc, z);
#pragma unroll
    for (int f = 0; f < 8; ++f) xch[threadIdx.x * 9 + f] = z[f];
  }
  __syncthreads();
  const int base = int(threadIdx.x) & ~7;
  cx<R>* out = static_cast<cx<R>*>(vol_ptr(vs.out, vol));
  if (active) {
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = xch[(base + i) * 9 + c];
    idct2_apply(nodes0, hph0, L, J, z);
  }
  if constexpr (!kC) {
    if (active) {
#pragma unroll
      for (int f = 0; f < 8; ++f)
        out[gpos(n, L, J, ((f >> 2) & 1) + 2 * ((c >> 2) & 1), ((f >> 1) & 1) + 2 * ((c >> 1) & 1),
                 (f & 1) + 2 * (c & 1))] = z[f];
    }
  } else {
    // the block's nodes, 8 values per cube, a node's 8 cubes 73 values apart
    cx<R>* ych = xch + blockDim.x * 9;
    if (active) {
#pragma unroll
      for (int f = 0; f < 8; ++f) ych[(threadIdx.x >> 3) * 73 + (threadIdx.x & 7) * 9 + f] = z[f];
    }
    __syncthreads();
    // the rows: thread (cube cc, node nd) with the node fastest forms the 8
    // rows of cube cc of node nd, so that the lanes of a wave share their
    // rows (two per wave with 32 nodes per block) and read the same entries
    const int NB = int(blockDim.x) >> 3;
    const int cc = int(threadIdx.x) / NB, nd = int(threadIdx.x) - cc * NB;
    const long long tgn = (long long)blockIdx.x * blockDim.x + nd * 8;  // the node's first cube thread
    if (tgn >= cubes * nvol) return;
    const long long voln = tgn / cubes, jn = (tgn - voln * cubes) >> 3;
    const int Jn[3] = {int(jn >> (2 * L)), int((jn >> L) & mask), int(jn & mask)};
    cx<R>* outn = static_cast<cx<R>*>(vol_ptr(vs.out, voln));
    cx<R> mono[kNumMono];
    node_mono(hph0, L, Jn, mono);
    const int a0 = (cc >> 2) & 1, a1 = (cc >> 1) & 1, a2 = cc & 1;
    const cx<R>* yn = ych + nd * 73;
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      // row (f, cube cc) of C_4 from the LDS copy: sources at node-local
      // (x, y, z) = def + 2 abc, i.e. cube abc's value def
      const int r = cc * 8 + f;
      const int e0 = t4.start[r], len = t4.len[r];
      cx<R> acc{R(0), R(0)};
      for (int e = 0; e < len; ++e) {
        const uint32_t en = t4.ent[e0 + e];
        const int x = ent_x(en), y = ent_y(en), zz = ent_z(en);
        const int q = ((x >> 1) << 2) | ((y >> 1) << 1) | (zz >> 1), def = ((x & 1) << 2) | ((y & 1) << 1) | (zz & 1);
        acc = acc + poly_value(t4.poly, lv.nconst, ent_pid(en), mono) * yn[q * 9 + def];
      }
      outn[gpos(n, L, Jn, ((f >> 2) & 1) + 2 * a0, ((f >> 1) & 1) + 2 * a1, (f & 1) + 2 * a2)] = acc;
    }
  }
}

// Inverse level L, second pass: x(kappa) = sum C_nl(phi)[kappa, (def,abc)] y(def + 2 abc),
// one thread per output kappa = i + 2 abc.
template <typename R, typename TO, bool kUni>
__global__ __launch_bounds__(256) void k_inv_basis(VolSet vs, int nvol, int n, int L, DevLevel lv,
                                                   const double2* __restrict__ hph, const NodeConst* nodes, GatherMap gm) {
  if constexpr (kUni) {
    // wave-uniform rows (see row_uniform): no LDS, no barrier
    const long long N = (long long)n * n * n;
    const long long tg = gather_block(gm.xcd) * blockDim.x + threadIdx.x;
    if (tg >= N * nvol) return;
    const long long vol = tg / N, t = tg - vol * N;
    const RowIdx ri = row_of(t, n, L, lv.c.order, 1, gm);
    cx<R> mono[kNumMono];
    load_mono(nodes, hph, L, ri.J, mono);
    const cx<R>* __restrict__ in = static_cast<const cx<R>*>(vol_ptr(vs.in, vol));
    TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, vol));
    const cx<R> x = row_uniform<R, cx<R>>(in, n, L, ri.J, lv.c, ri.cube * 8 + ri.f, lv.poly, lv.nconst, mono);
    IO<TO, R>::st(out, gpos(n, L, ri.J, ((ri.f >> 2) & 1) + 2 * ri.a[0], ((ri.f >> 1) & 1) + 2 * ri.a[1], (ri.f & 1) + 2 * ri.a[2]), x);
    return;
  }
  __shared__ double sp[kMaxPoly * kNumMono];
  const long long N = gm.balance ? gm.off[8] * ((1LL << (3 * L)) >> gm.lg) : (long long)n * n * n;  // threads per volume
  const long long tg = gather_block(gm.xcd) * blockDim.x + threadIdx.x;
  const bool active = tg < N * nvol;
  const long long vol = active ? tg / N : 0, t = tg - vol * N;
  RowIdx ri{};
  RowCursor rc{};
  cx<R> mono[kNumMono];
  int k = 0, kf = 0;
  if (active) {
    if (gm.balance) {
      const RowPart rp = row_part_of(t, n, L, lv.c.order, gm);
      ri = rp.r, k = rp.k, kf = rp.kf;
    } else {
      ri = row_of(t, n, L, lv.c.order, lv.S, gm, lv.c.perm);
    }
    const int slice = ri.cube / lv.S;
    row_begin(lv.c, lv.S, slice * 8 + ri.f, ri.cube - slice * lv.S, rc, k, kf);
    load_mono(nodes, hph, L, ri.J, mono);
  }
  load_polys(lv, sp);
  if (!active) return;
  const cx<R>* __restrict__ in = static_cast<const cx<R>*>(vol_ptr(vs.in, vol));
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, vol));
  cx<R> x = row_finish<R, cx<R>>(in, n, L, ri.J, lv.c, lv.S, rc, sp, lv.nconst, mono);
  if (gm.balance) x = combine_parts(x, kf);
  if (k == 0)
    IO<TO, R>::st(out, gpos(n, L, ri.J, ((ri.f >> 2) & 1) + 2 * ri.a[0], ((ri.f >> 1) & 1) + 2 * ri.a[1], (ri.f & 1) + 2 * ri.a[2]), x);
}

// ---------------------------------------------------------------------------
// Fused tail: the last levels (node size nl0 <= 16) of a group of G sibling nodes
// sibling nodes (consecutive J_z) run in LDS, one thread per 2x2x2 cube of
// every sub-level.  Sub-level l of the tail is global level Lt + l; its
// sub-nodes j' in [0, 2^l)^3 own the node-local positions j' + 2^l b, exactly
// as the global layout nests.
// ---------------------------------------------------------------------------
// LDS capacity in points of the two tail forms: node sizes up to 8 (two
// nodes of 8^3) and 16 (one node of 16^3, 64 KB in FP64).  A block has one
// thread per cube of its nodes: capacity / 8.
constexpr int kTailCapSmall = 1024;
constexpr int kTailCapBig = 4096;

struct TailLevels {
  DevLevel lv[4];             // CSR tables (S = 1) of node sizes nl0, nl0/2, ...
  const NodeConst* nodes[4];  // node tables of global levels Lt + l, or null
  const double2* hph[4];      // phase tables of global levels Lt + l
};

__device__ __forceinline__ int lpos(int nl0, int l, const int jp[3], int x, int y, int z) {
  return (((jp[0] + (x << l)) * nl0) + (jp[1] + (y << l))) * nl0 + (jp[2] + (z << l));
}

// One table row gathered from an LDS node buffer, in entry order.  The table
// lives in global memory: the row's entries are read in chunks of 8 with the
// next chunk in flight while the current one is summed (e0, len: the row's
// start and length, loaded by the caller for all 8 rows of a cube at once).
template <typename R>
__device__ __forceinline__ cx<R> lds_row(const cx<R>* buf, int nl0, int l, const int jp[3], const DevSide& sd, int e0,
                                         int len, const double* sp, int nconst, const cx<R> mono[kNumMono]) {
  cx<R> acc{R(0), R(0)};
  if (len <= 0) return acc;
  uint32_t e8[kChunk];
#pragma unroll
  for (int u = 0; u < kChunk; ++u) e8[u] = sd.ent[e0 + min(u, len - 1)];
  for (int c = 0; c < len; c += kChunk) {
    uint32_t en[kChunk];
    const bool more = c + kChunk < len;
    if (more) {
#pragma unroll
      for (int u = 0; u < kChunk; ++u) en[u] = sd.ent[e0 + min(c + kChunk + u, len - 1)];
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      if (c + u < len)
        acc = acc + poly_value(sp, nconst, ent_pid(e8[u]), mono) *
                        buf[lpos(nl0, l, jp, ent_x(e8[u]), ent_y(e8[u]), ent_z(e8[u]))];
    if (more) {
#pragma unroll
      for (int u = 0; u < kChunk; ++u) e8[u] = en[u];
    }
  }
  return acc;
}

struct TailGeom {
  int n, Lt, nl0, k, G;
};
// block -> (volume, first node J of the group)
__device__ __forceinline__ void tail_block(const TailGeom& tg, long long blk, long long* vol, int J[3]) {
  const long long groups = (1LL << (3 * tg.Lt)) / tg.G;
  *vol = blk / groups;
  const long long jf = (blk - *vol * groups) * tg.G;  // J_z fastest
  const int mask = (1 << tg.Lt) - 1;
  J[0] = int(jf >> (2 * tg.Lt));
  J[1] = int((jf >> tg.Lt) & mask);
  J[2] = int(jf & mask);
}
// thread -> (node g of the group, sub-node j', cube a) at sub-level l; G3 = global node
struct TailCube {
  int g, jp[3], a[3], G3[3];
};
__device__ __forceinline__ TailCube tail_cube(const TailGeom& tg, const int J[3], int l, int t) {
  const int cpn = tg.nl0 * tg.nl0 * tg.nl0 / 8;  // cubes per node
  const int m = (tg.nl0 >> l) >> 1, sub = 1 << l;
  TailCube c;
  c.g = t / cpn;
  const int rr = t - c.g * cpn;
  const int jf = rr & ((1 << (3 * l)) - 1), cube = rr >> (3 * l);
  c.jp[0] = jf >> (2 * l);
  c.jp[1] = (jf >> l) & (sub - 1);
  c.jp[2] = jf & (sub - 1);
  c.a[0] = cube / (m * m);
  c.a[1] = (cube / m) % m;
  c.a[2] = cube % m;
  c.G3[0] = J[0] + (c.jp[0] << tg.Lt);
  c.G3[1] = J[1] + (c.jp[1] << tg.Lt);
  c.G3[2] = J[2] + c.g + (c.jp[2] << tg.Lt);
  return c;
}
__device__ __forceinline__ long long node_index(const int G3[3], int Lg) {
  return ((long long)G3[0] << (2 * Lg)) | ((long long)G3[1] << Lg) | G3[2];
}
template <typename R>
__device__ __forceinline__ void tail_mono(const TailLevels& tl, int l, int Lg, const int G3[3], cx<R> mono[kNumMono]) {
  node_mono(tl.hph[l], Lg, G3, mono);
}
template <typename R>
__device__ __forceinline__ void tail_A(const TailLevels& tl, int l, int Lg, const int G3[3], cx<R> a4[4][4],
                                       cx<R> a3[3][3]) {
  if (tl.nodes[l]) {
    const NodeConst& nc = tl.nodes[l][node_index(G3, Lg)];
#pragma unroll
    for (int i = 0; i < 16; ++i) a4[i / 4][i % 4] = ldc<R>(nc.a4[i]);
#pragma unroll
    for (int i = 0; i < 9; ++i) a3[i / 3][i % 3] = ldc<R>(nc.a3[i]);
  } else {
    cx<R> Q[3][3];
    node_pos_powers(tl.hph[l], Lg, G3, Q);
    build_A(Q, a4, a3);
  }
}

template <typename R, typename TI>
__device__ __forceinline__ void tail_load(const TailGeom& tg, const int J[3], const TI* in, cx<R>* buf) {
  const int npts = tg.nl0 * tg.nl0 * tg.nl0;
  for (int t = threadIdx.x; t < tg.G * npts; t += blockDim.x) {
    const int g = t % tg.G, a = t / tg.G;
    const int ax = a / (tg.nl0 * tg.nl0), ay = (a / tg.nl0) % tg.nl0, az = a % tg.nl0;
    const long long gp = ((long long)(J[0] + (ax << tg.Lt)) * tg.n + (J[1] + (ay << tg.Lt))) * tg.n +
                         (J[2] + g + (az << tg.Lt));
    buf[g * npts + a] = IO<TI, R>::ld(in, gp);
  }
}
template <typename R, typename TO>
__device__ __forceinline__ void tail_store(const TailGeom& tg, const int J[3], const cx<R>* buf, TO* out) {
  const int npts = tg.nl0 * tg.nl0 * tg.nl0;
  for (int t = threadIdx.x; t < tg.G * npts; t += blockDim.x) {
    const int g = t % tg.G, a = t / tg.G;
    const int ax = a / (tg.nl0 * tg.nl0), ay = (a / tg.nl0) % tg.nl0, az = a % tg.nl0;
    const long long gp = ((long long)(J[0] + (ax << tg.Lt)) * tg.n + (J[1] + (ay << tg.Lt))) * tg.n +
                         (J[2] + g + (az << tg.Lt));
    IO<TO, R>::st(out, gp, buf[g * npts + a]);
  }
}

// Every thread owns at most one cube per sub-level (the block has at least
// G * nl0^3 / 8 threads), so each sub-level reads its cube into registers,
// waits, and writes back into the same LDS buffer.
template <typename R, typename TI, typename TO, int kCap>
__global__ __launch_bounds__(kCap / 8) void k_fwd_tail(VolSet vs, TailGeom tg, TailLevels tl) {
  __shared__ cx<R> buf[kCap];
  __shared__ double sp[kMaxPoly * kNumMono];
  long long vol;
  int J[3];
  tail_block(tg, blockIdx.x, &vol, J);
  tail_load<R>(tg, J, static_cast<const TI*>(vol_ptr(vs.in, vol)), buf);
  const int npts = tg.nl0 * tg.nl0 * tg.nl0, ncubes = tg.G * npts / 8;
  const int t = threadIdx.x;
  for (int l = 0; l < tg.k; ++l) {
    const int Lg = tg.Lt + l;
    const DevLevel& lv = tl.lv[l];
    __syncthreads();
    for (int i = t; i < lv.npoly * kNumMono; i += blockDim.x) sp[i] = lv.poly[i];
    __syncthreads();
    TailCube c{};
    cx<R> tt[8];
    if (t < ncubes) {
      c = tail_cube(tg, J, l, t);
      const int m = (tg.nl0 >> l) >> 1;
      const int cube = (c.a[0] * m + c.a[1]) * m + c.a[2];
      const cx<R>* src = buf + c.g * npts;
      cx<R> mono[kNumMono];
      tail_mono<R>(tl, l, Lg, c.G3, mono);
      int rs[8], rl[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) rs[f] = lv.b.start[cube * 8 + f], rl[f] = lv.b.len[cube * 8 + f];
      cx<R> y[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) y[f] = lds_row(src, tg.nl0, l, c.jp, lv.b, rs[f], rl[f], sp, lv.nconst, mono);
      if (tl.nodes[l]) {
        const NodeConst& nc = tl.nodes[l][node_index(c.G3, Lg)];
        const int c4[4] = {1, 3, 4, 6}, c3[3] = {2, 5, 7};
        tt[0] = y[0];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          cx<R> acc{R(0), R(0)};
#pragma unroll
          for (int j = 0; j < 4; ++j) acc = acc + ldc<R>(nc.a4[i * 4 + j]) * y[c4[j]];
          tt[c4[i]] = acc;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          cx<R> acc{R(0), R(0)};
#pragma unroll
          for (int j = 0; j < 3; ++j) acc = acc + ldc<R>(nc.a3[i * 3 + j]) * y[c3[j]];
          tt[c3[i]] = acc;
        }
      } else {
        cx<R> Q[3][3];
        node_pos_powers(tl.hph[l], Lg, c.G3, Q);
        apply_A(Q, y, tt);
      }
      hadamard8(tt);
    }
    __syncthreads();
    if (t < ncubes) {
      cx<R>* dst = buf + c.g * npts;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        dst[lpos(tg.nl0, l, c.jp, ((i >> 2) & 1) + 2 * c.a[0], ((i >> 1) & 1) + 2 * c.a[1], (i & 1) + 2 * c.a[2])] = tt[i];
    }
  }
  __syncthreads();
  tail_store<R>(tg, J, buf, static_cast<TO*>(vol_ptr(vs.out, vol)));
}

template <typename R, typename TI, typename TO, int kCap>
__global__ __launch_bounds__(kCap / 8) void k_inv_tail(VolSet vs, TailGeom tg, TailLevels tl) {
  __shared__ cx<R> buf[kCap];
  __shared__ double sp[kMaxPoly * kNumMono];
  long long vol;
  int J[3];
  tail_block(tg, blockIdx.x, &vol, J);
  tail_load<R>(tg, J, static_cast<const TI*>(vol_ptr(vs.in, vol)), buf);
  const int npts = tg.nl0 * tg.nl0 * tg.nl0, ncubes = tg.G * npts / 8;
  const int t = threadIdx.x;
  const int c4[4] = {1, 3, 4, 6}, c3[3] = {2, 5, 7};
  for (int l = tg.k - 1; l >= 0; --l) {
    const int Lg = tg.Lt + l;
    const DevLevel& lv = tl.lv[l];
    __syncthreads();
    for (int i = t; i < lv.npoly * kNumMono; i += blockDim.x) sp[i] = lv.poly[i];
    // DCT_2^{-1} on this thread's cube, in place
    TailCube c{};
    int cube = 0;
    if (t < ncubes) {
      c = tail_cube(tg, J, l, t);
      const int m = (tg.nl0 >> l) >> 1;
      cube = (c.a[0] * m + c.a[1]) * m + c.a[2];
      cx<R>* b = buf + c.g * npts;
      cx<R> z[8];
      int p[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        p[i] = lpos(tg.nl0, l, c.jp, ((i >> 2) & 1) + 2 * c.a[0], ((i >> 1) & 1) + 2 * c.a[1], (i & 1) + 2 * c.a[2]);
        z[i] = b[p[i]];
      }
      hadamard8(z);
      cx<R> a4[4][4], a3[3][3];
      tail_A<R>(tl, l, Lg, c.G3, a4, a3);
      cx<R> b4[4], b3[3];
#pragma unroll
      for (int i = 0; i < 4; ++i) b4[i] = R(0.125) * z[c4[i]];
#pragma unroll
      for (int i = 0; i < 3; ++i) b3[i] = R(0.125) * z[c3[i]];
      solve_small<R, 4>(a4, b4);
      solve_small<R, 3>(a3, b3);
      b[p[0]] = R(0.125) * z[0];
#pragma unroll
      for (int i = 0; i < 4; ++i) b[p[c4[i]]] = b4[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) b[p[c3[i]]] = b3[i];
    }
    __syncthreads();
    // C gather: the 8 outputs kappa = i + 2 abc of this thread's cube
    cx<R> x[8];
    if (t < ncubes) {
      const cx<R>* src = buf + c.g * npts;
      cx<R> mono[kNumMono];
      tail_mono<R>(tl, l, Lg, c.G3, mono);
      int rs[8], rl[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) rs[i] = lv.c.start[cube * 8 + i], rl[i] = lv.c.len[cube * 8 + i];
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = lds_row(src, tg.nl0, l, c.jp, lv.c, rs[i], rl[i], sp, lv.nconst, mono);
    }
    __syncthreads();
    if (t < ncubes) {
      cx<R>* dst = buf + c.g * npts;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        dst[lpos(tg.nl0, l, c.jp, ((i >> 2) & 1) + 2 * c.a[0], ((i >> 1) & 1) + 2 * c.a[1], (i & 1) + 2 * c.a[2])] = x[i];
    }
  }
  __syncthreads();
  tail_store<R>(tg, J, buf, static_cast<TO*>(vol_ptr(vs.out, vol)));
}

// n = 1: the transform is the 1x1 matrix [T_0] = [1].
template <typename TI, typename TO>
__global__ void k_copy1(VolSet vs, int nvol) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nvol) {
    cx<double> x = IO<TI, double>::ld(static_cast<const TI*>(vol_ptr(vs.in, v)), 0);
    IO<TO, double>::st(static_cast<TO*>(vol_ptr(vs.out, v)), 0, x);
  }
}

// FP64 round-trip residual: out[0] = max |x - y|, out[1] = max |x| over
// `count` elements (|.| of complex values for complex data).  out must be
// zeroed first; maxima of non-negative doubles are combined through their bit
// patterns (monotonic for non-negative IEEE values) with 64-bit atomic max.
template <typename T>
__global__ __launch_bounds__(256) void k_residual(const T* __restrict__ x, const T* __restrict__ y, long long count,
                                                  unsigned long long* out) {
  double dmax = 0.0, xmax = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x) {
    const cx<double> a = IO<T, double>::ld(x, i), b = IO<T, double>::ld(y, i);
    const double dx = a.x - b.x, dy = a.y - b.y;
    // a NaN difference counts as infinitely large (fmax below would drop it)
    double d = sqrt(dx * dx + dy * dy), m = sqrt(a.x * a.x + a.y * a.y);
    if (d != d) d = INFINITY;
    if (m != m) m = INFINITY;
    dmax = fmax(dmax, d);
    xmax = fmax(xmax, m);
  }
  __shared__ double sd[256], sx[256];
  sd[threadIdx.x] = dmax;
  sx[threadIdx.x] = xmax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
      sx[threadIdx.x] = fmax(sx[threadIdx.x], sx[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(sd[0]));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(sx[0]));
  }
}

// Synthetic operand in [-1, 1): a hash of the index (autotuning input).
template <typename T>
__global__ void k_fill(T* x, long long count, unsigned seed) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x) {
    unsigned h = unsigned(i) * 2654435761u ^ (unsigned(i >> 32) + seed) * 2246822519u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    x[i] = T(int(h >> 8) - (1 << 23)) / T(1 << 23);
  }
}

__global__ void k_zero2(unsigned long long* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0ull;
}

// FP64 half phases of every level: level L, axis d, J_d -> exp(i pi (rst_d + J_d) / 2^L).
__global__ void k_phase_table(double2* out, int D, double r0, double r1, double r2) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  // level L occupies [3 (2^L - 1), 3 (2^(L+1) - 1))
  for (int L = 0; L < D; ++L) {
    int base = 3 * ((1 << L) - 1), cnt = 3 << L;
    if (idx < base || idx >= base + cnt) continue;
    int d = (idx - base) >> L, J = (idx - base) & ((1 << L) - 1);
    double rd = d == 0 ? r0 : (d == 1 ? r1 : r2);
    double ang = (rd + J) / double(1 << L);  // in units of pi
    double s, c;
    sincospi(ang, &s, &c);
    out[idx] = make_double2(c, s);
  }
}

}  // namespace fcc

#include "orbit_level.hpp"
#include "fold_fft.hpp"
#include "base_fold.hpp"


// ===========================================================================
// Host side
// ===========================================================================
using namespace fcc;

namespace {

enum class DT { F32R, F64R, F32C, F64C };

// Coefficient polynomials of one node size on one device, in the fixed
// monomial order, constants first.
struct DevPolys {
  const double* poly = nullptr;
  int npoly = 0, nconst = 0;
  uint16_t zero_pid = 0;        // the zero polynomial that pads sliced tables
  std::vector<uint16_t> newid;  // host polynomial id -> device id
};
struct DevTablesCache {
  std::mutex mu;
  std::map<std::array<int, 2>, DevPolys> polys;  // (device, nl)
  std::map<std::array<int, 5>, DevSide> sides;   // (device, nl, cubes per slice, side, cube order)
  std::vector<void*> owned;
};
DevTablesCache& cache() {
  static DevTablesCache c;
  return c;
}

// Set FCC_VERBOSE=1 to print the HIP call that failed to stderr.
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("FCC_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}
fcc_status hip_fail(hipError_t e, const char* what, int line) {
  if (verbose()) std::fprintf(stderr, "fcc_dct: %s failed at line %d: %s\n", what, line, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? FCC_ERR_OOM : FCC_ERR_HIP;
}
#define HIPCHK(expr)                                              \
  do {                                                            \
    hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__);   \
  } while (0)
}  // namespace
hipError_t fcc::dev_malloc_raw(void** p, size_t bytes) {
  static std::mutex mu;
  static std::string armed;
  static long long count = 0;
  const char* v = std::getenv("FCC_FAIL_ALLOC_AT");
  {
    std::lock_guard<std::mutex> lock(mu);
    const std::string now = v ? v : "";
    if (now != armed) armed = now, count = 0;
    if (!armed.empty() && ++count == std::atoll(armed.c_str())) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  return hipMalloc(p, bytes);
}
namespace {
// FCC_POISON_SCRATCH set and not "0" (a debugging aid): freshly allocated
// scratch is filled with all-ones bytes, a NaN in FP32 and in FP64, so that a
// kernel reading scratch before writing it shows in the results.
void poison_scratch(void* ptr, size_t bytes) {
  const char* v = std::getenv("FCC_POISON_SCRATCH");
  if (v && *v && *v != '0' && ptr && bytes) {
    (void)hipMemset(ptr, 0xff, bytes);
    (void)hipDeviceSynchronize();  // done before any stream of the caller can use the buffer
  }
}
// Status of the launches just enqueued (stale errors are cleared on entry).
fcc_status launch_status(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FCC_OK : hip_fail(e, what, 0);
}

// Device copy of v; the allocation is recorded in *own (the table cache's list
// by default: kept until the process ends).
template <typename T>
fcc_status upload(const std::vector<T>& v, const T** out, std::vector<void*>* own = nullptr) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
  HIPCHK(dev_malloc(&p, bytes));
  if (!v.empty()) {
    hipError_t e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p);
      return hip_fail(e, "hipMemcpy(tables)", __LINE__);
    }
  }
  (own ? own : &cache().owned)->push_back(p);
  *out = static_cast<const T*>(p);
  return FCC_OK;
}

// Sliced copy of one side's gather rows (see DevSide).  rowptr is the CSR of
// rows cube * 8 + f; zero_pid names a polynomial equal to zero.
// Sliced device copy of one side (B or C) of the tables, cube order `ord`.
fcc_status upload_side(const std::vector<int>& rowptr, const std::vector<uint32_t>& src,
                       const std::vector<uint16_t>& pid, const DevPolys& dp, int S, CubeOrder ord,
                       const GatherBlocks* blocks, bool cside, DevSide* out, std::vector<void*>* own) {
  const int rows = int(rowptr.size()) - 1, cubes = rows / 8, slices = (cubes + S - 1) / S;
  int m = 1, lgm = 0;
  while (m * m * m < cubes) m *= 2, ++lgm;
  if (2 * m > 256) return FCC_ERR_UNSUPPORTED;  // coordinates of a packed entry have 8 bits
  // natural cube index of the q-th cube in the slice order
  std::vector<int> nat(cubes);
  for (int q = 0; q < cubes; ++q) {
    int a[3];
    cube_abc(q, lgm, ord, a);
    nat[q] = (a[0] * m + a[1]) * m + a[2];
  }
  std::vector<int> start(size_t(slices) * 8), len(size_t(slices) * 8);
  size_t total = 0;
  for (int sl = 0; sl < slices; ++sl)
    for (int f = 0; f < 8; ++f) {
      int mx = 0;
      for (int j = 0; j < S && sl * S + j < cubes; ++j) {
        const int r = nat[sl * S + j] * 8 + f;
        mx = std::max(mx, rowptr[r + 1] - rowptr[r]);
      }
      start[size_t(sl) * 8 + f] = int(total);
      len[size_t(sl) * 8 + f] = mx;
      total += size_t(mx) * S;
    }
  if (total > 0x7fffffffu) return FCC_ERR_UNSUPPORTED;
  // packed entries (x << 24) | (y << 16) | (z << 8) | polynomial; padding:
  // position 0 with the zero polynomial
  std::vector<uint32_t> sent(total, uint32_t(dp.zero_pid));
  for (int sl = 0; sl < slices; ++sl)
    for (int f = 0; f < 8; ++f)
      for (int j = 0; j < S && sl * S + j < cubes; ++j) {
        const int r = nat[sl * S + j] * 8 + f;
        for (int e = 0; e < rowptr[r + 1] - rowptr[r]; ++e) {
          const size_t q = size_t(start[size_t(sl) * 8 + f]) + size_t(e) * S + j;
          const uint32_t sv = src[rowptr[r] + e];
          sent[q] = ((sv >> 20) << 24) | (((sv >> 10) & 1023u) << 16) | ((sv & 1023u) << 8) |
                    uint32_t(dp.newid[pid[rowptr[r] + e]]);
        }
      }
  fcc_status s;
  if ((s = upload(start, &out->start, own)) != FCC_OK) return s;
  if ((s = upload(len, &out->len, own)) != FCC_OK) return s;
  if ((s = upload(sent, &out->ent, own)) != FCC_OK) return s;
  out->order = ord;
  out->perm = nullptr;
  if (S > 1 && blocks && slices % 4 == 0) {
    // Groups of 4 consecutive slices (one block of threads: neighbouring
    // tiles, which share cache lines in the CU) sorted by the first (in slice
    // order) block of B they touch, so that the groups holding one block
    // become neighbours.  A B row belongs to its cube's block; a C row kappa
    // to the block that reads kappa in B.
    std::vector<int> qof(cubes);
    for (int q = 0; q < cubes; ++q) qof[nat[q]] = q;
    const int groups = slices / 4;
    std::vector<std::pair<int, int>> key(groups);
    for (int gi = 0; gi < groups; ++gi) {
      int k = cubes;
      for (int j = 0; j < 4 * S; ++j) {
        const int c = nat[gi * 4 * S + j];
        if (!cside) {
          k = std::min(k, qof[blocks->cube[c]]);
          continue;
        }
        const int a = c / (m * m), b = (c / m) % m, cc = c % m, nl = 2 * m;
        for (int i = 0; i < 8; ++i) {
          const size_t kap = (size_t(2 * a + (i >> 2)) * nl + (2 * b + ((i >> 1) & 1))) * nl + (2 * cc + (i & 1));
          k = std::min(k, qof[blocks->kappa[kap]]);
        }
      }
      key[gi] = {k, gi};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> perm(groups);
    for (int i = 0; i < groups; ++i) perm[i] = key[i].second;
    if ((s = upload(perm, &out->perm, own)) != FCC_OK) return s;
  }
  return FCC_OK;
}

// The polynomials of node size nl on device dev (cached; caller holds the
// cache lock).
fcc_status device_polys(int dev, int nl, const DevPolys** out) {
  auto& C = cache();
  std::array<int, 2> key{dev, nl};
  auto it = C.polys.find(key);
  if (it != C.polys.end()) {
    *out = &it->second;
    return FCC_OK;
  }
  const LevelTables* T = level_tables(nl);
  if (!T) return FCC_ERR_OOM;
  // Remap the coefficient polynomials to the fixed monomial order
  // {1, c3, c1, c2, c1 c3} and sort them so that constants come first.
  auto slot_of = [](int e1, int e2, int e3) {
    if (e1 == 0 && e2 == 0 && e3 == 0) return 0;
    if (e1 == 0 && e2 == 0 && e3 == 1) return 1;
    if (e1 == 1 && e2 == 0 && e3 == 0) return 2;
    if (e1 == 0 && e2 == 1 && e3 == 0) return 3;
    if (e1 == 1 && e2 == 0 && e3 == 1) return 4;
    return -1;
  };
  std::vector<double> fixed(size_t(T->npoly) * kNumMono, 0.0);
  for (int q = 0; q < T->nmono; ++q) {
    int sl = slot_of(T->mono[3 * q], T->mono[3 * q + 1], T->mono[3 * q + 2]);
    if (sl < 0) return FCC_ERR_UNSUPPORTED;
    for (int p = 0; p < T->npoly; ++p) fixed[size_t(p) * kNumMono + sl] = T->poly[size_t(p) * T->nmono + q];
  }
  std::vector<int> order(T->npoly);
  for (int p = 0; p < T->npoly; ++p) order[p] = p;
  auto is_const = [&](int p) {
    for (int q = 1; q < kNumMono; ++q)
      if (fixed[size_t(p) * kNumMono + q] != 0.0) return false;
    return true;
  };
  std::stable_partition(order.begin(), order.end(), is_const);
  int nconst = 0;
  for (int p = 0; p < T->npoly; ++p) nconst += is_const(p) ? 1 : 0;
  // one extra constant polynomial equal to zero pads the sliced tables
  order.insert(order.begin() + nconst, -1);
  ++nconst;
  DevPolys dp;
  dp.zero_pid = uint16_t(nconst - 1);
  dp.newid.resize(T->npoly);
  std::vector<double> poly(fixed.size() + kNumMono, 0.0);
  for (int i = 0; i <= T->npoly; ++i) {
    if (order[i] < 0) continue;
    dp.newid[order[i]] = uint16_t(i);
    for (int q = 0; q < kNumMono; ++q) poly[size_t(i) * kNumMono + q] = fixed[size_t(order[i]) * kNumMono + q];
  }
  dp.nconst = nconst;
  dp.npoly = T->npoly + 1;
  if (dp.npoly > kMaxPoly) return FCC_ERR_UNSUPPORTED;
  fcc_status s = upload(poly, &dp.poly);
  if (s != FCC_OK) return s;
  *out = &C.polys.emplace(key, std::move(dp)).first->second;
  return FCC_OK;
}

// One side (0 = B, 1 = C) of node size nl, S cubes per slice, cube order ord.
// With own == nullptr the tables are cached for the process; otherwise they
// are built afresh and their allocations appended to *own for the caller to
// free.  The caller holds the cache lock.
fcc_status device_side(int dev, int nl, int S, int side, CubeOrder ord, DevSide* out, std::vector<void*>* own) {
  auto& C = cache();
  std::array<int, 5> key{dev, nl, S, side, (ord.la << 16) | (ord.lb << 8) | ord.lc};
  if (!own) {
    auto it = C.sides.find(key);
    if (it != C.sides.end()) {
      *out = it->second;
      return FCC_OK;
    }
  }
  const LevelTables* T = level_tables(nl);
  if (!T) return FCC_ERR_OOM;
  const DevPolys* dp = nullptr;
  fcc_status s = device_polys(dev, nl, &dp);
  if (s != FCC_OK) return s;
  const GatherBlocks* blocks = nullptr;
  if (S > 1 && !(blocks = gather_blocks(nl))) return FCC_ERR_OOM;
  s = side == 0 ? upload_side(T->b_rowptr, T->b_src, T->b_pid, *dp, S, ord, blocks, false, out, own)
                : upload_side(T->c_rowptr, T->c_src, T->c_pid, *dp, S, ord, blocks, true, out, own);
  if (s == FCC_OK && !own) C.sides.emplace(key, *out);
  return s;
}

// Both sides of node size nl (cached), B in order ob and C in order oc.
fcc_status device_level(int dev, int nl, int S, CubeOrder ob, CubeOrder oc, DevLevel* out) {
  const DevPolys* dp = nullptr;
  fcc_status s = device_polys(dev, nl, &dp);
  if (s != FCC_OK) return s;
  DevLevel lv{};
  if ((s = device_side(dev, nl, S, 0, ob, &lv.b, nullptr)) != FCC_OK) return s;
  if ((s = device_side(dev, nl, S, 1, oc, &lv.c, nullptr)) != FCC_OK) return s;
  lv.poly = dp->poly;
  lv.npoly = dp->npoly;
  lv.nconst = dp->nconst;
  lv.S = S;
  *out = lv;
  return FCC_OK;
}

// ---- orbit-block templates on the device (see orbit_level.hpp) --------------

// Cube slots of one kind in wavefront order: quads of 4 slots whose segments
// have the same lengths first (no lane of a wavefront waits for another),
// then the rest by decreasing total; -1 pads the last quad.
std::vector<int16_t> quad_order(const std::vector<int>& segptr, int nc) {
  constexpr int kSeg = 8 * kNumMono;  // segments per cube slot
  std::map<std::vector<int>, std::vector<int>> byprof;
  for (int j = 0; j < nc; ++j) {
    std::vector<int> pr(kSeg);
    for (int k = 0; k < kSeg; ++k) pr[k] = segptr[j * kSeg + k + 1] - segptr[j * kSeg + k];
    byprof[pr].push_back(j);
  }
  std::vector<int16_t> out;
  std::vector<std::pair<int, int>> rest;  // (-total, slot)
  for (const auto& kv : byprof) {
    int tot = 0;
    for (int v : kv.first) tot += v;
    const auto& js = kv.second;
    const size_t whole = js.size() / 4 * 4;
    for (size_t i = 0; i < whole; ++i) out.push_back(int16_t(js[i]));
    for (size_t i = whole; i < js.size(); ++i) rest.push_back({-tot, js[i]});
  }
  std::sort(rest.begin(), rest.end());
  for (const auto& r : rest) out.push_back(int16_t(r.second));
  while (out.size() % 4) out.push_back(-1);
  return out;
}

// Templates and representatives of node size nl on device dev (cached; the
// caller holds the cache lock).  Rows are split by monomial with integer
// coefficients (see DevOrbitLevel).  FCC_ERR_UNSUPPORTED if a kind does not
// fit the kernels' LDS arrays or a coefficient is not a 16-bit multiple of 1/144.
fcc_status device_orbit_level(int dev, int nl, DevOrbitLevel* out) {
  static std::map<std::array<int, 2>, DevOrbitLevel> levels;
  const std::array<int, 2> key{dev, nl};
  auto it = levels.find(key);
  if (it != levels.end()) {
    *out = it->second;
    return FCC_OK;
  }
  const OrbitBlocks* ob = orbit_blocks(nl);
  if (!ob) return FCC_ERR_UNSUPPORTED;
  std::vector<DevOrbitKind> kinds;
  std::vector<int16_t> perm;
  std::vector<uint16_t> rowptr;
  std::vector<uint32_t> ent;
  std::vector<int8_t> wmat;
  std::vector<uint32_t> reps;
  std::vector<int4> chunks[2];
  const auto& G = weyl_group();
  for (size_t t = 0; t < ob->templ.size(); ++t) {
    const OrbitTemplate& T = ob->templ[t];
    if (T.nc < 1 || T.nc > kOrbitMaxCubes) return FCC_ERR_UNSUPPORTED;
    DevOrbitKind k{};
    k.nc = T.nc;
    k.off_w = int(wmat.size());
    for (int j = 0; j < T.nc; ++j)
      for (int i = 0; i < 9; ++i) wmat.push_back(int8_t(G[T.w[j]][i]));
    while (wmat.size() % 16) wmat.push_back(0);
    // transposed sides: row s of B^T lists the rows r of B that read slot s
    // (with B's coefficient), and likewise for C^T
    auto transpose = [&](const std::vector<int>& rp, const std::vector<uint16_t>& en, std::vector<int>* trp,
                         std::vector<uint16_t>* ten) {
      const int rows = 8 * T.nc;
      std::vector<std::vector<uint16_t>> byrow(rows);
      for (int r = 0; r < rows; ++r)
        for (int e = rp[r]; e < rp[r + 1]; ++e) byrow[en[e] >> 8].push_back(uint16_t((r << 8) | (en[e] & 255u)));
      trp->assign(1, 0);
      ten->clear();
      for (int r = 0; r < rows; ++r) {
        ten->insert(ten->end(), byrow[r].begin(), byrow[r].end());
        trp->push_back(int(ten->size()));
      }
    };
    std::vector<int> bt_rp, ct_rp;
    std::vector<uint16_t> bt_en, ct_en;
    transpose(T.b_rowptr, T.b_ent, &bt_rp, &bt_en);
    transpose(T.c_rowptr, T.c_ent, &ct_rp, &ct_en);
    for (int side = 0; side < 4; ++side) {
      const std::vector<int>& rp = side == 0 ? T.b_rowptr : side == 1 ? T.c_rowptr : side == 2 ? bt_rp : ct_rp;
      const std::vector<uint16_t>& en = side == 0 ? T.b_ent : side == 1 ? T.c_ent : side == 2 ? bt_en : ct_en;
      std::vector<int> seg(1, 0);
      std::vector<uint32_t> se;
      for (int r = 0; r < 8 * T.nc; ++r)
        for (int q = 0; q < kNumMono; ++q) {
          for (int e = rp[r]; e < rp[r + 1]; ++e) {
            const double c = ob->poly[size_t(en[e] & 255u) * kNumMono + q] * 144.0;
            const long long kc = std::llround(c);
            if (kc == 0) continue;
            if (std::fabs(c - double(kc)) > 1e-9 || kc < -32768 || kc > 32767) return FCC_ERR_UNSUPPORTED;
            se.push_back((uint32_t(en[e] >> 8) << 16) | (uint32_t(kc) & 0xffffu));
          }
          seg.push_back(int(se.size()));
        }
      if (se.size() > size_t(kOrbitMaxEnt)) return FCC_ERR_UNSUPPORTED;
      k.off_rowptr[side] = int(rowptr.size());
      for (int v : seg) rowptr.push_back(uint16_t(v));
      while (rowptr.size() % 8) rowptr.push_back(0);
      k.off_ent[side] = int(ent.size());
      k.nent[side] = int(se.size());
      ent.insert(ent.end(), se.begin(), se.end());
      while (ent.size() % 4) ent.push_back(0);
      k.off_perm[side] = int(perm.size());
      const std::vector<int16_t> q = quad_order(seg, T.nc);
      perm.insert(perm.end(), q.begin(), q.end());
      while (perm.size() % 8) perm.push_back(-1);
    }
    kinds.push_back(k);
    const std::vector<uint32_t>& r = ob->reps[t];
    // one block's orbits per chunk: K = U (blocks of one node) or U / 8
    const int lgU = orbit_lg_units(T.nc);
    for (int gs = 0; gs < 2; ++gs) {
      const size_t K = size_t(1) << (gs == 0 ? lgU : lgU - 3);
      for (size_t r0 = 0; r0 < r.size(); r0 += K)
        chunks[gs].push_back(make_int4(int(t), int(reps.size() + r0), int(std::min(K, r.size() - r0)), lgU));
    }
    reps.insert(reps.end(), r.begin(), r.end());
  }
  DevOrbitLevel lv{};
  fcc_status s = FCC_OK;
  if (s == FCC_OK) s = upload(kinds, &lv.kinds);
  if (s == FCC_OK) s = upload(perm, &lv.perm);
  if (s == FCC_OK) s = upload(rowptr, &lv.rowptr);
  if (s == FCC_OK) s = upload(ent, &lv.ent);
  if (s == FCC_OK) s = upload(wmat, &lv.wmat);
  if (s == FCC_OK) s = upload(reps, &lv.reps);
  for (int gs = 0; gs < 2 && s == FCC_OK; ++gs) s = upload(chunks[gs], &lv.chunks[gs]);
  if (s != FCC_OK) return s;
  for (int gs = 0; gs < 2; ++gs) lv.nchunk[gs] = int(chunks[gs].size());
  lv.lgm = 0;
  while ((1 << lv.lgm) < ob->m) ++lv.lgm;
  levels.emplace(key, lv);
  *out = lv;
  return FCC_OK;
}

bool is_pow2(int n) { return n >= 1 && n <= 1024 && (n & (n - 1)) == 0; }

// Coinciding zeros: theta_j and theta_j' give the same (x,y,z) iff
// theta_j' = g^T theta_j mod Z^3 for some g in W (T_k(g^T theta) = T_k(theta)).
// With theta_j = (rst + j)/n this happens for some j != j' iff (g^T - I) rst is
// integral for some g whose induced map j -> g^T j + (g^T - I) rst (mod n) is
// not the identity.
bool singular_skew(int n, const double rst[3]) {
  if (n == 1) return false;
  for (const auto& g : weyl_group()) {
    int gt[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) gt[3 * i + j] = g[3 * j + i];
    bool ident = true;
    for (int i = 0; i < 9; ++i) ident &= gt[i] == ((i % 4) == 0 ? 1 : 0);
    if (ident) continue;
    double v[3];
    bool integral = true;
    for (int i = 0; i < 3; ++i) {
      v[i] = gt[3 * i] * rst[0] + gt[3 * i + 1] * rst[1] + gt[3 * i + 2] * rst[2] - rst[i];
      integral &= std::fabs(v[i] - std::nearbyint(v[i])) < 1e-12;
    }
    if (!integral) continue;
    bool identity_mod_n = true;
    for (int i = 0; i < 3; ++i) {
      long long vi = (long long)std::nearbyint(v[i]);
      if (((vi % n) + n) % n != 0) identity_mod_n = false;
      for (int j = 0; j < 3; ++j) {
        long long e = gt[3 * i + j] - (i == j ? 1 : 0);
        if (((e % n) + n) % n != 0) identity_mod_n = false;
      }
    }
    if (!identity_mod_n) return true;
  }
  return false;
}

}  // namespace

namespace {

DT in_type(const fcc_plan_s* p) {
  bool dbl = p->prec == FCC_PREC_FP64;
  if (p->flags & FCC_REAL_INPUT) return dbl ? DT::F64R : DT::F32R;
  return dbl ? DT::F64C : DT::F32C;
}
DT cplx_type(const fcc_plan_s* p) { return p->prec == FCC_PREC_FP64 ? DT::F64C : DT::F32C; }
DT stage_type(const fcc_plan_s* p) { return p->stages64 ? DT::F64C : DT::F32C; }
// Type of the buffer that holds the coefficient vectors of level L's nodes
// (the input of forward level L, the output of inverse level L).  With
// level0_fp32 the top level's result (level 1's input) is complex64; the
// in-place DCT_2^{-1} pass of level L then reads and writes elements of one
// size (buf_type(L+1) has the size of level L's arithmetic type) at every L.
DT buf_type(const fcc_plan_s* p, int L) { return (p->level0_fp32 && L == 1) ? DT::F32C : stage_type(p); }
bool arith64(const fcc_plan_s* p, int L) { return p->stages64 && !(p->level0_fp32 && L == 0); }

constexpr int kBlock = 256;

// Per-launch timing.  While a timer is active on this thread, every kernel of
// the transform is launched with its own start and stop event
// (hipExtLaunchKernelGGL records them at the kernel's start and end), so a
// slot's time is the kernel's own duration without the gaps between launches.
struct LaunchTimer {
  std::vector<hipEvent_t>* ev = nullptr;  // 2 per launch
  size_t next = 0;
};
thread_local LaunchTimer* t_timer = nullptr;
template <typename... KArgs, typename... Args>
void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, unsigned shmem, hipStream_t st, Args... args) {
  LaunchTimer* tm = t_timer;
  if (tm && tm->next + 2 <= tm->ev->size()) {
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, (*tm->ev)[tm->next], (*tm->ev)[tm->next + 1], 0, args...);
    tm->next += 2;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
  }
}


// One thread per 2x2x2 cube.  Small passes (fewer than 4 blocks of 256 per
// CU) use blocks of 64 threads so that they still reach every CU.
int cube_block(int n, int nvol) {
  const long long h = n >> 1;
  return h * h * h * nvol < 1024LL * kBlock ? 64 : kBlock;
}
dim3 grid_cubes(int n, int nvol) {
  const long long h = n >> 1, threads = h * h * h * nvol, b = cube_block(n, nvol);
  return dim3((unsigned)((threads + b - 1) / b), 1, 1);
}
dim3 grid_points(int n, int nvol) {  // one thread per point (gather row)
  long long threads = (long long)n * n * n * nvol;
  return dim3((unsigned)((threads + kBlock - 1) / kBlock), 1, 1);
}
const double2* phases(const fcc_plan_s* p, int L) { return p->hph + 3 * ((1 << L) - 1); }
const NodeConst* nodes_of(const fcc_plan_s* p, int L) {
  return (p->nodes && p->node_off[L] >= 0) ? static_cast<const NodeConst*>(p->nodes) + p->node_off[L] : nullptr;
}

// thread map of the gather pass of direction d (0 forward, 1 inverse) at level L
// (f_inner needs whole slices: the node must have at least S cubes)
GatherMap gmap(const fcc_plan_s* p, int d, int L) {
  const unsigned m = p->tune.map[d][L];
  const long long half = p->n >> (L + 1), cubes = half * half * half;
  const bool whole = cubes >= p->lv[L].S;
  GatherMap g{};
  g.xcd = (m & FCC_MAP_XCD16) ? 2 : int(m & FCC_MAP_XCD);
  g.f_inner = int(whole && (m & FCC_MAP_F_INNER) != 0);
  g.lg = 3 * L;
  // the clustered map runs blocks of 4 whole slices (levels 0 and 1 only)
  const long long S = p->lv[L].S;
  g.cluster = int((m & FCC_MAP_CLUSTER) && L <= 1 && S > 1 && cubes % (4 * S) == 0);
  if (g.cluster) g.f_inner = 0;
  if (L >= 2 && (m & FCC_MAP_NODES8)) g.lg = std::min(3, 3 * L);
  if (L >= 2 && (m & FCC_MAP_NODES64)) g.lg = std::min(6, 3 * L);
  if ((m & FCC_MAP_BALANCE) && !g.cluster) {
    g.balance = 1;
    g.f_inner = 0;
    // f by decreasing lanes per row keeps every row's lanes aligned
    int ord[8] = {0, 1, 2, 3, 4, 5, 6, 7};
    std::stable_sort(ord, ord + 8, [&](int a, int b) { return p->kf[d][L][a] > p->kf[d][L][b]; });
    const long long unit = cubes << g.lg;  // threads per lane slot of one f in a group
    g.off[0] = 0;
    for (int i = 0; i < 8; ++i) {
      g.forder[i] = (unsigned char)ord[i];
      g.kf[i] = p->kf[d][L][ord[i]];
      g.off[i + 1] = g.off[i] + (unit << g.kf[i]);
    }
  }
  return g;
}
// threads of a gather launch: one per row, or one per row part (balanced map)
dim3 grid_gather(const fcc_plan_s* p, const GatherMap& g, int L, int nvol) {
  if (!g.balance) return grid_points(p->n, nvol);
  const long long threads = g.off[8] * ((1LL << (3 * L)) >> g.lg) * nvol;
  return dim3(unsigned((threads + kBlock - 1) / kBlock));
}

// rows are wave-uniform: one cube per slice, 64 lanes in one node group, no parts
bool uniform_rows(const fcc_plan_s* p, const GatherMap& gm, int L) {
  return p->lv[L].S == 1 && gm.lg >= 6 && !gm.balance;
}
template <typename R, bool U>
void fwd_gather_launch(const fcc_plan_s* p, int L, DT ti, const VolSet& vs, int nvol, hipStream_t st,
                       const GatherMap& gm, dim3 g) {
  const double2* h = phases(p, L);
  const NodeConst* nc = nodes_of(p, L);
  switch (ti) {
    case DT::F32R: launch((k_fwd_gather<R, float, U>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm); break;
    case DT::F64R: launch((k_fwd_gather<R, double, U>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm); break;
    case DT::F32C: launch((k_fwd_gather<R, float2, U>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm); break;
    case DT::F64C: launch((k_fwd_gather<R, double2, U>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm); break;
  }
}
template <typename R>
void fwd_gather_dispatch(const fcc_plan_s* p, int L, DT ti, const VolSet& vs, int nvol, hipStream_t st) {
  const GatherMap gm = gmap(p, 0, L);
  const dim3 g = grid_gather(p, gm, L, nvol);
  if (uniform_rows(p, gm, L))
    fwd_gather_launch<R, true>(p, L, ti, vs, nvol, st, gm, g);
  else
    fwd_gather_launch<R, false>(p, L, ti, vs, nvol, st, gm, g);
}
template <typename R, typename TI>
void fwd_level_out(const fcc_plan_s* p, int L, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  dim3 g = grid_points(p->n, nvol);
  const double2* h = phases(p, L);
  const NodeConst* nc = nodes_of(p, L);
  const GatherMap gm = gmap(p, 0, L);
  if (nc) {
    if (to == DT::F32C)
      launch((k_fwd_level<R, TI, float2, true>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm);
    else
      launch((k_fwd_level<R, TI, double2, true>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm);
  } else {
    if (to == DT::F32C)
      launch((k_fwd_level<R, TI, float2, false>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm);
    else
      launch((k_fwd_level<R, TI, double2, false>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm);
  }
}
template <typename R>
void fwd_level_dispatch(const fcc_plan_s* p, int L, DT ti, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  switch (ti) {
    case DT::F32R: fwd_level_out<R, float>(p, L, to, vs, nvol, st); break;
    case DT::F64R: fwd_level_out<R, double>(p, L, to, vs, nvol, st); break;
    case DT::F32C: fwd_level_out<R, float2>(p, L, to, vs, nvol, st); break;
    case DT::F64C: fwd_level_out<R, double2>(p, L, to, vs, nvol, st); break;
  }
}
// Level L of direction d (0 forward, 1 inverse) runs as one orbit-block
// launch (orbit_level.hpp): the schedule asks for it, the node size is at
// least 16, the level is above the fused tail and its templates are on the GPU.
bool orbit_at(const fcc_plan_s* p, int d, int L) {
  return L < 10 && (p->tune.map[d][L] & FCC_MAP_ORBIT) && (p->n >> L) >= 8 && L < p->tail_Lt[d] &&
         L < int(p->olv.size()) && p->olv[L].kinds != nullptr && p->onodes && p->onode_off[L] >= 0;
}
bool fwd_split(const fcc_plan_s* p, int L) { return !orbit_at(p, 0, L) && (p->tune.map[0][L] & FCC_MAP_SPLIT) != 0; }
// The DCT_2 pass of level D - 2 and the last level run as one launch: the
// last level runs alone (fused depth 1) after a two-pass level D - 2 (D >= 3)
// in the same arithmetic.
bool fwd_last2(const fcc_plan_s* p) {
  return !p->fold_base && p->D >= 3 && p->tail_Lt[0] == p->D - 1 && fwd_split(p, p->D - 2) &&
         arith64(p, p->D - 2) == arith64(p, p->D - 1);
}
// The inverse counterpart: the last level alone, then the DCT_2^{-1} pass of
// level D - 2, as one launch.
bool orbit_at(const fcc_plan_s* p, int d, int L);
bool inv_last2(const fcc_plan_s* p) {
  return p->D >= 3 && p->tail_Lt[1] == p->D - 1 && buf_type(p, p->D - 1) == stage_type(p) && !orbit_at(p, 1, p->D - 2) &&
         arith64(p, p->D - 2) == arith64(p, p->D - 1);
}
// ... and the C gather of level D - 2 (node size 4) in the same launch, where
// that level's row table has one cube per slice (D - 2 >= 2).
bool inv_last2c(const fcc_plan_s* p) {
  const int L = p->D - 2;
  if (!(inv_last2(p) && L >= 2 && L < int(p->lv.size()) && p->lv[L].c.start != nullptr && p->lv[L].S == 1)) return false;
  const LevelTables* T = level_tables(4);  // one cube per slice: the device rows hold c_rowptr.back() entries
  return T && T->c_rowptr.size() == 65 && T->c_rowptr.back() <= kLast2cEnt && p->lv[L].npoly <= kLast2cPoly;
}
// number of launch slots of one transform in direction d (0 forward, 1 inverse)
// (Hermitian-packed plans add the pack launch after the forward and the
// unpack launch before the inverse.)
int slot_count(const fcc_plan_s* p, int d) {
  const int extra = p->hslot ? 1 : 0;
  if (p->fold) return p->n == 1 ? 1 : 4;
  if (p->dense) return 2;  // split of the input, GEMM
  if (p->n == 1) return 1 + extra;
  if (p->transposed) return p->D;
  int k = 1 + extra;
  if (d == 1) {
    for (int L = 0; L < p->tail_Lt[1]; ++L) k += orbit_at(p, 1, L) ? 1 : 2;
    return inv_last2c(p) ? k - 2 : (inv_last2(p) ? k - 1 : k);
  }
  for (int L = 0; L < p->tail_Lt[0]; ++L) k += fwd_split(p, L) ? 2 : 1;
  return fwd_last2(p) ? k - 1 : k;
}
// First launch slot of level L (L < tail_Lt[d]) in direction d.
int level_slot(const fcc_plan_s* p, int d, int L) {
  int k = 0;
  if (d == 0) {
    for (int l = 0; l < L; ++l) k += fwd_split(p, l) ? 2 : 1;
    return k;
  }
  k = 1;  // the tail, or the last level (with the DCT_2^{-1} pass of level D - 2)
  for (int l = p->tail_Lt[1] - 1; l > L; --l)
    k += orbit_at(p, 1, l) ? 1 : (l == p->D - 2 && inv_last2(p) ? (inv_last2c(p) ? 0 : 1) : 2);
  return k;
}

// Names and algorithmic element sizes of the launch slots of one transform in
// direction d, in launch order (the same decisions as enqueue_forward and
// enqueue_inverse).  A launch is priced by the method's own input and output:
// each element read once and written once, in the plan's data precision
// (real input 4 or 8 bytes, complex 8 or 16), whatever its stage precision.
struct SlotDesc {
  std::string name;
  int in_b, out_b;
};
std::vector<SlotDesc> describe_slots(const fcc_plan_s* p, int d) {
  const int r = p->prec == FCC_PREC_FP64 ? 8 : 4, c = 2 * r;
  const int rin = (p->flags & FCC_REAL_INPUT) ? r : c;
  std::vector<SlotDesc> v;
  auto L_ = [](int L) { return " L" + std::to_string(L); };
  if (p->hslot) {
    // the plain transform's slots, then the pack launch (forward), or the
    // unpack launch, then the plain slots (inverse): full spectrum <-> packed
    fcc_plan_s q = *p;
    q.hslot = nullptr;
    std::vector<SlotDesc> b = describe_slots(&q, d);
    if (d == 0)
      b.push_back({"k_hpack", c, c});
    else
      b.insert(b.begin(), {"k_hunpack", c, c});
    return b;
  }
  if (p->fold) {
    // priced like the other launches: each DFT pass reads and writes the volume once
    if (d == 0) {
      v.push_back({"k_fold", rin, c});
      if (p->n > 1)
        for (const char* a : {"k_dft c", "k_dft b", "k_dft a"}) v.push_back({a, c, c});
    } else {
      if (p->n > 1)
        for (const char* a : {"k_dft a", "k_dft b", "k_dft c"}) v.push_back({a, c, c});
      v.push_back({"k_unfold", c, rin});
    }
    return v;
  }
  if (p->n == 1) return {{d == 0 ? "k_copy1" : "k_copy1", d == 0 ? rin : c, d == 0 ? c : rin}};
  if (p->dense) {
    // the split of the input (read once, hi + lo written in 16 bits) and the GEMM
    const std::string t = p->prec == FCC_PREC_SPLIT_FP16 ? "<f16>" : "<bf16>";
    const int bi = d == 0 ? rin : c, bo = d == 0 ? c : rin;
    return {{"k_split_rows" + t, bi, bi}, {"k_split_gemm" + t, bi, bo}};
  }
  const int D = p->D;
  if (p->transposed) {
    if (d == 0) {
      v.push_back({"k_tr_last" + L_(D - 1), rin, c});
      for (int L = D - 2; L >= 0; --L) v.push_back({"k_tr_orbit" + L_(L), c, c});
    } else {
      for (int L = 0; L <= D - 2; ++L) v.push_back({"k_tr_inv_orbit" + L_(L), c, c});
      v.push_back({"k_tr_inv_last" + L_(D - 1), c, rin});
    }
    return v;
  }
  if (d == 0) {
    for (int L = 0; L < p->tail_Lt[0]; ++L) {
      const int bi = L == 0 ? rin : c;
      if (orbit_at(p, 0, L)) {
        v.push_back({"k_fwd_orbit" + L_(L), bi, c});
      } else if (fwd_split(p, L)) {
        v.push_back({"k_fwd_gather" + L_(L), bi, c});
        if (!(L == D - 2 && fwd_last2(p))) v.push_back({"k_fwd_dct2" + L_(L), c, c});
      } else {
        v.push_back({"k_fwd_level" + L_(L), bi, c});
      }
    }
    if (p->fold_base)
      v.push_back({"k_fwd_base L" + std::to_string(p->tail_Lt[0]) + "-" + std::to_string(D - 1),
                   p->tail_Lt[0] == 0 ? rin : c, c});
    else if (fwd_last2(p))
      v.push_back({"k_fwd_dct2_last2 L" + std::to_string(D - 2) + "-" + std::to_string(D - 1), c, c});
    else if (p->tail_Lt[0] == D - 1 && D >= 2)
      v.push_back({"k_fwd_dct2" + L_(D - 1), c, c});
    else
      v.push_back({"k_fwd_tail L" + std::to_string(p->tail_Lt[0]) + "-" + std::to_string(D - 1),
                   p->tail_Lt[0] == 0 ? rin : c, c});
    return v;
  }
  const int Lt = p->tail_Lt[1];
  if (inv_last2c(p))
    v.push_back({"k_inv_last2c L" + std::to_string(D - 1) + "-" + std::to_string(D - 2), c, c});
  else if (inv_last2(p))
    v.push_back({"k_inv_dct2_last2 L" + std::to_string(D - 1) + "-" + std::to_string(D - 2), c, c});
  else if (Lt == D - 1 && D >= 2 && buf_type(p, D - 1) == stage_type(p))
    v.push_back({"k_inv_dct2" + L_(D - 1), c, c});
  else
    v.push_back({"k_inv_tail L" + std::to_string(D - 1) + "-" + std::to_string(Lt), c, Lt == 0 ? rin : c});
  for (int L = Lt - 1; L >= 0; --L) {
    const int bo = L == 0 ? rin : c;
    if (L == D - 2 && inv_last2c(p)) continue;  // in the first slot
    if (orbit_at(p, 1, L)) {
      v.push_back({"k_inv_orbit" + L_(L), c, bo});
      continue;
    }
    if (!(L == D - 2 && inv_last2(p))) v.push_back({"k_inv_dct2" + L_(L), c, c});
    v.push_back({"k_inv_basis" + L_(L), c, bo});
  }
  return v;
}

// ---- orbit-block level launches -------------------------------------------
dim3 orbit_grid(const fcc_plan_s* p, int L, int nvol) {
  const long long total = orbit_blocks_total(p->olv[L].nchunk[L == 0 ? 0 : 1], L, nvol);
  return dim3(unsigned(((total + 7) >> 3) << 3));
}
const OrbitNode* onodes_of(const fcc_plan_s* p, int L) {
  return static_cast<const OrbitNode*>(p->onodes) + p->onode_off[L];
}
template <typename R, typename TI, typename TO, bool kT = false>
void fwd_orbit_launch(const fcc_plan_s* p, int L, const VolSet& vs, int nvol, hipStream_t st) {
  launch((k_fwd_orbit<R, TI, TO, kT>), orbit_grid(p, L, nvol), dim3(kOrbitThreads), 0, st, vs, nvol, p->n, L,
         p->olv[L], phases(p, L), onodes_of(p, L));
}
void fwd_orbit_dispatch(const fcc_plan_s* p, int L, DT ti, const VolSet& vs, int nvol, hipStream_t st) {
  if (arith64(p, L)) {
    switch (ti) {
      case DT::F32R: fwd_orbit_launch<double, float, double2>(p, L, vs, nvol, st); break;
      case DT::F64R: fwd_orbit_launch<double, double, double2>(p, L, vs, nvol, st); break;
      case DT::F32C: fwd_orbit_launch<double, float2, double2>(p, L, vs, nvol, st); break;
      case DT::F64C: fwd_orbit_launch<double, double2, double2>(p, L, vs, nvol, st); break;
    }
  } else {
    // FP32 arithmetic: FP32 data in, complex64 out (FP32 stages or FP32 top level)
    if (ti == DT::F32R)
      fwd_orbit_launch<float, float, float2>(p, L, vs, nvol, st);
    else
      fwd_orbit_launch<float, float2, float2>(p, L, vs, nvol, st);
  }
}
template <typename R, typename TI, typename TO, bool kT = false>
void inv_orbit_launch(const fcc_plan_s* p, int L, const VolSet& vs, int nvol, hipStream_t st) {
  launch((k_inv_orbit<R, TI, TO, kT>), orbit_grid(p, L, nvol), dim3(kOrbitThreads), 0, st, vs, nvol, p->n, L,
         p->olv[L], phases(p, L), onodes_of(p, L));
}
void inv_orbit_dispatch(const fcc_plan_s* p, int L, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  if (arith64(p, L)) {
    switch (to) {
      case DT::F32R: inv_orbit_launch<double, double2, float>(p, L, vs, nvol, st); break;
      case DT::F64R: inv_orbit_launch<double, double2, double>(p, L, vs, nvol, st); break;
      case DT::F32C: inv_orbit_launch<double, double2, float2>(p, L, vs, nvol, st); break;
      case DT::F64C: inv_orbit_launch<double, double2, double2>(p, L, vs, nvol, st); break;
    }
  } else {
    if (to == DT::F32R)
      inv_orbit_launch<float, float2, float>(p, L, vs, nvol, st);
    else
      inv_orbit_launch<float, float2, float2>(p, L, vs, nvol, st);
  }
}

template <typename R>
void fwd_dct2_dispatch(const fcc_plan_s* p, int L, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  dim3 g = grid_cubes(p->n, nvol);
  const double2* h = phases(p, L);
  const NodeConst* nc = nodes_of(p, L);
  if (to == DT::F32C)
    launch((k_fwd_dct2<R, float2>), g, dim3(cube_block(p->n, nvol)), 0, st, vs, nvol, p->n, L, h, nc);
  else
    launch((k_fwd_dct2<R, double2>), g, dim3(cube_block(p->n, nvol)), 0, st, vs, nvol, p->n, L, h, nc);
}

template <typename R>
void fwd_last2_dispatch(const fcc_plan_s* p, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  const int L = p->D - 2;
  const dim3 g = grid_cubes(p->n, nvol);
  const int b = cube_block(p->n, nvol);
  const unsigned sh = unsigned(b) * 9u * unsigned(sizeof(cx<R>));
  if (to == DT::F32C)
    launch((k_fwd_dct2_last2<R, float2>), g, dim3(b), sh, st, vs, nvol, p->n, L, phases(p, L), nodes_of(p, L),
           phases(p, L + 1), nodes_of(p, L + 1));
  else
    launch((k_fwd_dct2_last2<R, double2>), g, dim3(b), sh, st, vs, nvol, p->n, L, phases(p, L), nodes_of(p, L),
           phases(p, L + 1), nodes_of(p, L + 1));
}

template <typename R>
void inv_last2_dispatch(const fcc_plan_s* p, DT ti, const VolSet& vs, int nvol, hipStream_t st) {
  const int L = p->D - 2;
  const dim3 g = grid_cubes(p->n, nvol);
  const int b = cube_block(p->n, nvol);
  const bool fused = inv_last2c(p);
  // the exchange rows, and where fused the node rows (b / 8 nodes of 73 values)
  const unsigned sh = (unsigned(b) * 9u + (fused ? unsigned(b / 8) * 73u : 0u)) * unsigned(sizeof(cx<R>));
  if (fused) {
    if (ti == DT::F32C)
      launch((k_inv_dct2_last2<R, float2, true>), g, dim3(b), sh, st, vs, nvol, p->n, L, phases(p, L),
             nodes_of(p, L), phases(p, L + 1), nodes_of(p, L + 1), p->lv[L], level_tables(4)->c_rowptr.back());
    else
      launch((k_inv_dct2_last2<R, double2, true>), g, dim3(b), sh, st, vs, nvol, p->n, L, phases(p, L),
             nodes_of(p, L), phases(p, L + 1), nodes_of(p, L + 1), p->lv[L], level_tables(4)->c_rowptr.back());
  } else if (ti == DT::F32C) {
    launch((k_inv_dct2_last2<R, float2>), g, dim3(b), sh, st, vs, nvol, p->n, L, phases(p, L), nodes_of(p, L),
           phases(p, L + 1), nodes_of(p, L + 1), DevLevel{}, 0);
  } else {
    launch((k_inv_dct2_last2<R, double2>), g, dim3(b), sh, st, vs, nvol, p->n, L, phases(p, L), nodes_of(p, L),
           phases(p, L + 1), nodes_of(p, L + 1), DevLevel{}, 0);
  }
}

template <typename R>
void inv_dct2_dispatch(const fcc_plan_s* p, int L, DT ti, const VolSet& vs, int nvol, hipStream_t st) {
  dim3 g = grid_cubes(p->n, nvol);
  const double2* h = phases(p, L);
  const NodeConst* nc = nodes_of(p, L);
  if (ti == DT::F32C)
    launch((k_inv_dct2<R, float2>), g, dim3(cube_block(p->n, nvol)), 0, st, vs, nvol, p->n, L, h, nc);
  else
    launch((k_inv_dct2<R, double2>), g, dim3(cube_block(p->n, nvol)), 0, st, vs, nvol, p->n, L, h, nc);
}
template <typename R, bool U>
void inv_basis_launch(const fcc_plan_s* p, int L, DT to, const VolSet& vs, int nvol, hipStream_t st,
                      const GatherMap& gm, dim3 g) {
  const double2* h = phases(p, L);
  const NodeConst* nc = nodes_of(p, L);
  switch (to) {
    case DT::F32R: launch((k_inv_basis<R, float, U>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm); break;
    case DT::F64R: launch((k_inv_basis<R, double, U>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm); break;
    case DT::F32C: launch((k_inv_basis<R, float2, U>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm); break;
    case DT::F64C: launch((k_inv_basis<R, double2, U>), g, dim3(kBlock), 0, st, vs, nvol, p->n, L, p->lv[L], h, nc, gm); break;
  }
}
template <typename R>
void inv_basis_dispatch(const fcc_plan_s* p, int L, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  const GatherMap gm = gmap(p, 1, L);
  const dim3 g = grid_gather(p, gm, L, nvol);
  if (uniform_rows(p, gm, L))
    inv_basis_launch<R, true>(p, L, to, vs, nvol, st, gm, g);
  else
    inv_basis_launch<R, false>(p, L, to, vs, nvol, st, gm, g);
}

TailLevels tail_levels(const fcc_plan_s* p, int Lt) {
  TailLevels tl{};
  for (int l = 0; l < p->D - Lt; ++l) {
    tl.lv[l] = p->tlv[Lt + l];
    tl.nodes[l] = nodes_of(p, Lt + l);
    tl.hph[l] = phases(p, Lt + l);
  }
  return tl;
}
int tail_cap(int nl0) { return nl0 <= 8 ? kTailCapSmall : kTailCapBig; }
// As many sibling nodes per block as the LDS buffer holds (within one row of
// J_z), fewer while the launch would have under 2048 blocks.
TailGeom tail_geom(const fcc_plan_s* p, int Lt, int nvol) {
  TailGeom g;
  g.n = p->n;
  g.Lt = Lt;
  g.nl0 = p->n >> Lt;
  g.k = p->D - Lt;
  g.G = std::min(tail_cap(g.nl0) / (g.nl0 * g.nl0 * g.nl0), 1 << Lt);
  while (g.G > 1 && (1LL << (3 * g.Lt)) / g.G * nvol < 2048) g.G >>= 1;
  return g;
}
dim3 tail_grid(const TailGeom& g, int nvol) { return dim3(unsigned(((1LL << (3 * g.Lt)) / g.G) * nvol)); }
dim3 tail_block_dim(const TailGeom& g) { return dim3(unsigned(std::max(64, g.G * g.nl0 * g.nl0 * g.nl0 / 8))); }
template <typename R, typename TI>
void fwd_tail_out(const fcc_plan_s* p, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  const TailGeom g = tail_geom(p, p->tail_Lt[0], nvol);
  const TailLevels tl = tail_levels(p, p->tail_Lt[0]);
  const dim3 gr = tail_grid(g, nvol), bd = tail_block_dim(g);
  const bool big = tail_cap(g.nl0) == kTailCapBig;
  if (to == DT::F32C) {
    if (big)
      launch((k_fwd_tail<R, TI, float2, kTailCapBig>), gr, bd, 0, st, vs, g, tl);
    else
      launch((k_fwd_tail<R, TI, float2, kTailCapSmall>), gr, bd, 0, st, vs, g, tl);
  } else {
    if (big)
      launch((k_fwd_tail<R, TI, double2, kTailCapBig>), gr, bd, 0, st, vs, g, tl);
    else
      launch((k_fwd_tail<R, TI, double2, kTailCapSmall>), gr, bd, 0, st, vs, g, tl);
  }
}
template <typename R>
void fwd_tail_dispatch(const fcc_plan_s* p, DT ti, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  switch (ti) {
    case DT::F32R: fwd_tail_out<R, float>(p, to, vs, nvol, st); break;
    case DT::F64R: fwd_tail_out<R, double>(p, to, vs, nvol, st); break;
    case DT::F32C: fwd_tail_out<R, float2>(p, to, vs, nvol, st); break;
    case DT::F64C: fwd_tail_out<R, double2>(p, to, vs, nvol, st); break;
  }
}
template <typename R, typename TI>
void inv_tail_out(const fcc_plan_s* p, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  const TailGeom g = tail_geom(p, p->tail_Lt[1], nvol);
  const TailLevels tl = tail_levels(p, p->tail_Lt[1]);
  const dim3 gr = tail_grid(g, nvol), bd = tail_block_dim(g);
  if (tail_cap(g.nl0) == kTailCapBig) {
    switch (to) {
      case DT::F32R: launch((k_inv_tail<R, TI, float, kTailCapBig>), gr, bd, 0, st, vs, g, tl); break;
      case DT::F64R: launch((k_inv_tail<R, TI, double, kTailCapBig>), gr, bd, 0, st, vs, g, tl); break;
      case DT::F32C: launch((k_inv_tail<R, TI, float2, kTailCapBig>), gr, bd, 0, st, vs, g, tl); break;
      case DT::F64C: launch((k_inv_tail<R, TI, double2, kTailCapBig>), gr, bd, 0, st, vs, g, tl); break;
    }
  } else {
    switch (to) {
      case DT::F32R: launch((k_inv_tail<R, TI, float, kTailCapSmall>), gr, bd, 0, st, vs, g, tl); break;
      case DT::F64R: launch((k_inv_tail<R, TI, double, kTailCapSmall>), gr, bd, 0, st, vs, g, tl); break;
      case DT::F32C: launch((k_inv_tail<R, TI, float2, kTailCapSmall>), gr, bd, 0, st, vs, g, tl); break;
      case DT::F64C: launch((k_inv_tail<R, TI, double2, kTailCapSmall>), gr, bd, 0, st, vs, g, tl); break;
    }
  }
}
template <typename R>
void inv_tail_dispatch(const fcc_plan_s* p, DT ti, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  if (ti == DT::F32C)
    inv_tail_out<R, float2>(p, to, vs, nvol, st);
  else
    inv_tail_out<R, double2>(p, to, vs, nvol, st);
}

// ---- FCC_FOLD_BASE: the dense base of node size M = n >> tail_Lt[0] -------
int base_slot(int M) { return M == 4 ? 0 : (M == 8 ? 1 : 2); }
template <typename R, typename TI, int M>
void fwd_base_launch(const fcc_plan_s* p, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  const int Lt = p->tail_Lt[0];
  const int G = std::min(BaseShape<M>::G, 1 << Lt);
  const long long blocks = ((1LL << (3 * Lt)) / G) * nvol;
  const dim3 gr(unsigned(((blocks + 7) >> 3) << 3)), bd(256);
  const int2* reps = reinterpret_cast<const int2*>(p->breps) + p->brep_off[base_slot(M)];
  const int norb = p->brep_cnt[base_slot(M)];
  if constexpr (std::is_same<R, float>::value) {
    launch((k_fwd_base<R, TI, float2, M>), gr, bd, 0, st, vs, nvol, p->n, Lt, G, p->r8[0], p->r8[1], p->r8[2],
           reps, norb);
  } else {
    if (to == DT::F32C)
      launch((k_fwd_base<R, TI, float2, M>), gr, bd, 0, st, vs, nvol, p->n, Lt, G, p->r8[0], p->r8[1], p->r8[2],
             reps, norb);
    else
      launch((k_fwd_base<R, TI, double2, M>), gr, bd, 0, st, vs, nvol, p->n, Lt, G, p->r8[0], p->r8[1], p->r8[2],
             reps, norb);
  }
}
template <typename R, typename TI>
void fwd_base_m(const fcc_plan_s* p, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  const int M = p->n >> p->tail_Lt[0];
  if (M == 4)
    fwd_base_launch<R, TI, 4>(p, to, vs, nvol, st);
  else if (M == 8)
    fwd_base_launch<R, TI, 8>(p, to, vs, nvol, st);
  else
    fwd_base_launch<R, TI, 16>(p, to, vs, nvol, st);
}
// The base sits below at least one radix-2 level (tail_Lt[0] >= 1), so its
// input is a stage buffer: complex, FP64 or (FP32 stages, or level 1 of an
// FCC_LEVEL0_FP32 plan) FP32.
void fwd_base_dispatch(const fcc_plan_s* p, DT ti, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  if (!p->stages64)
    fwd_base_m<float, float2>(p, DT::F32C, vs, nvol, st);
  else if (ti == DT::F32C)
    fwd_base_m<double, float2>(p, to, vs, nvol, st);
  else
    fwd_base_m<double, double2>(p, to, vs, nvol, st);
}

template <typename TI, typename TO>
void launch_copy1(const VolSet& vs, int nvol, hipStream_t st) {
  launch((k_copy1<TI, TO>), dim3(unsigned((nvol + 63) / 64)), dim3(64), 0, st, vs, nvol);
}
void copy1_dispatch(DT ti, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  auto go = [&](auto tag_in) {
    using TI = decltype(tag_in);
    switch (to) {
      case DT::F32R: launch_copy1<TI, float>(vs, nvol, st); break;
      case DT::F64R: launch_copy1<TI, double>(vs, nvol, st); break;
      case DT::F32C: launch_copy1<TI, float2>(vs, nvol, st); break;
      case DT::F64C: launch_copy1<TI, double2>(vs, nvol, st); break;
    }
  };
  switch (ti) {
    case DT::F32R: go(float{}); break;
    case DT::F64R: go(double{}); break;
    case DT::F32C: go(float2{}); break;
    case DT::F64C: go(double2{}); break;
  }
}

// Optional per-launch timing: an event is recorded before the first launch and
// after every launch, so slot k's duration is ev[k+1] - ev[k].
// Enqueue the forward transform of nvol volumes that share plan p.
// ws0/ws1: two scratch arrays of n^3 stage-precision complex per volume.
fcc_status enqueue_transposed(const fcc_plan_s* p, int dir, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0,
                              VolPtrs ws1, hipStream_t st);
fcc_status enqueue_forward_plain(const fcc_plan_s* p, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0, VolPtrs ws1,
                                 hipStream_t st);
fcc_status enqueue_inverse_plain(const fcc_plan_s* p, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0, VolPtrs ws1,
                                 hipStream_t st);
// ---- FCC_FOLD_FFT: fold, three DFT passes; DFT passes, unfold ---------------
template <typename R, int N>
void dft_launch(int ax, int sgn, const VolSet& vs, int nvol, const cx<R>* w8n, int post_r8, hipStream_t st) {
  const dim3 g(unsigned(nvol * (N * N / dft_lines<R, N>()))), b(256);
  if (sgn > 0) {
    if (ax == 0) launch((k_dft<R, N, 0, 1>), g, b, 0, st, vs, nvol, w8n, post_r8);
    else if (ax == 1) launch((k_dft<R, N, 1, 1>), g, b, 0, st, vs, nvol, w8n, post_r8);
    else launch((k_dft<R, N, 2, 1>), g, b, 0, st, vs, nvol, w8n, post_r8);
  } else {
    if (ax == 0) launch((k_dft<R, N, 0, -1>), g, b, 0, st, vs, nvol, w8n, post_r8);
    else if (ax == 1) launch((k_dft<R, N, 1, -1>), g, b, 0, st, vs, nvol, w8n, post_r8);
    else launch((k_dft<R, N, 2, -1>), g, b, 0, st, vs, nvol, w8n, post_r8);
  }
}
template <typename R>
void dft_dispatch(int n, int ax, int sgn, const VolSet& vs, int nvol, const cx<R>* w8n, int post_r8, hipStream_t st) {
  switch (n) {
    case 2: dft_launch<R, 2>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    case 4: dft_launch<R, 4>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    case 8: dft_launch<R, 8>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    case 16: dft_launch<R, 16>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    case 32: dft_launch<R, 32>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    case 64: dft_launch<R, 64>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    case 128: dft_launch<R, 128>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    case 256: dft_launch<R, 256>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    case 512: dft_launch<R, 512>(ax, sgn, vs, nvol, w8n, post_r8, st); break;
    default: break;
  }
}
// Forward: k_fold (x -> out), then the DFT passes along c, b, a in place on
// out.  Inverse: the DFT passes along a (in -> ws0), b, c (in place, each with
// its axis phase), then k_unfold (ws0 -> out).
template <typename R>
fcc_status fold_run(const fcc_plan_s* p, int dir, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0, hipStream_t st) {
  const int n = p->n, lg = p->D;
  const cx<R>* w = static_cast<const cx<R>*>(p->fw8n);
  const int nrep = p->fnrep;
  // blocks of 64 lanes where 256 would leave CUs idle
  const int lanes = (long long)nrep * nvol >= 1024LL * kFoldLanes ? kFoldLanes : 64;
  const long long nblk = (long long)nvol * ((nrep + lanes - 1) / lanes);
  const dim3 gp(unsigned(((nblk + 7) >> 3) << 3)), b(lanes);
  const bool real = (p->flags & FCC_REAL_INPUT) != 0;
  const int* r8 = p->r8;
  const int* reps = static_cast<const int*>(p->freps);
  // the default skew's phases at compile time (only r8 mod 8 matters)
  const bool def = (r8[0] & 7) == 1 && (r8[1] & 7) == 0 && (r8[2] & 7) == 3;
  auto fold = [&](auto tin, auto dflt) {
    using TI = decltype(tin);
    launch((k_fold<R, TI, decltype(dflt)::value>), gp, b, 0, st, VolSet{in, out}, nvol, lg, r8[0], r8[1], r8[2], w,
           reps, nrep);
  };
  if (dir > 0) {
    if (real)
      def ? fold(R{}, std::true_type{}) : fold(R{}, std::false_type{});
    else
      def ? fold(cx<R>{}, std::true_type{}) : fold(cx<R>{}, std::false_type{});
    for (int ax = 2; n > 1 && ax >= 0; --ax) dft_dispatch<R>(n, ax, 1, VolSet{out, out}, nvol, w, 0, st);
    return launch_status("fold forward launch");
  }
  VolPtrs src = in;
  if (n > 1) {
    dft_dispatch<R>(n, 0, -1, VolSet{in, ws0}, nvol, w, r8[0], st);
    dft_dispatch<R>(n, 1, -1, VolSet{ws0, ws0}, nvol, w, r8[1], st);
    dft_dispatch<R>(n, 2, -1, VolSet{ws0, ws0}, nvol, w, r8[2], st);
    src = ws0;
  }
  const cx<R>* kt = static_cast<const cx<R>*>(p->fkt);
  auto unfold = [&](auto tout, auto dflt) {
    using TO = decltype(tout);
    launch((k_unfold<R, TO, decltype(dflt)::value>), gp, b, 0, st, VolSet{src, out}, nvol, lg, r8[0], r8[1], r8[2],
           kt, p->fnpat, reps, p->fpid, nrep);
  };
  if (real)
    def ? unfold(R{}, std::true_type{}) : unfold(R{}, std::false_type{});
  else
    def ? unfold(cx<R>{}, std::true_type{}) : unfold(cx<R>{}, std::false_type{});
  return launch_status("fold inverse launch");
}
fcc_status fold_enqueue(const fcc_plan_s* p, int dir, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0, hipStream_t st) {
  return p->prec == FCC_PREC_FP64 ? fold_run<double>(p, dir, nvol, in, out, ws0, st)
                                  : fold_run<float>(p, dir, nvol, in, out, ws0, st);
}

void hpack_launch(const fcc_plan_s* p, bool unpack, const void* src, void* dst, hipStream_t st) {
  const long long N = (long long)p->n * p->n * p->n;
  const dim3 g(unsigned((N + 255) / 256)), b(256);
  if (p->prec == FCC_PREC_FP64) {
    if (unpack)
      launch(k_hunpack<double2>, g, b, 0, st, static_cast<const double2*>(src), static_cast<double2*>(dst),
             static_cast<const int*>(p->hslot), N);
    else
      launch(k_hpack<double2>, g, b, 0, st, static_cast<const double2*>(src), static_cast<double2*>(dst),
             static_cast<const int*>(p->hslot), N);
  } else {
    if (unpack)
      launch(k_hunpack<float2>, g, b, 0, st, static_cast<const float2*>(src), static_cast<float2*>(dst),
             static_cast<const int*>(p->hslot), N);
    else
      launch(k_hpack<float2>, g, b, 0, st, static_cast<const float2*>(src), static_cast<float2*>(dst),
             static_cast<const int*>(p->hslot), N);
  }
}
// Enqueue the forward transform of nvol volumes that share plan p (the
// transposed transform for FCC_TRANSPOSED plans; FCC_HERMITIAN_PACKED plans
// serve one volume: the full spectrum goes to the plan's buffer, then packed).
fcc_status enqueue_forward(const fcc_plan_s* p, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0, VolPtrs ws1,
                           hipStream_t st) {
  if (p->fold) return fold_enqueue(p, 1, nvol, in, out, ws0, st);
  if (p->transposed) return enqueue_transposed(p, 1, nvol, in, out, ws0, ws1, st);
  if (p->hslot) {
    if (nvol != 1 || out.arr) return FCC_ERR_UNSUPPORTED;
    fcc_status s = enqueue_forward_plain(p, 1, in, VolPtrs{nullptr, p->hfull}, ws0, ws1, st);
    if (s != FCC_OK) return s;
    hpack_launch(p, false, p->hfull, out.one, st);
    return launch_status("pack launch");
  }
  return enqueue_forward_plain(p, nvol, in, out, ws0, ws1, st);
}
fcc_status enqueue_inverse(const fcc_plan_s* p, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0, VolPtrs ws1,
                           hipStream_t st) {
  if (p->fold) return fold_enqueue(p, -1, nvol, in, out, ws0, st);
  if (p->transposed) return enqueue_transposed(p, -1, nvol, in, out, ws0, ws1, st);
  if (p->hslot) {
    if (nvol != 1 || in.arr) return FCC_ERR_UNSUPPORTED;
    hpack_launch(p, true, in.one, p->hfull, st);
    fcc_status s = launch_status("unpack launch");
    if (s != FCC_OK) return s;
    return enqueue_inverse_plain(p, 1, VolPtrs{nullptr, p->hfull}, out, ws0, ws1, st);
  }
  return enqueue_inverse_plain(p, nvol, in, out, ws0, ws1, st);
}
fcc_status enqueue_forward_plain(const fcc_plan_s* p, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0, VolPtrs ws1,
                                 hipStream_t st) {
  if (p->n == 1) {
    copy1_dispatch(in_type(p), cplx_type(p), VolSet{in, out}, nvol, st);
    return launch_status("forward n=1 launch");
  }
  VolPtrs src = in;
  DT src_t = in_type(p);
  for (int L = 0; L < p->tail_Lt[0]; ++L) {
    VolPtrs a = (L & 1) ? ws1 : ws0;
    const DT to = buf_type(p, L + 1);
    if (orbit_at(p, 0, L)) {
      // basis change and DCT_2 over whole orbits, into a
      fwd_orbit_dispatch(p, L, src_t, VolSet{src, a}, nvol, st);
    } else if (!fwd_split(p, L)) {
      // basis change and DCT_2 in one launch, into a
      if (arith64(p, L))
        fwd_level_dispatch<double>(p, L, src_t, to, VolSet{src, a}, nvol, st);
      else
        fwd_level_dispatch<float>(p, L, src_t, to, VolSet{src, a}, nvol, st);
    } else {
      // pass 1: basis-change gather into a; pass 2: DCT_2 on the cubes of a, in place
      if (arith64(p, L))
        fwd_gather_dispatch<double>(p, L, src_t, VolSet{src, a}, nvol, st);
      else
        fwd_gather_dispatch<float>(p, L, src_t, VolSet{src, a}, nvol, st);
      if (L == p->D - 2 && fwd_last2(p)) {
        // this DCT_2 pass runs with the last level below
      } else if (arith64(p, L)) {
        fwd_dct2_dispatch<double>(p, L, to, VolSet{a, a}, nvol, st);
      } else {
        fwd_dct2_dispatch<float>(p, L, to, VolSet{a, a}, nvol, st);
      }
    }
    src = a;
    src_t = to;
  }
  // hybrid depth: one dense base per node of level tail_Lt[0]
  if (p->fold_base) {
    fwd_base_dispatch(p, src_t, cplx_type(p), VolSet{src, out}, nvol, st);
    return launch_status("forward base launch");
  }
  // the last level alone (node size 2, B_2 = I): DCT_2 on the cubes, with the
  // DCT_2 pass of level D - 2 where that level is two-pass
  if (fwd_last2(p)) {
    if (arith64(p, p->D - 1))
      fwd_last2_dispatch<double>(p, cplx_type(p), VolSet{src, out}, nvol, st);
    else
      fwd_last2_dispatch<float>(p, cplx_type(p), VolSet{src, out}, nvol, st);
    return launch_status("forward level launch");
  }
  if (p->tail_Lt[0] == p->D - 1 && p->D >= 2) {
    if (arith64(p, p->D - 1))
      fwd_dct2_dispatch<double>(p, p->D - 1, cplx_type(p), VolSet{src, out}, nvol, st);
    else
      fwd_dct2_dispatch<float>(p, p->D - 1, cplx_type(p), VolSet{src, out}, nvol, st);
    return launch_status("forward level launch");
  }
  // the last levels (node size <= 16) in one LDS-resident launch
  if (p->stages64)
    fwd_tail_dispatch<double>(p, src_t, cplx_type(p), VolSet{src, out}, nvol, st);
  else
    fwd_tail_dispatch<float>(p, src_t, cplx_type(p), VolSet{src, out}, nvol, st);
  return launch_status("forward level launch");
}

fcc_status enqueue_inverse_plain(const fcc_plan_s* p, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0, VolPtrs ws1,
                                 hipStream_t st) {
  DT real_or_cplx = (p->flags & FCC_REAL_INPUT) ? in_type(p) : cplx_type(p);
  if (p->n == 1) {
    copy1_dispatch(cplx_type(p), real_or_cplx, VolSet{in, out}, nvol, st);
    return launch_status("inverse n=1 launch");
  }
  // the last level alone (node size 2, C_2 = I): DCT_2^{-1} on the cubes
  // (its output type is the stage type of level D-1)
  const bool last_only = p->tail_Lt[1] == p->D - 1 && p->D >= 2 && buf_type(p, p->D - 1) == stage_type(p);
  const bool fused = inv_last2c(p);
  if (inv_last2(p)) {
    // with the DCT_2^{-1} pass of level D - 2 (its result lands in ws0, where
    // that pass would have written it), and where fused also with that
    // level's C gather (its result lands in ws1, the gather's destination)
    const VolPtrs dst = fused ? ws1 : ws0;
    if (arith64(p, p->D - 1))
      inv_last2_dispatch<double>(p, cplx_type(p), VolSet{in, dst}, nvol, st);
    else
      inv_last2_dispatch<float>(p, cplx_type(p), VolSet{in, dst}, nvol, st);
  } else if (last_only) {
    if (arith64(p, p->D - 1))
      inv_dct2_dispatch<double>(p, p->D - 1, cplx_type(p), VolSet{in, ws0}, nvol, st);
    else
      inv_dct2_dispatch<float>(p, p->D - 1, cplx_type(p), VolSet{in, ws0}, nvol, st);
  } else {
    // the last levels first, in one LDS-resident launch
    const int Lt = p->tail_Lt[1];
    VolPtrs dst = Lt == 0 ? out : ws0;
    DT to = Lt == 0 ? real_or_cplx : buf_type(p, Lt);
    if (p->stages64)
      inv_tail_dispatch<double>(p, cplx_type(p), to, VolSet{in, dst}, nvol, st);
    else
      inv_tail_dispatch<float>(p, cplx_type(p), to, VolSet{in, dst}, nvol, st);
  }
  VolPtrs cur = fused ? ws1 : ws0;
  bool cur_is_user = false;
  int which = fused ? 1 : 0;  // scratch array holding the current level's data
  for (int L = p->tail_Lt[1] - 1 - (fused ? 1 : 0); L >= 0; --L) {
    VolPtrs a = which ? ws1 : ws0;
    VolPtrs b = which ? ws0 : ws1;
    // the DCT_2^{-1} pass reads level L+1's result (or the user's X) and
    // writes level L's cube values in level L's arithmetic type
    DT ti = cur_is_user ? cplx_type(p) : buf_type(p, L + 1);
    if (orbit_at(p, 1, L)) {
      // DCT_2^{-1} and the basis change over whole orbits, cur -> dst
      VolPtrs dst = L == 0 ? out : b;
      DT to = L == 0 ? real_or_cplx : buf_type(p, L);
      inv_orbit_dispatch(p, L, to, VolSet{cur, dst}, nvol, st);
      cur = b;
      cur_is_user = false;
      which ^= 1;
      continue;
    }
    if (L == p->D - 2 && inv_last2(p)) {
      // done with the last level above
    } else if (arith64(p, L)) {
      inv_dct2_dispatch<double>(p, L, ti, VolSet{cur, a}, nvol, st);
    } else {
      inv_dct2_dispatch<float>(p, L, ti, VolSet{cur, a}, nvol, st);
    }
    VolPtrs dst = L == 0 ? out : b;
    DT to = L == 0 ? real_or_cplx : buf_type(p, L);
    if (arith64(p, L))
      inv_basis_dispatch<double>(p, L, to, VolSet{a, dst}, nvol, st);
    else
      inv_basis_dispatch<float>(p, L, to, VolSet{a, dst}, nvol, st);
    cur = b;
    cur_is_user = false;
    which ^= 1;
  }
  return launch_status("inverse level launch");
}

// The transposed transform (FCC_TRANSPOSED): forward X = F^T x runs the
// factors of eq. FastAlgorithm transposed, deepest level first (DCT_2^T per
// cube, then per level DCT_2^T and B^T over the orbits); the inverse
// x = F^{-T} X runs C^T and DCT_2^{-T} from the top level down.
template <typename R>
void tr_last_dispatch(const fcc_plan_s* p, bool inv, DT ti, DT to, const VolSet& vs, int nvol, hipStream_t st) {
  const int L = p->D - 1;
  const long long nodes = (1LL << (3 * L)) * nvol;
  const dim3 g(unsigned((nodes + 255) / 256)), b(256);
  const double2* h = phases(p, L);
  using RC = cx<R>;
  (void)sizeof(RC);
  auto go = [&](auto tin, auto tout) {
    using TI = decltype(tin);
    using TO = decltype(tout);
    if (inv)
      launch((k_tr_last<R, TI, TO, true>), g, b, 0, st, vs, nvol, p->n, L, h);
    else
      launch((k_tr_last<R, TI, TO, false>), g, b, 0, st, vs, nvol, p->n, L, h);
  };
  auto out_of = [&](auto tin) {
    switch (to) {
      case DT::F32R: go(tin, float{}); break;
      case DT::F64R: go(tin, double{}); break;
      case DT::F32C: go(tin, float2{}); break;
      case DT::F64C: go(tin, double2{}); break;
    }
  };
  switch (ti) {
    case DT::F32R: out_of(float{}); break;
    case DT::F64R: out_of(double{}); break;
    case DT::F32C: out_of(float2{}); break;
    case DT::F64C: out_of(double2{}); break;
  }
}
fcc_status enqueue_transposed(const fcc_plan_s* p, int dir, int nvol, VolPtrs in, VolPtrs out, VolPtrs ws0,
                              VolPtrs ws1, hipStream_t st) {
  const DT real_or_cplx = (p->flags & FCC_REAL_INPUT) ? in_type(p) : cplx_type(p);
  if (p->n == 1) {
    copy1_dispatch(dir > 0 ? in_type(p) : cplx_type(p), dir > 0 ? cplx_type(p) : real_or_cplx, VolSet{in, out}, nvol,
                   st);
    return launch_status("transposed n=1 launch");
  }
  const int D = p->D;
  const DT stg = stage_type(p);
  if (dir > 0) {
    VolPtrs dst = D == 1 ? out : ws0;
    if (p->stages64)
      tr_last_dispatch<double>(p, false, in_type(p), D == 1 ? cplx_type(p) : stg, VolSet{in, dst}, nvol, st);
    else
      tr_last_dispatch<float>(p, false, in_type(p), D == 1 ? cplx_type(p) : stg, VolSet{in, dst}, nvol, st);
    VolPtrs cur = ws0;
    int which = 1;
    for (int L = D - 2; L >= 0; --L) {
      VolPtrs d2 = L == 0 ? out : (which ? ws1 : ws0);
      const DT to = L == 0 ? cplx_type(p) : stg;
      if (p->stages64) {
        if (to == DT::F32C)
          inv_orbit_launch<double, double2, float2, true>(p, L, VolSet{cur, d2}, nvol, st);
        else
          inv_orbit_launch<double, double2, double2, true>(p, L, VolSet{cur, d2}, nvol, st);
      } else {
        inv_orbit_launch<float, float2, float2, true>(p, L, VolSet{cur, d2}, nvol, st);
      }
      cur = d2;
      which ^= 1;
    }
    return launch_status("transposed forward launch");
  }
  VolPtrs src = in;
  DT src_t = cplx_type(p);
  for (int L = 0; L <= D - 2; ++L) {
    VolPtrs d2 = (L & 1) ? ws1 : ws0;
    if (p->stages64) {
      if (src_t == DT::F32C)
        fwd_orbit_launch<double, float2, double2, true>(p, L, VolSet{src, d2}, nvol, st);
      else
        fwd_orbit_launch<double, double2, double2, true>(p, L, VolSet{src, d2}, nvol, st);
    } else {
      fwd_orbit_launch<float, float2, float2, true>(p, L, VolSet{src, d2}, nvol, st);
    }
    src = d2;
    src_t = stg;
  }
  if (p->stages64)
    tr_last_dispatch<double>(p, true, src_t, real_or_cplx, VolSet{src, out}, nvol, st);
  else
    tr_last_dispatch<float>(p, true, src_t, real_or_cplx, VolSet{src, out}, nvol, st);
  return launch_status("transposed inverse launch");
}

VolPtrs one_vol(const void* p) { return VolPtrs{nullptr, const_cast<void*>(p)}; }
VolPtrs many_vol(void* const* dev_arr) { return VolPtrs{dev_arr, nullptr}; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

namespace fcc {
fcc_status enqueue_inverse_arrays(const fcc_plan_s* p, int nvol, void* const* in_dev, void* const* out_dev,
                                  void* const* ws0_dev, void* const* ws1_dev, hipStream_t st) {
  return enqueue_inverse(p, nvol, many_vol(in_dev), many_vol(out_dev), many_vol(ws0_dev), many_vol(ws1_dev), st);
}
}  // namespace fcc

namespace {

// ---- batched execution: volumes grouped by plan configuration, recorded
// into a HIP graph on first use and replayed afterwards ----------------------
struct BatchGroup {
  const fcc_plan_s* p = nullptr;   // representative plan
  std::vector<int> vols;           // indices into the call's arrays
};

struct BatchExec {
  std::vector<uintptr_t> key;      // count, direction, plans, in, out
  std::vector<void*> allocations;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
};

std::mutex& batch_mu() {
  static std::mutex m;
  return m;
}
// Recorded graphs, most recently used last; at most kBatchCacheCap are kept
// (the oldest is freed when a new one is recorded).
constexpr size_t kBatchCacheCap = 4;
std::vector<BatchExec*>& batch_cache() {
  static std::vector<BatchExec*> c;
  return c;
}

void free_batch(BatchExec* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void* a : b->allocations) (void)hipFree(a);
  delete b;
}

bool same_config(const fcc_plan_s* a, const fcc_plan_s* b) {
  return a->n == b->n && a->prec == b->prec && a->flags == b->flags && a->stages64 == b->stages64 &&
         a->dense == b->dense && a->level0_fp32 == b->level0_fp32 && a->rst[0] == b->rst[0] &&
         a->rst[1] == b->rst[1] && a->rst[2] == b->rst[2] && std::memcmp(&a->tune, &b->tune, sizeof a->tune) == 0;
}

std::vector<BatchGroup> group_plans(const fcc_plan_t* plans, int count) {
  std::vector<BatchGroup> groups;
  for (int i = 0; i < count; ++i) {
    bool placed = false;
    for (auto& g : groups)
      if (same_config(g.p, plans[i])) {
        g.vols.push_back(i);
        placed = true;
        break;
      }
    if (!placed) {
      BatchGroup g;
      g.p = plans[i];
      g.vols.push_back(i);
      groups.push_back(g);
    }
  }
  return groups;
}

// A group's volumes run in chunks of at most this many points per launch; the
// chunks share one scratch pair (they run one after the other on the group's
// stream), which bounds the scratch of a group to ~2 x 2^25 stage values.
constexpr long long kBatchChunkPoints = 1LL << 25;
int chunk_volumes(const fcc_plan_s* p, int cnt) {
  const long long N = (long long)p->n * p->n * p->n;
  return int(std::max<long long>(1, std::min<long long>(cnt, kBatchChunkPoints / std::max<long long>(1, N))));
}

// Resources of one group, allocated before capture (no allocation or
// synchronous copy may happen while a stream is being captured).
struct GroupRes {
  void** rows = nullptr;   // device pointer arrays: in, out, scratch 0, scratch 1 (cnt each)
  // dense groups whose volumes are evenly spaced: first volume and spacing in
  // bytes of the in and out lists (0: not evenly spaced)
  char* base[2] = {nullptr, nullptr};
  long long stride[2] = {0, 0};
  void* aws = nullptr;     // dense: the split input of the group, either direction
  float* scale = nullptr;  // dense FP16: per-row scales
  void* ws = nullptr;      // fast path: one scratch pair per volume of a chunk
  size_t wb = 0;
  int chunk = 1;           // volumes per chunk
};

fcc_status prepare_group(std::vector<void*>* allocs, const BatchGroup& g, const void* const* in, void* const* out,
                         GroupRes* r) {
  const fcc_plan_s* p = g.p;
  const int cnt = int(g.vols.size());
  const bool scratch = !p->dense && p->n > 1;
  r->chunk = p->dense ? cnt : chunk_volumes(p, cnt);
  if (scratch) {
    const size_t N = size_t(p->n) * p->n * p->n;
    r->wb = N * (p->stages64 ? sizeof(double2) : sizeof(float2));
    if (dev_malloc(&r->ws, r->wb * 2 * r->chunk) != hipSuccess) return FCC_ERR_OOM;
    allocs->push_back(r->ws);
    poison_scratch(r->ws, r->wb * 2 * r->chunk);
  }
  std::vector<void*> ptr(size_t(4) * cnt, nullptr);
  for (int v = 0; v < cnt; ++v) {
    ptr[v] = const_cast<void*>(in[g.vols[v]]);
    ptr[cnt + v] = out[g.vols[v]];
    if (scratch) {
      const int slot = v % r->chunk;
      ptr[2 * cnt + v] = static_cast<char*>(r->ws) + r->wb * (2 * size_t(slot));
      ptr[3 * cnt + v] = static_cast<char*>(r->ws) + r->wb * (2 * size_t(slot) + 1);
    }
  }
  if (p->dense) {
    const size_t b = std::max(dense_ws_bytes(p->dfwd, cnt), dense_ws_bytes(p->dinv, cnt));
    if (dev_malloc(&r->aws, b) != hipSuccess) return FCC_ERR_OOM;
    allocs->push_back(r->aws);
    poison_scratch(r->aws, b);
  }
  if (p->dense && cnt > 1)
    for (int l = 0; l < 2; ++l) {
      char* b = static_cast<char*>(ptr[size_t(l) * cnt]);
      const long long st = static_cast<char*>(ptr[size_t(l) * cnt + 1]) - b;
      bool even = st > 0 && st % 16 == 0;
      for (int v = 2; v < cnt && even; ++v) even = static_cast<char*>(ptr[size_t(l) * cnt + v]) - b == st * v;
      if (even) {
        r->base[l] = b;
        r->stride[l] = st;
      }
    }
  void* d = nullptr;
  if (dev_malloc(&d, sizeof(void*) * ptr.size() + sizeof(float) * cnt) != hipSuccess) return FCC_ERR_OOM;
  allocs->push_back(d);
  r->rows = static_cast<void**>(d);
  r->scale = reinterpret_cast<float*>(r->rows + ptr.size());
  if (hipMemcpy(r->rows, ptr.data(), sizeof(void*) * ptr.size(), hipMemcpyHostToDevice) != hipSuccess)
    return FCC_ERR_HIP;
  return FCC_OK;
}

// Enqueue direction d (+1 forward in -> out, -1 inverse in -> out; the round
// trip calls forward, then inverse with in and out swapped) for one group,
// chunk by chunk.  ev (optional): start/stop events for every launch slot of
// every chunk (dense groups: around each GEMM).
fcc_status enqueue_group(const BatchGroup& g, const GroupRes& r, int d, bool swap, hipStream_t st,
                         std::vector<hipEvent_t>* ev, size_t* evpos) {
  const fcc_plan_s* p = g.p;
  const int cnt = int(g.vols.size());
  void** in = r.rows + (swap ? cnt : 0);
  void** out = r.rows + (swap ? 0 : cnt);
  void** w0 = r.rows + 2 * cnt;
  void** w1 = r.rows + 3 * cnt;
  fcc_status s = FCC_OK;
  if (p->dense) {
    hipEvent_t* e = ev ? &(*ev)[*evpos] : nullptr;
    if (ev) *evpos += 4;
    // evenly spaced volumes: base + row stride, else the pointer arrays
    const int li = swap ? 1 : 0, lo = swap ? 0 : 1;
    if (r.stride[0] && r.stride[1] && r.stride[li] % 4 == 0 && r.stride[lo] % 4 == 0)
      return dense_run(p, d > 0 ? p->dfwd : p->dinv, cnt, nullptr, nullptr, r.base[li], r.base[lo], r.scale, r.aws,
                       st, r.stride[li] / 4, r.stride[lo] / 4, e);
    return dense_run(p, d > 0 ? p->dfwd : p->dinv, cnt, in, out, nullptr, nullptr, r.scale, r.aws, st, 0, 0, e);
  }
  for (int v0 = 0; v0 < cnt && s == FCC_OK; v0 += r.chunk) {
    const int k = std::min(r.chunk, cnt - v0);
    LaunchTimer tm;
    if (ev) {
      tm.ev = ev;
      tm.next = *evpos;
      t_timer = &tm;
    }
    s = d > 0 ? enqueue_forward(p, k, many_vol(in + v0), many_vol(out + v0), many_vol(w0 + v0), many_vol(w1 + v0), st)
              : enqueue_inverse(p, k, many_vol(in + v0), many_vol(out + v0), many_vol(w0 + v0), many_vol(w1 + v0), st);
    t_timer = nullptr;
    if (ev) *evpos = tm.next;
  }
  return s;
}

fcc_status record_group(const BatchGroup& g, const GroupRes& r, int dir, hipStream_t st) {
  fcc_status s = FCC_OK;
  if (dir >= 0) s = enqueue_group(g, r, 1, false, st, nullptr, nullptr);
  if (s == FCC_OK && dir == 0) s = enqueue_group(g, r, -1, true, st, nullptr, nullptr);
  if (s == FCC_OK && dir < 0) s = enqueue_group(g, r, -1, false, st, nullptr, nullptr);
  return s;
}

// Up to this many branches of the graph run side by side: group k is
// recorded on branch k mod kBatchBranches, between a fork and a join.
constexpr int kBatchBranches = 4;

fcc_status build_batch(BatchExec* bx, const fcc_plan_t* plans, int count, const void* const* in, void* const* out,
                       int dir) {
  std::vector<BatchGroup> groups = group_plans(plans, count);
  // largest groups first: they start at once on their own branch
  std::stable_sort(groups.begin(), groups.end(), [](const BatchGroup& a, const BatchGroup& b) {
    return (long long)a.p->n * a.p->n * a.p->n * (long long)a.vols.size() >
           (long long)b.p->n * b.p->n * b.p->n * (long long)b.vols.size();
  });
  fcc_status s = FCC_OK;
  std::vector<GroupRes> res(groups.size());
  for (size_t gi = 0; gi < groups.size() && s == FCC_OK; ++gi)
    s = prepare_group(&bx->allocations, groups[gi], in, out, &res[gi]);
  if (s != FCC_OK) return s;
  // record on private default-priority streams (the caller's may be the
  // legacy default stream, which cannot be captured); kernels only, no
  // memset nodes
  const int nb = std::min<int>(kBatchBranches, int(groups.size()));
  std::vector<hipStream_t> br(nb, nullptr);
  std::vector<hipEvent_t> evs(1 + nb, nullptr);
  hipError_t e = hipSuccess;
  for (int i = 0; i < nb && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
  for (size_t i = 0; i < evs.size() && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&evs[i], hipEventDisableTiming);
  auto cleanup = [&]() {
    for (auto q : br)
      if (q) (void)hipStreamDestroy(q);
    for (auto v : evs)
      if (v) (void)hipEventDestroy(v);
  };
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "hipStreamCreate(batch branches)", __LINE__);
  }
  if ((e = hipStreamBeginCapture(br[0], hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    cleanup();
    return hip_fail(e, "hipStreamBeginCapture", __LINE__);
  }
  // fork: the other branches wait for an event of the capturing stream
  e = hipEventRecord(evs[0], br[0]);
  for (int i = 1; i < nb && e == hipSuccess; ++i) e = hipStreamWaitEvent(br[i], evs[0], 0);
  for (size_t gi = 0; gi < groups.size() && s == FCC_OK && e == hipSuccess; ++gi)
    s = record_group(groups[gi], res[gi], dir, br[gi % nb]);
  // join
  for (int i = 1; i < nb && s == FCC_OK && e == hipSuccess; ++i) {
    e = hipEventRecord(evs[i], br[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(br[0], evs[i], 0);
  }
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(br[0], &graph);
  cleanup();
  if (s != FCC_OK || e != hipSuccess || ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (s != FCC_OK) return s;
    return hip_fail(e != hipSuccess ? e : ee, "batch graph capture", __LINE__);
  }
  bx->graph = graph;
  e = hipGraphInstantiate(&bx->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate", __LINE__);
  return FCC_OK;
}

}  // namespace

extern "C" {

const char* fcc_status_string(fcc_status s) {
  switch (s) {
    case FCC_OK: return "FCC_OK: success";
    case FCC_ERR_INVALID_ARG: return "FCC_ERR_INVALID_ARG: null/misaligned pointer or bad argument";
    case FCC_ERR_NOT_POW2: return "FCC_ERR_NOT_POW2: n must be a power of two in [1, 1024]";
    case FCC_ERR_SINGULAR_SKEW: return "FCC_ERR_SINGULAR_SKEW: the skew (r,s,t) gives coinciding zeros";
    case FCC_ERR_OOM: return "FCC_ERR_OOM: allocation failed";
    case FCC_ERR_HIP: return "FCC_ERR_HIP: HIP runtime error";
    case FCC_ERR_UNSUPPORTED: return "FCC_ERR_UNSUPPORTED: valid request the library does not serve";
  }
  return "unknown fcc_status";
}

fcc_status fcc_asp_tables(int nl, fcc_level_tables* out) {
  if (!out) return FCC_ERR_INVALID_ARG;
  if (nl < 2 || !is_pow2(nl)) return FCC_ERR_NOT_POW2;
  const LevelTables* T = level_tables(nl);
  if (!T) return FCC_ERR_OOM;
  out->nl = T->nl;
  out->m = T->m;
  out->nmono = T->nmono;
  out->npoly = T->npoly;
  out->mono = T->mono.data();
  out->poly = T->poly.data();
  out->b_rowptr = T->b_rowptr.data();
  out->b_src = T->b_src.data();
  out->b_pid = T->b_pid.data();
  out->c_rowptr = T->c_rowptr.data();
  out->c_src = T->c_src.data();
  out->c_pid = T->c_pid.data();
  const GatherBlocks* gb = gather_blocks(nl);
  if (!gb) return FCC_ERR_OOM;
  out->cube_block = gb->cube.data();
  out->kappa_block = gb->kappa.data();
  return FCC_OK;
}

fcc_status fcc_asp_orbit_blocks(int nl, fcc_orbit_blocks* out) {
  if (!out) return FCC_ERR_INVALID_ARG;
  if (nl < 4 || !is_pow2(nl)) return FCC_ERR_NOT_POW2;
  const OrbitBlocks* B = orbit_blocks(nl);
  if (!B) return FCC_ERR_UNSUPPORTED;
  if (B->templ.size() > sizeof out->templ / sizeof out->templ[0]) return FCC_ERR_UNSUPPORTED;
  static const std::vector<int> group = [] {
    std::vector<int> g;
    for (const auto& w : weyl_group()) g.insert(g.end(), w.begin(), w.end());
    return g;
  }();
  *out = fcc_orbit_blocks{};
  out->nl = B->nl;
  out->m = B->m;
  out->npoly = B->npoly;
  out->nconst = B->nconst;
  out->ntempl = int(B->templ.size());
  out->poly = B->poly.data();
  out->group = group.data();
  for (size_t t = 0; t < B->templ.size(); ++t) {
    const OrbitTemplate& T = B->templ[t];
    fcc_orbit_template& o = out->templ[t];
    o.nc = T.nc;
    o.w = T.w.data();
    o.b_rowptr = T.b_rowptr.data();
    o.b_ent = T.b_ent.data();
    o.c_rowptr = T.c_rowptr.data();
    o.c_ent = T.c_ent.data();
    o.nrep = int(B->reps[t].size());
    o.rep = B->reps[t].data();
  }
  return FCC_OK;
}

}  // extern "C"

namespace {
void lookup_static_scratch(int dev);  // allocation-free entry point (below)
// Built-in schedule: the autotuner's choices on MI355X at n = 64, 128, 256.
fcc_tuning default_tuning(int n) {
  // The searches at n = 64, 128 and 256 (fcc_dct_autotune, reps 5), taken
  // for n <= 64, n = 128 and n >= 256; with orbit-block levels the forward
  // at n = 256 is faster with the last level fused to the DCT_2 pass of the
  // level above (3.04 ms) than with the two-level LDS tail (3.09 ms).
  constexpr unsigned X = FCC_MAP_XCD, FI = FCC_MAP_F_INNER, N8 = FCC_MAP_NODES8, N64 = FCC_MAP_NODES64,
                     SP = FCC_MAP_SPLIT, X16 = FCC_MAP_XCD16, CL = FCC_MAP_CLUSTER;
  struct Choice {
    int tail[2];
    int tile[2][2][3];  // [direction][level][side]
    unsigned map[2][10];
  };
  static const Choice small = {{1, 1},
                               {{{1, 2, 3}, {0, 1, 2}}, {{1, 2, 3}, {0, 0, 0}}},
                               {{SP, SP, SP, SP, SP | N64, SP | N64, SP | N64, SP | N64, SP | N64, SP | N64},
                                {X, X, X, X, X, N64 | X, N64 | X, N64 | X, N64 | X, N64 | X}}};
  static const Choice mid = {{1, 1},
                             {{{2, 2, 2}, {2, 2, 2}}, {{1, 2, 3}, {0, 0, 0}}},
                             {{SP, SP | X16, SP | N8 | X, SP | N64, SP, SP, SP | N64, SP | N64, SP | N64, SP | N64},
                              {CL | X, CL | X, N64 | X, X, 0, 0, 0, 0, 0, 0}}};
  static const Choice large = {{1, 1},
                               {{{2, 2, 2}, {2, 2, 2}}, {{2, 2, 2}, {0, 0, 0}}},
                               {{SP, SP | X16 | FI, SP | X16 | N64, SP | N64, SP | X16 | N64, SP | N64, SP | N64,
                                 SP | N64, SP | N64, SP | N64},
                                {CL | X, CL | X, N64 | X, N64 | X, 0, 0, X16 | N64, 0, 0, 0}}};
  const Choice& c = n <= 64 ? small : (n <= 128 ? mid : large);
  fcc_tuning t{};
  for (int d = 0; d < 2; ++d) {
    t.tail_levels[d] = c.tail[d];
    for (int L = 0; L < 2; ++L)
      for (int a = 0; a < 3; ++a) t.tile[d][L][a] = c.tile[d][L][a];
    // orbit-block launches for every level with node size >= 16 (with blocks
    // sized by the orbits' cube count they beat the row gathers there too)
    for (int L = 0; L < 10; ++L) t.map[d][L] = c.map[d][L] | ((n >> L) >= 16 ? unsigned(FCC_MAP_ORBIT) : 0u);
  }
  return t;
}
bool valid_tuning(const fcc_tuning& t) {
  for (int d = 0; d < 2; ++d) {
    if (t.tail_levels[d] < 1 || t.tail_levels[d] > 4) return false;
    for (int L = 0; L < 2; ++L)
      for (int a = 0; a < 3; ++a)
        if (t.tile[d][L][a] < 0 || t.tile[d][L][a] > 9) return false;
    for (int L = 0; L < 10; ++L) {
      const unsigned m = t.map[d][L];
      if (m & ~unsigned(FCC_MAP_XCD | FCC_MAP_F_INNER | FCC_MAP_NODES8 | FCC_MAP_NODES64 | FCC_MAP_SPLIT |
                        FCC_MAP_BALANCE | FCC_MAP_XCD16 | FCC_MAP_CLUSTER | FCC_MAP_ORBIT))
        return false;
      if ((m & FCC_MAP_NODES8) && (m & FCC_MAP_NODES64)) return false;
    }
  }
  return true;
}
// The plan's copy of the schedule, tile sides clamped to its node sizes.
void resolve_tuning(fcc_plan_s* p, const fcc_tuning& t) {
  p->tune = t;
  for (int d = 0; d < 2; ++d) {
    p->tail_Lt[d] = std::max(0, p->D - t.tail_levels[d]);
    for (int L = 0; L < 2; ++L)
      for (int a = 0; a < 3; ++a) p->tune.tile[d][L][a] = std::min(t.tile[d][L][a], std::max(0, p->D - L - 1));
  }
}
// Cube order of the gather tables of direction d at level L.
CubeOrder tile_order(const fcc_plan_s* p, int d, int L) {
  if (L > 1) return CubeOrder{0, 0, 0};
  return CubeOrder{p->tune.tile[d][L][0], p->tune.tile[d][L][1], p->tune.tile[d][L][2]};
}
int slice_cubes(int L) { return L == 0 ? 64 : (L == 1 ? 8 : 1); }

// Schedules found by fcc_dct_autotune, per (device, n, precision, flags).
std::mutex& tuned_mu() {
  static std::mutex m;
  return m;
}
std::map<std::array<int, 4>, fcc_tuning>& tuned() {
  static std::map<std::array<int, 4>, fcc_tuning> t;
  return t;
}
// Persistence (FCC_AUTOTUNE_CACHE=path): one text line per search,
//   fccdct-schedule 1 <arch> <n> <prec> <flags> <tail x2> <tile x12> <map x20>,
// appended by fcc_dct_autotune and read, for the device's architecture, at the
// first plan of each device in a process (later lines win).  Call with
// tuned_mu() held.
std::string device_arch(int dev) {
  hipDeviceProp_t pr{};
  if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
  std::string a(pr.gcnArchName);
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}
void save_schedule(int dev, int n, int prec, unsigned flags, const fcc_tuning& t) {
  const char* path = std::getenv("FCC_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "fccdct-schedule 1 %s %d %d %u %d %d", device_arch(dev).c_str(), n, prec, flags, t.tail_levels[0],
               t.tail_levels[1]);
  for (int d = 0; d < 2; ++d)
    for (int L = 0; L < 2; ++L)
      for (int a = 0; a < 3; ++a) std::fprintf(f, " %d", t.tile[d][L][a]);
  for (int d = 0; d < 2; ++d)
    for (int L = 0; L < 10; ++L) std::fprintf(f, " %u", t.map[d][L]);
  std::fprintf(f, "\n");
  std::fclose(f);
}
void load_schedules(int dev) {
  static std::vector<int> loaded;
  if (std::find(loaded.begin(), loaded.end(), dev) != loaded.end()) return;
  loaded.push_back(dev);
  const char* path = std::getenv("FCC_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  const std::string arch = device_arch(dev);
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    char tag[32], ar[64];
    int ver = 0, n = 0, prec = 0, used = 0;
    unsigned flags = 0;
    fcc_tuning t{};
    if (std::sscanf(line, "%31s %d %63s %d %d %u %d %d%n", tag, &ver, ar, &n, &prec, &flags, &t.tail_levels[0],
                    &t.tail_levels[1], &used) != 8 ||
        std::string(tag) != "fccdct-schedule" || ver != 1 || arch != ar)
      continue;
    const char* c = line + used;
    bool ok = true;
    for (int d = 0; d < 2 && ok; ++d)
      for (int L = 0; L < 2 && ok; ++L)
        for (int a = 0; a < 3 && ok; ++a) {
          int k = 0;
          ok = std::sscanf(c, "%d%n", &t.tile[d][L][a], &k) == 1;
          c += k;
        }
    for (int d = 0; d < 2 && ok; ++d)
      for (int L = 0; L < 10 && ok; ++L) {
        int k = 0;
        ok = std::sscanf(c, "%u%n", &t.map[d][L], &k) == 1;
        c += k;
      }
    if (ok && valid_tuning(t)) tuned()[{dev, n, prec, int(flags)}] = t;
  }
  std::fclose(f);
}
}  // namespace

extern "C" {

}  // extern "C"
namespace {
// Tables of an FCC_FOLD_FFT plan: the phases exp(2 pi i m / (8n)), the unfold
// rows (scaled by 1/n^3) and the per-point row index, all in the data
// precision; one n^3 complex scratch buffer for the inverse.
template <typename C>
fcc_status fold_upload(fcc_plan_s* p, const fcc::FoldTables& t) {
  const int n = p->n;
  std::vector<C> w(size_t(8) * n), k(t.K.size());
  for (int m = 0; m < 8 * n; ++m) {
    // exact at the multiples of pi/4, else the FP64 sine and cosine of the reduced angle
    const double a = 2.0 * M_PI * double(m) / (8.0 * n);
    w[m] = {decltype(C{}.x)(std::cos(a)), decltype(C{}.x)(std::sin(a))};
    if ((m * 8) % (8 * n) == 0) {
      static const double h = std::sqrt(0.5);
      const double cs[8][2] = {{1, 0}, {h, h}, {0, 1}, {-h, h}, {-1, 0}, {-h, -h}, {0, -1}, {h, -h}};
      const int q = (m * 8) / (8 * n);
      w[m] = {decltype(C{}.x)(cs[q][0]), decltype(C{}.x)(cs[q][1])};
    }
  }
  const double inv = 1.0 / (double(n) * n * n);
  for (size_t i = 0; i < t.K.size(); ++i) k[i] = {decltype(C{}.x)(t.K[i].real() * inv), decltype(C{}.x)(t.K[i].imag() * inv)};
  hipError_t e = dev_malloc(&p->fw8n, w.size() * sizeof(C));
  if (e == hipSuccess) e = hipMemcpy(p->fw8n, w.data(), w.size() * sizeof(C), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = dev_malloc(&p->fkt, k.size() * sizeof(C));
  if (e == hipSuccess) e = hipMemcpy(p->fkt, k.data(), k.size() * sizeof(C), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = dev_malloc(reinterpret_cast<void**>(&p->fpid), t.prid.size());
  if (e == hipSuccess) e = hipMemcpy(p->fpid, t.prid.data(), t.prid.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = dev_malloc(&p->freps, t.reps.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpy(p->freps, t.reps.data(), t.reps.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  p->fnrep = int(t.reps.size());
  if (e == hipSuccess) {
    p->ws_bytes = size_t(n) * n * n * sizeof(C);
    e = dev_malloc(&p->ws[0], p->ws_bytes);
    if (e == hipSuccess) poison_scratch(p->ws[0], p->ws_bytes);
  }
  return e == hipSuccess ? FCC_OK : hip_fail(e, "fold tables", __LINE__);
}
// FCC_FOLD_BASE: 8 rst integral; the orbit representatives of W on the
// M-torus (smallest flat index of each orbit) for M = 4, 8, 16; without an
// explicit schedule the forward's base has node size min(16, n).
fcc_status base_prepare(fcc_plan_s* p, const double r[3], bool default_schedule) {
  for (int i = 0; i < 3; ++i) {
    const double v = 8.0 * r[i];
    if (std::fabs(v - std::nearbyint(v)) > 1e-12) return FCC_ERR_UNSUPPORTED;
    p->r8[i] = int(std::nearbyint(v));
  }
  if (p->n > 1024) return FCC_ERR_UNSUPPORTED;  // the base's phase table holds 8 n / M entries
  p->fold_base = true;
  if (default_schedule) p->tune.tail_levels[0] = std::min(4, p->D - 1);
  if (p->tune.tail_levels[0] < 2 || p->tune.tail_levels[0] > p->D - 1) return FCC_ERR_INVALID_ARG;
  p->tail_Lt[0] = p->D - p->tune.tail_levels[0];
  std::vector<int> reps;  // (representative, mask of repeated images) pairs
  for (int m = 0; m < 3; ++m) {
    const int lg = m + 2, M = 1 << lg;
    p->brep_off[m] = int(reps.size()) / 2;
    std::vector<std::pair<int, int>> orb;
    for (int q = 0; q < M * M * M; ++q) {
      const int k[3] = {q >> (2 * lg), (q >> lg) & (M - 1), q & (M - 1)};
      int img[24], mask = 0;
      bool smallest = true;
      for (int u = 0; u < 24; ++u) {
        int v[3];
        for (int i = 0; i < 3; ++i)
          v[i] = (kFoldW[u].g[3 * i] * k[0] + kFoldW[u].g[3 * i + 1] * k[1] + kFoldW[u].g[3 * i + 2] * k[2]) & (M - 1);
        img[u] = (v[0] << (2 * lg)) | (v[1] << lg) | v[2];
        smallest = smallest && img[u] >= q;
        for (int w = 0; w < u; ++w)
          if (img[w] == img[u]) {
            mask |= 1 << u;
            break;
          }
      }
      if (smallest) orb.push_back({mask, q});
    }
    std::sort(orb.begin(), orb.end());
    for (const auto& o : orb) reps.push_back(o.second), reps.push_back(o.first);
    p->brep_cnt[m] = int(orb.size());
  }
  hipError_t e = dev_malloc(&p->breps, reps.size() * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(p->breps, reps.data(), reps.size() * sizeof(int), hipMemcpyHostToDevice);
  return e == hipSuccess ? FCC_OK : hip_fail(e, "base orbit table", __LINE__);
}
fcc_status fold_prepare(fcc_plan_s* p, const double r[3], hipStream_t) {
  p->fold = true;
  p->stages64 = p->prec == FCC_PREC_FP64;
  for (int i = 0; i < 3; ++i) {
    const double v = 8.0 * r[i];
    if (std::fabs(v - std::nearbyint(v)) > 1e-12) return FCC_ERR_UNSUPPORTED;
    p->r8[i] = int(std::nearbyint(v));
  }
  fcc::FoldTables t;
  const fcc_status s = fcc::fold_tables(p->n, p->r8, &t, true);
  if (s != FCC_OK) return s;
  if (t.npat > kFoldMaxPat) return FCC_ERR_UNSUPPORTED;
  p->fnpat = t.npat;
  return p->prec == FCC_PREC_FP64 ? fold_upload<double2>(p, t) : fold_upload<float2>(p, t);
}
}  // namespace
extern "C" {

fcc_status fcc_dct_plan(fcc_plan_t* plan, int n, const double rst[3], fcc_precision prec, unsigned flags,
                        void* hip_stream) {
  return fcc_dct_plan_tuned(plan, n, rst, prec, flags, nullptr, hip_stream);
}

fcc_status fcc_dct_get_tuning(fcc_plan_t p, fcc_tuning* out) {
  if (!p || !out) return FCC_ERR_INVALID_ARG;
  *out = p->tune;
  return FCC_OK;
}

fcc_status fcc_dct_plan_tuned(fcc_plan_t* plan, int n, const double rst[3], fcc_precision prec, unsigned flags,
                              const fcc_tuning* tuning, void* hip_stream) {
  if (!plan) return FCC_ERR_INVALID_ARG;
  *plan = nullptr;
  if (!is_pow2(n)) return FCC_ERR_NOT_POW2;
  if (prec < FCC_PREC_FP64 || prec > FCC_PREC_SPLIT_FP16) return FCC_ERR_INVALID_ARG;
  if ((flags & FCC_STAGES_FP32) && (flags & FCC_STAGES_FP64)) return FCC_ERR_INVALID_ARG;
  if (flags & ~(unsigned)(FCC_REAL_INPUT | FCC_STAGES_FP32 | FCC_STAGES_FP64 | FCC_LEVEL0_FP32 | FCC_TRANSPOSED |
                          FCC_HERMITIAN_PACKED | FCC_FOLD_FFT | FCC_FOLD_BASE))
    return FCC_ERR_INVALID_ARG;
  if ((flags & FCC_FOLD_FFT) && ((flags & ~(unsigned)(FCC_FOLD_FFT | FCC_REAL_INPUT)) ||
                                 (prec != FCC_PREC_FP32 && prec != FCC_PREC_FP64) || n > 512))
    return FCC_ERR_UNSUPPORTED;
  const bool split_prec = prec == FCC_PREC_SPLIT_BF16 || prec == FCC_PREC_SPLIT_FP16;
  if ((flags & FCC_TRANSPOSED) &&
      (split_prec || (flags & (FCC_LEVEL0_FP32 | FCC_HERMITIAN_PACKED)) || n > 256))
    return FCC_ERR_UNSUPPORTED;
  if ((flags & FCC_FOLD_BASE) && (split_prec || (flags & (FCC_TRANSPOSED | FCC_FOLD_FFT)) || n < 8))
    return FCC_ERR_UNSUPPORTED;
  if ((flags & FCC_FOLD_BASE) && tuning && tuning->tail_levels[0] < 2) return FCC_ERR_INVALID_ARG;
  if ((flags & FCC_HERMITIAN_PACKED) && !(flags & FCC_REAL_INPUT)) return FCC_ERR_INVALID_ARG;
  if ((flags & FCC_HERMITIAN_PACKED) && split_prec) return FCC_ERR_UNSUPPORTED;
  if (tuning && !valid_tuning(*tuning)) return FCC_ERR_INVALID_ARG;
  // per-row tables pack node-local coordinates in 8 bits: node sizes above 256
  // need orbit-block launches in both directions
  for (int L = 0; tuning && L < 10 && (n >> L) > 256; ++L)
    if (!(tuning->map[0][L] & tuning->map[1][L] & FCC_MAP_ORBIT)) return FCC_ERR_UNSUPPORTED;
  if ((prec == FCC_PREC_SPLIT_BF16 || prec == FCC_PREC_SPLIT_FP16) && n > 8) return FCC_ERR_UNSUPPORTED;
  double r[3] = {0.125, 0.0, 0.375};
  if (rst)
    for (int d = 0; d < 3; ++d) {
      if (!std::isfinite(rst[d])) return FCC_ERR_INVALID_ARG;
      r[d] = rst[d];
    }
  if (singular_skew(n, r)) return FCC_ERR_SINGULAR_SKEW;
  fcc_plan_s* p = new (std::nothrow) fcc_plan_s;
  if (!p) return FCC_ERR_OOM;
  p->n = n;
  p->prec = prec;
  p->flags = flags;
  for (int d = 0; d < 3; ++d) p->rst[d] = r[d];
  while ((1 << p->D) < n) ++p->D;
  // Stage precision.  FP32 stages lose accuracy with depth (the skew children
  // approach W-fixed points and their coefficient vectors become ill
  // conditioned); measured FP32-stage errors pass 1e-5 only up to n = 8.
  p->dense = prec == FCC_PREC_SPLIT_BF16 || prec == FCC_PREC_SPLIT_FP16;
  if (prec == FCC_PREC_FP64 || p->dense)
    p->stages64 = true;
  else if (flags & FCC_STAGES_FP32)
    p->stages64 = false;
  else if (flags & FCC_STAGES_FP64)
    p->stages64 = true;
  else
    p->stages64 = n > 4;
  // Opt-in: level 0 in FP32.  Rounding at the top level is not amplified by
  // the well-conditioned children, but it raises the round-trip error from
  // ~5e-8 to ~4e-6 at n = 32..128 (measured), so it is not the default.
  p->level0_fp32 = (flags & FCC_LEVEL0_FP32) && prec == FCC_PREC_FP32 && p->stages64 && p->D >= 2;
  {
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
      delete p;
      return hip_fail(e, "hipGetDevice", __LINE__);
    }
  }
  lookup_static_scratch(p->device);
  bool searched = false;  // the schedule is fcc_dct_autotune's
  if (tuning) {
    resolve_tuning(p, *tuning);
  } else {
    fcc_tuning t = default_tuning(n);
    {
      std::lock_guard<std::mutex> lock(tuned_mu());
      load_schedules(p->device);
      auto it = tuned().find({p->device, n, int(prec), int(flags)});
      if (it != tuned().end()) t = it->second, searched = true;
    }
    resolve_tuning(p, t);
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  fcc_status s = FCC_OK;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  if (flags & FCC_FOLD_BASE) {
    s = base_prepare(p, r, !tuning && !searched);
    if (s != FCC_OK) {
      fcc_dct_destroy(p);
      return s;
    }
  }
  if (flags & FCC_FOLD_FFT) {
    s = fold_prepare(p, r, st);
    if (s != FCC_OK) {
      fcc_dct_destroy(p);
      return s;
    }
    *plan = p;
    return FCC_OK;
  }
  // Levels that run as orbit-block launches in both directions read no
  // per-row table; the others need one, and its packed entries hold node-local
  // coordinates in 8 bits (node size <= 256).
  // (The transposed transform runs orbit-block launches at every level with
  // node size >= 4 and a per-cube pass at the last: no table anywhere.)
  p->transposed = (flags & FCC_TRANSPOSED) != 0;
  bool tables[16] = {};
  for (int L = 0; L < p->D; ++L) {
    const bool orb = (n >> L) >= 8 && L < 10 && (p->tune.map[0][L] & FCC_MAP_ORBIT) &&
                     (p->tune.map[1][L] & FCC_MAP_ORBIT);
    tables[L] = !orb && !p->transposed;
    if (tables[L] && (n >> L) > 256) {
      delete p;
      return FCC_ERR_UNSUPPORTED;
    }
  }
  {
    std::lock_guard<std::mutex> lock(cache().mu);
    p->olv.assign(p->D, DevOrbitLevel{});
    for (int L = 0; s == FCC_OK && L < p->D && L < 10; ++L)
      if (p->transposed ? (n >> L) >= 4
                        : ((n >> L) >= 8 && ((p->tune.map[0][L] | p->tune.map[1][L]) & FCC_MAP_ORBIT)))
        s = device_orbit_level(p->device, n >> L, &p->olv[L]);
    for (int L = 0; s == FCC_OK && L < p->D; ++L) {
      DevLevel lv{};
      if (tables[L])
        s = device_level(p->device, n >> L, slice_cubes(L), tile_order(p, 0, L), tile_order(p, 1, L), &lv);
      p->lv.push_back(lv);
    }
    // balanced map: lanes per row from the mean row length of each f
    for (int L = 0; s == FCC_OK && L < p->D; ++L) {
      if (!tables[L]) continue;
      const LevelTables* T = level_tables(n >> L);
      if (!T) {
        s = FCC_ERR_OOM;
        break;
      }
      for (int d = 0; d < 2; ++d) {
        const std::vector<int>& rp = d == 0 ? T->b_rowptr : T->c_rowptr;
        const long long cubes = (long long)(rp.size() - 1) / 8;
        for (int f = 0; f < 8; ++f) {
          long long tot = 0;
          for (long long c = 0; c < cubes; ++c) tot += rp[c * 8 + f + 1] - rp[c * 8 + f];
          const double mean = cubes ? double(tot) / double(cubes) : 0.0;
          p->kf[d][L][f] = mean > 20.0 ? 2 : (mean > 10.0 ? 1 : 0);
        }
      }
    }
    // plain-order tables with one cube per slice for every level a fused
    // tail may cover (node sizes <= 16); levels >= 2 have them already
    p->tlv.resize(p->D);
    for (int L = std::max(0, p->D - 4); s == FCC_OK && !p->transposed && L < p->D; ++L) {
      if (L >= 2 && tables[L])
        p->tlv[L] = p->lv[L];
      else
        s = device_level(p->device, n >> L, 1, CubeOrder{0, 0, 0}, CubeOrder{0, 0, 0}, &p->tlv[L]);
    }
  }
  if (s == FCC_OK && p->D > 0) {
    size_t cnt = 3 * ((size_t(1) << p->D) - 1);
    hipError_t e = dev_malloc(&p->hph, cnt * sizeof(double2));
    if (e != hipSuccess) s = hip_fail(e, "device allocation (phase table)", __LINE__);
    if (s == FCC_OK) {
      hipLaunchKernelGGL(k_phase_table, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, st, p->hph, p->D, r[0], r[1],
                         r[2]);
      s = launch_status("phase table launch");
    }
  }
  if (s == FCC_OK && p->D > 0) {
    // FP64 node constants for the levels with at most kNodeTableMax nodes
    long long total = 0;
    // (only where a node has at least 64 cubes, n >> L >= 8: with fewer cubes
    // per node the 400 bytes of a table entry cost more traffic than forming
    // A from the phases)
    for (int L = 0; L < p->D; ++L) {
      p->node_off[L] = -1;
      if ((1LL << (3 * L)) <= kNodeTableMax && (p->n >> L) >= 8) {
        p->node_off[L] = total;
        total += 1LL << (3 * L);
      }
    }
    hipError_t e = total > 0 ? dev_malloc(&p->nodes, sizeof(NodeConst) * total) : hipSuccess;
    if (e != hipSuccess) s = hip_fail(e, "device allocation (node table)", __LINE__);
    for (int L = 0; s == FCC_OK && L < p->D; ++L)
      if (p->node_off[L] >= 0) {
        const long long cnt = 1LL << (3 * L);
        hipLaunchKernelGGL(k_node_table, dim3(unsigned((cnt + 63) / 64)), dim3(64), 0, st,
                           static_cast<NodeConst*>(p->nodes) + p->node_off[L], L, phases(p, L));
        s = launch_status("node table launch");
      }
  }
  if (s == FCC_OK && p->D > 0) {
    // dense DCT_2 and inverse of every node of the orbit-block levels
    long long total = 0;
    for (int L = 0; L < p->D; ++L) {
      p->onode_off[L] = -1;
      if (L < int(p->olv.size()) && p->olv[L].kinds) {
        p->onode_off[L] = total;
        total += 1LL << (3 * L);
      }
    }
    hipError_t e = total > 0 ? dev_malloc(&p->onodes, sizeof(OrbitNode) * total) : hipSuccess;
    if (e != hipSuccess) s = hip_fail(e, "device allocation (orbit node table)", __LINE__);
    for (int L = 0; s == FCC_OK && L < p->D; ++L)
      if (p->onode_off[L] >= 0) {
        const long long cnt = 1LL << (3 * L);
        hipLaunchKernelGGL(k_orbit_nodes, dim3(unsigned((cnt + 63) / 64)), dim3(64), 0, st,
                           static_cast<OrbitNode*>(p->onodes) + p->onode_off[L], L, phases(p, L));
        s = launch_status("orbit node table launch");
      }
  }
  if (s == FCC_OK && p->D > 0) {
    size_t N = size_t(n) * n * n;
    p->ws_bytes = N * (p->stages64 ? sizeof(double2) : sizeof(float2));
    for (int b = 0; b < 2 && s == FCC_OK; ++b) {
      hipError_t e = dev_malloc(&p->ws[b], p->ws_bytes);
      if (e != hipSuccess) s = hip_fail(e, "device allocation (scratch)", __LINE__);
      else poison_scratch(p->ws[b], p->ws_bytes);
    }
  }
  if (s == FCC_OK && (flags & FCC_HERMITIAN_PACKED)) {
    // the pairing j' = (c - g^T j) mod n: g in W with c = -g^T rst - rst integral
    const auto& G = weyl_group();
    int gsel = -1;
    long long cv[3] = {0, 0, 0};
    for (int w = 0; w < 24 && gsel < 0; ++w) {
      bool ok = true;
      long long c[3];
      for (int i = 0; i < 3 && ok; ++i) {
        double v = -r[i];
        for (int k = 0; k < 3; ++k) v -= double(G[w][3 * k + i]) * r[k];  // (g^T rst)_i = sum_k g[k][i] rst_k
        ok = std::fabs(v - std::nearbyint(v)) < 1e-12;
        c[i] = (long long)std::nearbyint(v);
      }
      if (ok) {
        gsel = w;
        for (int i = 0; i < 3; ++i) cv[i] = c[i];
      }
    }
    if (gsel < 0) {
      s = FCC_ERR_UNSUPPORTED;
    } else {
      const long long N = (long long)n * n * n;
      std::vector<int> slot;
      try {
        slot.assign(size_t(N), 0);
      } catch (const std::bad_alloc&) {
        s = FCC_ERR_OOM;
      }
      if (s == FCC_OK) {
        const auto& g = G[gsel];
        auto partner = [&](long long j) {
          const long long v[3] = {j / ((long long)n * n), (j / n) % n, j % n};
          long long q[3];
          for (int i = 0; i < 3; ++i) {
            long long t = cv[i];
            for (int k = 0; k < 3; ++k) t -= (long long)g[3 * k + i] * v[k];
            q[i] = ((t % n) + n) % n;
          }
          return (q[0] * n + q[1]) * n + q[2];
        };
        long long k = 0;
        for (long long j = 0; j < N; ++j)
          if (j <= partner(j)) slot[size_t(j)] = int(k++);
        for (long long j = 0; j < N; ++j) {
          const long long q = partner(j);
          if (j > q) slot[size_t(j)] = -slot[size_t(q)] - 1;
        }
        p->hpacked = k;
        hipError_t e = dev_malloc(reinterpret_cast<void**>(&p->hslot), sizeof(int) * size_t(N));
        if (e == hipSuccess) e = hipMemcpy(p->hslot, slot.data(), sizeof(int) * size_t(N), hipMemcpyHostToDevice);
        if (e == hipSuccess)
          e = dev_malloc(&p->hfull, size_t(N) * (prec == FCC_PREC_FP64 ? sizeof(double2) : sizeof(float2)));
        if (e == hipSuccess)
          poison_scratch(p->hfull, size_t(N) * (prec == FCC_PREC_FP64 ? sizeof(double2) : sizeof(float2)));
        if (e != hipSuccess) s = hip_fail(e, "hermitian packing tables", __LINE__);
      }
    }
  }
  if (s == FCC_OK) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = hip_fail(e, "hipStreamSynchronize", __LINE__);
  }
  if (s == FCC_OK && p->dense) {
    s = dense_prepare(p, st);
    if (s == FCC_OK && dev_malloc(&p->rowscale, sizeof(float)) != hipSuccess) s = FCC_ERR_OOM;
    if (s == FCC_OK &&
        dev_malloc(&p->dws, std::max(dense_ws_bytes(p->dfwd, 1), dense_ws_bytes(p->dinv, 1))) != hipSuccess)
      s = FCC_ERR_OOM;
    if (s == FCC_OK) poison_scratch(p->dws, std::max(dense_ws_bytes(p->dfwd, 1), dense_ws_bytes(p->dinv, 1)));
    p->rows_cap = 1;
  }
  if (s != FCC_OK) {
    fcc_dct_destroy(p);
    return s;
  }
  *plan = p;
  return FCC_OK;
}

fcc_status fcc_dct_destroy(fcc_plan_t p) {
  if (!p) return FCC_OK;
  {
    std::lock_guard<std::mutex> lock(batch_mu());
    auto& c = batch_cache();
    for (size_t i = 0; i < c.size();) {
      bool uses = false;
      for (size_t k = 2; k < c[i]->key.size(); k += 3) uses |= c[i]->key[k] == reinterpret_cast<uintptr_t>(p);
      if (uses) {
        free_batch(c[i]);
        c.erase(c.begin() + i);
      } else {
        ++i;
      }
    }
  }
  dense_free(p);
  if (p->resid) (void)hipFree(p->resid);
  if (p->nodes) (void)hipFree(p->nodes);
  if (p->onodes) (void)hipFree(p->onodes);
  if (p->hslot) (void)hipFree(p->hslot);
  if (p->hfull) (void)hipFree(p->hfull);
  if (p->hph) (void)hipFree(p->hph);
  if (p->fw8n) (void)hipFree(p->fw8n);
  if (p->fkt) (void)hipFree(p->fkt);
  if (p->fpid) (void)hipFree(p->fpid);
  if (p->freps) (void)hipFree(p->freps);
  if (p->breps) (void)hipFree(p->breps);
  for (void* w : p->ws)
    if (w) (void)hipFree(w);
  delete p;
  return FCC_OK;
}

fcc_status fcc_dct_forward(fcc_plan_t p, const void* x, void* X, void* hip_stream) {
  if (!p || !x || !X || !aligned16(x) || !aligned16(X)) return FCC_ERR_INVALID_ARG;
  if (x == X) return FCC_ERR_UNSUPPORTED;
  (void)hipGetLastError();
  if (p->dense)
    return dense_run(p, p->dfwd, 1, nullptr, nullptr, x, X, p->rowscale, p->dws, static_cast<hipStream_t>(hip_stream));
  return enqueue_forward(p, 1, one_vol(x), one_vol(X), one_vol(p->ws[0]), one_vol(p->ws[1]),
                         static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

// ---- allocation-free forward: scratch in a static device array -------------
namespace {
// The two ping-pong buffers of fcc_dct_forward_static live in this array, one
// copy per device.  Host code never names it directly (the name is a host-side
// stand-in, not a device address): its address on each device is looked up
// once, with that device current, and kept in scratch_addr.
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex scratch_mu;
void* scratch_addr[kMaxDevices] = {};
hipError_t scratch_err[kMaxDevices] = {};
bool scratch_tried[kMaxDevices] = {};

// Called at plan set-up with the plan's device current.
void lookup_static_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_tried[dev]) return;
  scratch_tried[dev] = true;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  scratch_err[dev] = e;
  if (e == hipSuccess) scratch_addr[dev] = ptr;
}
void* static_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  return scratch_addr[dev];
}
}  // namespace

extern "C" {

fcc_status fcc_dct_forward_static(fcc_plan_t p, const void* x, void* X, void* hip_stream) {
  if (!p || !x || !X || !aligned16(x) || !aligned16(X)) return FCC_ERR_INVALID_ARG;
  if (x == X) return FCC_ERR_UNSUPPORTED;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device) return FCC_ERR_INVALID_ARG;
  (void)hipGetLastError();
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  char* base = static_cast<char*>(static_scratch(p->device));
  if (!base) return FCC_ERR_HIP;
  // dense path: its per-row input scale (one float) and, 256 bytes on, the split input
  if (p->dense) {
    if (256 + dense_ws_bytes(p->dfwd, 1) > kStaticScratchBytes) return FCC_ERR_UNSUPPORTED;
    return dense_run(p, p->dfwd, 1, nullptr, nullptr, x, X, reinterpret_cast<float*>(base), base + 256, st);
  }
  const size_t half = size_t(p->n) * p->n * p->n * (p->stages64 ? sizeof(double2) : sizeof(float2));
  // the two buffers, each 256-byte aligned
  const size_t stride = (half + 255) & ~size_t(255);
  if (2 * stride > kStaticScratchBytes) return FCC_ERR_UNSUPPORTED;
  return enqueue_forward(p, 1, one_vol(x), one_vol(X), one_vol(base), one_vol(base + stride), st);
}

fcc_status fcc_dct_inverse(fcc_plan_t p, const void* X, void* x, void* hip_stream) {
  if (!p || !x || !X || !aligned16(x) || !aligned16(X)) return FCC_ERR_INVALID_ARG;
  if (x == X) return FCC_ERR_UNSUPPORTED;
  (void)hipGetLastError();
  if (p->dense)
    return dense_run(p, p->dinv, 1, nullptr, nullptr, X, x, p->rowscale, p->dws, static_cast<hipStream_t>(hip_stream));
  return enqueue_inverse(p, 1, one_vol(X), one_vol(x), one_vol(p->ws[0]), one_vol(p->ws[1]),
                         static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

namespace {
// Average duration (ms) of each launch slot of `reps` transforms in direction
// +1 (forward) or -1 (inverse), timed with events around every launch.
fcc_status time_slots(const fcc_plan_s* p, const void* in, void* out, int direction, int reps, hipStream_t st,
                      std::vector<float>* ms) {
  const int slots = slot_count(p, direction > 0 ? 0 : 1);
  ms->assign(slots, 0.f);
  // the dense path records its events itself (around the split and the
  // GEMM); the fast path records a start and stop per kernel
  const bool whole = p->dense;
  std::vector<hipEvent_t> ev(size_t(2) * slots * reps, nullptr);
  fcc_status s = FCC_OK;
  for (auto& e : ev) {
    hipError_t he = hipEventCreate(&e);
    if (he != hipSuccess) {
      s = hip_fail(he, "hipEventCreate", __LINE__);
      break;
    }
  }
  for (int r = 0; r < reps && s == FCC_OK; ++r) {
    std::vector<hipEvent_t> sub(ev.begin() + size_t(r) * 2 * slots, ev.begin() + size_t(r + 1) * 2 * slots);
    if (whole) {
      s = dense_run(p, direction > 0 ? p->dfwd : p->dinv, 1, nullptr, nullptr, in, out, p->rowscale, p->dws, st, 0,
                    0, sub.data());
      continue;
    }
    LaunchTimer tm;
    tm.ev = &sub;
    t_timer = &tm;
    s = direction > 0 ? enqueue_forward(p, 1, one_vol(in), one_vol(out), one_vol(p->ws[0]), one_vol(p->ws[1]), st)
                      : enqueue_inverse(p, 1, one_vol(in), one_vol(out), one_vol(p->ws[0]), one_vol(p->ws[1]), st);
    t_timer = nullptr;
    if (s == FCC_OK && tm.next != sub.size()) s = FCC_ERR_HIP;  // launch count differs from the slot count
  }
  if (s == FCC_OK) {
    hipError_t he = hipStreamSynchronize(st);
    if (he != hipSuccess) s = hip_fail(he, "hipStreamSynchronize", __LINE__);
  }
  if (s == FCC_OK)
    for (int k = 0; k < slots; ++k) {
      double acc = 0.0;
      for (int r = 0; r < reps; ++r) {
        float t = 0.f;
        (void)hipEventElapsedTime(&t, ev[size_t(r) * 2 * slots + 2 * k], ev[size_t(r) * 2 * slots + 2 * k + 1]);
        acc += t;
      }
      (*ms)[k] = float(acc / reps);
    }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return s;
}
}  // namespace

extern "C" {

fcc_status fcc_dct_time_launches(fcc_plan_t p, const void* in, void* out, int direction, int reps, float* ms,
                                 int cap, int* count, void* hip_stream) {
  if (!p || !in || !out || !count || reps < 1 || (direction != 1 && direction != -1)) return FCC_ERR_INVALID_ARG;
  if (!aligned16(in) || !aligned16(out) || in == out) return FCC_ERR_INVALID_ARG;
  const int slots = slot_count(p, direction > 0 ? 0 : 1);
  *count = slots;
  if (!ms || cap < slots) return ms ? FCC_ERR_INVALID_ARG : FCC_OK;
  (void)hipGetLastError();
  std::vector<float> v;
  fcc_status s = time_slots(p, in, out, direction, reps, static_cast<hipStream_t>(hip_stream), &v);
  if (s == FCC_OK) std::copy(v.begin(), v.end(), ms);
  return s;
}

fcc_status fcc_dct_autotune(int n, const double rst[3], fcc_precision prec, unsigned flags, int reps,
                            fcc_tuning* best, void* hip_stream) {
  if (reps < 1) return FCC_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  fcc_plan_t p = nullptr;
  fcc_status s = fcc_dct_plan_tuned(&p, n, rst, prec, flags, nullptr, hip_stream);
  if (s != FCC_OK) return s;
  if (!p->dense && !p->fold && p->D >= 2) {
    // synthetic operands: the forward input and a complex array for the
    // forward output / inverse input
    const long long N = (long long)n * n * n;
    const size_t el = (p->prec == FCC_PREC_FP64) ? sizeof(double) : sizeof(float);
    void* a = nullptr;
    void* b = nullptr;
    hipError_t e = dev_malloc(&a, 2 * el * N);
    if (e == hipSuccess) e = dev_malloc(&b, 2 * el * N);
    if (e != hipSuccess) s = hip_fail(e, "device allocation (autotune operands)", __LINE__);
    if (s == FCC_OK) {
      const unsigned blocks = unsigned(std::min<long long>((2 * N + 255) / 256, 65535));
      if (el == sizeof(double)) {
        hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(256), 0, st, static_cast<double*>(a), 2 * N, 1u);
        hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(256), 0, st, static_cast<double*>(b), 2 * N, 2u);
      } else {
        hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(256), 0, st, static_cast<float*>(a), 2 * N, 1u);
        hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(256), 0, st, static_cast<float*>(b), 2 * N, 2u);
      }
      s = launch_status("autotune fill");
    }
    std::vector<float> ms;
    auto total = [&](int d, double* out) {
      fcc_status r = d == 0 ? time_slots(p, a, b, 1, reps, st, &ms) : time_slots(p, b, a, -1, reps, st, &ms);
      double t = 0.0;
      for (float v : ms) t += v;
      *out = t;
      return r;
    };
    for (int d = 0; d < 2 && s == FCC_OK; ++d) {
      // 1. fused tail depth, by whole-direction time
      int best_k = p->tune.tail_levels[d];
      double best_t = 1e30;
      for (int k = (d == 0 && p->fold_base) ? 2 : 1; k <= std::min(4, p->D - (d == 0 && p->fold_base)) && s == FCC_OK;
           ++k) {
        p->tune.tail_levels[d] = k;
        p->tail_Lt[d] = std::max(0, p->D - k);
        double t = 0.0;
        s = total(d, &t);
        if (verbose()) std::fprintf(stderr, "fcc_autotune n=%d dir=%d tail_levels=%d: %.4f ms\n", n, d, k, t);
        if (s == FCC_OK && t < best_t) best_t = t, best_k = k;
      }
      p->tune.tail_levels[d] = best_k;
      p->tail_Lt[d] = std::max(0, p->D - best_k);
      // 2. tile shape and thread map of the level-0 and level-1 gather
      // passes, by the time of that level's launches
      auto level_ms = [&](int L) {
        const int k = level_slot(p, d, L);
        if (d == 1) return double(ms[k + ((L == p->D - 2 && inv_last2(p)) ? 0 : 1)]);  // the C gather pass
        return double(ms[k]) + (fwd_split(p, L) ? double(ms[k + 1]) : 0.0);
      };
      static const int tiles0[][3] = {{0, 0, 0}, {2, 2, 2}, {1, 2, 3}, {0, 3, 3}, {3, 3, 3}, {2, 2, 4}};
      static const int tiles1[][3] = {{0, 0, 0}, {1, 1, 1}, {0, 1, 2}, {2, 2, 2}};
      static const unsigned top_fwd[] = {0u,
                                         FCC_MAP_XCD,
                                         FCC_MAP_SPLIT,
                                         FCC_MAP_SPLIT | FCC_MAP_XCD,
                                         FCC_MAP_SPLIT | FCC_MAP_F_INNER,
                                         FCC_MAP_SPLIT | FCC_MAP_F_INNER | FCC_MAP_XCD,
                                         FCC_MAP_SPLIT | FCC_MAP_BALANCE,
                                         FCC_MAP_SPLIT | FCC_MAP_BALANCE | FCC_MAP_XCD,
                                         FCC_MAP_SPLIT | FCC_MAP_XCD16,
                                         FCC_MAP_SPLIT | FCC_MAP_F_INNER | FCC_MAP_XCD16,
                                         FCC_MAP_SPLIT | FCC_MAP_CLUSTER,
                                         FCC_MAP_SPLIT | FCC_MAP_CLUSTER | FCC_MAP_XCD,
                                         FCC_MAP_SPLIT | FCC_MAP_CLUSTER | FCC_MAP_XCD16};
      static const unsigned top_inv[] = {0u,
                                         FCC_MAP_XCD,
                                         FCC_MAP_F_INNER,
                                         FCC_MAP_F_INNER | FCC_MAP_XCD,
                                         FCC_MAP_BALANCE,
                                         FCC_MAP_BALANCE | FCC_MAP_XCD,
                                         FCC_MAP_XCD16,
                                         FCC_MAP_F_INNER | FCC_MAP_XCD16,
                                         FCC_MAP_CLUSTER,
                                         FCC_MAP_CLUSTER | FCC_MAP_XCD,
                                         FCC_MAP_CLUSTER | FCC_MAP_XCD16};
      for (int L = 0; L < 2 && L < p->tail_Lt[d] && s == FCC_OK; ++L) {
        if (orbit_at(p, d, L)) continue;  // no table, no map to search
        const int lgm = p->D - L - 1;
        const int ntiles = L == 0 ? 6 : 4;
        DevSide& cur = d == 0 ? p->lv[L].b : p->lv[L].c;
        DevSide best_side = cur;
        fcc_tuning best_t2 = p->tune;
        double best_ms = 1e30;
        std::vector<void*> keep;  // allocations of the winning side if not cached
        for (int ti = 0; ti < ntiles && s == FCC_OK; ++ti) {
          const int* tt = L == 0 ? tiles0[ti] : tiles1[ti];
          const CubeOrder o{std::min(tt[0], lgm), std::min(tt[1], lgm), std::min(tt[2], lgm)};
          bool dup = false;  // the same clamped shape as an earlier candidate
          for (int tj = 0; tj < ti; ++tj) {
            const int* uu = L == 0 ? tiles0[tj] : tiles1[tj];
            dup |= std::min(uu[0], lgm) == o.la && std::min(uu[1], lgm) == o.lb && std::min(uu[2], lgm) == o.lc;
          }
          if (dup) continue;
          std::vector<void*> own;
          DevSide cand{};
          {
            std::lock_guard<std::mutex> lock(cache().mu);
            std::array<int, 5> key{p->device, n >> L, slice_cubes(L), d, (o.la << 16) | (o.lb << 8) | o.lc};
            auto it = cache().sides.find(key);
            if (it != cache().sides.end())
              cand = it->second;
            else
              s = device_side(p->device, n >> L, slice_cubes(L), d, o, &cand, &own);
          }
          bool won = false;
          const unsigned* maps = d == 0 ? top_fwd : top_inv;
          const int nmaps = d == 0 ? int(sizeof top_fwd / sizeof top_fwd[0]) : int(sizeof top_inv / sizeof top_inv[0]);
          for (int mi = 0; mi < nmaps && s == FCC_OK; ++mi) {
            cur = cand;
            p->tune.tile[d][L][0] = o.la;
            p->tune.tile[d][L][1] = o.lb;
            p->tune.tile[d][L][2] = o.lc;
            p->tune.map[d][L] = maps[mi];
            s = d == 0 ? time_slots(p, a, b, 1, reps, st, &ms) : time_slots(p, b, a, -1, reps, st, &ms);
            if (s != FCC_OK) break;
            const double t = level_ms(L);
            if (verbose())
              std::fprintf(stderr, "fcc_autotune n=%d dir=%d level=%d tile=(%d,%d,%d) map=%u: %.4f ms\n", n, d, L, o.la,
                           o.lb, o.lc, maps[mi], t);
            if (t < best_ms) {
              best_ms = t;
              best_side = cand;
              best_t2 = p->tune;
              won = true;
            }
          }
          if (won) {
            for (void* q : keep) (void)hipFree(q);
            keep = own;
          } else {
            for (void* q : own) (void)hipFree(q);
          }
        }
        cur = best_side;
        p->tune = best_t2;
        if (!keep.empty()) {
          // the winner becomes the cached table of its key
          std::lock_guard<std::mutex> lock(cache().mu);
          const CubeOrder o{best_t2.tile[d][L][0], best_t2.tile[d][L][1], best_t2.tile[d][L][2]};
          cache().sides.emplace(std::array<int, 5>{p->device, n >> L, slice_cubes(L), d,
                                                   (o.la << 16) | (o.lb << 8) | o.lc},
                                best_side);
          cache().owned.insert(cache().owned.end(), keep.begin(), keep.end());
        }
      }
      // 3. thread map of the gather passes from level 2 on (plain-order
      // tables, so only the map changes)
      static const unsigned deep_fwd[] = {0u,
                                          FCC_MAP_XCD,
                                          FCC_MAP_NODES8,
                                          FCC_MAP_NODES8 | FCC_MAP_XCD,
                                          FCC_MAP_NODES64,
                                          FCC_MAP_NODES64 | FCC_MAP_XCD,
                                          FCC_MAP_SPLIT,
                                          FCC_MAP_SPLIT | FCC_MAP_NODES8 | FCC_MAP_XCD,
                                          FCC_MAP_SPLIT | FCC_MAP_NODES64,
                                          FCC_MAP_SPLIT | FCC_MAP_BALANCE | FCC_MAP_NODES64,
                                          FCC_MAP_SPLIT | FCC_MAP_BALANCE | FCC_MAP_NODES64 | FCC_MAP_XCD,
                                          FCC_MAP_SPLIT | FCC_MAP_NODES64 | FCC_MAP_XCD16};
      static const unsigned deep_inv[] = {0u,
                                          FCC_MAP_XCD,
                                          FCC_MAP_NODES8,
                                          FCC_MAP_NODES8 | FCC_MAP_XCD,
                                          FCC_MAP_NODES64,
                                          FCC_MAP_NODES64 | FCC_MAP_XCD,
                                          FCC_MAP_NODES8 | FCC_MAP_F_INNER | FCC_MAP_XCD,
                                          FCC_MAP_BALANCE | FCC_MAP_NODES64 | FCC_MAP_XCD,
                                          FCC_MAP_BALANCE | FCC_MAP_XCD,
                                          FCC_MAP_NODES64 | FCC_MAP_XCD16};
      for (int L = 2; L < p->tail_Lt[d] && s == FCC_OK; ++L) {
        if (orbit_at(p, d, L) || (d == 1 && L == p->D - 2 && inv_last2c(p))) continue;
        unsigned best_m = p->tune.map[d][L];
        double best_ms = 1e30;
        const unsigned* maps = d == 0 ? deep_fwd : deep_inv;
        const int nmaps = d == 0 ? 12 : 10;
        for (int mi = 0; mi < nmaps; ++mi) {
          p->tune.map[d][L] = maps[mi];
          s = d == 0 ? time_slots(p, a, b, 1, reps, st, &ms) : time_slots(p, b, a, -1, reps, st, &ms);
          if (s != FCC_OK) break;
          const double t = level_ms(L);
          if (verbose())
            std::fprintf(stderr, "fcc_autotune n=%d dir=%d level=%d map=%u: %.4f ms\n", n, d, L, maps[mi], t);
          if (t < best_ms) best_ms = t, best_m = maps[mi];
        }
        p->tune.map[d][L] = best_m;
      }
    }
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
  }
  fcc_tuning t = p->tune;
  if (s == FCC_OK) {
    std::lock_guard<std::mutex> lock(tuned_mu());
    load_schedules(p->device);
    tuned()[{p->device, n, int(prec), int(flags)}] = t;
    save_schedule(p->device, n, int(prec), flags, t);
    if (best) *best = t;
  }
  fcc_dct_destroy(p);
  return s;
}

fcc_status fcc_dct_roundtrip_residual(fcc_plan_t p, const void* x, const void* y, double* result,
                                      void* hip_stream) {
  if (!p || !x || !y || !result || !aligned16(x) || !aligned16(y)) return FCC_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();
  const long long N = (long long)p->n * p->n * p->n;
  if (!p->resid) {
    hipError_t ea = dev_malloc(reinterpret_cast<void**>(&p->resid), 2 * sizeof(unsigned long long));
    if (ea != hipSuccess) return hip_fail(ea, "device allocation (residual)", __LINE__);
  }
  unsigned long long* d = p->resid;
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, st, d);
  const unsigned blocks = unsigned(std::min<long long>((N + 255) / 256, 2048));
  switch (in_type(p)) {
    case DT::F32R: hipLaunchKernelGGL(k_residual<float>, dim3(blocks), dim3(256), 0, st, static_cast<const float*>(x), static_cast<const float*>(y), N, d); break;
    case DT::F64R: hipLaunchKernelGGL(k_residual<double>, dim3(blocks), dim3(256), 0, st, static_cast<const double*>(x), static_cast<const double*>(y), N, d); break;
    case DT::F32C: hipLaunchKernelGGL(k_residual<float2>, dim3(blocks), dim3(256), 0, st, static_cast<const float2*>(x), static_cast<const float2*>(y), N, d); break;
    case DT::F64C: hipLaunchKernelGGL(k_residual<double2>, dim3(blocks), dim3(256), 0, st, static_cast<const double2*>(x), static_cast<const double2*>(y), N, d); break;
  }
  fcc_status s = launch_status("residual launch");
  unsigned long long h[2] = {0ull, 0ull};
  if (s == FCC_OK) {
    e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = hip_fail(e, "residual copy", __LINE__);
  }
  if (s != FCC_OK) return s;
  double dmax, xmax;
  std::memcpy(&dmax, &h[0], 8);
  std::memcpy(&xmax, &h[1], 8);
  *result = xmax > 0.0 ? dmax / xmax : dmax;
  return FCC_OK;
}

fcc_status fcc_dct_batched(const fcc_plan_t* plans, int count, const void* const* in, void* const* out,
                           int direction, void* hip_stream) {
  if (!plans || !in || !out || count < 1) return FCC_ERR_INVALID_ARG;
  if (direction < -1 || direction > 1) return FCC_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i)
    if (!plans[i] || !in[i] || !out[i] || !aligned16(in[i]) || !aligned16(out[i]) || in[i] == out[i])
      return FCC_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i)
    if (plans[i]->hslot) return FCC_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();
  std::vector<uintptr_t> key;
  key.reserve(3 * size_t(count) + 2);
  key.push_back(uintptr_t(count));
  key.push_back(uintptr_t(direction + 1));
  for (int i = 0; i < count; ++i) {
    key.push_back(reinterpret_cast<uintptr_t>(plans[i]));
    key.push_back(reinterpret_cast<uintptr_t>(in[i]));
    key.push_back(reinterpret_cast<uintptr_t>(out[i]));
  }
  std::lock_guard<std::mutex> lock(batch_mu());
  auto& cache_v = batch_cache();
  BatchExec* bx = nullptr;
  for (size_t i = 0; i < cache_v.size(); ++i)
    if (cache_v[i]->key == key) {
      bx = cache_v[i];
      cache_v.erase(cache_v.begin() + i);
      cache_v.push_back(bx);  // most recently used last
      break;
    }
  if (!bx) {
    if (cache_v.size() >= kBatchCacheCap) {
      // the oldest graph may still run on a stream: wait for the device first
      (void)hipDeviceSynchronize();
      free_batch(cache_v.front());
      cache_v.erase(cache_v.begin());
    }
    bx = new (std::nothrow) BatchExec;
    if (!bx) return FCC_ERR_OOM;
    bx->key = key;
    fcc_status s = build_batch(bx, plans, count, in, out, direction);
    if (s != FCC_OK) {
      free_batch(bx);
      return s;
    }
    cache_v.push_back(bx);
  }
  hipError_t e = hipGraphLaunch(bx->exec, st);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch", __LINE__);
  return FCC_OK;
}

fcc_status fcc_dct_packed_size(fcc_plan_t p, long long* count) {
  if (!p || !count) return FCC_ERR_INVALID_ARG;
  *count = p->hslot ? p->hpacked : (long long)p->n * p->n * p->n;
  return FCC_OK;
}

fcc_status fcc_dct_batched_release(void) {
  std::lock_guard<std::mutex> lock(batch_mu());
  auto& c = batch_cache();
  if (c.empty()) return FCC_OK;
  hipError_t e = hipDeviceSynchronize();
  for (BatchExec* b : c) free_batch(b);
  c.clear();
  return e == hipSuccess ? FCC_OK : hip_fail(e, "hipDeviceSynchronize", __LINE__);
}

fcc_status fcc_dct_describe_launches(fcc_plan_t p, int direction, fcc_launch_info* info, int cap, int* count) {
  if (!p || !count || (direction != 1 && direction != -1)) return FCC_ERR_INVALID_ARG;
  const std::vector<SlotDesc> v = describe_slots(p, direction > 0 ? 0 : 1);
  *count = int(v.size());
  if (!info) return FCC_OK;
  if (cap < int(v.size())) return FCC_ERR_INVALID_ARG;
  const long long N = (long long)p->n * p->n * p->n;
  for (size_t i = 0; i < v.size(); ++i) {
    std::memset(&info[i], 0, sizeof info[i]);
    std::snprintf(info[i].name, sizeof info[i].name, "%s", v[i].name.c_str());
    info[i].points = N;
    info[i].in_bytes = v[i].in_b;
    info[i].out_bytes = v[i].out_b;
  }
  return FCC_OK;
}

fcc_status fcc_dct_batched_time_launches(const fcc_plan_t* plans, int count, const void* const* in,
                                         void* const* out, int direction, int reps, float* ms,
                                         fcc_launch_info* info, int cap, int* nslots, void* hip_stream) {
  if (!plans || !in || !out || count < 1 || !nslots || reps < 1) return FCC_ERR_INVALID_ARG;
  if (direction < -1 || direction > 1) return FCC_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i)
    if (!plans[i] || !in[i] || !out[i] || !aligned16(in[i]) || !aligned16(out[i]) || in[i] == out[i])
      return FCC_ERR_INVALID_ARG;
  std::vector<BatchGroup> groups = group_plans(plans, count);
  // the slots: per group, the forward then the inverse launches of every chunk
  std::vector<fcc_launch_info> slots;
  std::vector<int> per_run;  // slots of one pass over all groups
  for (const BatchGroup& g : groups) {
    const int cnt = int(g.vols.size());
    const int chunk = g.p->dense ? cnt : chunk_volumes(g.p, cnt);
    for (int d = 0; d < 2; ++d) {
      if ((d == 0 && direction < 0) || (d == 1 && direction > 0)) continue;
      const std::vector<SlotDesc> v = describe_slots(g.p, d);
      for (int v0 = 0; v0 < cnt; v0 += chunk) {
        const int k = std::min(chunk, cnt - v0);
        for (const SlotDesc& sd : v) {
          fcc_launch_info li{};
          std::snprintf(li.name, sizeof li.name, "n%d x%d %s", g.p->n, k, sd.name.c_str());
          li.points = (long long)k * g.p->n * g.p->n * g.p->n;
          li.in_bytes = sd.in_b;
          li.out_bytes = sd.out_b;
          slots.push_back(li);
        }
      }
    }
  }
  *nslots = int(slots.size());
  if (!ms) return FCC_OK;
  if (cap < int(slots.size())) return FCC_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();
  std::vector<void*> allocs;
  std::vector<GroupRes> res(groups.size());
  fcc_status s = FCC_OK;
  for (size_t gi = 0; gi < groups.size() && s == FCC_OK; ++gi) s = prepare_group(&allocs, groups[gi], in, out, &res[gi]);
  std::vector<hipEvent_t> ev(size_t(2) * slots.size() * reps, nullptr);
  for (size_t i = 0; i < ev.size() && s == FCC_OK; ++i) {
    hipError_t he = hipEventCreate(&ev[i]);
    if (he != hipSuccess) s = hip_fail(he, "hipEventCreate", __LINE__);
  }
  size_t pos = 0;
  for (int r = 0; r < reps && s == FCC_OK; ++r)
    for (size_t gi = 0; gi < groups.size() && s == FCC_OK; ++gi) {
      if (direction >= 0) s = enqueue_group(groups[gi], res[gi], 1, false, st, &ev, &pos);
      if (s == FCC_OK && direction == 0) s = enqueue_group(groups[gi], res[gi], -1, true, st, &ev, &pos);
      if (s == FCC_OK && direction < 0) s = enqueue_group(groups[gi], res[gi], -1, false, st, &ev, &pos);
    }
  if (s == FCC_OK && pos != ev.size()) s = FCC_ERR_HIP;  // launch count differs from the slot count
  if (s == FCC_OK) {
    hipError_t he = hipStreamSynchronize(st);
    if (he != hipSuccess) s = hip_fail(he, "hipStreamSynchronize", __LINE__);
  }
  if (s == FCC_OK) {
    const size_t ns = slots.size();
    for (size_t k = 0; k < ns; ++k) {
      double acc = 0.0;
      for (int r = 0; r < reps; ++r) {
        float t = 0.f;
        (void)hipEventElapsedTime(&t, ev[(size_t(r) * ns + k) * 2], ev[(size_t(r) * ns + k) * 2 + 1]);
        acc += t;
      }
      ms[k] = float(acc / reps);
      if (info) info[k] = slots[k];
    }
  } else {
    (void)hipStreamSynchronize(st);
  }
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  for (void* a : allocs) (void)hipFree(a);
  return s;
}

}  // extern "C"
