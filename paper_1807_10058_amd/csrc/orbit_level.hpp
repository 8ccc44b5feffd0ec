// Orbit-block form of one radix-2x2x2 level (Sec. IV-B, eq. FastAlgorithm),
// basis change and DCT_2 (x) I fused into one launch.
//
// Let W act on the cube grid [0,m)^3 of a node of size nl = 2m by
// q -> (g q) mod m.  For an orbit O the rows (def, q), q in O, of B_nl read
// exactly the sources q' + m o (q' in O, o in {0,1}^3) and nothing else, and
// the 8 rows of a cube are all in the block, so
//
//   forward : load the 8|O| sources of the orbit once, form the 8 rows of
//             every cube from them (the orbit kind's template), apply
//             DCT_2(phi) to each cube and store its 8 values;
//   inverse : load the 8 values of every cube of the orbit, apply
//             DCT_2(phi)^{-1} (per-cube solves), then form every output
//             x(q' + m o) from the orbit's 8|O| cube values (C_nl's block).
//
// A block takes 16 orbits of one kind ("units") of one node J.  Their sources
// (or cube values) sit in LDS as [slot][unit], slot = cube slot * 8 + o (or
// def).  The rows are summed by wavefronts of 64 lanes = 4 cube slots x 16
// units; the template orders the cube slots so that the 4 slots of a wavefront
// have identical row lengths (generic orbits: groups of 4 cubes with the same
// profile), so the lanes of a wavefront run the same trip counts.  Blocks are
// numbered so that each XCD works through one contiguous range (consecutive
// nodes, then consecutive chunks of orbits in Morton order of their
// representatives), which keeps the cache lines that neighbouring blocks share
// in one L2.
#pragma once

namespace fcc {

constexpr int kOrbitUnits = 16;                   // orbits per block
constexpr int kOrbitThreads = 384;                // 6 wavefronts: 24 cube slots x 16 units
constexpr int kOrbitMaxCubes = 24;
constexpr int kOrbitMaxSlots = 8 * kOrbitMaxCubes;  // 192
constexpr int kOrbitMaxEnt = 2560;                // entries of one kind's B (C) block

// Logical block of an orbit launch: blocks i, i+8, i+16, ... run on one XCD,
// which gets one contiguous range of the total.  Returns -1 past the end.
__device__ __forceinline__ long long orbit_block(long long total) {
  const long long per = (total + 7) >> 3;
  const long long b = (long long)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  return b < total ? b : -1;
}

// Cube q_j = (G[w_j] p0) mod m of unit representative p0.
__device__ __forceinline__ void orbit_cube(const int8_t* g, uint32_t pr, int mask, int q[3]) {
  const int p0[3] = {int(pr >> 20), int((pr >> 10) & 1023u), int(pr & 1023u)};
#pragma unroll
  for (int d = 0; d < 3; ++d) q[d] = (g[3 * d] * p0[0] + g[3 * d + 1] * p0[1] + g[3 * d + 2] * p0[2]) & mask;
}

// Block set-up shared by both directions: decode (volume, chunk, node), copy
// the kind's side `sd` of the template to LDS and form the node's coefficient
// values.  Returns false for padding blocks (the whole block leaves).
template <typename R>
struct OrbitBlock {
  long long vol;
  int J[3];
  int kind, first, cnt, nc;
};
template <typename R>
__device__ __forceinline__ bool orbit_setup(const DevOrbitLevel& ol, int n, int L, int nvol, int sd,
                                            const double2* __restrict__ hph, OrbitBlock<R>& ob, cx<R>* coef,
                                            uint16_t* ent, uint16_t* rowptr, int16_t* perm, int8_t* wm) {
  const long long nnode = 1LL << (3 * L);
  const long long b = orbit_block((long long)ol.nchunk * nnode * nvol);
  if (b < 0) return false;
  const long long node = b % nnode, rest = b / nnode;
  const int chunk = int(rest % ol.nchunk);
  ob.vol = rest / ol.nchunk;
  const int mask = (1 << L) - 1;
  ob.J[0] = int(node >> (2 * L));
  ob.J[1] = int((node >> L) & mask);
  ob.J[2] = int(node & mask);
  const int4 ch = ol.chunks[chunk];
  ob.kind = ch.x;
  ob.first = ch.y;
  ob.cnt = ch.z;
  const DevOrbitKind kd = ol.kinds[ob.kind];
  ob.nc = kd.nc;
  const int rows = 8 * kd.nc;
  const int tid = threadIdx.x;
  for (int i = tid; i <= rows; i += blockDim.x) rowptr[i] = ol.rowptr[kd.off_rowptr[sd] + i];
  const int nent = ol.rowptr[kd.off_rowptr[sd] + rows];
  for (int i = tid; i < nent; i += blockDim.x) ent[i] = ol.ent[kd.off_ent[sd] + i];
  const int np = 4 * ((kd.nc + 3) >> 2);
  for (int i = tid; i < np; i += blockDim.x) perm[i] = ol.perm[kd.off_perm[sd] + i];
  for (int i = tid; i < 9 * kd.nc; i += blockDim.x) wm[i] = ol.wmat[kd.off_w + i];
  if (tid < ol.npoly) {
    cx<R> mono[kNumMono];
    node_mono(hph, L, ob.J, mono);
    coef[tid] = poly_value(ol.poly, ol.nconst, tid, mono);
  }
  return true;
}

// Forward level L: y = B_nl(c) x on the orbits of one chunk, then
// z = DCT_2(phi) y per cube, stored at the cube's 8 positions.
template <typename R, typename TI, typename TO>
__global__ __launch_bounds__(kOrbitThreads) void k_fwd_orbit(VolSet vs, int nvol, int n, int L, DevOrbitLevel ol,
                                                             const double2* __restrict__ hph,
                                                             const NodeConst* nodes) {
  __shared__ cx<R> src[kOrbitMaxSlots * kOrbitUnits];
  __shared__ cx<R> coef[kMaxPoly];
  __shared__ uint16_t ent[kOrbitMaxEnt];
  __shared__ uint16_t rowptr[kOrbitMaxSlots + 1];
  __shared__ int16_t perm[kOrbitMaxCubes];
  __shared__ int8_t wm[9 * kOrbitMaxCubes];
  OrbitBlock<R> ob;
  if (!orbit_setup<R>(ol, n, L, nvol, 0, hph, ob, coef, ent, rowptr, perm, wm)) return;
  __syncthreads();
  const int mask = (1 << ol.lgm) - 1;
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, ob.vol));
  // sources: slot s = j * 8 + o of unit u is q_j(u) + m o
  for (int it = threadIdx.x; it < ob.nc * 8 * kOrbitUnits; it += kOrbitThreads) {
    const int u = it & (kOrbitUnits - 1), s = it >> 4;
    if (u < ob.cnt) {
      int q[3];
      orbit_cube(wm + 9 * (s >> 3), ol.reps[ob.first + u], mask, q);
      const int o = s & 7;
      src[it] = IO<TI, R>::ld(in, gpos(n, L, ob.J, q[0] + (((o >> 2) & 1) << ol.lgm),
                                        q[1] + (((o >> 1) & 1) << ol.lgm), q[2] + ((o & 1) << ol.lgm)));
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, u = lane & (kOrbitUnits - 1);
  if (w >= ((ob.nc + 3) >> 2) || u >= ob.cnt) return;
  const int j = perm[4 * w + (lane >> 4)];
  if (j < 0) return;
  cx<R> y[8];
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    cx<R> acc{R(0), R(0)};
    const int e1 = rowptr[j * 8 + f + 1];
    for (int e = rowptr[j * 8 + f]; e < e1; ++e) {
      const uint16_t v = ent[e];
      acc = acc + coef[v & 255u] * src[(v >> 8) * kOrbitUnits + u];
    }
    y[f] = acc;
  }
  dct2_apply(nodes, hph, L, ob.J, y);
  int q[3];
  orbit_cube(wm + 9 * j, ol.reps[ob.first + u], mask, q);
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, ob.vol));
#pragma unroll
  for (int i = 0; i < 8; ++i)
    IO<TO, R>::st(out, gpos(n, L, ob.J, 2 * q[0] + ((i >> 2) & 1), 2 * q[1] + ((i >> 1) & 1), 2 * q[2] + (i & 1)),
                  y[i]);
}

// Inverse level L: y = DCT_2(phi)^{-1} z per cube of the chunk's orbits, then
// x(q' + m o) = row (q', o) of C_nl(c) applied to the orbit's cube values.
template <typename R, typename TI, typename TO>
__global__ __launch_bounds__(kOrbitThreads) void k_inv_orbit(VolSet vs, int nvol, int n, int L, DevOrbitLevel ol,
                                                             const double2* __restrict__ hph,
                                                             const NodeConst* nodes) {
  __shared__ cx<R> ys[kOrbitMaxSlots * kOrbitUnits];
  __shared__ cx<R> coef[kMaxPoly];
  __shared__ uint16_t ent[kOrbitMaxEnt];
  __shared__ uint16_t rowptr[kOrbitMaxSlots + 1];
  __shared__ int16_t perm[kOrbitMaxCubes];
  __shared__ int8_t wm[9 * kOrbitMaxCubes];
  OrbitBlock<R> ob;
  if (!orbit_setup<R>(ol, n, L, nvol, 1, hph, ob, coef, ent, rowptr, perm, wm)) return;
  __syncthreads();
  const int mask = (1 << ol.lgm) - 1;
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, ob.vol));
  // cube values: slot s = j * 8 + def of unit u, from position def + 2 q_j(u)
  for (int it = threadIdx.x; it < ob.nc * kOrbitUnits; it += kOrbitThreads) {
    const int u = it & (kOrbitUnits - 1), j = it >> 4;
    if (u < ob.cnt) {
      int q[3];
      orbit_cube(wm + 9 * j, ol.reps[ob.first + u], mask, q);
      cx<R> z[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        z[i] = IO<TI, R>::ld(in, gpos(n, L, ob.J, 2 * q[0] + ((i >> 2) & 1), 2 * q[1] + ((i >> 1) & 1),
                                       2 * q[2] + (i & 1)));
      idct2_apply(nodes, hph, L, ob.J, z);
#pragma unroll
      for (int f = 0; f < 8; ++f) ys[(j * 8 + f) * kOrbitUnits + u] = z[f];
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, u = lane & (kOrbitUnits - 1);
  if (w >= ((ob.nc + 3) >> 2) || u >= ob.cnt) return;
  const int j = perm[4 * w + (lane >> 4)];
  if (j < 0) return;
  int q[3];
  orbit_cube(wm + 9 * j, ol.reps[ob.first + u], mask, q);
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, ob.vol));
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    cx<R> acc{R(0), R(0)};
    const int e1 = rowptr[j * 8 + o + 1];
    for (int e = rowptr[j * 8 + o]; e < e1; ++e) {
      const uint16_t v = ent[e];
      acc = acc + coef[v & 255u] * ys[(v >> 8) * kOrbitUnits + u];
    }
    IO<TO, R>::st(out, gpos(n, L, ob.J, q[0] + (((o >> 2) & 1) << ol.lgm), q[1] + (((o >> 1) & 1) << ol.lgm),
                            q[2] + ((o & 1) << ol.lgm)),
                  acc);
  }
}

}  // namespace fcc
