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
// A block takes U "units" = K orbits of one kind x G nodes (G = 1 at level
// 0, 8 below; the nodes are consecutive in J, so for one source slot the
// units of one orbit read consecutive addresses); U grows as the kind's orbits
// shrink (8 units for orbits of more than 12 cubes, 16 up to 12, 32 up to 6,
// 64 up to 3), so that every block fills its 192 threads and its LDS whatever
// the stabiliser of its orbits.  The sources (or cube values) sit in LDS as
// [slot][unit], slot = cube slot * 8 + o (or def).  The rows are summed by
// wavefronts of 64 lanes = 64 / U cube slots x U units; a
// template row is split by monomial of the node's coefficient polynomials
// into 5 segments of integer coefficients (the row's rational coefficients
// times 144), and the cube slots are ordered so that the slots of a wavefront
// have identical segment lengths (generic orbits: groups of 4 cubes with the
// same profile), so the lanes of a wavefront run the same trip counts.  The
// node's DCT_2 (and its inverse) comes from a per-node table of 64 complex
// entries each.
// Blocks are numbered so that each XCD works through one contiguous range
// (consecutive node groups, then consecutive orbits in Morton order of their
// representatives), which keeps cache lines that neighbouring blocks share in
// one L2.
#pragma once

namespace fcc {

constexpr int kOrbitThreads = 192;                  // 3 wavefronts: cube slots x units, nc U <= 192
constexpr int kOrbitMaxCubes = 24;
constexpr int kOrbitMaxSlots = 8 * kOrbitMaxCubes;  // 192
constexpr int kOrbitVal = 8 * kOrbitMaxSlots;       // LDS values: 8 nc U <= 1536
constexpr int kOrbitMaxOrbits = 64;                 // orbits per block (level 0, U = 64)
constexpr int kOrbitSeg = 8 * kNumMono;             // segments per cube slot
constexpr int kOrbitMaxEnt = 2560;                  // entries of one kind's B (C) block
constexpr int kOrbitMaxNodes = 8;

// Units of a block for orbits of nc cubes (8 nc U <= kOrbitVal).
__host__ __device__ __forceinline__ int orbit_lg_units(int nc) { return nc > 12 ? 3 : (nc > 6 ? 4 : (nc > 3 ? 5 : 6)); }
// Blocks of an orbit launch at level L: one per chunk (of the level's chunk
// table) and group of G = min(8^L, 8) nodes.
__host__ __device__ __forceinline__ long long orbit_blocks_total(int nchunk, int L, int nvol) {
  return (long long)nchunk * (L == 0 ? 1LL : (1LL << (3 * (L - 1)))) * nvol;
}

// Logical block of an orbit launch: blocks i, i+8, i+16, ... run on one XCD,
// which gets one contiguous range of the total.  Returns -1 past the end.
__device__ __forceinline__ long long orbit_block(long long total) {
  const long long per = (total + 7) >> 3;
  const long long b = (long long)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  return b < total ? b : -1;
}

// Cube q_j = (G[w_j] p0) mod m of representative p0.
__device__ __forceinline__ void orbit_cube(const int8_t* g, uint32_t pr, int mask, int q[3]) {
  const int p0[3] = {int(pr >> 20), int((pr >> 10) & 1023u), int(pr & 1023u)};
#pragma unroll
  for (int d = 0; d < 3; ++d) q[d] = (g[3 * d] * p0[0] + g[3 * d + 1] * p0[1] + g[3 * d + 2] * p0[2]) & mask;
}

// LDS state of a block.
template <typename R>
struct OrbitShared {
  cx<R> val[kOrbitVal];  // sources (forward) or cube values (inverse), [slot][unit]
  alignas(16) cx<R> mono[kOrbitMaxNodes][kNumMono];  // monomials / 144, per node
  alignas(16) uint32_t ent[kOrbitMaxEnt];
  alignas(16) uint16_t seg[kOrbitMaxCubes * kOrbitSeg + 8];
  alignas(16) int16_t perm[kOrbitMaxCubes];
  alignas(16) int8_t wm[9 * kOrbitMaxCubes + 8];
  uint32_t rep[kOrbitMaxOrbits];
};

struct OrbitBlock {
  long long vol;
  long long node0;  // first node of the block's group of G
  int G, K;         // nodes and orbits of the block
  int U, lgU;       // units (K G)
  int nc, nact;     // cubes of the kind; active units (orbit index < chunk count)
};

// Node J (flat index) -> coordinates.
__device__ __forceinline__ void node_coords(long long node, int L, int J[3]) {
  const int mask = (1 << L) - 1;
  J[0] = int(node >> (2 * L));
  J[1] = int((node >> L) & mask);
  J[2] = int(node & mask);
}

// Block set-up shared by both directions: decode (volume, chunk, orbit
// sub-range, node group), then copy the kind's side `sd` of the template and
// the orbits' representatives to LDS and form each node's monomials.  Every
// copy is a 16-byte load issued before the first wait (one memory round
// trip).  Returns false for blocks with nothing to do (the whole block leaves).
constexpr int kOrbitPieces = 5;  // 16-byte pieces per thread
template <typename R>
__device__ __forceinline__ bool orbit_setup(const DevOrbitLevel& ol, int L, int nvol, int sd,
                                            const double2* __restrict__ hph, OrbitBlock& ob, OrbitShared<R>& sh) {
  const long long nnode = 1LL << (3 * L);
  ob.G = int(nnode < kOrbitMaxNodes ? nnode : kOrbitMaxNodes);
  const int gs = ob.G == 1 ? 0 : 1;
  const int nch = ol.nchunk[gs];
  const long long b = orbit_block(orbit_blocks_total(nch, L, nvol));
  if (b < 0) return false;
  const long long ngroups = nnode / ob.G;
  const long long ng = b % ngroups;
  const long long rest = b / ngroups;
  const int chunk = int(rest % nch);
  ob.vol = rest / nch;
  ob.node0 = ng * ob.G;
  const int4 ch = ol.chunks[gs][chunk];
  ob.lgU = ch.w;
  ob.U = 1 << ch.w;
  ob.K = ob.U / ob.G;
  const int first = ch.y;
  const int norb = ch.z;
  ob.nact = norb * ob.G;
  const DevOrbitKind kd = ol.kinds[ch.x];
  ob.nc = kd.nc;
  const int tid = threadIdx.x;
  // pieces: segment starts, entries, slot order, slot matrices
  const int o1 = (kOrbitSeg * kd.nc + 1 + 7) >> 3;
  const int o2 = o1 + ((kd.nent[sd] + 3) >> 2);
  const int o3 = o2 + ((kd.nc + 7) >> 3);
  const int total = o3 + ((9 * kd.nc + 15) >> 4);
  const uint4* g_seg = reinterpret_cast<const uint4*>(ol.rowptr + kd.off_rowptr[sd]);
  const uint4* g_ent = reinterpret_cast<const uint4*>(ol.ent + kd.off_ent[sd]);
  const uint4* g_perm = reinterpret_cast<const uint4*>(ol.perm + kd.off_perm[sd]);
  const uint4* g_wm = reinterpret_cast<const uint4*>(ol.wmat + kd.off_w);
  // (pieces past the total re-read the first one, so every load is unconditional)
  uint4 t[kOrbitPieces];
#pragma unroll
  for (int c = 0; c < kOrbitPieces; ++c) {
    const int k = tid + c * kOrbitThreads;
    const uint4* src = k >= total ? g_seg
                       : k < o1   ? g_seg + k
                       : k < o2   ? g_ent + (k - o1)
                       : k < o3   ? g_perm + (k - o2)
                                  : g_wm + (k - o3);
    t[c] = *src;
  }
  uint32_t r = 0;
  if (tid < norb) r = ol.reps[first + tid];
  if (tid < ob.G) {
    int J[3];
    node_coords(ob.node0 + tid, L, J);
    cx<R> mono[kNumMono];
    node_mono(hph, L, J, mono);
#pragma unroll
    for (int q = 0; q < kNumMono; ++q) sh.mono[tid][q] = R(1.0 / 144.0) * mono[q];
  }
#pragma unroll
  for (int c = 0; c < kOrbitPieces; ++c) {
    const int k = tid + c * kOrbitThreads;
    if (k < total) {
      uint4* dst = k < o1   ? reinterpret_cast<uint4*>(sh.seg) + k
                   : k < o2 ? reinterpret_cast<uint4*>(sh.ent) + (k - o1)
                   : k < o3 ? reinterpret_cast<uint4*>(sh.perm) + (k - o2)
                            : reinterpret_cast<uint4*>(sh.wm) + (k - o3);
      *dst = t[c];
    }
  }
  if (tid < norb) sh.rep[tid] = r;
  return true;
}

// One row of B (C) for unit u: sum_q (mono_q / 144) * sum_{segment q} k_e val[slot_e][u].
template <typename R>
__device__ __forceinline__ cx<R> orbit_row(const OrbitShared<R>& sh, int s0, int u, int lgU, const cx<R>* mono) {
  cx<R> y{R(0), R(0)};
  const char* vbase = reinterpret_cast<const char*>(sh.val) + u * sizeof(cx<R>);
#pragma unroll
  for (int q = 0; q < kNumMono; ++q) {
    cx<R> a{R(0), R(0)};
    const int e1 = sh.seg[s0 + q + 1];
#pragma unroll 2
    for (int e = sh.seg[s0 + q]; e < e1; ++e) {
      const uint32_t v = sh.ent[e];
      const cx<R> x = *reinterpret_cast<const cx<R>*>(vbase + ((v >> 16) << lgU) * sizeof(cx<R>));
      const R c = R(int(int16_t(v & 0xffffu)));
      a.x = a.x + c * x.x;
      a.y = a.y + c * x.y;
    }
    y = y + mono[q] * a;
  }
  return y;
}

// Forward level L: y = B_nl(c) x on the block's orbits and nodes, then
// z = DCT_2(phi) y per cube, stored at the cube's 8 positions.
// kT: the transposed transform's inverse level instead: rows of C^T (side 3),
// then DCT_2(phi)^{-T} per cube.
template <typename R, typename TI, typename TO, bool kT>
__global__ __launch_bounds__(kOrbitThreads) void k_fwd_orbit(VolSet vs, int nvol, int n, int L, DevOrbitLevel ol,
                                                             const double2* __restrict__ hph,
                                                             const OrbitNode* __restrict__ onodes) {
  __shared__ OrbitShared<R> sh;
  OrbitBlock ob;
  if (!orbit_setup<R>(ol, L, nvol, kT ? 3 : 0, hph, ob, sh)) return;
  __syncthreads();
  const int mask = (1 << ol.lgm) - 1;
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, ob.vol));
  // sources: slot s = j * 8 + o of unit u = k * G + g is q_j(orbit k) + m o in
  // node node0 + g; every load of a thread is issued before the first wait
  constexpr int kPer = kOrbitVal / kOrbitThreads;
  cx<R> v[kPer];
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int it = threadIdx.x + c * kOrbitThreads, u = it & (ob.U - 1), s = it >> ob.lgU;
    if (it < ob.nc * 8 * ob.U && u < ob.nact) {
      int q[3], J[3];
      orbit_cube(sh.wm + 9 * (s >> 3), sh.rep[u / ob.G], mask, q);
      node_coords(ob.node0 + u % ob.G, L, J);
      const int o = s & 7;
      v[c] = IO<TI, R>::ld(in, gpos(n, L, J, q[0] + (((o >> 2) & 1) << ol.lgm), q[1] + (((o >> 1) & 1) << ol.lgm),
                                    q[2] + ((o & 1) << ol.lgm)));
    }
  }
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int it = threadIdx.x + c * kOrbitThreads;
    if (it < ob.nc * 8 * ob.U && (it & (ob.U - 1)) < ob.nact) sh.val[it] = v[c];
  }
  __syncthreads();
  // wavefront w: cube slots 64 / U * w ... of the slot order, U units each
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, u = lane & (ob.U - 1);
  if (w >= ((ob.nc << ob.lgU) + 63) >> 6 || u >= ob.nact) return;
  const int j = sh.perm[((64 >> ob.lgU) * w) + (lane >> ob.lgU)];
  if (j < 0) return;
  int J[3];
  node_coords(ob.node0 + u % ob.G, L, J);
  const cx<R>* mono = sh.mono[u % ob.G];
  // z = DCT_2(phi) y, one column per row of B as the rows complete (column
  // f + 1 is loaded while row f is summed)
  const OrbitNode& on = onodes[ob.node0 + u % ob.G];
  cx<R> y[8];
  // column f of the matrix: D[f * 8 + i] (forward), or row f of DCT_2^{-1},
  // Dinv[i * 8 + f] (transposed inverse)
  auto col = [&](int f, int i) { return kT ? on.Dinv[i * 8 + f] : on.D[f * 8 + i]; };
  double2 dcol[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    y[i] = {R(0), R(0)};
    dcol[i] = col(0, i);
  }
#pragma unroll 1
  for (int f = 0; f < 8; ++f) {
    double2 cur[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) cur[i] = dcol[i];
    if (f < 7) {
#pragma unroll
      for (int i = 0; i < 8; ++i) dcol[i] = col(f + 1, i);
    }
    const cx<R> yf = orbit_row(sh, (j * 8 + f) * kNumMono, u, ob.lgU, mono);
#pragma unroll
    for (int i = 0; i < 8; ++i) y[i] = y[i] + ldc<R>(cur[i]) * yf;
  }
  int q[3];
  orbit_cube(sh.wm + 9 * j, sh.rep[u / ob.G], mask, q);
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, ob.vol));
#pragma unroll
  for (int i = 0; i < 8; ++i)
    IO<TO, R>::st(out, gpos(n, L, J, 2 * q[0] + ((i >> 2) & 1), 2 * q[1] + ((i >> 1) & 1), 2 * q[2] + (i & 1)),
                  y[i]);
}

// Inverse level L: y = DCT_2(phi)^{-1} z per cube of the block's orbits and
// nodes, then x(q' + m o) = row (q', o) of C_nl(c) applied to the orbit's cube
// values.
// kT: the transposed transform's level instead: DCT_2(phi)^T per cube, then
// the rows of B^T (side 2).
template <typename R, typename TI, typename TO, bool kT>
__global__ __launch_bounds__(kOrbitThreads) void k_inv_orbit(VolSet vs, int nvol, int n, int L, DevOrbitLevel ol,
                                                             const double2* __restrict__ hph,
                                                             const OrbitNode* __restrict__ onodes) {
  __shared__ OrbitShared<R> sh;
  OrbitBlock ob;
  if (!orbit_setup<R>(ol, L, nvol, kT ? 2 : 1, hph, ob, sh)) return;
  __syncthreads();
  const int mask = (1 << ol.lgm) - 1;
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, ob.vol));
  // cube values: slot s = j * 8 + def of unit u, from position def + 2 q_j
  for (int it = threadIdx.x; it < ob.nc * ob.U; it += kOrbitThreads) {
    const int u = it & (ob.U - 1), j = it >> ob.lgU;
    if (u < ob.nact) {
      int q[3], J[3];
      orbit_cube(sh.wm + 9 * j, sh.rep[u / ob.G], mask, q);
      node_coords(ob.node0 + u % ob.G, L, J);
      cx<R> z[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        z[i] = IO<TI, R>::ld(in, gpos(n, L, J, 2 * q[0] + ((i >> 2) & 1), 2 * q[1] + ((i >> 1) & 1),
                                       2 * q[2] + (i & 1)));
      // y = DCT_2(phi)^{-1} z (transposed transform: DCT_2(phi)^T z)
      const OrbitNode& on = onodes[ob.node0 + u % ob.G];
      cx<R> y[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) y[f] = {R(0), R(0)};
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int f = 0; f < 8; ++f) y[f] = y[f] + ldc<R>(kT ? on.D[f * 8 + i] : on.Dinv[i * 8 + f]) * z[i];
#pragma unroll
      for (int f = 0; f < 8; ++f) sh.val[((j * 8 + f) << ob.lgU) + u] = y[f];
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, u = lane & (ob.U - 1);
  if (w >= ((ob.nc << ob.lgU) + 63) >> 6 || u >= ob.nact) return;
  const int j = sh.perm[((64 >> ob.lgU) * w) + (lane >> ob.lgU)];
  if (j < 0) return;
  int J[3];
  node_coords(ob.node0 + u % ob.G, L, J);
  const cx<R>* mono = sh.mono[u % ob.G];
  int q[3];
  orbit_cube(sh.wm + 9 * j, sh.rep[u / ob.G], mask, q);
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, ob.vol));
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const cx<R> x = orbit_row(sh, (j * 8 + o) * kNumMono, u, ob.lgU, mono);
    IO<TO, R>::st(out, gpos(n, L, J, q[0] + (((o >> 2) & 1) << ol.lgm), q[1] + (((o >> 1) & 1) << ol.lgm),
                            q[2] + ((o & 1) << ol.lgm)),
                  x);
  }
}

}  // namespace fcc
