// Dense base of the hybrid-depth forward (FCC_FOLD_BASE): the recursion of
// Sec. IV-B stops at node size M (n = 2^Lt M, the stepwise decomposition with
// n = 2^Lt * M), and every node J of level Lt applies its own DCT_M(phi_J),
// phi_J = ((r,s,t) + J) / 2^Lt, in one LDS-resident launch.
//
// DCT_M(phi) is taken from the explicit matrix (Sec. IV-A, eq.
// SU4ChebyshevTransformExplicitForm, Lemma 2 with the node's skew): with the
// two sums exchanged,
//   X[j] = sum_mu Fh[mu] e(mu.j / M),      e(t) = exp(2 pi i t),
//   Fh[mu] = (1/24) sum_{(k, g): g k = mu mod M} x[k] e((g k).phi / M),
// a twiddled fold of the node onto the M-torus and an unnormalised inverse
// DFT_M^3 shared by all nodes.  With 8 (r,s,t) = r8 integral and
// rho = r8 + 8 J, (g k).phi / M = (g k).rho / (8 n), so every phase is a root
// of unity of order 8n.  A lane owns one orbit of W on the M-torus (its
// representative r) and all 24 images u r = k_u + M W_u (k_u in [0, M)^3):
//   Fh[k_h] = (1/24) A(k_h) sum_u x[k_u] T[(W_h . rho - Z_u . (h^T rho)) mod P],
//   Z_u = u^{-1} W_u,  A(k) = e(k.rho / (8n)),  T[t] = e(t / P),  P = 8 * 2^Lt,
// (the term of g = h u^{-1}: g k_u = k_h + M (W_h - h Z_u)).  The sum over u
// runs over every g once, so images that coincide (orbits with a stabiliser)
// receive the same value.  A lane reads its orbit's 24 inputs before it
// writes any output, and orbits are disjoint, so the fold runs in place.
//
// The base is well conditioned in itself (a fold with unit-modulus weights
// and a DFT), but its input carries the growth of the levels above it, so
// the stage precision rule of the plan applies unchanged.
#pragma once
#include <hip/hip_runtime.h>

#include "fold_fft.hpp"
#include "kernels.hpp"

namespace fcc {

// M^3-point nodes, G = 256 / M^2 of them per block (consecutive J_z), 256 * M
// points in LDS; z-lines padded by one element so that the line passes along
// every axis run without bank conflicts.
template <int M>
struct BaseShape {
  static constexpr int lg = M == 4 ? 2 : (M == 8 ? 3 : 4);
  static constexpr int G = 256 / (M * M);
  static constexpr int row = M + 1;
  static constexpr int node = M * M * row;
  static constexpr int maxP = 8192 / M;  // phase table entries, P = 8 * 2^Lt for n <= 1024
};

template <int M>
__device__ __forceinline__ int base_idx(int a0, int a1, int a2) {
  return (a0 * M + a1) * BaseShape<M>::row + a2;
}

// One DFT_M pass along axis AX (0: a, 1: b, 2: c) of every line of the block,
// in place, kernel exp(+2 pi i j k / M).
template <typename R, int M, int AX>
__device__ __forceinline__ void base_dft_axis(cx<R>* buf, int G) {
  using S = BaseShape<M>;
  for (int l = threadIdx.x; l < G * M * M; l += blockDim.x) {
    const int g = l / (M * M), p = (l / M) % M, q = l % M;
    int base, stride;
    if constexpr (AX == 2) {
      base = g * S::node + (p * M + q) * S::row;
      stride = 1;
    } else if constexpr (AX == 1) {
      base = g * S::node + p * M * S::row + q;
      stride = S::row;
    } else {
      base = g * S::node + p * S::row + q;
      stride = M * S::row;
    }
    cx<R> v[M];
#pragma unroll
    for (int i = 0; i < M; ++i) v[i] = buf[base + i * stride];
    RegDFT<R, M, 1>::run(v);
#pragma unroll
    for (int i = 0; i < M; ++i) buf[base + i * stride] = v[i];
  }
}

// acc += a b in four fused multiply-adds
template <typename R>
__device__ __forceinline__ void base_cmac(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

typedef short base_s2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ base_s2 base_pack(int lo, int hi) { return base_s2{short(lo), short(hi)}; }

// The base of nvol volumes: in holds the output of level Lt - 1, out receives
// X.  orb: per orbit of W on the M-torus its representative (flat index) and
// the mask of the images h whose point an earlier image already has (orbits
// sorted by mask, so that the lanes of a wave skip the same images).
// G = min(BaseShape<M>::G, 2^Lt) nodes per logical block; launches have a
// multiple of 8 blocks (fold_block).
template <typename R, typename TI, typename TO, int M>
__global__ __launch_bounds__(256) void k_fwd_base(VolSet vs, int nvol, int n, int Lt, int G, int r80, int r81,
                                                  int r82, const int2* __restrict__ orb, int norb) {
  using S = BaseShape<M>;
  __shared__ cx<R> buf[S::G * S::node];
  __shared__ cx<R> tw[S::maxP];
  __shared__ cx<R> ax[S::G * 3 * M];
  const int P = 8 << Lt, mask = (1 << Lt) - 1;
  const long long groups = (1LL << (3 * Lt)) / G;
  const long long blk = fold_block(groups * nvol);
  if (blk < 0) return;
  const long long vol = blk / groups;
  const long long jf = (blk - vol * groups) * G;  // first node of the block, J_z fastest
  const int J0 = int(jf >> (2 * Lt)), J1 = int((jf >> Lt) & mask), J2 = int(jf & mask);
  const int r8[3] = {r80, r81, r82};
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, vol));
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, vol));
  constexpr int lg = S::lg, M3 = M * M * M;
  // every load of a thread in flight before the first store to LDS
  constexpr int kLd = S::G * M3 / 256;
  cx<R> ld[kLd];
#pragma unroll
  for (int c = 0; c < kLd; ++c) {
    const int t = threadIdx.x + c * 256;
    if (t < G * M3) {
      const int g = t % G, a = t / G;
      const int a0 = a >> (2 * lg), a1 = (a >> lg) & (M - 1), a2 = a & (M - 1);
      ld[c] = IO<TI, R>::ld(in, ((long long)(J0 + (a0 << Lt)) * n + (J1 + (a1 << Lt))) * n + (J2 + g + (a2 << Lt)));
    }
  }
  // the phase tables while the loads are in flight
  for (int t = threadIdx.x; t < P; t += blockDim.x) {
    double s, c;
    sincospi(2.0 * double(t) / double(P), &s, &c);
    tw[t] = {R(c), R(s)};
  }
  for (int t = threadIdx.x; t < G * 3 * M; t += blockDim.x) {
    const int g = t / (3 * M), d = (t / M) % 3, k = t % M;
    const int Jd = d == 0 ? J0 : (d == 1 ? J1 : J2 + g);
    const long long e = ((long long)k * (r8[d] + 8 * Jd)) & (8LL * n - 1);
    double s, c;
    sincospi(2.0 * double(e) / double(8LL * n), &s, &c);
    ax[t] = {R(c), R(s)};
  }
#pragma unroll
  for (int c = 0; c < kLd; ++c) {
    const int t = threadIdx.x + c * 256;
    if (t < G * M3) {
      const int g = t % G, a = t / G;
      buf[g * S::node + base_idx<M>(a >> (2 * lg), (a >> lg) & (M - 1), a & (M - 1))] = ld[c];
    }
  }
  __syncthreads();
  if (int(threadIdx.x) < G * norb) {
    const int g = threadIdx.x / norb, o = threadIdx.x - g * norb;
    const int2 ob = orb[o];
    const int k[3] = {ob.x >> (2 * lg), (ob.x >> lg) & (M - 1), ob.x & (M - 1)};
    const int rho[3] = {r8[0] + 8 * J0, r8[1] + 8 * J1, r8[2] + 8 * (J2 + g)};
    cx<R>* nb = buf + g * S::node;
    const cx<R>* axg = ax + g * 3 * M;
    cx<R> xv[24];
    // Z_u as 16-bit pairs: (z0, z1) per u, z2 of u = 2i, 2i+1 in one word
    base_s2 za[24], zb[12];
#pragma unroll
    for (int u = 0; u < 24; ++u) {
      int v[3];
      fold_act(u, k, v);
      xv[u] = nb[base_idx<M>(v[0] & (M - 1), v[1] & (M - 1), v[2] & (M - 1))];
      const int w[3] = {v[0] >> lg, v[1] >> lg, v[2] >> lg};
      int z[3];
      fold_act(kFoldWinv[u], w, z);
      za[u] = base_pack(z[0], z[1]);
      if (u & 1)
        zb[u >> 1].y = short(z[2]);
      else
        zb[u >> 1] = base_pack(z[2], 0);
    }
    const unsigned dup = unsigned(ob.y);
    // one output image per iteration (the group element from a table in
    // constant memory), all 24 sources in registers
#pragma nounroll
    for (int h = 0; h < 24; ++h) {
      if ((dup >> h) & 1u) continue;
      int v[3];
      fold_act(h, k, v);
      const int kh[3] = {v[0] & (M - 1), v[1] & (M - 1), v[2] & (M - 1)};
      const int* gh = kFoldW[h].g;
      int q[3];  // h^T rho
#pragma unroll
      for (int i = 0; i < 3; ++i) q[i] = gh[i] * rho[0] + gh[3 + i] * rho[1] + gh[6 + i] * rho[2];
      const int base = (v[0] >> lg) * rho[0] + (v[1] >> lg) * rho[1] + (v[2] >> lg) * rho[2];  // W_h . rho
      const base_s2 qa = base_pack(-q[0], -q[1]), qe = base_pack(-q[2], 0), qo = base_pack(0, -q[2]);
      // eight phase loads in flight, two accumulators
      cx<R> acc[2] = {{R(0), R(0)}, {R(0), R(0)}};
#pragma unroll
      for (int c = 0; c < 24; c += 8) {
        cx<R> t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int u = c + i;
          const int e = __builtin_amdgcn_sdot2(za[u], qa, __builtin_amdgcn_sdot2(zb[u >> 1], (u & 1) ? qo : qe, base, false),
                                               false);
          t[i] = tw[e & (P - 1)];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) base_cmac(acc[i & 1], xv[c + i], t[i]);
      }
      const cx<R> sum = acc[0] + acc[1];
      const cx<R> a = axg[kh[0]] * axg[M + kh[1]] * axg[2 * M + kh[2]];
      nb[base_idx<M>(kh[0], kh[1], kh[2])] = (R(1) / R(24)) * (a * sum);
    }
  }
  __syncthreads();
  base_dft_axis<R, M, 2>(buf, G);
  __syncthreads();
  base_dft_axis<R, M, 1>(buf, G);
  __syncthreads();
  base_dft_axis<R, M, 0>(buf, G);
  __syncthreads();
  for (int t = threadIdx.x; t < G * M3; t += blockDim.x) {
    const int g = t % G, a = t / G;
    const int a0 = a >> (2 * lg), a1 = (a >> lg) & (M - 1), a2 = a & (M - 1);
    const long long gp = ((long long)(J0 + (a0 << Lt)) * n + (J1 + (a1 << Lt))) * n + (J2 + g + (a2 << Lt));
    IO<TO, R>::st(out, gp, buf[g * S::node + base_idx<M>(a0, a1, a2)]);
  }
}

}  // namespace fcc
