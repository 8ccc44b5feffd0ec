// Device side of the fold+FFT formulation (FCC_FOLD_FFT; a variant that
// follows from the explicit matrix of Sec. IV-A, not the paper's
// factorisation).  With 8 rst = r8 integral:
//
// forward  X = N IDFT_3(Fh), and for g^{-1} mu = k_g + n w_g (k_g in [0,n)^3)
//          Fh[mu] = (1/24) exp(2 pi i mu.rst / n) sum_g w8^{-(w_g . g^T r8)} x[k_g]
//          (w8 = exp(2 pi i / 8)): one gather pass (k_fold), then one DFT pass
//          per axis (k_dft, in place on the output);
// inverse  Fh' = DFT_3(X) exp(-2 pi i mu.rst / n) (the phase applied per axis
//          by the DFT passes), then per point
//          x[k] = sum_u K[pid[k]][u] w8^{-(f_u . r8)} Fh'[u k mod n],  u k = (u k mod n) + n f_u,
//          with the host-built unfold rows K (scaled by 1/N; fold_plan.hpp).
//
// DFT passes: a block owns a tile of whole lines along one axis (4096 points
// in FP32, 2048 in FP64) and runs a Stockham autosort FFT on it, radix 8 or
// 16 in registers per stage, LDS between stages; the first stage reads global
// memory and the last writes it, so a pass moves each element once in and
// once out.  Lines along the strided axes are taken in runs of consecutive c
// so that every global access is a contiguous run.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace fcc {

struct FoldW {
  int g[9];
};
#define FCC_FOLD_G(u, a0, a1, a2, a3, a4, a5, a6, a7, a8, ui) FoldW{{a0, a1, a2, a3, a4, a5, a6, a7, a8}},
constexpr FoldW kFoldW[24] = {FCC_GROUP(FCC_FOLD_G)};
#undef FCC_FOLD_G
#define FCC_FOLD_GI(u, a0, a1, a2, a3, a4, a5, a6, a7, a8, ui) ui,
constexpr int kFoldWinv[24] = {FCC_GROUP(FCC_FOLD_GI)};
#undef FCC_FOLD_GI

constexpr int kFoldMaxPat = 64;  // unfold rows held in LDS

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// a * exp(-i pi m / 4) for m in [0, 8)
template <typename R>
__device__ __forceinline__ cx<R> rot8m(cx<R> a, int m) {
  constexpr R h = R(0.70710678118654752440);
  if (m & 1) a = {(a.x + a.y) * h, (a.y - a.x) * h};
  if (m & 2) a = {a.y, -a.x};
  if (m & 4) a = {-a.x, -a.y};
  return a;
}

// a * exp(S 2 pi i Q / 16), Q in [0, 8)
template <typename R, int Q, int S>
__device__ __forceinline__ cx<R> twq(cx<R> a) {
  constexpr R h = R(0.70710678118654752440), c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173);
  if constexpr (Q == 0) {
    return a;
  } else if constexpr (Q == 4) {
    return S > 0 ? cx<R>{-a.y, a.x} : cx<R>{a.y, -a.x};
  } else if constexpr (Q == 2) {
    return {(a.x - S * a.y) * h, (a.y + S * a.x) * h};
  } else if constexpr (Q == 6) {
    return {(-a.x - S * a.y) * h, (-a.y + S * a.x) * h};
  } else {
    constexpr R c = Q == 1 ? c1 : Q == 3 ? s1 : Q == 5 ? -s1 : -c1;
    constexpr R s = R(S) * (Q == 1 ? s1 : Q == 3 ? c1 : Q == 5 ? c1 : s1);
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

// In-register DFT of size M (power of two <= 16) with kernel exp(S 2 pi i jk / M).
template <typename R, int M, int S>
struct RegDFT {
  static __device__ __forceinline__ void run(cx<R>* v) {
    cx<R> e[M / 2], o[M / 2];
#pragma unroll
    for (int i = 0; i < M / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    RegDFT<R, M / 2, S>::run(e);
    RegDFT<R, M / 2, S>::run(o);
    static_for<0, M / 2>([&](auto K) {
      constexpr int k = decltype(K)::value;
      const cx<R> t = twq<R, k*(16 / M), S>(o[k]);
      v[k] = e[k] + t;
      v[k + M / 2] = e[k] - t;
    });
  }
};
template <typename R, int S>
struct RegDFT<R, 1, S> {
  static __device__ __forceinline__ void run(cx<R>*) {}
};

// Radices of the DFT of size N, first stage first.
template <int N>
struct FftPlan;
template <> struct FftPlan<2> { static constexpr int ns = 1; static constexpr int r[3] = {2, 1, 1}; };
template <> struct FftPlan<4> { static constexpr int ns = 1; static constexpr int r[3] = {4, 1, 1}; };
template <> struct FftPlan<8> { static constexpr int ns = 1; static constexpr int r[3] = {8, 1, 1}; };
template <> struct FftPlan<16> { static constexpr int ns = 1; static constexpr int r[3] = {16, 1, 1}; };
template <> struct FftPlan<32> { static constexpr int ns = 2; static constexpr int r[3] = {8, 4, 1}; };
template <> struct FftPlan<64> { static constexpr int ns = 2; static constexpr int r[3] = {8, 8, 1}; };
template <> struct FftPlan<128> { static constexpr int ns = 2; static constexpr int r[3] = {16, 8, 1}; };
template <> struct FftPlan<256> { static constexpr int ns = 2; static constexpr int r[3] = {16, 16, 1}; };
template <> struct FftPlan<512> { static constexpr int ns = 3; static constexpr int r[3] = {8, 8, 8}; };

template <int N, int S>
constexpr int fft_span() {
  int p = 1;
  for (int i = 0; i < S; ++i) p *= FftPlan<N>::r[i];
  return p;
}

template <typename R>
constexpr int fold_tile() {
  return sizeof(R) == 4 ? 4096 : 2048;
}
template <typename R, int N>
constexpr int dft_lines() {  // lines per block
  return fold_tile<R>() / N < N * N ? fold_tile<R>() / N : N * N;
}

// One DFT pass of size N along axis AX (0: a, stride N^2; 1: b, stride N;
// 2: c, contiguous) with kernel exp(S 2 pi i mu j / N), on every line of nvol
// volumes; may run in place.  With post_r8 != 0 the outputs are multiplied by
// exp(-2 pi i mu post_r8 / (8N)) (mu the output index along the axis).
template <typename R, int N, int AX, int S>
__global__ __launch_bounds__(256) void k_dft(VolSet vs, int nvol, const cx<R>* __restrict__ w8n, int post_r8) {
  constexpr int L = dft_lines<R, N>();
  constexpr int P = L * N;  // points per block
  constexpr int PADN = N + 1;
  constexpr int blocks_per_vol = N * N / L;
  __shared__ cx<R> lds[L * PADN];
  __shared__ cx<R> tw[N];
  const int vol = blockIdx.x / blocks_per_vol;
  const int blk = blockIdx.x - vol * blocks_per_vol;
  if (vol >= nvol) return;
  const cx<R>* in = static_cast<const cx<R>*>(vol_ptr(vs.in, vol));
  cx<R>* out = static_cast<cx<R>*>(vol_ptr(vs.out, vol));
  for (int m = threadIdx.x; m < N; m += 256) {
    const cx<R> w = w8n[8 * m];
    tw[m] = S > 0 ? w : conj(w);
  }
  // global offset of position pos of block line l
  auto goff = [&](int l, int pos) -> long long {
    const long long gl = (long long)blk * L + l;
    if constexpr (AX == 2) {
      return gl * N + pos;
    } else {
      const long long e = gl / N, c = gl - e * N;
      return AX == 1 ? e * N * N + (long long)pos * N + c : e * N + (long long)pos * N * N + c;
    }
  };
  static_for<0, FftPlan<N>::ns>([&](auto SI) {
    constexpr int s = decltype(SI)::value;
    constexpr int RS = FftPlan<N>::r[s];
    constexpr int Ns = fft_span<N, s>();  // product of the earlier radices
    constexpr int NR = N / RS;
    constexpr int ITEMS = (P / RS + 255) / 256;
    constexpr bool first = s == 0, last = s == FftPlan<N>::ns - 1;
    cx<R> v[ITEMS][RS];
    int li[ITEMS], ji[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int item = threadIdx.x + it * 256;
      int l, j;
      if constexpr (AX == 2) {
        l = item / NR;
        j = item - l * NR;
      } else {
        j = item / L;
        l = item - j * L;
      }
      li[it] = l;
      ji[it] = j;
      if (item < P / RS) {
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          if constexpr (first)
            v[it][r] = in[goff(l, j + r * NR)];
          else
            v[it][r] = lds[l * PADN + j + r * NR];
        }
      }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      if (threadIdx.x + it * 256 < P / RS) {
        if constexpr (!first) {
          const int k = ji[it] % Ns;
#pragma unroll
          for (int r = 1; r < RS; ++r) v[it][r] = v[it][r] * tw[r * k * (N / (Ns * RS))];
        }
        RegDFT<R, RS, S>::run(v[it]);
      }
    }
    // Every read of this stage is consumed before any write: LDS reads of a
    // later stage, or (one stage only) global reads of a pass in place.
    if constexpr (!first || last) __syncthreads();
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      if (threadIdx.x + it * 256 < P / RS) {
        const int j = ji[it], l = li[it];
        const int idx = (j / Ns) * Ns * RS + j % Ns;
#pragma unroll
        for (int r = 0; r < RS; ++r) {
          const int pos = idx + r * Ns;
          if constexpr (last) {
            cx<R> o = v[it][r];
            if (post_r8) o = o * conj(w8n[(pos * post_r8) & (8 * N - 1)]);
            out[goff(l, pos)] = o;
          } else {
            lds[l * PADN + pos] = v[it][r];
          }
        }
      }
    }
    if constexpr (!last) __syncthreads();
  });
}

// Orbit lanes.  Each lane owns one orbit of W on the torus, by its
// representative rep (ordered by box, so a wave's orbits are close), and all
// 24 images u rep mod n = u rep - n W_u (W_u = floor(u rep / n)): it loads the
// input at every image once, forms the 24 outputs from them in registers and
// stores them.  With the image index in the unrolled loops a compile-time
// constant, the phase of each (output h, source u) pair costs a few integer
// operations:
//   forward  Fh[h rep] = (1/24) e(h rep) sum_u w8^{-(Z_u . h^T r8 - W_h . r8)} x[u rep],
//            Z_u = u^{-1} W_u,
//   inverse  x[h rep] = sum_u K[pid][u] w8^{-(W_{uh} . r8 - W_h . u^T r8)} Fh'[(u h) rep],
// (e(mu) = exp(2 pi i mu.rst / n); w8^{-j} from an 8-entry table in LDS).
// Images that coincide (orbits with a stabiliser) are stored once per image
// by the same lane, last one kept.
constexpr int kFoldLanes = 256;  // lanes per block (64 for small launches)

struct FoldMul {
  unsigned char m[24][24];
};
// m[a][b] = index of W[a] W[b]
constexpr FoldMul fold_mul() {
  FoldMul t{};
  for (int a = 0; a < 24; ++a)
    for (int b = 0; b < 24; ++b) {
      int P[9] = {};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) P[3 * i + j] += kFoldW[a].g[3 * i + k] * kFoldW[b].g[3 * k + j];
      for (int c = 0; c < 24; ++c) {
        bool eq = true;
        for (int q = 0; q < 9; ++q) eq = eq && kFoldW[c].g[q] == P[q];
        if (eq) t.m[a][b] = (unsigned char)c;
      }
    }
  return t;
}
constexpr FoldMul kFoldMul = fold_mul();

// Logical block: launches have a multiple of 8 blocks, blocks i, i+8, ...
// run on one XCD and take one contiguous range of orbits, so that the
// neighbouring orbits that share cache lines meet in one L2.
__device__ __forceinline__ long long fold_block(long long total) {
  const long long per = (total + 7) >> 3;
  const long long b = (long long)(blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  return b < total ? b : -1;
}

__device__ __forceinline__ void fold_act(int u, const int k[3], int v[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    v[i] = kFoldW[u].g[3 * i] * k[0] + kFoldW[u].g[3 * i + 1] * k[1] + kFoldW[u].g[3 * i + 2] * k[2];
}
// z . (g^T r8) with g = W[u]: the default skew r8 = (1, 0, 3) folds to constants
template <bool DEF>
__device__ __forceinline__ int fold_qdot(int u, const int z[3], const int r8[3]) {
  const int* g = kFoldW[u].g;
  if constexpr (DEF) {
    return (g[0] + 3 * g[6]) * z[0] + (g[1] + 3 * g[7]) * z[1] + (g[2] + 3 * g[8]) * z[2];
  } else {
    int s = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) s += (g[i] * r8[0] + g[3 + i] * r8[1] + g[6 + i] * r8[2]) * z[i];
    return s;
  }
}
template <bool DEF>
__device__ __forceinline__ int fold_rdot(const int w[3], const int r8[3]) {
  if constexpr (DEF) return w[0] + 3 * w[2];
  return w[0] * r8[0] + w[1] * r8[1] + w[2] * r8[2];
}
// A copy of k the compiler cannot see through, so that the images a later
// loop needs are recomputed there instead of being held from an earlier one.
__device__ __forceinline__ void fold_launder(const int k[3], int o[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    int t = k[i];
    asm volatile("" : "+v"(t));
    o[i] = t;
  }
}
template <typename R>
__device__ __forceinline__ void fold_rot_table(cx<R>* t) {
  if (threadIdx.x < 8) {
    constexpr R h = R(0.70710678118654752440);
    const R c[8] = {1, h, 0, -h, -1, -h, 0, h};
    t[threadIdx.x] = {c[threadIdx.x], -c[(threadIdx.x + 6) & 7]};  // exp(-i pi j / 4)
  }
}

// Forward fold of nvol volumes (out is complex R).
template <typename R, typename TI, bool DEF>
__global__ __launch_bounds__(kFoldLanes) void k_fold(VolSet vs, int nvol, int lg, int r80, int r81, int r82,
                                                     const cx<R>* __restrict__ w8n, const int* __restrict__ reps,
                                                     int nrep) {
  __shared__ cx<R> rot[8];
  fold_rot_table(rot);
  __syncthreads();
  const int lanes = blockDim.x, bpv = (nrep + lanes - 1) / lanes;
  const long long blk = fold_block((long long)bpv * nvol);
  if (blk < 0) return;
  const int vol = int(blk / bpv);
  const int r = int(blk - (long long)vol * bpv) * lanes + threadIdx.x;
  const int n = 1 << lg, mask = n - 1;
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, vol));
  cx<R>* __restrict__ out = static_cast<cx<R>*>(vol_ptr(vs.out, vol));
  const int r8[3] = {r80, r81, r82};
  const int rep = reps[min(r, nrep - 1)];
  const int k[3] = {rep >> (2 * lg), (rep >> lg) & mask, rep & mask};
  // real input stays real: each term is then two multiply-adds
  constexpr bool kReal = std::is_same<TI, float>::value || std::is_same<TI, double>::value;
  using V = typename std::conditional<kReal, R, cx<R>>::type;
  V xv[24];
  int A8[3] = {0, 0, 0};  // W_u . r8 mod 8, eight 4-bit fields per word
#pragma unroll
  for (int u = 0; u < 24; ++u) {
    int v[3];
    fold_act(u, k, v);
    const cx<R> t = IO<TI, R>::ld(in, ((long long)(v[0] & mask) * n + (v[1] & mask)) * n + (v[2] & mask));
    if constexpr (kReal)
      xv[u] = t.x;
    else
      xv[u] = t;
    const int w[3] = {v[0] >> lg, v[1] >> lg, v[2] >> lg};
    A8[u >> 3] |= (fold_rdot<DEF>(w, r8) & 7) << (4 * (u & 7));
  }
  cx<R> acc[24];
#pragma unroll
  for (int h = 0; h < 24; ++h) acc[h] = {R(0), R(0)};
  int k1[3], k2[3];
  fold_launder(k, k1);
#pragma unroll
  for (int u = 0; u < 24; ++u) {
    int v[3];
    fold_act(u, k1, v);
    const int w[3] = {v[0] >> lg, v[1] >> lg, v[2] >> lg};
    int z[3];  // u^{-1} W_u
    fold_act(kFoldWinv[u], w, z);
#pragma unroll
    for (int h = 0; h < 24; ++h) {
      const cx<R> c = rot[(fold_qdot<DEF>(h, z, r8) - (A8[h >> 3] >> (4 * (h & 7)))) & 7];
      if constexpr (kReal)
        acc[h] = {acc[h].x + c.x * xv[u], acc[h].y + c.y * xv[u]};
      else
        acc[h] = acc[h] + c * xv[u];
    }
  }
  if (r >= nrep) return;
  fold_launder(k, k2);
#pragma unroll
  for (int h = 0; h < 24; ++h) {
    int v[3];
    fold_act(h, k2, v);
    const int mu[3] = {v[0] & mask, v[1] & mask, v[2] & mask};
    const int e = (mu[0] * r8[0] + mu[1] * r8[1] + mu[2] * r8[2]) & (8 * n - 1);
    out[((long long)mu[0] * n + mu[1]) * n + mu[2]] = (R(1) / R(24)) * (w8n[e] * acc[h]);
  }
}

// Inverse unfold: x[k] from Fh' (complex R) with the unfold rows K.
template <typename R, typename TO, bool DEF>
__global__ __launch_bounds__(kFoldLanes) void k_unfold(VolSet vs, int nvol, int lg, int r80, int r81, int r82,
                                                       const cx<R>* __restrict__ kt, int npat,
                                                       const int* __restrict__ reps,
                                                       const unsigned char* __restrict__ prid, int nrep) {
  __shared__ cx<R> ks[kFoldMaxPat * 24];
  __shared__ cx<R> rot[8];
  for (int q = threadIdx.x; q < npat * 24; q += blockDim.x) ks[q] = kt[q];
  fold_rot_table(rot);
  __syncthreads();
  const int lanes = blockDim.x, bpv = (nrep + lanes - 1) / lanes;
  const long long blk = fold_block((long long)bpv * nvol);
  if (blk < 0) return;
  const int vol = int(blk / bpv);
  const int r = int(blk - (long long)vol * bpv) * lanes + threadIdx.x;
  const int rc = min(r, nrep - 1);
  const int n = 1 << lg, mask = n - 1;
  const cx<R>* __restrict__ in = static_cast<const cx<R>*>(vol_ptr(vs.in, vol));
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, vol));
  const int r8[3] = {r80, r81, r82};
  const int rep = reps[rc];
  const int k[3] = {rep >> (2 * lg), (rep >> lg) & mask, rep & mask};
  cx<R> y[24];
  int B8[3] = {0, 0, 0}, pr4[6] = {0, 0, 0, 0, 0, 0};  // W_v . r8 mod 8 (4-bit fields); row indices (bytes)
#pragma unroll
  for (int v = 0; v < 24; ++v) {
    int t[3];
    fold_act(v, k, t);
    y[v] = in[((long long)(t[0] & mask) * n + (t[1] & mask)) * n + (t[2] & mask)];
    const int w[3] = {t[0] >> lg, t[1] >> lg, t[2] >> lg};
    B8[v >> 3] |= (fold_rdot<DEF>(w, r8) & 7) << (4 * (v & 7));
    pr4[v >> 2] |= int(prid[(long long)v * nrep + rc]) << (8 * (v & 3));
  }
  int k1[3];
  fold_launder(k, k1);
#pragma unroll
  for (int h = 0; h < 24; ++h) {
    int t[3];
    fold_act(h, k1, t);
    const int w[3] = {t[0] >> lg, t[1] >> lg, t[2] >> lg};
    const cx<R>* krow = ks + 24 * ((pr4[h >> 2] >> (8 * (h & 3))) & 255);
    cx<R> acc{R(0), R(0)};
#pragma unroll
    for (int u = 0; u < 24; ++u) {
      const int v = kFoldMul.m[u][h];
      const cx<R> c = krow[u] * rot[(((B8[v >> 3] >> (4 * (v & 7))) & 7) - fold_qdot<DEF>(u, w, r8)) & 7];
      acc = acc + c * y[v];
    }
    if (r < nrep) IO<TO, R>::st(out, ((long long)(t[0] & mask) * n + (t[1] & mask)) * n + (t[2] & mask), acc);
  }
}

}  // namespace fcc
