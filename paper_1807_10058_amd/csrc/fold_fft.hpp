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

// Orbit blocks.  A block takes kFoldReps orbits of W on the torus (by their
// representatives, ordered by 8^3 box so that a block's orbits are close)
// and all 24 images h r of each: it loads the input at every image once into
// LDS, forms each output from the 24 members of its orbit there, and stores
// it.  Lane (h, i) owns image h of orbit i; a wave holds one h, so the LDS
// slot of a source (an element of W fixed by g and h) is the same for the
// whole wave.  Images that coincide (orbits with a stabiliser) are loaded and
// stored more than once, with equal values.
constexpr int kFoldReps = 64;
constexpr int kFoldItems = 24 * kFoldReps / 256;

struct FoldMul {
  unsigned char m[24][24];
};
// m[a][b] = index of W[a]^{inv ? -1 : 1} W[b]
constexpr FoldMul fold_mul(bool inv) {
  FoldMul t{};
  for (int a = 0; a < 24; ++a)
    for (int b = 0; b < 24; ++b) {
      const int* A = kFoldW[inv ? kFoldWinv[a] : a].g;
      const int* B = kFoldW[b].g;
      int P[9] = {};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) P[3 * i + j] += A[3 * i + k] * B[3 * k + j];
      for (int c = 0; c < 24; ++c) {
        bool eq = true;
        for (int q = 0; q < 9; ++q) eq = eq && kFoldW[c].g[q] == P[q];
        if (eq) t.m[a][b] = (unsigned char)c;
      }
    }
  return t;
}
constexpr FoldMul kFoldMulInv = fold_mul(true);   // g^{-1} h
constexpr FoldMul kFoldMul = fold_mul(false);     // u h
#define FCC_FOLD_GC(u, a0, a1, a2, a3, a4, a5, a6, a7, a8, ui) {a0, a1, a2, a3, a4, a5, a6, a7, a8},
__constant__ int kFoldWc[24][9] = {FCC_GROUP(FCC_FOLD_GC)};
#undef FCC_FOLD_GC

// Image h of representative rep (flat index), reduced mod n.
__device__ __forceinline__ void fold_image(int h, int rep, int lg, int mu[3]) {
  const int n = 1 << lg;
  const int k[3] = {rep >> (2 * lg), (rep >> lg) & (n - 1), rep & (n - 1)};
#pragma unroll
  for (int i = 0; i < 3; ++i)
    mu[i] = (kFoldWc[h][3 * i] * k[0] + kFoldWc[h][3 * i + 1] * k[1] + kFoldWc[h][3 * i + 2] * k[2]) & (n - 1);
}

// Forward fold of nvol volumes (out is complex R).
template <typename R, typename TI>
__global__ __launch_bounds__(256) void k_fold(VolSet vs, int nvol, int lg, int r80, int r81, int r82,
                                              const cx<R>* __restrict__ w8n, const int* __restrict__ reps,
                                              int nrep) {
  __shared__ cx<R> xs[24][kFoldReps];
  __shared__ unsigned char tab[24 * 24];
  const int bpv = (nrep + kFoldReps - 1) / kFoldReps;
  const int vol = blockIdx.x / bpv, r0 = (blockIdx.x - vol * bpv) * kFoldReps;
  if (vol >= nvol) return;
  const int n = 1 << lg;
  const TI* __restrict__ in = static_cast<const TI*>(vol_ptr(vs.in, vol));
  cx<R>* __restrict__ out = static_cast<cx<R>*>(vol_ptr(vs.out, vol));
  for (int q = threadIdx.x; q < 24 * 24; q += 256) tab[q] = kFoldMulInv.m[q / 24][q % 24];
  int mu[kFoldItems][3];
#pragma unroll
  for (int it = 0; it < kFoldItems; ++it) {
    const int item = threadIdx.x + it * 256;
    const int h = __builtin_amdgcn_readfirstlane(item / kFoldReps), i = item % kFoldReps;
    const int r = min(r0 + i, nrep - 1);
    fold_image(h, reps[r], lg, mu[it]);
    xs[h][i] = IO<TI, R>::ld(in, ((long long)mu[it][0] * n + mu[it][1]) * n + mu[it][2]);
  }
  __syncthreads();
  const int r8[3] = {r80, r81, r82};
#pragma unroll 1
  for (int it = 0; it < kFoldItems; ++it) {
    const int item = threadIdx.x + it * 256;
    const int h = __builtin_amdgcn_readfirstlane(item / kFoldReps), i = item % kFoldReps;
    cx<R> acc{R(0), R(0)};
    static_for<0, 24>([&](auto G) {
      constexpr int g = decltype(G)::value;
      constexpr FoldW gi = kFoldW[kFoldWinv[g]];
      constexpr FoldW gg = kFoldW[g];
      int w[3];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        w[d] = (gi.g[3 * d] * mu[it][0] + gi.g[3 * d + 1] * mu[it][1] + gi.g[3 * d + 2] * mu[it][2]) >> lg;
      int m = 0;  // (g w) . r8
#pragma unroll
      for (int d = 0; d < 3; ++d) m += (gg.g[3 * d] * w[0] + gg.g[3 * d + 1] * w[1] + gg.g[3 * d + 2] * w[2]) * r8[d];
      acc = acc + rot8m(xs[tab[g * 24 + h]][i], m & 7);
    });
    if (r0 + i < nrep) {
      const int e = (mu[it][0] * r8[0] + mu[it][1] * r8[1] + mu[it][2] * r8[2]) & (8 * n - 1);
      out[((long long)mu[it][0] * n + mu[it][1]) * n + mu[it][2]] = (R(1) / R(24)) * (w8n[e] * acc);
    }
  }
}

// Inverse unfold: x[k] from Fh' (complex R) with the unfold rows K.
template <typename R, typename TO>
__global__ __launch_bounds__(256) void k_unfold(VolSet vs, int nvol, int lg, int r80, int r81, int r82,
                                                const cx<R>* __restrict__ kt, int npat,
                                                const int* __restrict__ reps, const unsigned char* __restrict__ prid,
                                                int nrep) {
  __shared__ cx<R> fs[24][kFoldReps];
  __shared__ cx<R> ks[kFoldMaxPat * 24];
  __shared__ unsigned char tab[24 * 24];
  const int bpv = (nrep + kFoldReps - 1) / kFoldReps;
  const int vol = blockIdx.x / bpv, r0 = (blockIdx.x - vol * bpv) * kFoldReps;
  if (vol >= nvol) return;
  const int n = 1 << lg;
  const cx<R>* __restrict__ in = static_cast<const cx<R>*>(vol_ptr(vs.in, vol));
  TO* __restrict__ out = static_cast<TO*>(vol_ptr(vs.out, vol));
  for (int q = threadIdx.x; q < npat * 24; q += 256) ks[q] = kt[q];
  for (int q = threadIdx.x; q < 24 * 24; q += 256) tab[q] = kFoldMul.m[q / 24][q % 24];
  int kk[kFoldItems][3];
  int pr[kFoldItems];
#pragma unroll
  for (int it = 0; it < kFoldItems; ++it) {
    const int item = threadIdx.x + it * 256;
    const int h = __builtin_amdgcn_readfirstlane(item / kFoldReps), i = item % kFoldReps;
    const int r = min(r0 + i, nrep - 1);
    fold_image(h, reps[r], lg, kk[it]);
    pr[it] = prid[(long long)h * nrep + r];
    fs[h][i] = in[((long long)kk[it][0] * n + kk[it][1]) * n + kk[it][2]];
  }
  __syncthreads();
  const int r8[3] = {r80, r81, r82};
#pragma unroll 1
  for (int it = 0; it < kFoldItems; ++it) {
    const int item = threadIdx.x + it * 256;
    const int h = __builtin_amdgcn_readfirstlane(item / kFoldReps), i = item % kFoldReps;
    const cx<R>* krow = ks + 24 * pr[it];
    cx<R> acc{R(0), R(0)};
    static_for<0, 24>([&](auto U) {
      constexpr int u = decltype(U)::value;
      constexpr FoldW g = kFoldW[u];
      int m = 0;  // floor(u k / n) . r8
#pragma unroll
      for (int d = 0; d < 3; ++d)
        m += ((g.g[3 * d] * kk[it][0] + g.g[3 * d + 1] * kk[it][1] + g.g[3 * d + 2] * kk[it][2]) >> lg) * r8[d];
      acc = acc + krow[u] * rot8m(fs[tab[u * 24 + h]][i], m & 7);
    });
    if (r0 + i < nrep) IO<TO, R>::st(out, ((long long)kk[it][0] * n + kk[it][1]) * n + kk[it][2], acc);
  }
}

}  // namespace fcc
