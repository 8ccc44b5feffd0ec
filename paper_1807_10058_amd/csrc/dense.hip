// Dense base transform on the MFMA units (FCC_PREC_SPLIT_BF16 / _FP16).
//
// For small n the whole skew transform is one dense matrix (Sec. IV-A,
// eq. SU4ChebyshevTransformExplicitForm): F[j][k] = T_k(theta_j), N = n^3 rows
// and columns.  Many independent blocks x_b of the same size are transformed at
// once as a real GEMM
//     out[b, :] = W in[b, :],
// with W the real form of F (or of F^{-1}): complex rows and columns are
// interleaved (re, im), so FP32 real or interleaved complex64 blocks are read
// and written in place, with no separate pack pass.
//
// Precision: operands are split into 16-bit hi + lo parts (hi = round(v),
// lo = round(v - hi)); each 16x16 output tile accumulates hi*hi + hi*lo + lo*hi
// in FP32 on v_mfma_f32_16x16x32_{bf16,f16}.  W is scaled by a power of two
// to max |W| = 1 before the split; for FP16 every input row is also scaled by
// a power of two (per-block scaling) so that its largest entry is in [0.5, 1].
//
// Tables: F is evaluated in FP64 on the GPU from the orbit sums; F^{-1} is
// obtained by running the FP64 fast inverse (the level kernels) on the unit
// vectors; W is assembled and split on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "asp_tables.hpp"
#include "plan.hpp"

namespace fcc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct GroupArg {
  int g[24 * 9];
};

// F[j][k] = T_k(theta_j) = (1/24) sum_g exp(2 pi i (g k).(rst + j) / n), FP64.
__global__ void k_dense_matrix(double2* F, int n, double r0, double r1, double r2, GroupArg G) {
  const long long N = (long long)n * n * n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * N) return;
  const long long j = idx / N, k = idx % N;
  const int jv[3] = {int(j / (n * n)), int((j / n) % n), int(j % n)};
  const int kv[3] = {int(k / (n * n)), int((k / n) % n), int(k % n)};
  const double r[3] = {r0, r1, r2};
  double re = 0.0, im = 0.0;
  for (int q = 0; q < 24; ++q) {
    const int* g = G.g + 9 * q;
    long long ip = 0;
    double fp = 0.0;
    for (int i = 0; i < 3; ++i) {
      long long lam = (long long)g[3 * i] * kv[0] + (long long)g[3 * i + 1] * kv[1] + (long long)g[3 * i + 2] * kv[2];
      ip += lam * jv[i];
      fp += double(lam) * r[i];
    }
    ip %= n;
    double a = (double(ip) + fp) / double(n);
    a -= floor(a);
    double s, c;
    sincospi(2.0 * a, &s, &c);
    re += c;
    im += s;
  }
  F[idx] = make_double2(re / 24.0, im / 24.0);
}

// e_j for j in [j0, j0 + cnt): volume v is the unit vector of column j0 + v.
__global__ void k_unit_vectors(double2* E, long long N, long long j0, int cnt) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * cnt) return;
  const long long v = idx / N, e = idx % N;
  E[idx] = make_double2(e == j0 + v ? 1.0 : 0.0, 0.0);
}

// Power-of-two scale per input row so that its largest |entry| lies in [0.5, 1].
__global__ __launch_bounds__(256) void k_rowscale(const float* const* rows, const float* base, long long ld, int K,
                                                  float* scale) {
  const int r = blockIdx.x;
  const float* p = rows ? rows[r] : base + (long long)r * ld;
  float mx = 0.f;
  for (int k = threadIdx.x; k < K; k += blockDim.x) mx = fmaxf(mx, fabsf(p[k]));
  __shared__ float red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float m = red[0];
    scale[r] = (m > 0.f && isfinite(m)) ? ldexpf(1.0f, -ilogbf(m) - 1) : 1.0f;
  }
}

template <typename T16>
struct Vec8;
template <>
struct Vec8<__bf16> {
  typedef bf16x8 type;
  static __device__ __forceinline__ f32x4 mfma(type a, type b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Vec8<_Float16> {
  typedef f16x8 type;
  static __device__ __forceinline__ f32x4 mfma(type a, type b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

constexpr int BM = 128, BN = 128, BK = 32, LDSK = BK + 8;
constexpr int KP_ALIGN = 2 * BK;  // padded K of the stored operands: an even number of K tiles

// The input rows split once into 16-bit hi and lo parts (scaled by the row's
// power of two for FP16), M rounded up to BM with zero rows and K to Kp with
// zeros, so the GEMM reads both operands the same way and masks nothing.
// One block per row, 4 values per thread.
template <typename T16, bool kRows>
__global__ __launch_bounds__(128) void k_split_rows(const float* const* a_rows, const float* a_base, long long lda,
                                                    int M, int K, int Kp, const float* __restrict__ rowscale,
                                                    T16* __restrict__ a_hi, T16* __restrict__ a_lo) {
  const int r = blockIdx.x;
  const bool ok = r < M;
  const float* ap = ok ? (kRows ? a_rows[r] : a_base + (long long)r * lda) : nullptr;
  const float s = (ok && rowscale) ? rowscale[r] : 1.0f;
  for (int k = threadIdx.x * 4; k < Kp; k += 128 * 4) {
    T16 h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float v = (ok && k + i < K) ? ap[k + i] * s : 0.f;
      h[i] = T16(v);
      l[i] = T16(v - float(h[i]));
    }
    T16* hp = a_hi + (long long)r * Kp + k;
    T16* lp = a_lo + (long long)r * Kp + k;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      hp[i] = h[i];
      lp[i] = l[i];
    }
  }
}

// One K tile of both operands in registers: 16 entries of an A row and of a
// W row, hi and lo.  Named members, no arrays, so that nothing is addressed
// through scratch.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct GemmTile {
  u32x4 ah0, ah1, al0, al1, wh0, wh1, wl0, wl1;
};
template <typename T16>
__device__ __forceinline__ void gemm_load(const T16* ahp, const T16* alp, const T16* bhp, const T16* blp, int k0,
                                          GemmTile& t) {
  const u32x4* a = reinterpret_cast<const u32x4*>(ahp + k0);
  const u32x4* b = reinterpret_cast<const u32x4*>(alp + k0);
  const u32x4* c = reinterpret_cast<const u32x4*>(bhp + k0);
  const u32x4* d = reinterpret_cast<const u32x4*>(blp + k0);
  t.ah0 = a[0], t.ah1 = a[1];
  t.al0 = b[0], t.al1 = b[1];
  t.wh0 = c[0], t.wh1 = c[1];
  t.wl0 = d[0], t.wl1 = d[1];
}
template <typename T16>
__device__ __forceinline__ void gemm_store(const GemmTile& t, T16* ahi, T16* alo, T16* bhi, T16* blo) {
  u32x4* a = reinterpret_cast<u32x4*>(ahi);
  u32x4* b = reinterpret_cast<u32x4*>(alo);
  u32x4* c = reinterpret_cast<u32x4*>(bhi);
  u32x4* d = reinterpret_cast<u32x4*>(blo);
  a[0] = t.ah0, a[1] = t.ah1;
  b[0] = t.al0, b[1] = t.al1;
  c[0] = t.wh0, c[1] = t.wh1;
  d[0] = t.wl0, d[1] = t.wl1;
}

// An output row pointer read from memory is a generic (flat) pointer, whose
// stores are counted with the LDS operations; rebuilt as an offset from a
// kernel argument (hidden from the optimiser, which would fold it back) its
// stores are global ones.
template <typename T, typename B>
__device__ __forceinline__ T* gemm_global(T* p, const B* base) {
  long long off = reinterpret_cast<const char*>(p) - reinterpret_cast<const char*>(base);
  asm volatile("" : "+v"(off));
  return reinterpret_cast<T*>(const_cast<char*>(reinterpret_cast<const char*>(base)) + off);
}

template <typename T16>
struct GemmStage {
  T16 a_hi[BM][LDSK], a_lo[BM][LDSK], b_hi[BN][LDSK], b_lo[BN][LDSK];
};

// One K tile: store the prefetched operands into stage S, barrier, start the
// loads of tile kt + 2 into the same registers, multiply from S.
template <typename T16>
__device__ __forceinline__ void gemm_step(GemmStage<T16>& S, GemmTile& cur, f32x4 (&acc)[4][4], int kt, int nk,
                                          int ar, int kc, int lane, int wm, int wn, const T16* ahp, const T16* alp,
                                          const T16* bhp, const T16* blp) {
  typedef typename Vec8<T16>::type V8;
  gemm_store<T16>(cur, &S.a_hi[ar][kc], &S.a_lo[ar][kc], &S.b_hi[ar][kc], &S.b_lo[ar][kc]);
  __syncthreads();
  gemm_load<T16>(ahp, alp, bhp, blp, min(kt + 2, nk - 2 + (kt & 1)) * BK, cur);  // in flight during the MFMAs
  const int kq = (lane >> 4) * 8;
  V8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int r = wm * 64 + mt * 16 + (lane & 15);
    ah[mt] = *reinterpret_cast<const V8*>(&S.a_hi[r][kq]);
    al[mt] = *reinterpret_cast<const V8*>(&S.a_lo[r][kq]);
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int c = wn * 64 + nt * 16 + (lane & 15);
    bh[nt] = *reinterpret_cast<const V8*>(&S.b_hi[c][kq]);
    bl[nt] = *reinterpret_cast<const V8*>(&S.b_lo[c][kq]);
  }
  // hi*hi, then hi*lo, then lo*hi: 16 independent tiles between dependent MFMAs
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = Vec8<T16>::mfma(ah[mt], bh[nt], acc[mt][nt]);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = Vec8<T16>::mfma(ah[mt], bl[nt], acc[mt][nt]);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = Vec8<T16>::mfma(al[mt], bh[nt], acc[mt][nt]);
}

// out[r, c] = (sum_k A[r, k] W[c, k]) * w_unscale / rowscale[r]  for r < M, c < Nc,
// with A and W given as hi + lo (rows of Kp entries; A has a multiple of BM
// rows).  Block 256 threads = 4 waves as 2 (rows) x 2 (cols); each wave owns a
// 64 x 64 tile = 4 x 4 MFMA 16x16 tiles, one 32-deep MFMA step per K tile.
// Operand layout of v_mfma_f32_16x16x32: A lane l holds A[l % 16][8 (l / 16) + i],
// B lane l holds B[8 (l / 16) + i][l % 16], D lane l holds D[4 (l / 16) + v][l % 16].
// Two LDS stages: K tile t is stored into stage t & 1 while the MFMAs of tile
// t - 1 may still read the other one, so one barrier per K tile suffices;
// the operands of tile t + 2 are loaded into registers while tile t is
// multiplied.
template <typename T16, bool kRows>
__global__ __launch_bounds__(256) void k_split_gemm(float* const* c_rows, float* c_base, long long ldc,
                                                    const T16* __restrict__ a_hi, const T16* __restrict__ a_lo,
                                                    const T16* __restrict__ w_hi, const T16* __restrict__ w_lo,
                                                    int M, int Nc, int Kp, const float* __restrict__ rowscale,
                                                    float w_unscale) {
  typedef typename Vec8<T16>::type V8;
  __shared__ __attribute__((aligned(16))) GemmStage<T16> st[2];
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  // thread -> A row m0 + ar and W row n0 + ar, 16 consecutive k from kc
  const int ar = tid >> 1, kc = (tid & 1) * 16;
  const T16* ahp = a_hi + (long long)(m0 + ar) * Kp + kc;
  const T16* alp = a_lo + (long long)(m0 + ar) * Kp + kc;
  const T16* bhp = w_hi + (long long)(n0 + ar) * Kp + kc;
  const T16* blp = w_lo + (long long)(n0 + ar) * Kp + kc;
  // Kp is a multiple of 2 BK: an even number of K tiles, so both steps of the
  // loop body run unconditionally; the prefetch index is clamped (the last
  // two reloads are unused).
  const int nk = Kp / BK;

  GemmTile t0, t1;
  gemm_load<T16>(ahp, alp, bhp, blp, 0, t0);
  gemm_load<T16>(ahp, alp, bhp, blp, BK, t1);
  for (int kt = 0; kt < nk; kt += 2) {
    gemm_step<T16>(st[0], t0, acc, kt, nk, ar, kc, lane, wm, wn, ahp, alp, bhp, blp);
    gemm_step<T16>(st[1], t1, acc, kt + 1, nk, ar, kc, lane, wm, wn, ahp, alp, bhp, blp);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = m0 + wm * 64 + mt * 16 + (lane >> 4) * 4 + v;
      if (r >= M) continue;
      float* cp = kRows ? gemm_global(c_rows[r], w_hi) : c_base + (long long)r * ldc;
      const float f = w_unscale / (rowscale ? rowscale[r] : 1.0f);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int c = n0 + wn * 64 + nt * 16 + (lane & 15);
        if (c < Nc) cp[c] = acc[mt][nt][v] * f;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

uint16_t to_bf16(float f) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
float from_bf16(uint16_t h) {
  uint32_t u = uint32_t(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint16_t to_f16(float f) {
  _Float16 h = (_Float16)f;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}
float from_f16(uint16_t u) {
  _Float16 h;
  std::memcpy(&h, &u, 2);
  return (float)h;
}

// Real GEMM operand of a complex matrix Mc (rows = outputs, cols = inputs,
// element (o, i) at Mc[o * so + i * si]).
std::vector<double> real_form(const std::vector<double2>& Mc, long long so, long long si, int nout, int nin,
                              bool cplx_in, bool cplx_out, int* K, int* Nc) {
  *K = cplx_in ? 2 * nin : nin;
  *Nc = cplx_out ? 2 * nout : nout;
  std::vector<double> W(size_t(*Nc) * *K);
  for (int r = 0; r < *Nc; ++r) {
    const int o = cplx_out ? r / 2 : r, po = cplx_out ? r % 2 : 0;
    for (int c = 0; c < *K; ++c) {
      const int i = cplx_in ? c / 2 : c, pi = cplx_in ? c % 2 : 0;
      const double2 m = Mc[size_t(o) * so + size_t(i) * si];
      double v;
      if (po == 0 && pi == 0) v = m.x;        // re <- re
      else if (po == 0 && pi == 1) v = -m.y;  // re <- im
      else if (po == 1 && pi == 0) v = m.y;   // im <- re
      else v = m.x;                           // im <- im
      W[size_t(r) * *K + c] = v;
    }
  }
  return W;
}

fcc_status upload_split(const std::vector<double>& W, int K, int Nc, bool fp16, DenseOp* op) {
  op->K = K;
  op->Nc = Nc;
  op->Kp = (K + KP_ALIGN - 1) / KP_ALIGN * KP_ALIGN;
  op->Ncp = (Nc + BN - 1) / BN * BN;
  double mx = 0.0;
  for (double v : W) mx = std::max(mx, std::fabs(v));
  const int e = mx > 0.0 ? std::ilogb(mx) + 1 : 0;  // scaled max in [0.5, 1)
  op->w_unscale = std::ldexp(1.0f, e);
  std::vector<uint16_t> hi(size_t(op->Ncp) * op->Kp, 0), lo(hi.size(), 0);
  for (int r = 0; r < Nc; ++r)
    for (int c = 0; c < K; ++c) {
      const double v = std::ldexp(W[size_t(r) * K + c], -e);
      const uint16_t h = fp16 ? to_f16(float(v)) : to_bf16(float(v));
      const double hv = fp16 ? from_f16(h) : from_bf16(h);
      const uint16_t l = fp16 ? to_f16(float(v - hv)) : to_bf16(float(v - hv));
      hi[size_t(r) * op->Kp + c] = h;
      lo[size_t(r) * op->Kp + c] = l;
    }
  const size_t bytes = hi.size() * sizeof(uint16_t);
  if (dev_malloc(&op->w_hi, bytes) != hipSuccess || dev_malloc(&op->w_lo, bytes) != hipSuccess) return FCC_ERR_OOM;
  if (hipMemcpy(op->w_hi, hi.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(op->w_lo, lo.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
    return FCC_ERR_HIP;
  return FCC_OK;
}

}  // namespace

void dense_free(fcc_plan_s* p) {
  for (DenseOp* op : {&p->dfwd, &p->dinv}) {
    if (op->w_hi) (void)hipFree(op->w_hi);
    if (op->w_lo) (void)hipFree(op->w_lo);
    op->w_hi = op->w_lo = nullptr;
  }
  if (p->rowscale) (void)hipFree(p->rowscale);
  p->rowscale = nullptr;
  if (p->dws) (void)hipFree(p->dws);
  p->dws = nullptr;
}

fcc_status dense_prepare(fcc_plan_s* p, hipStream_t st) {
  const int n = p->n;
  const long long N = (long long)n * n * n;
  const bool fp16 = p->prec == FCC_PREC_SPLIT_FP16;
  // forward matrix in FP64 on the GPU
  GroupArg G;
  const auto& W = weyl_group();
  for (int q = 0; q < 24; ++q)
    for (int i = 0; i < 9; ++i) G.g[9 * q + i] = W[q][i];
  double2* F = nullptr;
  double2* E = nullptr;
  double2* Finv = nullptr;
  double2* scratch = nullptr;
  void** parr = nullptr;
  fcc_status s = FCC_OK;
  auto fail = [&](fcc_status e) {
    if (parr) (void)hipFree(parr);
    if (F) (void)hipFree(F);
    if (E) (void)hipFree(E);
    if (Finv) (void)hipFree(Finv);
    if (scratch) (void)hipFree(scratch);
    return e;
  };
  if (dev_malloc(&F, sizeof(double2) * N * N) != hipSuccess) return fail(FCC_ERR_OOM);
  hipLaunchKernelGGL(k_dense_matrix, dim3(unsigned((N * N + 255) / 256)), dim3(256), 0, st, F, n, p->rst[0],
                     p->rst[1], p->rst[2], G);
  if (hipGetLastError() != hipSuccess) return fail(FCC_ERR_HIP);
  // inverse matrix: FP64 fast inverse of the unit vectors (column j of F^{-1})
  if (dev_malloc(&Finv, sizeof(double2) * N * N) != hipSuccess) return fail(FCC_ERR_OOM);
  if (n == 1) {
    const double2 one = make_double2(1.0, 0.0);
    if (hipMemcpy(Finv, &one, sizeof one, hipMemcpyHostToDevice) != hipSuccess) return fail(FCC_ERR_HIP);
  } else {
    fcc_plan_s sub;
    sub.n = p->n;
    sub.D = p->D;
    sub.device = p->device;
    std::memcpy(sub.rst, p->rst, sizeof sub.rst);
    sub.prec = FCC_PREC_FP64;
    sub.flags = 0;
    sub.stages64 = true;
    sub.lv = p->lv;
    sub.hph = p->hph;
    sub.tune = p->tune;
    sub.tail_Lt[0] = p->tail_Lt[0];
    sub.tail_Lt[1] = p->tail_Lt[1];
    sub.tlv = p->tlv;
    // all N unit vectors in one launch sequence; pointer arrays on the device
    if (dev_malloc(&E, sizeof(double2) * N * N) != hipSuccess) return fail(FCC_ERR_OOM);
    if (dev_malloc(&scratch, sizeof(double2) * N * N * 2) != hipSuccess) return fail(FCC_ERR_OOM);
    hipLaunchKernelGGL(k_unit_vectors, dim3(unsigned((N * N + 255) / 256)), dim3(256), 0, st, E, N, 0LL, int(N));
    std::vector<void*> ptr(size_t(4) * N);
    for (long long v = 0; v < N; ++v) {
      ptr[v] = E + N * v;
      ptr[N + v] = Finv + N * v;  // column v of F^{-1}, stored contiguously
      ptr[2 * N + v] = scratch + N * (2 * v);
      ptr[3 * N + v] = scratch + N * (2 * v + 1);
    }
    if (dev_malloc(&parr, sizeof(void*) * ptr.size()) != hipSuccess) return fail(FCC_ERR_OOM);
    if (hipMemcpy(parr, ptr.data(), sizeof(void*) * ptr.size(), hipMemcpyHostToDevice) != hipSuccess)
      return fail(FCC_ERR_HIP);
    s = enqueue_inverse_arrays(&sub, int(N), parr, parr + N, parr + 2 * N, parr + 3 * N, st);
    if (s != FCC_OK) return fail(s);
  }
  if (hipStreamSynchronize(st) != hipSuccess) return fail(FCC_ERR_HIP);
  std::vector<double2> hF(N * N), hFi(N * N);
  if (hipMemcpy(hF.data(), F, sizeof(double2) * N * N, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hFi.data(), Finv, sizeof(double2) * N * N, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(FCC_ERR_HIP);
  fail(FCC_OK);
  const bool real = p->flags & FCC_REAL_INPUT;
  int K, Nc;
  // forward: rows j (outputs), cols k (inputs): F[j * N + k]
  std::vector<double> Wf = real_form(hF, N, 1, int(N), int(N), !real, true, &K, &Nc);
  if ((s = upload_split(Wf, K, Nc, fp16, &p->dfwd)) != FCC_OK) return s;
  // inverse: F^{-1}[k][j] is stored at Finv[j * N + k] (column j contiguous)
  std::vector<double> Wi = real_form(hFi, 1, N, int(N), int(N), true, !real, &K, &Nc);
  if ((s = upload_split(Wi, K, Nc, fp16, &p->dinv)) != FCC_OK) return s;
  return FCC_OK;
}

size_t dense_ws_bytes(const DenseOp& op, int M) {
  const size_t mp = (size_t(std::max(M, 1)) + BM - 1) / BM * BM;
  return 2 * mp * size_t(op.Kp) * sizeof(uint16_t);
}

fcc_status dense_run(const fcc_plan_s* p, const DenseOp& op, int M, const void* const* in_rows_dev,
                     void* const* out_rows_dev, const void* in_base, void* out_base, float* rowscale, void* aws,
                     hipStream_t st, long long lda, long long ldc, hipEvent_t* ev) {
  if (lda <= 0) lda = op.K;
  if (ldc <= 0) ldc = op.Nc;
  if (!aws) return FCC_ERR_INVALID_ARG;
  const bool fp16 = p->prec == FCC_PREC_SPLIT_FP16;
  const float* const* ar = reinterpret_cast<const float* const*>(in_rows_dev);
  float* const* cr = reinterpret_cast<float* const*>(out_rows_dev);
  const float* ab = static_cast<const float*>(in_base);
  float* cb = static_cast<float*>(out_base);
  if (fp16 && !rowscale) return FCC_ERR_INVALID_ARG;
  if (!fp16) rowscale = nullptr;
  if (ev) (void)hipEventRecord(ev[0], st);
  if (fp16) hipLaunchKernelGGL(k_rowscale, dim3(M), dim3(256), 0, st, ar, ab, lda, op.K, rowscale);
  const int mp = (M + BM - 1) / BM * BM;
  const bool rows = ar != nullptr;
  auto go = [&](auto t16) {
    using T = decltype(t16);
    T* ahi = static_cast<T*>(aws);
    T* alo = ahi + size_t(mp) * op.Kp;
    const T* wh = static_cast<const T*>(op.w_hi);
    const T* wl = static_cast<const T*>(op.w_lo);
    if (rows)
      hipLaunchKernelGGL((k_split_rows<T, true>), dim3(mp), dim3(128), 0, st, ar, ab, lda, M, op.K, op.Kp, rowscale,
                         ahi, alo);
    else
      hipLaunchKernelGGL((k_split_rows<T, false>), dim3(mp), dim3(128), 0, st, ar, ab, lda, M, op.K, op.Kp,
                         rowscale, ahi, alo);
    const dim3 grid(op.Ncp / BN, mp / BM);
    if (ev) {
      (void)hipEventRecord(ev[1], st);
      (void)hipEventRecord(ev[2], st);
    }
    if (cr)
      hipLaunchKernelGGL((k_split_gemm<T, true>), grid, dim3(256), 0, st, cr, cb, ldc, ahi, alo, wh, wl, M, op.Nc,
                         op.Kp, rowscale, op.w_unscale);
    else
      hipLaunchKernelGGL((k_split_gemm<T, false>), grid, dim3(256), 0, st, cr, cb, ldc, ahi, alo, wh, wl, M, op.Nc,
                         op.Kp, rowscale, op.w_unscale);
  };
  if (fp16)
    go(_Float16{});
  else
    go(__bf16{});
  if (ev) (void)hipEventRecord(ev[3], st);
  return hipGetLastError() == hipSuccess ? FCC_OK : FCC_ERR_HIP;
}

}  // namespace fcc
