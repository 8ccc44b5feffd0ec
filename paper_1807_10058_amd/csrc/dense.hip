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

constexpr int BM = 64, BN = 128, BK = 64, LDSK = BK + 8;

// One K tile of the split GEMM's operands in registers: 16 floats of an A row
// (from k0 + akc) and 32 entries of a W row, hi and lo (from k0).  Named
// members, no arrays, so that nothing is addressed through scratch.
struct GemmTile {
  float4 a0, a1, a2, a3;
  uint4 h0, h1, h2, h3, l0, l1, l2, l3;
};
template <bool kVec>
__device__ __forceinline__ float4 gemm_a4(const float* arp, int K, int kk) {
  if constexpr (kVec) {
    // K % 4 == 0: a float4 is wholly in range or wholly out
    return (arp && kk < K) ? *reinterpret_cast<const float4*>(arp + kk) : make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    float4 v;
    v.x = (arp && kk < K) ? arp[kk] : 0.f;
    v.y = (arp && kk + 1 < K) ? arp[kk + 1] : 0.f;
    v.z = (arp && kk + 2 < K) ? arp[kk + 2] : 0.f;
    v.w = (arp && kk + 3 < K) ? arp[kk + 3] : 0.f;
    return v;
  }
}
template <bool kVec, typename T16>
__device__ __forceinline__ void gemm_load(const float* arp, int K, int k0, int akc, const T16* bhp, const T16* blp,
                                          GemmTile& t) {
  const int kk = k0 + akc;
  t.a0 = gemm_a4<kVec>(arp, K, kk);
  t.a1 = gemm_a4<kVec>(arp, K, kk + 4);
  t.a2 = gemm_a4<kVec>(arp, K, kk + 8);
  t.a3 = gemm_a4<kVec>(arp, K, kk + 12);
  const uint4* hp = reinterpret_cast<const uint4*>(bhp + k0);
  const uint4* lp = reinterpret_cast<const uint4*>(blp + k0);
  t.h0 = hp[0], t.h1 = hp[1], t.h2 = hp[2], t.h3 = hp[3];
  t.l0 = lp[0], t.l1 = lp[1], t.l2 = lp[2], t.l3 = lp[3];
}
// 8 floats, scaled, as hi and lo 16-bit vectors
template <typename T16>
__device__ __forceinline__ void gemm_split8(float4 x, float4 y, float s, typename Vec8<T16>::type& hi,
                                            typename Vec8<T16>::type& lo) {
  const float v[8] = {x.x * s, x.y * s, x.z * s, x.w * s, y.x * s, y.y * s, y.z * s, y.w * s};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const T16 t = T16(v[i]);
    hi[i] = t;
    lo[i] = T16(v[i] - float(t));
  }
}
template <typename T16>
__device__ __forceinline__ void gemm_store(const GemmTile& t, float as, T16* ahi, T16* alo, T16* bhi, T16* blo) {
  typedef typename Vec8<T16>::type V8;
  V8 hi, lo;
  gemm_split8<T16>(t.a0, t.a1, as, hi, lo);
  *reinterpret_cast<V8*>(ahi) = hi;
  *reinterpret_cast<V8*>(alo) = lo;
  gemm_split8<T16>(t.a2, t.a3, as, hi, lo);
  *reinterpret_cast<V8*>(ahi + 8) = hi;
  *reinterpret_cast<V8*>(alo + 8) = lo;
  uint4* bh = reinterpret_cast<uint4*>(bhi);
  uint4* bl = reinterpret_cast<uint4*>(blo);
  bh[0] = t.h0, bh[1] = t.h1, bh[2] = t.h2, bh[3] = t.h3;
  bl[0] = t.l0, bl[1] = t.l1, bl[2] = t.l2, bl[3] = t.l3;
}

// out[r, c] = (sum_k in[r, k] W[c, k]) * w_unscale  for r < M, c < Nc.
// Block 256 threads = 4 waves as 2 (rows) x 2 (cols); each wave owns a 32 x 64
// tile = 2 x 4 MFMA 16x16 tiles, two 32-deep MFMA steps per K tile of 64.
// Operand layout of v_mfma_f32_16x16x32: A lane l holds A[l % 16][8 (l / 16) + i],
// B lane l holds B[8 (l / 16) + i][l % 16], D lane l holds D[4 (l / 16) + v][l % 16].
// The next K tile of A (16 floats per thread) and W (hi and lo, 64 bytes each
// per thread) is loaded into registers while the current one is multiplied
// from LDS; A is split into hi + lo when it is stored to LDS.  kVec: rows are
// read as float4 (K a multiple of 4).
template <typename T16, bool kVec>
__global__ __launch_bounds__(256) void k_split_gemm(const float* const* a_rows, const float* a_base, long long lda,
                                                    float* const* c_rows, float* c_base, long long ldc,
                                                    const T16* __restrict__ w_hi, const T16* __restrict__ w_lo,
                                                    int M, int K, int Nc, int Kp, const float* __restrict__ rowscale,
                                                    float w_unscale) {
  typedef typename Vec8<T16>::type V8;
  __shared__ __attribute__((aligned(16))) T16 sa_hi[BM][LDSK];
  __shared__ __attribute__((aligned(16))) T16 sa_lo[BM][LDSK];
  __shared__ __attribute__((aligned(16))) T16 sb_hi[BN][LDSK];
  __shared__ __attribute__((aligned(16))) T16 sb_lo[BN][LDSK];
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  f32x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  // A: thread -> row arow, 16 consecutive k from akc; W: row brow, 32 k from bkc
  const int arow = tid >> 2, akc = (tid & 3) * 16;
  const float* arp = nullptr;
  float as = 1.0f;
  if (m0 + arow < M) {
    arp = a_rows ? a_rows[m0 + arow] : a_base + (long long)(m0 + arow) * lda;
    if (rowscale) as = rowscale[m0 + arow];
  }
  const int brow = tid >> 1, bkc = (tid & 1) * 32;
  const T16* bhp = w_hi + (long long)(n0 + brow) * Kp + bkc;
  const T16* blp = w_lo + (long long)(n0 + brow) * Kp + bkc;

  GemmTile tile;
  gemm_load<kVec>(arp, K, 0, akc, bhp, blp, tile);
  for (int k0 = 0; k0 < K; k0 += BK) {
    gemm_store<T16>(tile, as, &sa_hi[arow][akc], &sa_lo[arow][akc], &sb_hi[brow][bkc], &sb_lo[brow][bkc]);
    __syncthreads();
    if (k0 + BK < K) gemm_load<kVec>(arp, K, k0 + BK, akc, bhp, blp, tile);  // in flight during the MFMAs below
#pragma unroll
    for (int ks = 0; ks < BK; ks += 32) {
      const int kq = ks + (lane >> 4) * 8;
      V8 ah[2], al[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const int r = wm * 32 + mt * 16 + (lane & 15);
        ah[mt] = *reinterpret_cast<const V8*>(&sa_hi[r][kq]);
        al[mt] = *reinterpret_cast<const V8*>(&sa_lo[r][kq]);
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const int c = wn * 64 + nt * 16 + (lane & 15);
        const V8 wh = *reinterpret_cast<const V8*>(&sb_hi[c][kq]);
        const V8 wl = *reinterpret_cast<const V8*>(&sb_lo[c][kq]);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          acc[mt][nt] = Vec8<T16>::mfma(ah[mt], wh, acc[mt][nt]);
          acc[mt][nt] = Vec8<T16>::mfma(ah[mt], wl, acc[mt][nt]);
          acc[mt][nt] = Vec8<T16>::mfma(al[mt], wh, acc[mt][nt]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = m0 + wm * 32 + mt * 16 + (lane >> 4) * 4 + v;
      if (r >= M) continue;
      float* cp = c_rows ? c_rows[r] : c_base + (long long)r * ldc;
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
  op->Kp = (K + BK - 1) / BK * BK;
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
  if (hipMalloc(&op->w_hi, bytes) != hipSuccess || hipMalloc(&op->w_lo, bytes) != hipSuccess) return FCC_ERR_OOM;
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
  if (hipMalloc(&F, sizeof(double2) * N * N) != hipSuccess) return fail(FCC_ERR_OOM);
  hipLaunchKernelGGL(k_dense_matrix, dim3(unsigned((N * N + 255) / 256)), dim3(256), 0, st, F, n, p->rst[0],
                     p->rst[1], p->rst[2], G);
  if (hipGetLastError() != hipSuccess) return fail(FCC_ERR_HIP);
  // inverse matrix: FP64 fast inverse of the unit vectors (column j of F^{-1})
  if (hipMalloc(&Finv, sizeof(double2) * N * N) != hipSuccess) return fail(FCC_ERR_OOM);
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
    if (hipMalloc(&E, sizeof(double2) * N * N) != hipSuccess) return fail(FCC_ERR_OOM);
    if (hipMalloc(&scratch, sizeof(double2) * N * N * 2) != hipSuccess) return fail(FCC_ERR_OOM);
    hipLaunchKernelGGL(k_unit_vectors, dim3(unsigned((N * N + 255) / 256)), dim3(256), 0, st, E, N, 0LL, int(N));
    std::vector<void*> ptr(size_t(4) * N);
    for (long long v = 0; v < N; ++v) {
      ptr[v] = E + N * v;
      ptr[N + v] = Finv + N * v;  // column v of F^{-1}, stored contiguously
      ptr[2 * N + v] = scratch + N * (2 * v);
      ptr[3 * N + v] = scratch + N * (2 * v + 1);
    }
    if (hipMalloc(&parr, sizeof(void*) * ptr.size()) != hipSuccess) return fail(FCC_ERR_OOM);
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

fcc_status dense_run(const fcc_plan_s* p, const DenseOp& op, int M, const void* const* in_rows_dev,
                     void* const* out_rows_dev, const void* in_base, void* out_base, float* rowscale,
                     hipStream_t st) {
  const bool fp16 = p->prec == FCC_PREC_SPLIT_FP16;
  const float* const* ar = reinterpret_cast<const float* const*>(in_rows_dev);
  float* const* cr = reinterpret_cast<float* const*>(out_rows_dev);
  const float* ab = static_cast<const float*>(in_base);
  float* cb = static_cast<float*>(out_base);
  if (fp16) {
    if (!rowscale) return FCC_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_rowscale, dim3(M), dim3(256), 0, st, ar, ab, (long long)op.K, op.K, rowscale);
  } else {
    rowscale = nullptr;
  }
  dim3 grid(op.Ncp / BN, (M + BM - 1) / BM);
  const bool vec = (op.K & 3) == 0;
#define FCC_GEMM(T, V)                                                                                           \
  hipLaunchKernelGGL((k_split_gemm<T, V>), grid, dim3(256), 0, st, ar, ab, (long long)op.K, cr, cb,              \
                     (long long)op.Nc, static_cast<const T*>(op.w_hi), static_cast<const T*>(op.w_lo), M, op.K, \
                     op.Nc, op.Kp, rowscale, op.w_unscale)
  if (fp16) {
    if (vec)
      FCC_GEMM(_Float16, true);
    else
      FCC_GEMM(_Float16, false);
  } else {
    if (vec)
      FCC_GEMM(__bf16, true);
    else
      FCC_GEMM(__bf16, false);
  }
#undef FCC_GEMM
  return hipGetLastError() == hipSuccess ? FCC_OK : FCC_ERR_HIP;
}

}  // namespace fcc
