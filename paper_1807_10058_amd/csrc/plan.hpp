// Private plan state shared by the translation units of libfccdct.so.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "fcc_dct.h"
#include "kernels.hpp"

// Dense path (FCC_PREC_SPLIT_*): the whole transform as one matrix W applied by
// a split-precision MFMA GEMM  out[b, :] = W in[b, :]  (see dense.hip).
struct DenseOp {
  int K = 0, Nc = 0;       // logical GEMM sizes: in row length, out row length (floats)
  int Kp = 0, Ncp = 0;     // padded sizes of the stored operand
  void* w_hi = nullptr;    // Ncp x Kp, 16-bit (bf16 or fp16), row-major
  void* w_lo = nullptr;
  float w_unscale = 1.0f;  // the stored W is the true one times 1/w_unscale
};

struct fcc_plan_s {
  int n = 0, D = 0, device = 0;
  double rst[3] = {0.125, 0.0, 0.375};
  fcc_precision prec = FCC_PREC_FP64;
  unsigned flags = 0;
  bool stages64 = true;
  bool level0_fp32 = false;        // level 0 (top node) in FP32 arithmetic and storage
  std::vector<fcc::DevLevel> lv;  // per level L: tables of nl = n >> L
  double2* hph = nullptr;         // phase tables, all levels
  void* ws[2] = {nullptr, nullptr};
  size_t ws_bytes = 0;
  bool dense = false;             // FCC_PREC_SPLIT_*: dense matrix on MFMA
  DenseOp dfwd, dinv;
  float* rowscale = nullptr;      // per-row input scales (FP16 split), rows_cap entries
  void* dws = nullptr;            // split input of one row, dense_ws_bytes(op, 1) for either direction
  int rows_cap = 0;
  unsigned long long* resid = nullptr;  // 2 words for fcc_dct_roundtrip_residual
  void* nodes = nullptr;                // FP64 node constants of the upper levels
  long long node_off[16] = {};          // per level offset into nodes, -1 if none
  fcc_tuning tune{};                    // the schedule, sizes clamped to this n
  int tail_Lt[2] = {0, 0};              // first level of the fused LDS tail: [0] forward, [1] inverse
  std::vector<fcc::DevLevel> tlv;
  std::vector<fcc::DevOrbitLevel> olv;  // per level L: orbit templates of nl = n >> L (orbit levels only)
  bool transposed = false;              // FCC_TRANSPOSED: the transform's transpose (and its inverse)
  int* hslot = nullptr;                 // FCC_HERMITIAN_PACKED: per point, packed slot (see k_hpack)
  void* hfull = nullptr;                // FCC_HERMITIAN_PACKED: the full spectrum
  long long hpacked = 0;                // FCC_HERMITIAN_PACKED: complex values of the packed spectrum
  void* onodes = nullptr;               // dense DCT_2 and inverse per node of the orbit-block levels
  long long onode_off[16] = {};         // per level offset into onodes, -1 if none       // per level from min(tail_Lt) on: plain-order tables, S = 1
  unsigned char kf[2][16][8] = {};      // balanced map: log2 lanes per row, per side, level and f
  // FCC_FOLD_FFT (the fold+FFT variant): tables in the data precision
  bool fold = false;
  int r8[3] = {1, 0, 3};                // 8 rst
  void* fw8n = nullptr;                 // exp(2 pi i m / (8n)), m < 8n
  void* fkt = nullptr;                  // unfold rows, fnpat x 24, scaled by 1/n^3
  unsigned char* fpid = nullptr;        // unfold row per image of each orbit representative (24 x fnrep)
  void* freps = nullptr;                // orbit representatives (flat index), by 8^3 box
  int fnpat = 0, fnrep = 0;
  // FCC_FOLD_BASE (hybrid depth): the forward's last levels as one dense base
  // per node of size M = n >> tail_Lt[0] (4, 8 or 16)
  bool fold_base = false;
  int* breps = nullptr;                 // per orbit of W on the M-torus (M = 4, 8, 16 in turn): representative, mask of repeated images
  int brep_off[3] = {}, brep_cnt[3] = {};  // in orbits
};

namespace fcc {
// Every device allocation of the library.  FCC_FAIL_ALLOC_AT=k (testing the
// error paths) makes the k-th allocation counted since the variable last
// changed fail as if the device were out of memory.
hipError_t dev_malloc_raw(void** p, size_t bytes);
template <typename T>
hipError_t dev_malloc(T** p, size_t bytes) {
  return dev_malloc_raw(reinterpret_cast<void**>(p), bytes);
}
// dense.hip
fcc_status dense_prepare(fcc_plan_s* p, hipStream_t st);
// in_base / out_base rows are lda / ldc floats apart (0: the operator's row
// lengths); aws: dense_ws_bytes(op, M) bytes of device workspace (the split
// input); ev (optional): 4 events recorded around the split and the GEMM
// (the two launch slots of a dense transform)
fcc_status dense_run(const fcc_plan_s* p, const DenseOp& op, int M, const void* const* in_rows_dev,
                     void* const* out_rows_dev, const void* in_base, void* out_base, float* rowscale, void* aws,
                     hipStream_t st, long long lda = 0, long long ldc = 0, hipEvent_t* ev = nullptr);
size_t dense_ws_bytes(const DenseOp& op, int M);
void dense_free(fcc_plan_s* p);
// fcc_dct.hip: the level-by-level fast inverse for nvol volumes of plan p,
// with device arrays of per-volume pointers
fcc_status enqueue_inverse_arrays(const fcc_plan_s* p, int nvol, void* const* in_dev, void* const* out_dev,
                                  void* const* ws0_dev, void* const* ws1_dev, hipStream_t st);
}  // namespace fcc
