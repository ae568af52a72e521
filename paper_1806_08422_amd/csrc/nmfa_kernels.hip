// NMFA hot-path kernels for gfx950.
//
// One iteration of Algorithm 1 (paper Sec. II) for every spin i and replica r:
//   Phi_i = (h_i + sum_j J_ij s_j) / sqrt(h_i^2 + sum_j J_ij^2) + N(0, sigma)
//   s^_i  = -tanh(Phi_i / T_t)
//   s_i  <- alpha s^_i + (1 - alpha) s_i          (after all s^ of the iteration are known)
// The contraction sum_j J_ij s_j over all replicas is the matrix product J . S and runs on
// MFMA; the normalisation, noise, Boltzmann factor and damped update are fused into the MFMA
// epilogue in registers. After the last iteration the sign readout s~_i = s_i/|s_i| and the
// energy of Eq. 1 are evaluated.
//
// Kernels:
//   anneal_small<P>   persistent: one workgroup owns 16 replicas and all N <= 256 spins for the
//                     whole anneal. J sits in LDS, the operand copy of S is double-buffered in
//                     LDS, the master state lives in registers; one barrier per iteration.
//   anneal_step<P>    one iteration for large N (FP32; FP64 only for shapes the tiled FP64
//                     kernel does not take): each wave owns 16 rows x 64 replicas, reads J and S
//                     straight from global memory (L2), updates the master state in HBM and
//                     writes the next operand copy of S.
//   anneal_step_tiled, anneal_step_tiled_f64
//                     the same iteration as tiled matrix products through LDS (BF16 operands on
//                     256 x 128 workgroup tiles, FP64 on 128 x 64), with the fused epilogue.
//   anneal_sparse*    degree-d graphs with J in ELL rows (see their own comments).
//   readout_kernel    s~ = sign(s) (s = 0 reads +1).
//   energy_kernel     exact integer energies for integral J (int8) and integral h, or an
//                     integral pair term plus an FP64 field term summed in ascending i; with
//                     FP64 couplings the pair sums in FP64 (exact integers for integral J).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "nmfa_device.h"
#include "nmfa_internal.h"

namespace nmfa {

// ------------------------------------------------------------------------------------------
// Shared epilogue: from the accumulated field of four consecutive rows of one replica to the
// updated master state. acc[v] = sum_j J_ij s_j for row i = row0 + v.
// ------------------------------------------------------------------------------------------
template <int P>
struct Epilogue;

template <>
struct Epilogue<PREC_FP64> {
  __device__ static __forceinline__ void apply(const double acc[4], const double inv[4],
                                               const double h[4], double s[4], const AnnealArgs& a,
                                               double coef_t, uint32_t q, uint32_t r, uint32_t t) {
    // every operation rounded on its own (no contraction into FMAs), so that all kernels that
    // share this epilogue round alike, whatever the surrounding code lets the compiler fuse
#pragma clang fp contract(off)
    double z[4];
    gauss4_f64(philox4x32_10(q, r, t, 0u, a.key0, a.key1), z);
    const double sg = a.negate_noise ? -a.sigma : a.sigma;
    const double oma = 1.0 - a.alpha;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double phi = (h[v] + acc[v]) * inv[v] + sg * z[v];
      const double s_hat = -tanh(phi * coef_t);
      s[v] = a.alpha * s_hat + oma * s[v];
    }
  }
};

template <int P>
struct EpilogueF32 {
  __device__ static __forceinline__ void apply(const float acc[4], const float inv[4],
                                               const float hinv[4], float s[4], const AnnealArgs& a,
                                               float coef_t, uint32_t q, uint32_t r, uint32_t t) {
    float z[4];
    const float sg = (float)a.sigma;
    sigma_gauss4_f32(philox4x32_10(q, r, t, 0u, a.key0, a.key1), -2.0f * 0.6931471805599453f * sg * sg,
                     z);
    const float alpha = (float)a.alpha;
    const float oma = (float)(1.0 - a.alpha);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float x = fmaf(acc[v], inv[v], hinv[v]);
      const float phi = a.negate_noise ? x - z[v] : x + z[v];
      const float s_hat = neg_tanh_from_exp2_arg(phi * coef_t);
      s[v] = fmaf(alpha, s_hat, oma * s[v]);
    }
  }
};
template <>
struct Epilogue<PREC_FP32> : EpilogueF32<PREC_FP32> {};
template <>
struct Epilogue<PREC_BF16> : EpilogueF32<PREC_BF16> {};

// ------------------------------------------------------------------------------------------
// anneal_small<P, J8>: see the file header. Block = 64 * (Mp/16) threads, wave w owns rows
// [16w, 16w+16); grid = ceil(R / 16) workgroups, workgroup b owns replicas [16b, 16b+16).
// LDS: Js[Mp][js] (op_t), Ss[2][16][js] (op_t), with js = padded row stride in elements.
// J8: the global copy of J is FP8 e4m3 and is widened to BF16 while it is staged into LDS.
// The body is shared with anneal_small_batched, where one launch carries replica blocks of many
// jobs (serving): a workgroup may then have more waves than its job has row tiles, and the extra
// waves only take part in the barriers.
// ------------------------------------------------------------------------------------------
template <int P, bool J8>
__device__ __forceinline__ void anneal_small_body(const AnnealArgs& a, const int rblock) {
  using Tr = Traits<P>;
  using op_t = typename Tr::op_t;
  using acc_t = typename Tr::acc_t;
  using frag_t = typename Tr::frag_t;
  using acc4_t = typename Tr::acc4_t;
  constexpr int KW = Tr::KW;
  constexpr int VEC = 16 / (KW * (int)sizeof(op_t));  // MFMA steps per 16-byte LDS read

  extern __shared__ __align__(16) unsigned char smem[];
  const int N = a.N, Mp = a.Mp, Kp = a.Kp, js = a.lds_stride;
  op_t* Js = reinterpret_cast<op_t*>(smem);
  op_t* Ss = Js + (size_t)Mp * js;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4;
  const int c = lane & 15;
  const int r = rblock * 16 + c;       // replica of this lane
  const bool act = wave < (Mp >> 4);   // this wave owns a row tile of the job
  const int row0 = wave * 16 + 4 * g;  // first of this lane's four rows (accumulator layout)
  const int arow = wave * 16 + Tr::a_row(c);  // row this lane supplies to the A operand
  const int Kq = Kp >> 2;

  // ---- stage J into LDS (16-byte chunks), zero both S buffers --------------------------------
  {
    const int chunks_per_row = (Kp * (int)sizeof(op_t)) / 16;
    const int total = Mp * chunks_per_row;
    for (int ch = tid; ch < total; ch += blockDim.x) {
      const int row = ch / chunks_per_row;
      const int cc = ch - row * chunks_per_row;
      uint4 v;
      if constexpr (J8) {
        const uint8_t* src = reinterpret_cast<const uint8_t*>(a.J) + (size_t)row * Kp + cc * 8;
        const uint2 raw = *reinterpret_cast<const uint2*>(src);
        __bf16 w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t byte = ((k < 4 ? raw.x : raw.y) >> (8 * (k & 3))) & 0xffu;
          w[k] = (__bf16)fp8e4m3_to_float(byte);
        }
        v = *reinterpret_cast<const uint4*>(w);
      } else {
        v = reinterpret_cast<const uint4*>(a.J)[(size_t)row * chunks_per_row + cc];
      }
      *reinterpret_cast<uint4*>(reinterpret_cast<unsigned char*>(Js + (size_t)row * js) + cc * 16) = v;
    }
    const int s_words = (2 * 16 * js * (int)sizeof(op_t)) / 4;
    uint32_t* Sw = reinterpret_cast<uint32_t*>(Ss);
    for (int k = tid; k < s_words; k += blockDim.x) Sw[k] = 0u;
  }

  // ---- per-lane constants and initial state ----------------------------------------------
  acc_t inv[4], hv[4], s[4];
  const acc_t* inv_g = reinterpret_cast<const acc_t*>(a.inv_norm);
  const acc_t* h_g = reinterpret_cast<const acc_t*>(a.hterm);
  acc_t* state = reinterpret_cast<acc_t*>(a.state);
  const bool live_r = act && r < a.R;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    inv[v] = act ? inv_g[row0 + v] : (acc_t)0;
    hv[v] = act ? h_g[row0 + v] : (acc_t)0;
    const bool live = live_r && (row0 + v) < N;
    s[v] = (a.load_state && live) ? state[(size_t)r * N + row0 + v] : (acc_t)0;
  }
  __syncthreads();
  if (a.load_state && act) {
#pragma unroll
    for (int v = 0; v < 4; ++v) Ss[(size_t)c * js + row0 + v] = (op_t)s[v];
  }
  __syncthreads();

  const acc_t* coef = reinterpret_cast<const acc_t*>(a.coef);
  acc_t* traj = reinterpret_cast<acc_t*>(a.traj);
  int cur = 0;
  for (int t = a.t_begin; t <= a.t_end; ++t) {
    if (!act) {  // spare wave of a batched launch
      __syncthreads();
      continue;
    }
    // ---- mean field: D = J[rows of this wave] . S[:, replicas of this block] ----------------
    acc4_t acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = (acc_t)0;
    const op_t* Arow = Js + (size_t)arow * js + g * Kq;
    const op_t* Bcol = Ss + (size_t)cur * 16 * js + (size_t)c * js + g * Kq;
    for (int m = 0; m < Kq; m += VEC * KW) {
      const uint4 av = *reinterpret_cast<const uint4*>(Arow + m);
      const uint4 bv = *reinterpret_cast<const uint4*>(Bcol + m);
      const frag_t* af = reinterpret_cast<const frag_t*>(&av);
      const frag_t* bf = reinterpret_cast<const frag_t*>(&bv);
#pragma unroll
      for (int u = 0; u < VEC; ++u) acc = Tr::mfma(af[u], bf[u], acc);
    }
    // ---- fused epilogue ------------------------------------------------------------------
    acc_t fld[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) fld[v] = acc[v];
    Epilogue<P>::apply(fld, inv, hv, s, a, coef[t - 1], (uint32_t)(row0 >> 2), (uint32_t)r,
                       (uint32_t)t);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (row0 + v >= N) s[v] = (acc_t)0;  // padding rows stay empty
    const int nxt = cur ^ 1;
    op_t* Sn = Ss + (size_t)nxt * 16 * js + (size_t)c * js + row0;
#pragma unroll
    for (int v = 0; v < 4; ++v) Sn[v] = (op_t)s[v];
    const int k = t - a.t_begin;
    if (traj && k < a.record && live_r) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (row0 + v < N) traj[((size_t)k * a.R + r) * N + row0 + v] = s[v];
    }
    __syncthreads();
    cur = nxt;
  }

  // ---- final state and sign readout -------------------------------------------------------
  if (live_r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (row0 + v < N) {
        state[(size_t)r * N + row0 + v] = s[v];
        if (a.spins) a.spins[(size_t)r * N + row0 + v] = (s[v] >= (acc_t)0) ? (int8_t)1 : (int8_t)-1;
      }
    }
  }
}

template <int P, bool J8>
__global__ __launch_bounds__(1024) void anneal_small(AnnealArgs a) {
  anneal_small_body<P, J8>(a, (int)blockIdx.x);
}

// One launch for replica blocks of many jobs: tasks[b] = (job index, replica block).
template <int P, bool J8>
__global__ __launch_bounds__(1024) void anneal_small_batched(const AnnealArgs* __restrict__ jobs,
                                                             const int2* __restrict__ tasks) {
  const int2 tk = tasks[blockIdx.x];
  const AnnealArgs a = jobs[tk.x];
  anneal_small_body<P, J8>(a, tk.y);
}

// ------------------------------------------------------------------------------------------
// anneal_step<P>: one iteration t for large N. Block = 256 threads (4 waves); workgroup
// (bx, by) owns rows [64 bx, 64 bx + 64) and replicas [64 by, 64 by + 64); wave w owns the 16
// rows [64 bx + 16 w, +16) for all 64 replicas (four 16x16 MFMA tiles sharing one A fragment).
// Operands come straight from global memory: J as [Mp][Kp] op_t, S_cur as [Rp][Kp] op_t
// (replica-major, k contiguous). Writes S_next and the master state (in place).
// ------------------------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void anneal_step(AnnealArgs a, const void* S_cur_v, void* S_next_v,
                                                   int t) {
  using Tr = Traits<P>;
  using op_t = typename Tr::op_t;
  using acc_t = typename Tr::acc_t;
  using frag_t = typename Tr::frag_t;
  using acc4_t = typename Tr::acc4_t;
  constexpr int KW = Tr::KW;
  constexpr int VEC = 16 / (KW * (int)sizeof(op_t));
  const op_t* J = reinterpret_cast<const op_t*>(a.J);
  const op_t* S_cur = reinterpret_cast<const op_t*>(S_cur_v);
  op_t* S_next = reinterpret_cast<op_t*>(S_next_v);
  const int N = a.N, Kp = a.Kp, Kq = Kp >> 2;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int c = lane & 15;
  const int rowbase = blockIdx.x * 64 + wave * 16;
  const int arow = rowbase + Tr::a_row(c);
  const int row0 = rowbase + 4 * g;
  const int rbase = blockIdx.y * 64;

  acc4_t acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[ct][v] = (acc_t)0;

  const op_t* Arow = J + (size_t)arow * Kp + g * Kq;
  const op_t* B0 = S_cur + (size_t)(rbase + c) * Kp + g * Kq;
  for (int m = 0; m < Kq; m += VEC * KW) {
    const uint4 av = *reinterpret_cast<const uint4*>(Arow + m);
    const frag_t* af = reinterpret_cast<const frag_t*>(&av);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const uint4 bv = *reinterpret_cast<const uint4*>(B0 + (size_t)ct * 16 * Kp + m);
      const frag_t* bf = reinterpret_cast<const frag_t*>(&bv);
#pragma unroll
      for (int u = 0; u < VEC; ++u) acc[ct] = Tr::mfma(af[u], bf[u], acc[ct]);
    }
  }

  const acc_t* inv_g = reinterpret_cast<const acc_t*>(a.inv_norm);
  const acc_t* h_g = reinterpret_cast<const acc_t*>(a.hterm);
  acc_t* state = reinterpret_cast<acc_t*>(a.state);
  acc_t* traj = reinterpret_cast<acc_t*>(a.traj);
  const acc_t coef_t = reinterpret_cast<const acc_t*>(a.coef)[t - 1];
  acc_t inv[4], hv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    inv[v] = inv_g[row0 + v];
    hv[v] = h_g[row0 + v];
  }
  const int k_rec = t - a.t_begin;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int r = rbase + ct * 16 + c;
    const bool live_r = r < a.R;
    acc_t s[4], fld[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      fld[v] = acc[ct][v];
      s[v] = (live_r && row0 + v < N) ? state[(size_t)r * N + row0 + v] : (acc_t)0;
    }
    Epilogue<P>::apply(fld, inv, hv, s, a, coef_t, (uint32_t)(row0 >> 2), (uint32_t)r, (uint32_t)t);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (row0 + v >= N || !live_r) s[v] = (acc_t)0;
    op_t* dst = S_next + (size_t)r * Kp + row0;
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[v] = (op_t)s[v];
    if (live_r) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (row0 + v < N) {
          state[(size_t)r * N + row0 + v] = s[v];
          if (traj && k_rec < a.record) traj[((size_t)k_rec * a.R + r) * N + row0 + v] = s[v];
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Operand copy of a master state: S[r][i] = (op_t) state[r][i] for i < N, r < R; zero padding.
// ------------------------------------------------------------------------------------------
template <typename op_t, typename acc_t>
__global__ void pack_state_kernel(const acc_t* __restrict__ state, op_t* __restrict__ S, int N, int R,
                                  int Kp, int ld, int Rp, int zero) {
  const size_t total = (size_t)Rp * Kp;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx / Kp);
    const int i = (int)(idx - (size_t)r * Kp);
    acc_t v = 0;
    if (!zero && r < R && i < N) v = state[(size_t)r * N + i];
    S[(size_t)r * ld + i] = (op_t)v;
  }
}

// FP8 E4M3 operand copy (the FP8-spin precision), rounded as the annealing kernel's epilogue
// rounds (v_cvt_pk_fp8_f32: nearest even, saturating), so a resumed run continues bit-exactly.
__global__ void pack_state_fp8_kernel(const float* __restrict__ state, uint8_t* __restrict__ S, int N, int R, int Kp,
                                      int ld, int Rp, int zero) {
  const size_t total = (size_t)Rp * Kp;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx / Kp);
    const int i = (int)(idx - (size_t)r * Kp);
    float v = 0.0f;
    if (!zero && r < R && i < N) v = state[(size_t)r * N + i];
    S[(size_t)r * ld + i] = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xff);
  }
}

// ------------------------------------------------------------------------------------------
// Readout: s~ = +1 if s >= 0 (including -0.0), else -1.
// ------------------------------------------------------------------------------------------
template <typename acc_t>
__global__ void readout_kernel(const acc_t* __restrict__ state, int8_t* __restrict__ spins, size_t count) {
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count;
       idx += (size_t)gridDim.x * blockDim.x)
    spins[idx] = (state[idx] >= (acc_t)0) ? (int8_t)1 : (int8_t)-1;
}

// ------------------------------------------------------------------------------------------
// Energy of Eq. 1 (pairs i < j) for R spin vectors, E = (1/2) sum_i s_i y_i + sum_i h_i s_i with
// y_i = sum_j J_ij s_j. Integral J (int8): y and the pair term are exact int32/int64. Block =
// 256 threads handles one replica; thread i accumulates y_i by reading J column i (= row i by
// symmetry, so consecutive threads read consecutive bytes), then the products s_i y_i are
// reduced with wavefront shuffles and one LDS step. The field term uses integer h when h is
// integral; otherwise lane 0 sums h_i s_i in double in ascending i.
// FP64 J (non-integral couplings): y_i in double, reduced in a fixed tree order.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void energy_kernel(const int8_t* __restrict__ J8,
                                                     const double* __restrict__ J64,
                                                     const double* __restrict__ h,
                                                     int h_integral,
                                                     const int8_t* __restrict__ spins, int N, int R,
                                                     long long* __restrict__ E_int,
                                                     double* __restrict__ E) {
  __shared__ int8_t s_sh[8192];
  __shared__ long long part_i[4];
  __shared__ double part_d[4];
  const int r = blockIdx.x;
  if (r >= R) return;
  const int8_t* s = spins + (size_t)r * N;
  // spins of this replica in LDS, in chunks of 8192
  long long pair2 = 0;   // sum_i s_i y_i (integral J)
  double pair2_d = 0.0;  // same, FP64 J
  long long fld_i = 0;
  for (int base = 0; base < N; base += 8192) {
    const int len = min(8192, N - base);
    __syncthreads();
    for (int k = threadIdx.x; k < len; k += blockDim.x) s_sh[k] = s[base + k];
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      if (J8) {
        int y = 0;
        const int8_t* col = J8 + (size_t)base * N + i;
        for (int j = 0; j < len; ++j) y += (int)col[(size_t)j * N] * (int)s_sh[j];
        pair2 += (long long)y * (long long)s[i];
      } else {
        double y = 0.0;
        const double* col = J64 + (size_t)base * N + i;
        for (int j = 0; j < len; ++j) y += col[(size_t)j * N] * (double)s_sh[j];
        pair2_d += y * (double)s[i];
      }
    }
  }
  if (h && h_integral) {
    for (int i = threadIdx.x; i < N; i += blockDim.x) fld_i += (long long)h[i] * (long long)s[i];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long long v = wave_sum_i64(pair2 + 2 * fld_i);
  double vd = wave_sum_f64(pair2_d);
  if (lane == 0) {
    part_i[wave] = v;
    part_d[wave] = vd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    double totd = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      tot += part_i[w];
      totd += part_d[w];
    }
    if (J8) {
      const long long e2 = tot;  // 2 * (pair + integral field)
      double field_real = 0.0;
      if (h && !h_integral) {
        for (int i = 0; i < N; ++i) field_real += h[i] * (double)s[i];
      }
      if (E_int) E_int[r] = e2 / 2;
      E[r] = (h && !h_integral) ? (double)(e2 / 2) + field_real : (double)(e2 / 2);
    } else {
      double field = 0.0;
      if (h) {
        for (int i = 0; i < N; ++i) field += h[i] * (double)s[i];
      }
      // integral couplings and fields (the caller checked that every sum stays below 2^53): the
      // FP64 sums above are exact integers
      if (E_int) E_int[r] = h_integral ? (long long)totd / 2 + (long long)field : 0;
      E[r] = 0.5 * totd + field;
    }
  }
}

// ------------------------------------------------------------------------------------------
// anneal_sparse<P>: sparse couplings (degree-d graphs). J is stored row by row in ELL form, the
// nonzeros of row i in ascending column order padded to D entries with zero weights, so the
// field sum_j J_ij s_j is the dense sum with its exact zero terms left out (bit-identical up to
// the FMA contraction of each term). One workgroup owns RB replicas and all N spins for the whole
// anneal: the state of its replicas sits in LDS, double-buffered by iteration parity (layout
// [Nq][RB], replica fastest, so the threads of one spin gather consecutive words), and a
// workgroup barrier separates iterations. Thread tasks are (quad q of 4 consecutive spins,
// replica): one Philox call draws exactly the quad's noise, and the update is the shared
// Epilogue. FP64 precision runs in FP64; the other precisions run in FP32.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float fma_acc(float x, float y, float z) { return __builtin_fmaf(x, y, z); }
__device__ __forceinline__ double fma_acc(double x, double y, double z) { return __builtin_fma(x, y, z); }

template <int P>
__global__ __launch_bounds__(P == PREC_FP64 ? 512 : 1024) void anneal_sparse(AnnealArgs a,
                                                                             const int* __restrict__ ell_col,
                                                     const void* __restrict__ ell_val, int D, int RB) {
  using acc_t = typename Traits<P>::acc_t;
  extern __shared__ __align__(16) unsigned char smem_sp[];
  const int N = a.N, Nq = (N + 3) / 4;
  acc_t* buf0 = reinterpret_cast<acc_t*>(smem_sp);
  acc_t* buf1 = buf0 + (size_t)4 * Nq * RB;
  const acc_t* val = reinterpret_cast<const acc_t*>(ell_val);
  const acc_t* inv_g = reinterpret_cast<const acc_t*>(a.inv_norm);
  const acc_t* h_g = reinterpret_cast<const acc_t*>(a.hterm);
  const acc_t* coef = reinterpret_cast<const acc_t*>(a.coef);
  acc_t* state = reinterpret_cast<acc_t*>(a.state);
  acc_t* traj = reinterpret_cast<acc_t*>(a.traj);
  const int r0 = blockIdx.x * RB;
  const int slots = 4 * Nq * RB;
  for (int idx = threadIdx.x; idx < slots; idx += blockDim.x) {
    const int i = idx / RB, rr = idx - i * RB, r = r0 + rr;
    buf0[idx] = (a.load_state && r < a.R && i < N) ? state[(size_t)r * N + i] : (acc_t)0;
  }
  __syncthreads();
  int cur = 0;
  const int tasks = Nq * RB;
  for (int t = a.t_begin; t <= a.t_end; ++t) {
    const acc_t coef_t = coef[t - 1];
    const acc_t* sc = cur ? buf1 : buf0;
    acc_t* sn = cur ? buf0 : buf1;
    const int k_rec = t - a.t_begin;
    for (int task = threadIdx.x; task < tasks; task += blockDim.x) {
      const int q = task / RB, rr = task - q * RB, r = r0 + rr;
      acc_t acc[4], inv[4], hv[4], sv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * q + v;
        acc_t f = (acc_t)0;
        if (i < N) {
          const int* cl = ell_col + (size_t)i * D;
          const acc_t* vl = val + (size_t)i * D;
          for (int d = 0; d < D; ++d) f = fma_acc(vl[d], sc[cl[d] * RB + rr], f);
          inv[v] = inv_g[i];
          hv[v] = h_g[i];
        } else {
          inv[v] = (acc_t)0;
          hv[v] = (acc_t)0;
        }
        acc[v] = f;
        sv[v] = sc[i * RB + rr];
      }
      Epilogue<P>::apply(acc, inv, hv, sv, a, coef_t, (uint32_t)q, (uint32_t)r, (uint32_t)t);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * q + v;
        sn[i * RB + rr] = (i < N) ? sv[v] : (acc_t)0;
        if (traj && k_rec < a.record && r < a.R && i < N) traj[((size_t)k_rec * a.R + r) * N + i] = sv[v];
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  const acc_t* sf = cur ? buf1 : buf0;
  for (int idx = threadIdx.x; idx < slots; idx += blockDim.x) {
    const int i = idx / RB, rr = idx - i * RB, r = r0 + rr;
    if (r < a.R && i < N) {
      state[(size_t)r * N + i] = sf[idx];
      if (a.spins) a.spins[(size_t)r * N + i] = (sf[idx] >= (acc_t)0) ? (int8_t)1 : (int8_t)-1;
    }
  }
}

// ------------------------------------------------------------------------------------------
// anneal_sparse_rq<P, RB, DM, QP>: the sparse kernel with the couplings in registers. A thread
// owns the quads q = tid + k * blockDim.x (k < QP) for all RB replicas of its workgroup and for
// the whole anneal: its ELL rows (DM entries each, those beyond D zero-weight) are read from
// global memory once, the quads' own state stays in registers, and one neighbour read is one
// vector LDS load of that spin's RB replica values (layout [4 Nq][RB], replica fastest, as in
// anneal_sparse). Each replica's arithmetic (terms in ELL order, one FMA each, noise counters,
// epilogue) is that of anneal_sparse; a zero-weight term adds a signed zero to a sum that starts
// at +0 and so changes nothing. Both kernels therefore give bit-identical trajectories, whatever
// RB and whichever kernel the launcher picks.
// ------------------------------------------------------------------------------------------
template <typename T, int RB>
struct alignas(sizeof(T) * RB) RepVec {
  T v[RB];
};

template <int P, int RB, int DM, int QP>
__global__ __launch_bounds__(512) void anneal_sparse_rq(AnnealArgs a, const int* __restrict__ ell_col,
                                                       const void* __restrict__ ell_val, int D) {
  using acc_t = typename Traits<P>::acc_t;
  using V = RepVec<acc_t, RB>;
  extern __shared__ __align__(16) unsigned char smem_sp[];
  const int N = a.N, Nq = (N + 3) / 4;
  const int buf_bytes = 4 * Nq * (int)sizeof(V);
  const acc_t* val = reinterpret_cast<const acc_t*>(ell_val);
  const acc_t* inv_g = reinterpret_cast<const acc_t*>(a.inv_norm);
  const acc_t* h_g = reinterpret_cast<const acc_t*>(a.hterm);
  const acc_t* coef = reinterpret_cast<const acc_t*>(a.coef);
  acc_t* state = reinterpret_cast<acc_t*>(a.state);
  acc_t* traj = reinterpret_cast<acc_t*>(a.traj);
  const int r0 = blockIdx.x * RB;

  int off[QP][4][DM];  // byte offset of the neighbour's replica vector within a state buffer
  acc_t w[QP][4][DM];
  acc_t inv[QP][4], hv[QP][4], s[QP][RB][4];
#pragma unroll
  for (int k = 0; k < QP; ++k) {
    const int q = threadIdx.x + k * blockDim.x;
    const bool own = q < Nq;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * q + v;  // < 4 Nq = Mp when own: inv_g and h_g hold Mp entries
      const bool live = own && i < N;
      inv[k][v] = own ? inv_g[i] : (acc_t)0;
      hv[k][v] = own ? h_g[i] : (acc_t)0;
#pragma unroll
      for (int d = 0; d < DM; ++d) {
        const bool e = live && d < D;
        off[k][v][d] = e ? ell_col[(size_t)i * D + d] * (int)sizeof(V) : 0;
        w[k][v][d] = e ? val[(size_t)i * D + d] : (acc_t)0;
      }
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const int r = r0 + rr;
        s[k][rr][v] = (a.load_state && live && r < a.R) ? state[(size_t)r * N + i] : (acc_t)0;
      }
    }
    if (own) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        V y;
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) y.v[rr] = s[k][rr][v];
        *reinterpret_cast<V*>(smem_sp + (4 * q + v) * (int)sizeof(V)) = y;
      }
    }
  }
  __syncthreads();
  int cur = 0;
  for (int t = a.t_begin; t <= a.t_end; ++t) {
    const acc_t coef_t = coef[t - 1];
    const unsigned char* sc = smem_sp + (cur ? buf_bytes : 0);
    unsigned char* sn = smem_sp + (cur ? 0 : buf_bytes);
    const int k_rec = t - a.t_begin;
#pragma unroll
    for (int k = 0; k < QP; ++k) {
      const int q = threadIdx.x + k * blockDim.x;
      if (q >= Nq) continue;
      acc_t acc[RB][4];
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[rr][v] = (acc_t)0;
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int d = 0; d < DM; ++d) {
          const V x = *reinterpret_cast<const V*>(sc + off[k][v][d]);
#pragma unroll
          for (int rr = 0; rr < RB; ++rr) acc[rr][v] = fma_acc(w[k][v][d], x.v[rr], acc[rr][v]);
        }
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
        Epilogue<P>::apply(acc[rr], inv[k], hv[k], s[k][rr], a, coef_t, (uint32_t)q, (uint32_t)(r0 + rr),
                           (uint32_t)t);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool live = 4 * q + v < N;
        V y;
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) y.v[rr] = live ? s[k][rr][v] : (acc_t)0;
        *reinterpret_cast<V*>(sn + (4 * q + v) * (int)sizeof(V)) = y;
      }
      if (traj && k_rec < a.record) {
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
          const int r = r0 + rr;
          if (r >= a.R) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (4 * q + v < N) traj[((size_t)k_rec * a.R + r) * N + 4 * q + v] = s[k][rr][v];
        }
      }
    }
    __syncthreads();
    cur ^= 1;
  }
#pragma unroll
  for (int k = 0; k < QP; ++k) {
    const int q = threadIdx.x + k * blockDim.x;
    if (q >= Nq) continue;
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int r = r0 + rr;
      if (r >= a.R) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * q + v;
        if (i >= N) continue;
        state[(size_t)r * N + i] = s[k][rr][v];
        if (a.spins) a.spins[(size_t)r * N + i] = (s[k][rr][v] >= (acc_t)0) ? (int8_t)1 : (int8_t)-1;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Exact energies on the matrix cores, for integral couplings |J_ij| <= 127 (int8): the pair term
// sum_i s_i y_i with y = J s is an int8 x int8 -> int32 matrix product (v_mfma_i32_16x16x64_i8),
// exact in any summation order. Operands are zero-padded copies: J8p [Np][Np] and the signs
// Sp [Rp][Np] (Np a multiple of 64, Rp of 64), so the kernel needs no bounds checks. Each wave
// computes y for 16 rows x 64 replicas, forms s_i y_i for its rows and adds the per-replica sums
// to E2 with 64-bit integer atomics (exact, order-free). A finishing pass adds the field term
// with the arithmetic of energy_kernel, so both paths give identical energies.
// ------------------------------------------------------------------------------------------
typedef int i32x4 __attribute__((ext_vector_type(4)));

__global__ void pad_spins_kernel(const int8_t* __restrict__ s, int N, int R, int8_t* __restrict__ Sp, int Np,
                                 int Rp) {
  const size_t total = (size_t)Rp * Np;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx / Np), i = (int)(idx - (size_t)r * Np);
    Sp[idx] = (r < R && i < N) ? s[(size_t)r * N + i] : (int8_t)0;
  }
}

__global__ void zero_u64_kernel(unsigned long long* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// grid (Np / 64, Rp / 64), block 256: wave w owns rows 64*bx + 16w .. +15, replicas 64*by .. +63
__global__ __launch_bounds__(256) void energy_pairs_i8(const int8_t* __restrict__ J8p, const int8_t* __restrict__ Sp,
                                                       int Np, int R, unsigned long long* __restrict__ E2) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, g4 = lane >> 4;
  const int row0 = blockIdx.x * 64 + wave * 16;
  const int rep0 = blockIdx.y * 64;
  // lane group g4 supplies k = 16 g4 .. 16 g4 + 15 of every 64-k step, for A (J) and B (signs) alike
  const int8_t* a_ptr = J8p + (size_t)(row0 + c) * Np + 16 * g4;
  i32x4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = i32x4{0, 0, 0, 0};
  for (int k0 = 0; k0 < Np; k0 += 64) {
    const i32x4 av = *reinterpret_cast<const i32x4*>(a_ptr + k0);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const i32x4 bv = *reinterpret_cast<const i32x4*>(Sp + (size_t)(rep0 + 16 * ct + c) * Np + 16 * g4 + k0);
      acc[ct] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bv, acc[ct], 0, 0, 0);
    }
  }
  // lane (c, g4) holds y of rows row0 + 4 g4 + v for replica rep0 + 16 ct + c
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int r = rep0 + 16 * ct + c;
    const int sv = *reinterpret_cast<const int*>(Sp + (size_t)r * Np + row0 + 4 * g4);  // 4 signs
    int part = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) part += (int)(int8_t)(sv >> (8 * v)) * acc[ct][v];
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (g4 == 0 && r < R) atomicAdd(&E2[r], (unsigned long long)(long long)part);
  }
}

// E_int = (sum_i s_i y_i) / 2 + integral field term; E as energy_kernel computes it
__global__ void energy_finish_kernel(const unsigned long long* __restrict__ E2, const double* __restrict__ h,
                                     int h_integral, const int8_t* __restrict__ spins, int N, int R,
                                     long long* __restrict__ E_int, double* __restrict__ E) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int8_t* s = spins + (size_t)r * N;
  long long fld = 0;
  double field_real = 0.0;
  if (h && h_integral) {
    for (int i = 0; i < N; ++i) fld += (long long)h[i] * (long long)s[i];
  } else if (h) {
    for (int i = 0; i < N; ++i) field_real += h[i] * (double)s[i];
  }
  const long long e2 = (long long)E2[r] + 2 * fld;
  if (E_int) E_int[r] = e2 / 2;
  E[r] = (h && !h_integral) ? (double)(e2 / 2) + field_real : (double)(e2 / 2);
}

// ------------------------------------------------------------------------------------------
// Noise words / values for a range of spins (library utility and test hook for the stream).
// words: out[(k*n + i)] for replica r0 + k ... see nmfa.h.
// ------------------------------------------------------------------------------------------
__global__ void noise_words_kernel(uint32_t key0, uint32_t key1, uint32_t t, uint32_t r0, int nrep,
                                   int nq, uint32_t* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nrep * nq) return;
  const int k = idx / nq, q = idx - k * nq;
  const Philox4 w = philox4x32_10((uint32_t)q, r0 + (uint32_t)k, t, 0u, key0, key1);
  out[4 * (size_t)idx + 0] = w.x0;
  out[4 * (size_t)idx + 1] = w.x1;
  out[4 * (size_t)idx + 2] = w.x2;
  out[4 * (size_t)idx + 3] = w.x3;
}

__global__ void noise_values_kernel(uint32_t key0, uint32_t key1, uint32_t t, uint32_t r0, int nrep,
                                    int nq, int fp64, double* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nrep * nq) return;
  const int k = idx / nq, q = idx - k * nq;
  const Philox4 w = philox4x32_10((uint32_t)q, r0 + (uint32_t)k, t, 0u, key0, key1);
  if (fp64) {
    double z[4];
    gauss4_f64(w, z);
    for (int v = 0; v < 4; ++v) out[4 * (size_t)idx + v] = z[v];
  } else {
    float z[4];
    // sigma = 1: -2 ln 2 * 1
    sigma_gauss4_f32(w, -2.0f * 0.6931471805599453f, z);
    for (int v = 0; v < 4; ++v) out[4 * (size_t)idx + v] = (double)z[v];
  }
}

// ------------------------------------------------------------------------------------------
// Host-side launchers.
// ------------------------------------------------------------------------------------------
template <int P, bool J8>
static hipError_t launch_small_t(const AnnealArgs& a, hipStream_t st) {
  const int waves = a.Mp / 16;
  const size_t es = (P == PREC_FP64) ? 8 : (P == PREC_FP32 ? 4 : 2);
  const size_t lds = ((size_t)a.Mp + 32) * a.lds_stride * es;
  hipError_t e = hipFuncSetAttribute((const void*)anneal_small<P, J8>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int blocks = (a.R + 15) / 16;
  hipLaunchKernelGGL((anneal_small<P, J8>), dim3(blocks), dim3(64 * waves), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_anneal_small(int prec, const AnnealArgs& a, hipStream_t st) {
  switch (prec) {
    case PREC_FP64: return launch_small_t<PREC_FP64, false>(a, st);
    case PREC_FP32: return launch_small_t<PREC_FP32, false>(a, st);
    case PREC_BF16: return launch_small_t<PREC_BF16, false>(a, st);
    case PREC_FP8J_BF16S: return launch_small_t<PREC_BF16, true>(a, st);
  }
  return hipErrorInvalidValue;
}

template <int P, bool J8>
static hipError_t launch_small_batched_t(const AnnealArgs* jobs, const int2* tasks, int n_tasks, int max_Mp,
                                         size_t lds, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void*)anneal_small_batched<P, J8>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((anneal_small_batched<P, J8>), dim3(n_tasks), dim3(64 * (max_Mp / 16)), lds, st, jobs, tasks);
  return hipGetLastError();
}

hipError_t launch_anneal_small_batched(int prec, const AnnealArgs* jobs, const int2* tasks, int n_tasks, int max_Mp,
                                       size_t lds, hipStream_t st) {
  switch (prec) {
    case PREC_FP64: return launch_small_batched_t<PREC_FP64, false>(jobs, tasks, n_tasks, max_Mp, lds, st);
    case PREC_FP32: return launch_small_batched_t<PREC_FP32, false>(jobs, tasks, n_tasks, max_Mp, lds, st);
    case PREC_BF16: return launch_small_batched_t<PREC_BF16, false>(jobs, tasks, n_tasks, max_Mp, lds, st);
    case PREC_FP8J_BF16S: return launch_small_batched_t<PREC_BF16, true>(jobs, tasks, n_tasks, max_Mp, lds, st);
  }
  return hipErrorInvalidValue;
}

size_t small_lds_bytes(int prec, int Mp, int stride) {
  const size_t es = (prec == PREC_FP64) ? 8 : (prec == PREC_FP32 ? 4 : 2);
  return ((size_t)Mp + 32) * stride * es;
}

// ------------------------------------------------------------------------------------------
// anneal_step_tiled: one iteration for large N with BF16 operands (BF16 and FP8-J precisions),
// as a tiled matrix product with the fused epilogue. Workgroup (bx, by) owns rows [256 bx, +256)
// x replicas [128 by, +128) with eight waves (two per SIMD); wave w owns rows 64 (w / 2) .. +63
// and replicas 64 (w % 2) .. +63 (4 x 4 MFMA tiles of 16 x 16). J [Mp][Kp] and S_cur [Rp][Kp]
// (both k contiguous) stream through an LDS ring of 64-k blocks (256 rows of J and 128 replicas
// of S per stage) filled by direct-to-LDS loads: with BF16 J, 2 stages, one barrier per block and
// the next block issued at each barrier (a third stage measured 3.5% slower); with FP8 / FP4 J,
// 4 stages and one barrier per two blocks, the two blocks of a group with no branch between them
// so that the second block's fragment reads are scheduled under the first block's MFMAs (25.0 ->
// 23.9 ms; 4 stages of BF16 J do not fit in LDS). Unit u (8 k) of S row q sits at
// u ^ ((q >> 1) & 7) of its 128-byte row, so the 16 lanes a ds_read_b128 serves hit distinct bank
// groups. At N = 8192, R = 1024 this is one workgroup per CU, and a quarter fewer bytes per flop
// come from L2 than with 128 x 128 tiles (measured 28.7 against 36.4 ms per 200-iteration
// anneal). Needs Mp % 256 == 0 and S buffers of roundup(R, 128) rows (padding rows zero). Each
// wave loads its tile of the FP32 master state before the k loop, so that the epilogue does not
// wait for it (27.1 -> 25.0 ms).
// JFMT: format of J in memory and LDS, the narrowest that holds the couplings exactly (0 = BF16,
// 1 = FP8 E4M3, 2 = FP4 E2M1), widened to BF16 in registers: FP8 / FP4 rows of 64 / 32 bytes per
// block cut the J bytes each block moves into LDS to a half / a quarter (stages of 32 / 24 KB
// against 48; 29.3 -> 27.0 ms with FP4). Unit u (16 bytes) of J row q sits at u ^ f(q) with
// f = (q >> 1) & 7, (q >> 2) & 3, (q >> 3) & 1 for the three formats, so the 16 rows one fragment
// read spans hit distinct banks.
// ------------------------------------------------------------------------------------------
constexpr int ST_M = 256;                 // rows per workgroup
constexpr int ST_R = 128;                 // replicas per workgroup
constexpr int ST_K = 64;                  // k per block
constexpr int ST_STAGES = 2;                // ring stages with one barrier per block (BF16 J)

template <int JFMT>
struct StFmt {
  static constexpr int JRB = JFMT == 0 ? 128 : (JFMT == 1 ? 64 : 32);  // bytes of a J row per block
  static constexpr int JT = ST_M * JRB;                               // bytes of the J tile
  static constexpr int STAGE = JT + ST_R * ST_K * 2;                  // J tile + S tile (128-byte rows)
  static constexpr int JB = JT / 1024;                                // 1 KB blocks of the J tile
  static constexpr int LPW = STAGE / 1024 / 8;                        // 1 KB loads per wave and block
  static constexpr int UPR = JRB / 16;                                // 16-byte units per J row
  // blocks per barrier: two where four stages fit in LDS (FP8 / FP4 J), else one
  static constexpr int G = JFMT == 0 ? 1 : 2;
  static constexpr int NS = G > 1 ? 2 * G : ST_STAGES;                // stages of the LDS ring
  __device__ static __forceinline__ int swz(int q) {
    return JFMT == 0 ? ((q >> 1) & 7) : (JFMT == 1 ? ((q >> 2) & 3) : ((q >> 3) & 1));
  }
};
static_assert(StFmt<0>::LPW * 8 * 1024 == StFmt<0>::STAGE && StFmt<1>::LPW * 8 * 1024 == StFmt<1>::STAGE &&
                  StFmt<2>::LPW * 8 * 1024 == StFmt<2>::STAGE,
              "every wave issues the same number of 1 KB loads per block");
static_assert(StFmt<0>::NS * StFmt<0>::STAGE <= 160 * 1024 && StFmt<1>::NS * StFmt<1>::STAGE <= 160 * 1024 &&
                  StFmt<2>::NS * StFmt<2>::STAGE <= 160 * 1024 && StFmt<1>::G <= 2 && StFmt<2>::G <= 2,
              "the ring fits in LDS; the first wait of the grouped loop covers up to two blocks per group");

// 8 FP8 E4M3 (two words) or 8 FP4 E2M1 values (one word; value 2b in the low nibble of byte b)
// widened to BF16 (exact for every value of either format)
__device__ __forceinline__ bf16x8 tiled_widen_fp8(uint2 v) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v.x, 1.0f, false);
  const bf16x2 p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v.x, 1.0f, true);
  const bf16x2 p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v.y, 1.0f, false);
  const bf16x2 p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(v.y, 1.0f, true);
  return bf16x8{p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
}
__device__ __forceinline__ bf16x8 tiled_widen_fp4(uint32_t w) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 0);
  const bf16x2 p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 1);
  const bf16x2 p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 2);
  const bf16x2 p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 3);
  return bf16x8{p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
}

template <bool B>
struct StBool {
  static constexpr bool value = B;
};

template <int NV>
__device__ __forceinline__ void step_wait_vm() {
  static_assert(NV >= 0 && NV <= 63, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0xF70 | (NV & 15) | ((NV >> 4) << 14));
}

// The body takes the kernel arguments by reference, which measured 2% faster than the same code in
// the kernel itself (the compiler then reads the arguments where they are used).
template <int JFMT>
__device__ __forceinline__ void step_tiled_body(const AnnealArgs& a, const __bf16* __restrict__ S_cur,
                                                __bf16* __restrict__ S_next, int t) {
  using F = StFmt<JFMT>;
  constexpr int NS = F::NS, G = F::G;
  constexpr int LPW = F::LPW, JB = F::JB, JRB = F::JRB, UPR = F::UPR;
  extern __shared__ __align__(16) unsigned char smem_st[];  // NS x (J tile, S tile)
  const int N = a.N, Kp = a.Kp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g4 = lane >> 4, c = lane & 15;
  const int m0 = blockIdx.x * ST_M, r0 = blockIdx.y * ST_R;
  const int wm = 64 * (wave >> 1), wr = 64 * (wave & 1);

  // direct-to-LDS loads: blocks 0 .. JB - 1 hold the J tile (1024 / JRB rows each), JB .. JB + 15
  // the S tile (eight 128-byte rows each); wave w issues blocks LPW w .. LPW w + LPW - 1. Lane l
  // fills position l % (units per row) of row (rows per block) b' + l / (units per row) (b' the
  // block within its tile) with the global unit the swizzle puts there.
  const size_t jrow = (size_t)Kp * JRB / ST_K;  // bytes of one J row in memory
  size_t goff[LPW];
#pragma unroll
  for (int u = 0; u < LPW; ++u) {
    const int b = LPW * wave + u;
    if (b < JB) {
      const int q = (1024 / JRB) * b + lane / UPR;
      const int unit = (lane % UPR) ^ F::swz(q);
      goff[u] = (size_t)(m0 + q) * jrow + unit * 16;
    } else {
      const int q = 8 * (b - JB) + (lane >> 3);
      const int unit = (lane & 7) ^ ((q >> 1) & 7);
      goff[u] = (size_t)(r0 + q) * Kp * 2 + unit * 16;
    }
  }
  const unsigned char* Jb = reinterpret_cast<const unsigned char*>(a.J);
  const unsigned char* Sb = reinterpret_cast<const unsigned char*>(S_cur);
  unsigned char* ring = smem_st;
  auto issue = [&](int kb, int stage) {
#pragma unroll
    for (int u = 0; u < LPW; ++u) {
      const int b = LPW * wave + u;
      __builtin_amdgcn_global_load_lds(
          reinterpret_cast<const uint32_t*>((b < JB ? Jb + (size_t)kb * JRB : Sb + (size_t)kb * ST_K * 2) + goff[u]),
          ring + stage * F::STAGE + b * 1024, 16, 0, 0);
    }
  };
  // fragment offsets within a 16-row tile: lane (c, g4) reads k octet o = 4 s + g4 of row c at k
  // step s (the swizzle of row q depends on q mod 16 only): S and BF16 J in unit o, FP8 J in half
  // o % 2 of unit o / 2, FP4 J in quarter o % 4 of unit o / 4
  int foff[2], joff[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int o = 4 * s + g4;
    foff[s] = c * 128 + ((o ^ ((c >> 1) & 7)) * 16);
    if (JFMT == 0) joff[s] = foff[s];
    else if (JFMT == 1) joff[s] = c * 64 + (((o >> 1) ^ F::swz(c)) * 16) + (o & 1) * 8;
    else joff[s] = c * 32 + (((o >> 2) ^ F::swz(c)) * 16) + (o & 3) * 4;
  }

  f32x4 acc[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[rt][ct][v] = 0.0f;

  const int nkb = Kp / ST_K;
  // This wave's 64 x 64 master states are loaded before the k loop, so that their latency hides
  // under the matrix work rather than stalling the epilogue. They are issued ahead of the first
  // blocks, so the first block's wait also covers them. When the wave's tile lies inside N x R and
  // N % 4 == 0 (a wave-uniform test), a lane's four rows are one 16-byte load and store.
  float* state = reinterpret_cast<float*>(a.state);
  const bool full = (N & 3) == 0 && (reinterpret_cast<uintptr_t>(state) & 15) == 0 && m0 + wm + 64 <= N &&
                    r0 + wr + 64 <= a.R;
  float st[4][4][4];
  if (full) {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const float4 v4 = *reinterpret_cast<const float4*>(state + (size_t)(r0 + wr + 16 * ct + c) * N + m0 + wm +
                                                           16 * rt + 4 * g4);
        st[rt][ct][0] = v4.x;
        st[rt][ct][1] = v4.y;
        st[rt][ct][2] = v4.z;
        st[rt][ct][3] = v4.w;
      }
  } else {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int row0 = m0 + wm + 16 * rt + 4 * g4;
        const int r = r0 + wr + 16 * ct + c;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          st[rt][ct][v] = (r < a.R && row0 + v < N) ? state[(size_t)r * N + row0 + v] : 0.0f;
      }
  }

  // one 64-k block: both k steps' fragments are read up front, so that the second step's reads
  // land under the first step's MFMAs
  auto compute = [&](int stage) {
    const unsigned char* At = ring + stage * F::STAGE + wm * JRB;
    const unsigned char* Bt = ring + stage * F::STAGE + F::JT + wr * 128;
    bf16x8 af[2][4], bfr[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const unsigned char* ap = At + 16 * JRB * i + joff[s];
        if constexpr (JFMT == 0) af[s][i] = *reinterpret_cast<const bf16x8*>(ap);
        else if constexpr (JFMT == 1) af[s][i] = tiled_widen_fp8(*reinterpret_cast<const uint2*>(ap));
        else af[s][i] = tiled_widen_fp4(*reinterpret_cast<const uint32_t*>(ap));
        bfr[s][i] = *reinterpret_cast<const bf16x8*>(Bt + 2048 * i + foff[s]);
      }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[s][rt], bfr[s][ct], acc[rt][ct], 0, 0, 0);
  };

  if constexpr (G > 1) {
    // Groups of G blocks share one barrier, over a ring of 2G stages: the barrier at group kb
    // finds blocks kb .. kb + G - 1 landed and the previous group's stages read, and the next
    // group's blocks (issued at the previous barrier, or up front) have a whole group's work to
    // land. Two blocks per barrier measured 2% faster than one.
#pragma unroll
    for (int p = 0; p < NS; ++p)
      if (p < nkb) issue(p, p);
    int kb = 0;
    for (; kb + G <= nkb; kb += G) {
      if (kb == 0) {
        // blocks G .. 2G - 1 of the up-front issue may still be in flight
        const int ahead = nkb - G;
        if (ahead >= G) step_wait_vm<LPW * G>();
        else if (ahead == 1) step_wait_vm<LPW>();
        else step_wait_vm<0>();
      } else {
        step_wait_vm<0>();
      }
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      if (kb > 0) {
#pragma unroll
        for (int j = 0; j < G; ++j)
          if (kb + G + j < nkb) issue(kb + G + j, (kb + G + j) % NS);
      }
      // a whole group with no branch between its blocks, so that the next block's fragment reads
      // can be scheduled under the current block's MFMAs
#pragma unroll
      for (int j = 0; j < G; ++j) compute((kb + j) % NS);
      // the reads of this group are complete before the next barrier frees its stages
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (kb < nkb) {
      // the last nkb % G blocks, issued at the previous barrier (or up front)
      step_wait_vm<0>();
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < G - 1; ++j)
        if (kb + j < nkb) compute((kb + j) % NS);
    }
  } else {
    constexpr int LA = NS - 1;  // blocks issued ahead
    static_assert(LA >= 1 && LA <= 3, "the waits below cover up to two blocks in flight");
#pragma unroll
    for (int p = 0; p < LA; ++p)
      if (p < nkb) issue(p, p);
    for (int kb = 0; kb < nkb; ++kb) {
      // this wave's part of block kb has landed (the blocks after it may still be in flight)
      const int rem = nkb - 1 - kb;
      if (rem >= LA - 1) step_wait_vm<LPW * (LA - 1)>();
      else if (rem == 0) step_wait_vm<0>();
      else if (rem == 1) step_wait_vm<LPW>();
      else step_wait_vm<2 * LPW>();
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_barrier();  // every wave's part landed; every wave is done with block kb - 1
      __builtin_amdgcn_sched_barrier(0);
      if (kb + LA < nkb) issue(kb + LA, (kb + LA) % NS);
      compute(kb % NS);
      // the reads of this block are complete before the next barrier frees its buffer
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // ---- fused epilogue (the FP32 epilogue shared by every kernel) --------------------------------
  const float* inv_g = reinterpret_cast<const float*>(a.inv_norm);
  const float* h_g = reinterpret_cast<const float*>(a.hterm);
  float* traj = reinterpret_cast<float*>(a.traj);
  if (!(traj && t - a.t_begin < a.record)) traj = nullptr;
  else traj += (size_t)(t - a.t_begin) * a.R * N;
  const bool vec_traj = full && (reinterpret_cast<uintptr_t>(traj) & 15) == 0;
  const float coef_t = reinterpret_cast<const float*>(a.coef)[t - 1];
  // two copies of the epilogue, so that the bounds tests of a partial tile stay out of the full one
  auto epilogue = [&](auto full_c) {
    constexpr bool FULL = decltype(full_c)::value;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int row0 = m0 + wm + 16 * rt + 4 * g4;
      // inv_norm and hterm hold Mp entries (zero past N) and row0 is a multiple of 4
      const float4 inv4 = *reinterpret_cast<const float4*>(inv_g + row0);
      const float4 h4 = *reinterpret_cast<const float4*>(h_g + row0);
      const float inv[4] = {inv4.x, inv4.y, inv4.z, inv4.w};
      const float hv[4] = {h4.x, h4.y, h4.z, h4.w};
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int r = r0 + wr + 16 * ct + c;
        const bool live_r = FULL || r < a.R;
        float* sv = st[rt][ct];
        float fld[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) fld[v] = acc[rt][ct][v];
        Epilogue<PREC_BF16>::apply(fld, inv, hv, sv, a, coef_t, (uint32_t)(row0 >> 2), (uint32_t)r, (uint32_t)t);
        __bf16 outv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (!FULL && (row0 + v >= N || !live_r)) sv[v] = 0.0f;
          outv[v] = (__bf16)sv[v];
        }
        *reinterpret_cast<uint2*>(S_next + (size_t)r * Kp + row0) = *reinterpret_cast<const uint2*>(outv);
        float* sp = state + (size_t)r * N + row0;
        float* tp = traj + (size_t)r * N + row0;
        if constexpr (FULL) {
          const float4 o4 = make_float4(sv[0], sv[1], sv[2], sv[3]);
          *reinterpret_cast<float4*>(sp) = o4;
          if (traj) {
            if (vec_traj) *reinterpret_cast<float4*>(tp) = o4;
            else
#pragma unroll
              for (int v = 0; v < 4; ++v) tp[v] = sv[v];
          }
        } else if (live_r) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (row0 + v < N) {
              sp[v] = sv[v];
              if (traj) tp[v] = sv[v];
            }
        }
      }
    }
  };
  if (full) epilogue(StBool<true>{});
  else epilogue(StBool<false>{});
}

template <int JFMT>
__global__ __launch_bounds__(512, 1) void anneal_step_tiled(AnnealArgs a, const __bf16* __restrict__ S_cur,
                                                            __bf16* __restrict__ S_next, int t) {
  step_tiled_body<JFMT>(a, S_cur, S_next, t);
}

// ------------------------------------------------------------------------------------------
// anneal_step_tiled_f64: one FP64 iteration as a tiled matrix product with the fused FP64
// epilogue (the validation path for large N). Workgroup (bx, by) owns rows [128 bx, +128) x
// replicas [64 by, +64); wave w owns rows 32 w .. +31 (two 16-row tiles) for all 64 replicas
// (four 16-column tiles): eight v_mfma_f64_16x16x4f64 accumulators. J [Mp][Kp] and S_cur
// [Rp][Kp] (FP64, k contiguous) stream through a 3-stage LDS ring of 32-k blocks (32 KB of J and
// 16 KB of S per stage), filled by direct-to-LDS loads issued two blocks ahead. A block is four
// 8-k windows of two MFMA steps; in window i, step s, lane group g carries k = 8 i + 2 g + s for
// A and B alike (a dot product does not depend on the order of its terms), so every lane reads
// both steps' operands with one ds_read_b128. The 16-byte unit u of tile row q is stored at
// u ^ (q & 15) of its 256-byte row, so the 8 lanes one LDS cycle serves hit 8 distinct bank
// groups (the A rows of a 16-row tile are permuted as the FP64 instruction's output needs, which
// keeps them distinct modulo 16). Needs Mp % 128 == 0, Kp % 32 == 0 and S buffers of Rp rows
// (padding rows zero).
// ------------------------------------------------------------------------------------------
constexpr int SF_M = 128;                     // rows per workgroup
constexpr int SF_R = 64;                      // replicas per workgroup
constexpr int SF_K = 32;                      // k per block
constexpr int SF_STAGES = 3;
constexpr int SF_JT = SF_M * SF_K * 8;        // bytes of the J tile of one block (32 KB)
constexpr int SF_STAGE = SF_JT + SF_R * SF_K * 8;  // J tile + S tile (48 KB)
constexpr int SF_LPW = SF_STAGE / 1024 / 4;   // 1 KB direct-to-LDS loads per wave and block (12)

__global__ __launch_bounds__(256, 1) void anneal_step_tiled_f64(AnnealArgs a, const double* __restrict__ S_cur,
                                                                double* __restrict__ S_next, int t) {
  using Tr = Traits<PREC_FP64>;
  extern __shared__ __align__(16) unsigned char smem_sf[];  // SF_STAGES x (J tile, S tile)
  const int N = a.N, Kp = a.Kp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int m0 = blockIdx.x * SF_M, r0 = blockIdx.y * SF_R;

  // direct-to-LDS loads: 48 blocks of 1 KB per stage (blocks 0..31 the J tile, 32..47 the S
  // tile, four tile rows each); wave w issues blocks 12 w .. 12 w + 11. Lane l fills position
  // l % 16 of tile row 4 (b % 32) + l / 16 with the global unit the swizzle puts there.
  size_t goff[SF_LPW];
#pragma unroll
  for (int u = 0; u < SF_LPW; ++u) {
    const int b = SF_LPW * wave + u;
    const bool is_j = b < 32;
    const int q = 4 * (is_j ? b : b - 32) + (lane >> 4);
    const int unit = (lane & 15) ^ (q & 15);
    goff[u] = is_j ? ((size_t)(m0 + q) * Kp + 2 * unit) * 8 : ((size_t)(r0 + q) * Kp + 2 * unit) * 8;
  }
  const unsigned char* Jb = reinterpret_cast<const unsigned char*>(a.J);
  const unsigned char* Sb = reinterpret_cast<const unsigned char*>(S_cur);
  unsigned char* ring = smem_sf;
  auto issue = [&](int kb, int stage) {
#pragma unroll
    for (int u = 0; u < SF_LPW; ++u) {
      const int b = SF_LPW * wave + u;
      const unsigned char* src = (b < 32 ? Jb : Sb) + goff[u] + (size_t)kb * SF_K * 8;
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint32_t*>(src), ring + stage * SF_STAGE + b * 1024,
                                       16, 0, 0);
    }
  };
  // fragment offsets within a stage: A row 32 wave + 16 rt + a_row(c), B replica 16 ct + c; window
  // i reads unit 4 i + g of its row
  int aoff[2][4], boff[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int q = 32 * wave + 16 * rt + Tr::a_row(c);
      aoff[rt][i] = q * 256 + (((4 * i + g) ^ (q & 15)) * 16);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int q = 16 * ct + c;
      boff[ct][i] = SF_JT + q * 256 + (((4 * i + g) ^ (q & 15)) * 16);
    }
  }

  f64x4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[rt][ct][v] = 0.0;

  const int nkb = Kp / SF_K;
  issue(0, 0);
  if (nkb > 1) issue(1, 1);
  for (int kb = 0; kb < nkb; ++kb) {
    // this wave's part of block kb has landed (block kb + 1 may still be in flight)
    if (kb + 1 < nkb) step_wait_vm<SF_LPW>();
    else step_wait_vm<0>();
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_barrier();  // every wave's part landed; every wave is done with block kb - 1
    __builtin_amdgcn_sched_barrier(0);
    if (kb + 2 < nkb) issue(kb + 2, (kb + 2) % SF_STAGES);
    const unsigned char* base = ring + (kb % SF_STAGES) * SF_STAGE;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double2 af[2], bfr[4];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) af[rt] = *reinterpret_cast<const double2*>(base + aoff[rt][i]);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) bfr[ct] = *reinterpret_cast<const double2*>(base + boff[ct][i]);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          acc[rt][ct] = Tr::mfma(af[rt].x, bfr[ct].x, acc[rt][ct]);
          acc[rt][ct] = Tr::mfma(af[rt].y, bfr[ct].y, acc[rt][ct]);
        }
    }
    // the reads of this block are complete before the next barrier frees its buffer
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_sched_barrier(0);
  }

  // ---- fused FP64 epilogue (the one every FP64 kernel shares) ----------------------------------
  const double* inv_g = reinterpret_cast<const double*>(a.inv_norm);
  const double* h_g = reinterpret_cast<const double*>(a.hterm);
  double* state = reinterpret_cast<double*>(a.state);
  double* traj = reinterpret_cast<double*>(a.traj);
  const double coef_t = reinterpret_cast<const double*>(a.coef)[t - 1];
  const int k_rec = t - a.t_begin;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int row0 = m0 + 32 * wave + 16 * rt + 4 * g;
    double inv[4], hv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      inv[v] = inv_g[row0 + v];
      hv[v] = h_g[row0 + v];
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int r = r0 + 16 * ct + c;
      const bool live_r = r < a.R;
      double s[4], fld[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        fld[v] = acc[rt][ct][v];
        s[v] = (live_r && row0 + v < N) ? state[(size_t)r * N + row0 + v] : 0.0;
      }
      Epilogue<PREC_FP64>::apply(fld, inv, hv, s, a, coef_t, (uint32_t)(row0 >> 2), (uint32_t)r, (uint32_t)t);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (row0 + v >= N || !live_r) s[v] = 0.0;
      double* dst = S_next + (size_t)r * Kp + row0;
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[v] = s[v];
      if (live_r) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (row0 + v < N) {
            state[(size_t)r * N + row0 + v] = s[v];
            if (traj && k_rec < a.record) traj[((size_t)k_rec * a.R + r) * N + row0 + v] = s[v];
          }
      }
    }
  }
}

template <int JFMT>
static hipError_t launch_step_tiled(const AnnealArgs& a, const void* S_cur, void* S_next, int t, hipStream_t st) {
  const size_t lds = (size_t)StFmt<JFMT>::NS * StFmt<JFMT>::STAGE;
  hipError_t e = hipFuncSetAttribute((const void*)anneal_step_tiled<JFMT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid(a.Mp / ST_M, (a.R + ST_R - 1) / ST_R);
  hipLaunchKernelGGL(anneal_step_tiled<JFMT>, grid, dim3(512), lds, st, a, (const __bf16*)S_cur, (__bf16*)S_next, t);
  return hipGetLastError();
}

hipError_t launch_anneal_step(int prec, int jfmt, const AnnealArgs& a, const void* S_cur, void* S_next, int t,
                              hipStream_t st) {
  if (prec == PREC_BF16 || prec == PREC_FP8J_BF16S) {
    if (a.Mp % ST_M == 0 && a.Kp % ST_K == 0) {
      if (jfmt == 2) return launch_step_tiled<2>(a, S_cur, S_next, t, st);
      if (jfmt == 1) return launch_step_tiled<1>(a, S_cur, S_next, t, st);
      return launch_step_tiled<0>(a, S_cur, S_next, t, st);
    }
    if (jfmt != 0) return hipErrorInvalidValue;  // the direct kernel below reads BF16 J
  }
  if (prec == PREC_FP64 && a.Mp % SF_M == 0 && a.Kp % SF_K == 0 && a.Rp % SF_R == 0) {
    const size_t lds = (size_t)SF_STAGES * SF_STAGE;
    hipError_t e = hipFuncSetAttribute((const void*)anneal_step_tiled_f64,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const dim3 grid(a.Mp / SF_M, a.Rp / SF_R);
    hipLaunchKernelGGL(anneal_step_tiled_f64, grid, dim3(256), lds, st, a, (const double*)S_cur, (double*)S_next, t);
    return hipGetLastError();
  }
  const dim3 grid(a.Mp / 64, a.Rp / 64);
  switch (prec) {
    case PREC_FP64:
      hipLaunchKernelGGL((anneal_step<PREC_FP64>), grid, dim3(256), 0, st, a, S_cur, S_next, t);
      break;
    case PREC_FP32:
      hipLaunchKernelGGL((anneal_step<PREC_FP32>), grid, dim3(256), 0, st, a, S_cur, S_next, t);
      break;
    case PREC_BF16:
    case PREC_FP8J_BF16S:
      hipLaunchKernelGGL((anneal_step<PREC_BF16>), grid, dim3(256), 0, st, a, S_cur, S_next, t);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t sparse_lds_bytes(int prec, int N, int RB) {
  return (size_t)2 * 4 * ((N + 3) / 4) * RB * (prec == PREC_FP64 ? 8 : 4);
}

// Register-ELL variants: RB replicas per thread (4, 2, 1), DM = D rounded up to 4 / 8 / 16,
// QP quads per thread (1 up to 512 quads, 2 up to 1024), with QP * DM * (value words + 1) <= 32.
// FP64 keeps RB <= 2, and RB = 2 only for DM = 4, QP = 1: its epilogue, unrolled over the
// replicas, would spill otherwise.
template <int P, int RB>
static const void* rq_fn_d(int DM, int QP) {
  if (QP == 1) {
    if (DM == 4) return (const void*)anneal_sparse_rq<P, RB, 4, 1>;
    if (DM == 8) return (const void*)anneal_sparse_rq<P, RB, 8, 1>;
    if constexpr (P != PREC_FP64)
      if (DM == 16) return (const void*)anneal_sparse_rq<P, RB, 16, 1>;
  } else if (QP == 2) {
    if (DM == 4) return (const void*)anneal_sparse_rq<P, RB, 4, 2>;
    if constexpr (P != PREC_FP64)
      if (DM == 8) return (const void*)anneal_sparse_rq<P, RB, 8, 2>;
  }
  return nullptr;
}

static const void* rq_fn(int prec, int RB, int DM, int QP) {
  if (prec == PREC_FP64) {
    if (RB == 2) return DM == 4 && QP == 1 ? (const void*)anneal_sparse_rq<PREC_FP64, 2, 4, 1> : nullptr;
    return RB == 1 ? rq_fn_d<PREC_FP64, 1>(DM, QP) : nullptr;
  }
  if (RB == 4) return rq_fn_d<PREC_FP32, 4>(DM, QP);
  if (RB == 2) return rq_fn_d<PREC_FP32, 2>(DM, QP);
  return RB == 1 ? rq_fn_d<PREC_FP32, 1>(DM, QP) : nullptr;
}

struct SparseRq {
  const void* fn;
  int RB, threads;
  size_t lds;
};

// Picks the variant for (prec, N, D, R): the largest RB whose state fits in LDS and whose grid
// still covers every CU (RB = 1 when none does); then RB = 4 gives way to RB = 2 when it leaves
// the CUs under 16 resident waves and two RB = 2 workgroups fit on a CU (more waves hide the LDS
// and transcendental latencies better than a third and fourth replica per thread). Returns 0
// where the generic kernel must run.
static int sparse_rq_pick(int prec, int N, int D, int R, SparseRq* o) {
  const int Nq = (N + 3) / 4;
  const int QP = Nq <= 512 ? 1 : (Nq <= 1024 ? 2 : 0);
  const int DM = D <= 4 ? 4 : (D <= 8 ? 8 : (D <= 16 ? 16 : 0));
  if (!QP || !DM || QP * DM * (prec == PREC_FP64 ? 3 : 2) > 32) return 0;
  int dev = 0, cus = 256, max_lds = 65536;
  if (hipGetDevice(&dev) == hipSuccess) {
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  }
  const size_t word = prec == PREC_FP64 ? 8 : 4;
  const int threads = ((Nq + QP - 1) / QP + 63) / 64 * 64;
  auto lds_of = [&](int rb) { return (size_t)2 * 4 * Nq * rb * word; };
  auto fits = [&](int rb) { return lds_of(rb) <= (size_t)max_lds && rq_fn(prec, rb, DM, QP) != nullptr; };
  auto per_cu = [&](int rb) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, rq_fn(prec, rb, DM, QP), threads, lds_of(rb)) != hipSuccess)
      return 0;
    return nb;
  };
  int RB = 0;
  for (int rb : {4, 2, 1}) {
    if (!fits(rb)) continue;
    RB = rb;
    if ((R + rb - 1) / rb >= cus) break;
  }
  if (!RB) return 0;
  if (RB == 4 && fits(2)) {
    const int g4 = (R + 3) / 4, g2 = (R + 1) / 2, waves = threads / 64;
    const long res4 = (long)std::min(g4, cus * std::max(per_cu(4), 1)) * waves;
    if (res4 < 16L * cus && g2 >= 2 * cus && per_cu(2) >= 2) RB = 2;
  }
  o->fn = rq_fn(prec, RB, DM, QP);
  o->RB = RB;
  o->threads = threads;
  o->lds = lds_of(RB);
  return o->fn != nullptr;
}

int sparse_rq_applies(int prec, int N, int D) {
  SparseRq c;
  return sparse_rq_pick(prec, N, D, 1, &c);
}

hipError_t launch_anneal_sparse(int prec, const AnnealArgs& a, const int* ell_col, const void* ell_val, int D,
                                int RB, int allow_rq, int* used_rq, hipStream_t st) {
  SparseRq c;
  const bool rq = allow_rq && sparse_rq_pick(prec, a.N, D, a.R, &c);
  if (used_rq) *used_rq = rq ? 1 : 0;
  if (rq) {
    hipError_t e = hipFuncSetAttribute(c.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
    if (e != hipSuccess) return e;
    AnnealArgs args = a;
    const void* col = ell_col;
    const void* val = ell_val;
    int d = D;
    void* kargs[] = {&args, &col, &val, &d};
    return hipLaunchKernel(c.fn, dim3((a.R + c.RB - 1) / c.RB), dim3(c.threads), kargs, c.lds, st);
  }
  const int grid = (a.R + RB - 1) / RB;
  const size_t lds = sparse_lds_bytes(prec, a.N, RB);
  const void* fn = prec == PREC_FP64 ? (const void*)anneal_sparse<PREC_FP64> : (const void*)anneal_sparse<PREC_FP32>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  // 16 waves per workgroup (4 per SIMD; 8 waves in FP64, whose epilogue needs more registers): the
  // gathers and the epilogue of one wave hide behind the others
  if (prec == PREC_FP64)
    hipLaunchKernelGGL((anneal_sparse<PREC_FP64>), dim3(grid), dim3(512), lds, st, a, ell_col, ell_val, D, RB);
  else
    hipLaunchKernelGGL((anneal_sparse<PREC_FP32>), dim3(grid), dim3(1024), lds, st, a, ell_col, ell_val, D, RB);
  return hipGetLastError();
}

hipError_t launch_energy_i8(const int8_t* J8p, int Np, const double* h, int h_integral, const int8_t* spins,
                            int N, int R, int8_t* Sp, unsigned long long* E2, long long* E_int, double* E,
                            hipStream_t st) {
  const int Rp = (R + 63) / 64 * 64;
  const size_t total = (size_t)Rp * Np;
  const int pb = (int)std::min<size_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(pad_spins_kernel, dim3(pb), dim3(256), 0, st, spins, N, R, Sp, Np, Rp);
  hipLaunchKernelGGL(zero_u64_kernel, dim3((R + 255) / 256), dim3(256), 0, st, E2, R);
  hipLaunchKernelGGL(energy_pairs_i8, dim3(Np / 64, Rp / 64), dim3(256), 0, st, J8p, (const int8_t*)Sp, Np, R, E2);
  hipLaunchKernelGGL(energy_finish_kernel, dim3((R + 127) / 128), dim3(128), 0, st, (const unsigned long long*)E2,
                     h, h_integral, spins, N, R, E_int, E);
  return hipGetLastError();
}

hipError_t launch_pack_state(int prec, const void* state, void* S, int N, int R, int Kp, int ld, int Rp, int zero,
                             hipStream_t st) {
  const size_t total = (size_t)Rp * Kp;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
  switch (prec) {
    case PREC_FP64:
      hipLaunchKernelGGL((pack_state_kernel<double, double>), dim3(blocks), dim3(256), 0, st,
                         (const double*)state, (double*)S, N, R, Kp, ld, Rp, zero);
      break;
    case PREC_FP32:
      hipLaunchKernelGGL((pack_state_kernel<float, float>), dim3(blocks), dim3(256), 0, st,
                         (const float*)state, (float*)S, N, R, Kp, ld, Rp, zero);
      break;
    case PREC_FP8J_FP8S:
      hipLaunchKernelGGL(pack_state_fp8_kernel, dim3(blocks), dim3(256), 0, st, (const float*)state, (uint8_t*)S, N,
                         R, Kp, ld, Rp, zero);
      break;
    default:
      hipLaunchKernelGGL((pack_state_kernel<__bf16, float>), dim3(blocks), dim3(256), 0, st,
                         (const float*)state, (__bf16*)S, N, R, Kp, ld, Rp, zero);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_readout(int prec, const void* state, int8_t* spins, size_t count, hipStream_t st) {
  const int blocks = (int)std::min<size_t>((count + 255) / 256, 8192);
  if (prec == PREC_FP64)
    hipLaunchKernelGGL((readout_kernel<double>), dim3(blocks), dim3(256), 0, st, (const double*)state,
                       spins, count);
  else
    hipLaunchKernelGGL((readout_kernel<float>), dim3(blocks), dim3(256), 0, st, (const float*)state,
                       spins, count);
  return hipGetLastError();
}

hipError_t launch_energy(const int8_t* J8, const double* J64, const double* h, int h_integral,
                         const int8_t* spins, int N, int R, long long* E_int, double* E, hipStream_t st) {
  hipLaunchKernelGGL(energy_kernel, dim3(R), dim3(256), 0, st, J8, J64, h, h_integral, spins, N, R,
                     E_int, E);
  return hipGetLastError();
}

hipError_t launch_noise_words(uint32_t k0, uint32_t k1, uint32_t t, uint32_t r0, int nrep, int nq,
                              uint32_t* out, hipStream_t st) {
  const int total = nrep * nq;
  hipLaunchKernelGGL(noise_words_kernel, dim3((total + 255) / 256), dim3(256), 0, st, k0, k1, t, r0, nrep,
                     nq, out);
  return hipGetLastError();
}

hipError_t launch_noise_values(uint32_t k0, uint32_t k1, uint32_t t, uint32_t r0, int nrep, int nq,
                               int fp64, double* out, hipStream_t st) {
  const int total = nrep * nq;
  hipLaunchKernelGGL(noise_values_kernel, dim3((total + 255) / 256), dim3(256), 0, st, k0, k1, t, r0,
                     nrep, nq, fp64, out);
  return hipGetLastError();
}

}  // namespace nmfa
