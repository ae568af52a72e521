// Persistent large-N NMFA kernel for gfx950: replica groups annealed by the workgroups of one XCD.
//
// Algorithm 1 (paper Sec. II) is synchronous: every iteration needs all N spins of the previous
// one. For large N a replica group is therefore spread over P workgroups (one per CU) that each
// own 64 rows of J; after each iteration the group exchanges its new spins through memory and
// meets at a barrier.
//
//   * J: the workgroup's 64 rows stay in LDS for the whole anneal, in the narrowest format that
//     holds them exactly: FP4 E2M1 (couplings in {0, +-1/2, +-1, +-3/2, +-2, +-3, +-4, +-6}), FP8
//     E4M3, or BF16; chunks of 8 values XOR-swizzled by row so the A-fragment reads are conflict
//     free. Every format is widened to BF16 in registers for the MFMA.
//   * S: the operand copy (BF16) of the group's spins lives in global memory, double-buffered by
//     iteration parity, layout [replica][Kp]. Each iteration the workgroup streams it through
//     LDS with the direct-to-LDS loads of gfx950 (global_load_lds_dwordx4) in chunks of 64 k
//     (16 KB), through a ring of up to 6 buffers (what the LDS beside J allows), so several
//     chunks are in flight from L2 while the MFMAs consume the oldest one. The fragments of the
//     next chunk are read from LDS into a second register set while the MFMAs of the current
//     chunk run, so LDS latency is hidden behind matrix work.
//   * Wave (a, b) of the 8 waves (two per SIMD, so one hides the other's LDS latency) computes 32
//     rows (two 16-row tiles) x 32 replicas (two 16-column tiles) with v_mfma_f32_16x16x32_bf16.
//   * The epilogue (normalisation, Philox noise, tanh, damped update) runs in registers on the
//     accumulator layout; the FP32 master state never leaves the registers between iterations.
//   * Barrier: the P workgroups of a group count arrivals with a device-scope atomic and poll it
//     with device-scope loads. When every group sits inside one XCD (checked at start-up from
//     the XCC_ID hardware register) the new spins are exchanged through that XCD's L2: stores
//     complete before the arrival, and readers invalidate their L1 after the barrier. Otherwise
//     the workgroups fall back to device-scope release/acquire fences.
//   * Every wait is bounded; a timeout raises an abort flag that ends every workgroup's loop and
//     is reported to the host as an error.
#include <hip/hip_runtime.h>

#include <utility>

#include "nmfa_device.h"
#include "nmfa_internal.h"

namespace nmfa {

// control block layout (uint32 words)
enum : int {
  CTL_REG = 0,        // [16] workgroups registered per XCD
  CTL_TOTAL = 16,     // workgroups registered
  CTL_ABORT = 17,     // barrier timeout
  CTL_MODE = 18,      // 1 = XCD-local exchange, 2 = device-scope fences (written by workgroup 0)
  CTL_BAR = 64,       // group barrier counters, one per 16 words
  CTL_WG = 64 + 16 * 256,  // per workgroup: group, row block, exchange mode (4 words each)
  CTL_WORDS = 64 + 16 * 256 + 4 * 256,
};

constexpr int XCD_ROWS = 64;   // rows of J per workgroup
constexpr int XCD_RG = 128;    // replicas per group
constexpr int XCD_KC = 64;     // k per streamed spin chunk

constexpr unsigned SPIN_LIMIT = 1u << 22;  // about a second of polling

__device__ __forceinline__ unsigned ld_dev(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Widen 8 FP8 E4M3 values (two 32-bit words) to 8 BF16 (exact for every FP8 value).
__device__ __forceinline__ bf16x8 fp8x8_to_bf16x8(uint32_t lo, uint32_t hi) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 1.0f, false);
  const bf16x2 p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 1.0f, true);
  const bf16x2 p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 1.0f, false);
  const bf16x2 p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 1.0f, true);
  bf16x8 r;
  r[0] = p0[0]; r[1] = p0[1]; r[2] = p1[0]; r[3] = p1[1];
  r[4] = p2[0]; r[5] = p2[1]; r[6] = p3[0]; r[7] = p3[1];
  return r;
}

// Widen 8 FP4 E2M1 values (one 32-bit word, value 2b in the low nibble of byte b) to 8 BF16.
__device__ __forceinline__ bf16x8 fp4x8_to_bf16x8(uint32_t w) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 0);
  const bf16x2 p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 1);
  const bf16x2 p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 2);
  const bf16x2 p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp4(w, 1.0f, 3);
  bf16x8 r;
  r[0] = p0[0]; r[1] = p0[1]; r[2] = p1[0]; r[3] = p1[1];
  r[4] = p2[0]; r[5] = p2[1]; r[6] = p3[0]; r[7] = p3[1];
  return r;
}

// Wait until at most N of this wave's vector-memory operations are outstanding (N <= 63: the
// counter's low four bits sit in bits 3:0 of the immediate, the high two in bits 15:14; LDS and
// export counters are not waited on).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N <= 63, "vmcnt immediate");
  __builtin_amdgcn_s_waitcnt(0xF70 | (N & 15) | ((N >> 4) << 14));
}

// Wait until this wave's LDS reads (and scalar loads) are complete; vector-memory counters are
// left alone.
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Workgroup barrier without the memory fence of __syncthreads (which would also wait for the
// chunks still in flight); the asm statements keep the compiler from moving LDS accesses across.
__device__ __forceinline__ void bare_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Where a workgroup sits: its replica group, its row block and the exchange mode.
struct XcdSlot {
  unsigned my_group;  // group index within this launch
  int rb;             // row block
  bool xcd_mode;      // spins exchanged through the XCD's L2 (no device-scope fences)
  bool aborted;
};

// Registration: every workgroup reports its XCD (HW_REG_XCC_ID); when each XCD holds a multiple
// of P workgroups, groups are formed inside XCDs, else by launch order with device-scope fences.
// Thread 0 does the work; the result is broadcast through this workgroup's control words.
__device__ XcdSlot xcd_register(const XcdArgs& x, int tid) {
  unsigned* ctl = x.ctl;
  const unsigned P = (unsigned)x.P;
  if (tid == 0) {
    const unsigned xcc = __builtin_amdgcn_s_getreg((20) | (0 << 6) | (15 << 11)) & 0xfu;
    const unsigned slot = atomicAdd(&ctl[CTL_REG + xcc], 1u);
    atomicAdd(&ctl[CTL_TOTAL], 1u);
    unsigned spins = 0;
    while (ld_dev(&ctl[CTL_TOTAL]) < gridDim.x) {
      if (++spins > SPIN_LIMIT) {
        atomicExch(&ctl[CTL_ABORT], 1u);
        break;
      }
    }
    // XCD-local exchange needs every XCD's workgroup count to be a multiple of P.
    unsigned base = 0, ok = 1;
    for (unsigned k = 0; k < 16; ++k) {
      const unsigned cnt = ld_dev(&ctl[CTL_REG + k]);
      if (cnt % P) ok = 0;
      if (k < xcc) base += cnt;
    }
    unsigned* info = &ctl[CTL_WG + 4 * blockIdx.x];
    info[0] = ok ? (base + slot) / P : blockIdx.x / P;
    info[1] = ok ? slot % P : blockIdx.x % P;
    info[2] = (ok && !x.force_fenced) ? 1u : 0u;
    if (blockIdx.x == 0) atomicMax(&ctl[CTL_MODE], (ok && !x.force_fenced) ? 1u : 2u);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  XcdSlot r;
  r.my_group = __builtin_amdgcn_readfirstlane(ld_dev(&ctl[CTL_WG + 4 * blockIdx.x]));
  r.rb = (int)__builtin_amdgcn_readfirstlane(ld_dev(&ctl[CTL_WG + 4 * blockIdx.x + 1]));
  r.xcd_mode = ld_dev(&ctl[CTL_WG + 4 * blockIdx.x + 2]) != 0;
  r.aborted = ld_dev(&ctl[CTL_ABORT]) != 0;
  return r;
}

// Group barrier after the new spins are stored, in two halves so that work which does not
// depend on the other workgroups can run in between. Arrive: this workgroup's stores are
// complete (and released to the device when the group spans XCDs); one thread adds to the
// group's counter.
__device__ __forceinline__ void xcd_group_arrive(unsigned* bar, bool xcd_mode, int tid) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores of the new spins are complete
  __syncthreads();
  if (tid == 0) {
    if (!xcd_mode) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Wait: one thread polls until all P workgroups have arrived for this epoch (bounded), then the
// other workgroups' spins are made visible. Returns whether the anneal was aborted (a wait timed
// out somewhere).
__device__ __forceinline__ bool xcd_group_wait(const XcdArgs& x, unsigned* bar, unsigned epoch, bool xcd_mode,
                                               int tid) {
  unsigned* ctl = x.ctl;
  if (tid == 0) {
    const unsigned target = (unsigned)x.P * epoch;
    unsigned spins = 0;
    while (ld_dev(bar) < target) {
      if (++spins > SPIN_LIMIT || ld_dev(&ctl[CTL_ABORT])) {
        atomicExch(&ctl[CTL_ABORT], 1u);
        break;
      }
    }
    if (!xcd_mode) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (xcd_mode) asm volatile("buffer_inv sc0" ::: "memory");  // drop stale L1 lines
  return ld_dev(&ctl[CTL_ABORT]) != 0;
}

// Wait of the register-J kernel, which keeps the round trips to L2 off its critical path: the
// caller polls the counter once ahead (seen, read while it draws the next noise), the polling
// thread reads the abort word only every 64 polls, and its decision reaches the other waves
// through an LDS word (abort_word) rather than a load of the control block by every thread.
// Every wave of the workgroup therefore sees the same decision.
__device__ __forceinline__ bool xrj_group_wait(const XcdArgs& x, unsigned* bar, unsigned epoch, bool xcd_mode,
                                               int tid, unsigned seen, unsigned* abort_word) {
  unsigned* ctl = x.ctl;
  if (tid == 0) {
    const unsigned target = (unsigned)x.P * epoch;
    unsigned ab = 0;
    if (seen < target) {
      unsigned spins = 0;
      while (ld_dev(bar) < target) {
        if ((++spins & 63u) == 0 && (spins > SPIN_LIMIT || ld_dev(&ctl[CTL_ABORT]))) {
          atomicExch(&ctl[CTL_ABORT], 1u);
          ab = 1;
          break;
        }
      }
    }
    if (!xcd_mode) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *abort_word = ab;
  }
  __syncthreads();
  if (xcd_mode) asm volatile("buffer_inv sc0" ::: "memory");  // drop stale L1 lines
  return *abort_word != 0;
}

__device__ __forceinline__ bool xcd_group_barrier(const XcdArgs& x, unsigned* bar, unsigned epoch,
                                                  bool xcd_mode, int tid) {
  xcd_group_arrive(bar, xcd_mode, tid);
  return xcd_group_wait(x, bar, epoch, xcd_mode, tid);
}

// Raw J fragment of one lane for one k-step: 8 values as 16 (BF16), 8 (FP8) or 4 (FP4) bytes.
template <int JFMT> struct JRaw;
template <> struct JRaw<0> { typedef bf16x8 T; };
template <> struct JRaw<1> { typedef uint2 T; };
template <> struct JRaw<2> { typedef uint32_t T; };

template <int JFMT>
__device__ __forceinline__ bf16x8 widen(const typename JRaw<JFMT>::T& v);
template <> __device__ __forceinline__ bf16x8 widen<0>(const bf16x8& v) { return v; }
template <> __device__ __forceinline__ bf16x8 widen<1>(const uint2& v) { return fp8x8_to_bf16x8(v.x, v.y); }
template <> __device__ __forceinline__ bf16x8 widen<2>(const uint32_t& v) { return fp4x8_to_bf16x8(v); }

// JFMT: 0 = BF16, 1 = FP8 E4M3, 2 = FP4 E2M1 (format of J in global memory and in LDS);
// NB: spin chunk buffers in LDS.
template <int JFMT, int NB>
__global__ __launch_bounds__(512, 1) void anneal_xcd(AnnealArgs a, XcdArgs x) {
  extern __shared__ __align__(16) unsigned char smem[];  // all of LDS: J rows + S chunk ring
  constexpr int KC = XCD_KC;
  constexpr int CHUNK_BYTES = XCD_RG * KC * 2;  // 128 replicas x KC k, BF16
  constexpr int ROW_B = KC * 2;                 // bytes of one replica row in a chunk
  constexpr int COLS = KC / 8;                  // 16-byte columns per row
  constexpr int DPW = CHUNK_BYTES / 1024 / 8;   // 1 KB direct-to-LDS loads per wave and chunk
  constexpr int KSTEPS = KC / 32;
  constexpr int CB = JFMT == 0 ? 16 : (JFMT == 1 ? 8 : 4);  // bytes of 8 J values
  typedef typename JRaw<JFMT>::T AT;
  const int N = a.N, Kp = a.Kp, P = x.P, ks = x.ks;
  const int jrow = JFMT == 0 ? Kp * 2 : (JFMT == 1 ? Kp : Kp / 2);  // bytes of one J row
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g4 = lane >> 4, c = lane & 15;
  const int wa = wave >> 2, wb = wave & 3;  // rows 32*wa.., replicas 32*wb..
  unsigned* ctl = x.ctl;

  // ---- registration: find the XCD of every workgroup, then agree on the mapping -------------
  const XcdSlot slot = xcd_register(x, tid);
  const unsigned my_group = slot.my_group;
  const int group = (int)my_group + x.group_base;
  const int rb = slot.rb;
  const bool xcd_mode = slot.xcd_mode;
  bool aborted = slot.aborted;

  // ---- LDS: J rows (swizzled), ring of S chunk buffers -----------------------------------
  unsigned char* Jl = smem;                           // [64][jrow]
  unsigned char* Sl = smem + (size_t)XCD_ROWS * jrow;  // [NB][128][KC] bf16
  {
    // chunks of 8 values: 16 bytes (BF16), 8 (FP8) or 4 (FP4); XOR-swizzled with the row
    constexpr int cb = JFMT == 0 ? 16 : (JFMT == 1 ? 8 : 4);
    const int chunks_per_row = Kp / 8;
    const unsigned char* Jg = reinterpret_cast<const unsigned char*>(a.J) + (size_t)rb * XCD_ROWS * jrow;
    for (int idx = tid; idx < XCD_ROWS * chunks_per_row; idx += blockDim.x) {
      const int row = idx / chunks_per_row, ch = idx - row * chunks_per_row;
      const int sw = JFMT == 0 ? (ch ^ (row & 7)) : (ch ^ (row & 15));
      unsigned char* dst = Jl + (size_t)row * jrow + sw * cb;
      const unsigned char* src = Jg + (size_t)row * jrow + ch * cb;
      if (JFMT == 0) *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(src);
      else if (JFMT == 1) *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(src);
      else *reinterpret_cast<uint32_t*>(dst) = *reinterpret_cast<const uint32_t*>(src);
    }
  }

  // ---- per-lane constants and state ----------------------------------------------------------
  const float* inv_g = reinterpret_cast<const float*>(a.inv_norm);
  const float* h_g = reinterpret_cast<const float*>(a.hterm);
  float* state = reinterpret_cast<float*>(a.state);
  float* traj = reinterpret_cast<float*>(a.traj);
  const float* coef = reinterpret_cast<const float*>(a.coef);
  float inv[2][4], hv[2][4], s[2][2][4];
  int row0[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    row0[rt] = rb * XCD_ROWS + 32 * wa + 16 * rt + 4 * g4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      inv[rt][v] = inv_g[row0[rt] + v];
      hv[rt][v] = h_g[row0[rt] + v];
    }
  }
  const int rgroup0 = group * XCD_RG + 32 * wb;  // first replica of this wave
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int r = rgroup0 + 16 * ct + c;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0[rt] + v;
        s[rt][ct][v] = (a.load_state && r < a.R && i < N) ? state[(size_t)r * N + i] : 0.0f;
      }
  }

  const float sg = (float)a.sigma;
  const float neg2ln2_s2 = -2.0f * 0.6931471805599453f * sg * sg;
  const float alpha = (float)a.alpha, oma = (float)(1.0 - a.alpha);
  const int nchunks = Kp / KC;

  // loop-invariant LDS byte offsets of this lane's fragments. A (J): 8-value chunk
  // c8 = 8ch + 4ks + g4 of row lrow, stored at ((c8 & ~M) | ((c8 & M) ^ (lrow & M))) with
  // M = 7 (BF16) or 15 (FP8/FP4). With M = 15 an odd chunk flips bit 3 of the stored index,
  // i.e. offset bit 8*CB, which is clear in lrow*jrow (jrow is a multiple of 16*CB).
  constexpr int M = JFMT == 0 ? 7 : 15;
  int aoff[KSTEPS][2];
#pragma unroll
  for (int ks = 0; ks < KSTEPS; ++ks)
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int lrow = 32 * wa + 16 * rt + c;
      const int within = 4 * ks + g4;
      const int sw = (within & ~M) | ((within & M) ^ (lrow & M));
      aoff[ks][rt] = lrow * jrow + sw * CB;
    }
  // B (spins): replica rep, 16-byte column col = 4ks + g4 of the chunk row stored at
  // col ^ (rep & (COLS - 1)), so 16 consecutive replicas hit distinct banks
  int boff[KSTEPS][2];
#pragma unroll
  for (int ks = 0; ks < KSTEPS; ++ks)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int rep = 32 * wb + 16 * ct + c;
      const int col = 4 * ks + g4;
      boff[ks][ct] = rep * ROW_B + (col ^ (rep & (COLS - 1))) * 16;
    }
  // DMA: lane l of a 1 KB block fills row l / COLS, column l % COLS, taking the global column
  // that the swizzle puts there; blocks DPW * wave + u.
  int dma_src[DPW];
  int dma_dst[DPW];
#pragma unroll
  for (int u = 0; u < DPW; ++u) {
    const int blk = DPW * wave + u;
    const int rep = blk * (1024 / ROW_B) + lane / COLS;
    const int pos = lane % COLS;
    dma_src[u] = rep * ks + (pos ^ (rep & (COLS - 1))) * 8;  // elements within the group's block
    dma_dst[u] = blk * 1024;
  }
  __bf16* S0 = reinterpret_cast<__bf16*>(x.S[0]);
  __bf16* S1 = reinterpret_cast<__bf16*>(x.S[1]);
  unsigned* bar = &ctl[CTL_BAR + 16 * (int)my_group];  // per launch: < 256 groups
  int epoch = 0;
  __syncthreads();

  for (int t = a.t_begin; t <= a.t_end && !aborted; ++t) {
    const __bf16* Scur = (t & 1) ? S1 : S0;
    __bf16* Snext = (t & 1) ? S0 : S1;
    const __bf16* Sgrp = Scur + (size_t)group * XCD_RG * ks;

    // DMA of chunk ch into buffer buf: DPW wave-instructions of 1 KB per wave
    auto issue_chunk = [&](int ch, int buf) {
#pragma unroll
      for (int u = 0; u < DPW; ++u)
        __builtin_amdgcn_global_load_lds(Sgrp + dma_src[u] + ch * KC,
                                         Sl + (size_t)buf * CHUNK_BYTES + dma_dst[u], 16, 0, 0);
    };
    // this lane's fragments of chunk ch (in buffer buf) into registers
    auto load_frags = [&](AT (&fa)[KSTEPS][2], bf16x8 (&fb)[KSTEPS][2], int ch, int buf) {
      const unsigned char* Sb = Sl + (size_t)buf * CHUNK_BYTES;
      const int px = (M == 15) ? (ch & 1) * 8 * CB : 0;
      const unsigned char* Ja = Jl + ((JFMT == 0) ? ch * (KC / 8) * 16 : (ch >> 1) * 16 * CB);
#pragma unroll
      for (int ks = 0; ks < KSTEPS; ++ks) {
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) fa[ks][rt] = *reinterpret_cast<const AT*>(Ja + (aoff[ks][rt] ^ px));
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) fb[ks][ct] = *reinterpret_cast<const bf16x8*>(Sb + boff[ks][ct]);
      }
    };

    f32x4 acc[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[rt][ct][v] = 0.0f;
    auto compute = [&](const AT (&fa)[KSTEPS][2], const bf16x8 (&fb)[KSTEPS][2]) {
#pragma unroll
      for (int ks = 0; ks < KSTEPS; ++ks) {
        bf16x8 af[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) af[rt] = widen<JFMT>(fa[ks][rt]);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[rt], fb[ks][ct], acc[rt][ct], 0, 0, 0);
      }
    };

    AT fa0[KSTEPS][2], fa1[KSTEPS][2];
    bf16x8 fb0[KSTEPS][2], fb1[KSTEPS][2];
    const int prologue = min(NB - 1, nchunks);
    for (int q = 0; q < prologue; ++q) issue_chunk(q, q);
    if constexpr (NB == 2) {
      // two buffers: wait for chunk ch, refill the other buffer, read and use chunk ch
      for (int ch = 0; ch < nchunks; ++ch) {
        wait_vm<0>();
        bare_barrier();  // chunk ch visible to all waves; the other buffer is free
        if (ch + 1 < nchunks) issue_chunk(ch + 1, (ch + 1) & 1);
        load_frags(fa0, fb0, ch, ch & 1);
        compute(fa0, fb0);
      }
    } else {
      // chunk ch+1 is read into registers while chunk ch is multiplied; the DMA ring runs
      // NB - 2 chunks ahead of the register prefetch.
      if (NB - 2 <= nchunks - 1) wait_vm<DPW * (NB - 2)>();
      else wait_vm<0>();
      bare_barrier();
      load_frags(fa0, fb0, 0, 0);
      int rbuf = 1;       // buffer of chunk ch + 1
      int wbuf = NB - 1;  // buffer of chunk ch + NB - 1 (= that of chunk ch - 1)
      auto step = [&](int ch, const AT (&ca)[KSTEPS][2], const bf16x8 (&cb)[KSTEPS][2],
                      AT (&na)[KSTEPS][2], bf16x8 (&nb)[KSTEPS][2]) {
        if (ch + NB - 2 <= nchunks - 1) wait_vm<DPW * (NB - 3)>();  // chunk ch + 1 has landed
        else wait_vm<0>();
        bare_barrier();  // ... for every wave, and every wave is done with chunk ch - 1's buffer
        if (ch + NB - 1 < nchunks) issue_chunk(ch + NB - 1, wbuf);
        load_frags(na, nb, min(ch + 1, nchunks - 1), rbuf);
        compute(ca, cb);
        rbuf = (rbuf + 1 == NB) ? 0 : rbuf + 1;
        wbuf = (wbuf + 1 == NB) ? 0 : wbuf + 1;
      };
      for (int ch = 0; ch < nchunks; ch += 2) {  // nchunks is even (Kp is a multiple of 128)
        step(ch, fa0, fb0, fa1, fb1);
        step(ch + 1, fa1, fb1, fa0, fb0);
      }
    }

    // ---- fused epilogue --------------------------------------------------------------------
    const float coef_t = coef[t - 1];
    const int k_rec = t - a.t_begin;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int r = rgroup0 + 16 * ct + c;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        float z[4];
        sigma_gauss4_f32(philox4x32_10((uint32_t)(row0[rt] >> 2), (uint32_t)r, (uint32_t)t, 0u, a.key0, a.key1),
                         neg2ln2_s2, z);
        __bf16 outv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float xf = fmaf(acc[rt][ct][v], inv[rt][v], hv[rt][v]);
          const float phi = a.negate_noise ? xf - z[v] : xf + z[v];
          const float sh = neg_tanh_from_exp2_arg(phi * coef_t);
          float sv = fmaf(alpha, sh, oma * s[rt][ct][v]);
          if (row0[rt] + v >= N) sv = 0.0f;
          s[rt][ct][v] = sv;
          outv[v] = (__bf16)sv;
        }
        *reinterpret_cast<uint2*>(Snext + (size_t)r * ks + row0[rt]) = *reinterpret_cast<const uint2*>(outv);
        if (traj && k_rec < a.record && r < a.R) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (row0[rt] + v < N) traj[((size_t)k_rec * a.R + r) * N + row0[rt] + v] = s[rt][ct][v];
        }
      }
    }

    // ---- group barrier ----------------------------------------------------------------------
    if (t < a.t_end) aborted = xcd_group_barrier(x, bar, (unsigned)++epoch, xcd_mode, tid);
  }

  // ---- final state and readout ---------------------------------------------------------------
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int r = rgroup0 + 16 * ct + c;
    if (r >= a.R) continue;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0[rt] + v;
        if (i < N) {
          state[(size_t)r * N + i] = s[rt][ct][v];
          if (a.spins) a.spins[(size_t)r * N + i] = (s[rt][ct][v] >= 0.0f) ? (int8_t)1 : (int8_t)-1;
        }
      }
  }
}

// ---- register-resident J ------------------------------------------------------------------
// For couplings that FP4 E2M1 holds exactly and N <= 2048. A workgroup covers 128 rows x 64
// replicas (groups of 64 replicas over P = Mp / 128 workgroups), keeps its rows of J in registers
// as FP4 (one 32-bit register per 8 couplings) for the whole anneal, and uses the whole LDS as a
// ring of 16 KB spin chunks (64 replicas x 128 k), of which XRJ_LA are loaded ahead of the one
// being read. Eight waves, two per SIMD, so that the vector work of one (widening J, noise,
// epilogue) issues while the other's MFMAs run: the waves form 4 row groups of 32 rows times 2
// halves of k. Wave (rg, kh) keeps rows 32 rg .. 32 rg + 31 of J for the two 32-k steps 2 kh and
// 2 kh + 1 of every chunk (64 registers at Kp = 2048) and reads only those steps' spin fragments.
// The two partial sums of each output meet in LDS (in the ring, idle after the k loop): wave
// (rg, kh) owns row tile kh of its row group for the epilogue and adds the partner's partial sum of
// that tile in the fixed order (k half 0) + (k half 1), the same on every workgroup, so results do
// not depend on placement. The k loop is unrolled over all chunks, which makes every register
// index, buffer index, wait count and load offset a compile-time constant.
constexpr int XRJ_ROWS = 128;                  // rows of J per workgroup (32 per row group)
constexpr int XRJ_RG = 64;                     // replicas per group
constexpr int XRJ_KC = 128;                    // k per spin chunk (four 32-k MFMA steps)
constexpr int XRJ_NB = 8;                      // spin chunk buffers in LDS
constexpr int XRJ_LA = 4;                      // chunks in flight ahead of the one being read
constexpr int XRJ_CHB = XRJ_RG * XRJ_KC * 2;   // bytes of one chunk: 64 replicas x 128 k, BF16

template <class F, int... I>
__device__ __forceinline__ void static_for(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}

// NCH: number of 128-k chunks (Kp = 128 NCH).
template <int NCH>
__global__ __launch_bounds__(512, 1) void anneal_xrj(AnnealArgs a, XcdArgs x) {
  constexpr int KS = 2, RTW = 2, NRG = 4;  // k halves; 16-row tiles per wave; row groups
  constexpr int NC = NCH, KPW = 2;         // chunks; 32-k steps per wave and chunk
  constexpr int CHB = XRJ_CHB, NB = XRJ_NB, LA = XRJ_LA;
  static_assert(8 * (KS - 1) * 4 * 64 * 16 <= XRJ_NB * XRJ_CHB, "the partial sums fit in the ring");
  extern __shared__ __align__(16) unsigned char smem[];  // the chunk ring
  __shared__ unsigned abort_word;                        // the group barrier's decision
  constexpr int DPW = CHB / 1024 / 8;  // 1 KB direct-to-LDS loads per wave and chunk (2)
  static_assert(DPW * (LA - 1) <= 63, "wait counts fit the vmcnt field");
  const int N = a.N, ks = x.ks;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar registers
  const int rg = wave % NRG, kh = wave / NRG;  // row group, k half
  const int g4 = lane >> 4, c = lane & 15;

  const XcdSlot slot = xcd_register(x, tid);
  const unsigned my_group = slot.my_group;
  const int group = (int)my_group + x.group_base;
  const int rb = slot.rb;
  const bool xcd_mode = slot.xcd_mode;
  bool aborted = slot.aborted;

  // J of this wave: jr[ch][u][rt] = the 8 FP4 couplings of row rb*128 + 32 rg + 16 rt + c at
  // k = 128 ch + 8 (4 g4 + 2 kh + u) .. +7: in step 2 kh + u of chunk ch, lane group g4 supplies
  // the 16-byte unit 4 g4 + 2 kh + u of every spin row (a dot product does not depend on the order
  // of its terms).
  uint32_t jr[NC][KPW][RTW];
  {
    const int jrow = 64 * NCH;  // bytes of one FP4 row (Kp / 2)
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt) {
      const unsigned char* p = reinterpret_cast<const unsigned char*>(a.J) +
                               (size_t)(rb * XRJ_ROWS + 16 * (RTW * rg + rt) + c) * jrow + 16 * g4 + 8 * kh;
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) {
        const uint2 v = *reinterpret_cast<const uint2*>(p + 64 * ch);
        jr[ch][0][rt] = v.x;
        jr[ch][1][rt] = v.y;
      }
    }
  }

  const float* inv_g = reinterpret_cast<const float*>(a.inv_norm);
  const float* h_g = reinterpret_cast<const float*>(a.hterm);
  float* state = reinterpret_cast<float*>(a.state);
  float* traj = reinterpret_cast<float*>(a.traj);
  const float* coef = reinterpret_cast<const float*>(a.coef);
  // outputs of this wave: rows row0 .. row0 + 3 (row tile kh of its row group), replicas
  // rgroup0 + 16 ct + c
  const int row0 = rb * XRJ_ROWS + 16 * (RTW * rg + kh) + 4 * g4;
  float s[4][4];
  const int rgroup0 = group * XRJ_RG;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int r = rgroup0 + 16 * ct + c;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = row0 + v;
      s[ct][v] = (a.load_state && r < a.R && i < N) ? state[(size_t)r * N + i] : 0.0f;
    }
  }
  const float sg = (float)a.sigma;
  const float neg2ln2_s2 = -2.0f * 0.6931471805599453f * sg * sg;
  const float alpha = (float)a.alpha, oma = (float)(1.0 - a.alpha);
  // sigma * z for this lane's 4 x 4 outputs of iteration tt (drawn ahead, while the group barrier
  // of the previous iteration completes)
  float zn[4][4];
  auto draw_noise_half = [&](int tt, int ct0) {
#pragma unroll
    for (int ct = ct0; ct < ct0 + 2; ++ct)
      sigma_gauss4_f32(philox4x32_10((uint32_t)(row0 >> 2), (uint32_t)(rgroup0 + 16 * ct + c), (uint32_t)tt, 0u,
                                     a.key0, a.key1),
                       neg2ln2_s2, zn[ct]);
  };
  auto pin_noise_half = [&](int ct0) {
#pragma unroll
    for (int ct = ct0; ct < ct0 + 2; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) asm volatile("" ::"v"(zn[ct][v]));
  };
  draw_noise_half(a.t_begin, 0);
  draw_noise_half(a.t_begin, 2);

  // Spin chunks: replica rows of 16 units of 16 bytes; unit u of replica q sits at u ^ (q & 15),
  // so the 16 lanes that one ds_read_b128 serves at a time (replicas c = 0..15, one unit) hit all
  // 64 banks once.
  int boff[KPW];
#pragma unroll
  for (int u = 0; u < KPW; ++u) boff[u] = c * 256 + ((4 * g4 + 2 * kh + u) ^ c) * 16;
  // Direct-to-LDS loads: a chunk is 16 loads of 1 KB (4 replicas each); wave w issues loads
  // 2 w and 2 w + 1. Lane l fills position l % 16 of replica 4 blk + l / 16 with the global unit
  // the swizzle puts there.
  unsigned dma_off[DPW];
#pragma unroll
  for (int u = 0; u < DPW; ++u) {
    const int blk = DPW * wave + u;
    const int q = 4 * blk + lane / 16;
    const int pu = lane % 16;
    dma_off[u] = (unsigned)(q * ks + (pu ^ (q & 15)) * 8) * 2u;
  }

  const __bf16* S0 = reinterpret_cast<const __bf16*>(x.S[0]);
  const __bf16* S1 = reinterpret_cast<const __bf16*>(x.S[1]);
  unsigned char* ring = smem;
  unsigned* bar = &x.ctl[CTL_BAR + 16 * (int)my_group];
  int epoch = 0;
  __syncthreads();

  for (int t = a.t_begin; t <= a.t_end && !aborted; ++t) {
    const unsigned char* Sg =
        reinterpret_cast<const unsigned char*>(((t & 1) ? S1 : S0) + (size_t)group * XRJ_RG * ks);
    __bf16* Snext = const_cast<__bf16*>((t & 1) ? S0 : S1);

    auto issue = [&](int ch, int buf) {
#pragma unroll
      for (int u = 0; u < DPW; ++u)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const __bf16*>(Sg + dma_off[u] + ch * 2 * XRJ_KC),
                                         ring + buf * CHB + (DPW * wave + u) * 1024, 16, 0, 0);
    };
    bf16x8 fb[2][4];  // [register set][column tile]: the spins of one 32-k step
    // spin fragments of this wave's step st (chunk st / 2, unit 2 kh + st % 2) into set st % 2
    auto load = [&](int st) {
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
        fb[st & 1][ct] = *reinterpret_cast<const bf16x8*>(smem + ((st / KPW) % NB) * CHB + boff[st % KPW] + 4096 * ct);
    };
    f32x4 acc[RTW][4];

    constexpr int PRO = LA < NC ? LA : NC;
    static_assert(LA <= NB - 1, "a chunk may only be loaded into a buffer that every wave is done with");
#pragma unroll
    for (int p = 0; p < PRO; ++p) issue(p, p);
    wait_vm<DPW * (PRO - 1)>();
    bare_barrier();
    load(0);
    // step st: the spins of step st+1 are read into the other register set while the MFMAs of
    // step st run. Before the first read of chunk c+1 (in the last step of chunk c) the workgroup
    // meets at a barrier: chunk c+1 has landed for every wave, and every wave is done reading
    // chunk c-1, whose buffer then takes chunk c-1+NB.
    static_for(
        [&](auto kc) {
          constexpr int st = decltype(kc)::value;
          constexpr int ch = st / KPW;
          if constexpr (st % KPW == KPW - 1 && ch + 1 < NC) {
            constexpr int last_issued = (ch + LA - 1 < NC - 1) ? ch + LA - 1 : NC - 1;
            wait_vm<DPW * (last_issued - (ch + 1))>();
            __builtin_amdgcn_sched_barrier(0);
            bare_barrier();
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (ch + LA < NC) issue(ch + LA, (ch + LA) % NB);
          }
          wait_lds();
          if constexpr (st + 1 < KPW * NC) load(st + 1);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int rt = 0; rt < RTW; ++rt) {
            const bf16x8 af = fp4x8_to_bf16x8(jr[ch][st % KPW][rt]);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
              acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  af, fb[st & 1][ct], st == 0 ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : acc[rt][ct], 0, 0, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
        },
        std::make_integer_sequence<int, KPW * NC>{});

    // Lane-dependent values after the k loop are derived afresh from an opaque copy of the lane
    // index: computed once before the iteration loop they would stay live across the k loop,
    // where J, the accumulators and the spin fragments need nearly every register.
    int lane_e = lane;
    asm volatile("" : "+v"(lane_e));
    const int c_e = lane_e & 15;
    const int row0e = rb * XRJ_ROWS + 16 * (RTW * rg + kh) + 4 * (lane_e >> 4);

    // ---- the two partial sums of each output --------------------------------------------------
    // Every wave is past its last read of the ring (the last barrier of the k loop came before the
    // last chunk's reads, so meet again); then each writes its partial sums of the row tiles the
    // other waves of its row group own: slot ((rg, kh), j, ct) holds tile j (j-th tile other than kh).
    bare_barrier();
    f32x4 own[4];  // selected with compile-time indices (a register array indexed by kh would go to scratch)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) own[ct] = acc[0][ct];
#pragma unroll
    for (int qq = 1; qq < RTW; ++qq)
      if (qq == kh) {
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) own[ct] = acc[qq][ct];
      }
    f32x4* slots = reinterpret_cast<f32x4*>(smem);
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt) {
      if (rt == kh) continue;
      const int j = rt < kh ? rt : rt - 1;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) slots[(((rg * KS + kh) * (KS - 1) + j) * 4 + ct) * 64 + lane_e] = acc[rt][ct];
    }
    __syncthreads();
    f32x4 tot[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      f32x4 sum = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int w = 0; w < KS; ++w) {
        f32x4 pv;
        if (w == kh) {
          pv = own[ct];
        } else {
          const int j = kh < w ? kh : kh - 1;
          pv = slots[(((rg * KS + w) * (KS - 1) + j) * 4 + ct) * 64 + lane_e];
        }
        sum = (w == 0) ? pv : sum + pv;  // k half 0, then k half 1
      }
      tot[ct] = sum;
    }

    // ---- fused epilogue --------------------------------------------------------------------
    const float coef_t = coef[t - 1];
    const int k_rec = t - a.t_begin;
    // the normalisers of this lane's rows, re-read every iteration (cache hits) rather than held
    // in registers across the k loop
    const f32x4 inv = *reinterpret_cast<const f32x4*>(inv_g + row0e);
    const f32x4 hv = *reinterpret_cast<const f32x4*>(h_g + row0e);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int r = rgroup0 + 16 * ct + c_e;
      __bf16 outv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float xf = fmaf(tot[ct][v], inv[v], hv[v]);
        const float phi = a.negate_noise ? xf - zn[ct][v] : xf + zn[ct][v];
        const float sh = neg_tanh_from_exp2_arg(phi * coef_t);
        float sv = fmaf(alpha, sh, oma * s[ct][v]);
        if (row0e + v >= N) sv = 0.0f;
        s[ct][v] = sv;
        outv[v] = (__bf16)sv;
      }
      *reinterpret_cast<uint2*>(Snext + (size_t)r * ks + row0e) = *reinterpret_cast<const uint2*>(outv);
      if (traj && k_rec < a.record && r < a.R) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (row0e + v < N) traj[((size_t)k_rec * a.R + r) * N + row0e + v] = s[ct][v];
      }
    }

    if (t < a.t_end) {
      // arrive, draw the next iteration's noise, wait (as in anneal_xrj); the wait ends with a
      // workgroup barrier, after which the ring (and the partial sums in it) may be overwritten
      xcd_group_arrive(bar, xcd_mode, tid);
      draw_noise_half(t + 1, 0);
      pin_noise_half(0);
      unsigned seen = 0;
      __builtin_amdgcn_sched_barrier(0);
      if (tid == 0) seen = ld_dev(bar);
      __builtin_amdgcn_sched_barrier(0);
      draw_noise_half(t + 1, 2);
      pin_noise_half(2);
      aborted = xrj_group_wait(x, bar, (unsigned)++epoch, xcd_mode, tid, seen, &abort_word);
    }
  }

  // ---- final state and readout ---------------------------------------------------------------
  int lane_f = lane;
  asm volatile("" : "+v"(lane_f));
  const int row0f = rb * XRJ_ROWS + 16 * (RTW * rg + kh) + 4 * (lane_f >> 4);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int r = rgroup0 + 16 * ct + (lane_f & 15);
    if (r >= a.R) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = row0f + v;
      if (i < N) {
        state[(size_t)r * N + i] = s[ct][v];
        if (a.spins) a.spins[(size_t)r * N + i] = (s[ct][v] >= 0.0f) ? (int8_t)1 : (int8_t)-1;
      }
    }
  }
}

// ---- register-resident J, FP8 spins ----------------------------------------------------------
// The FP8-spin precision on the same decomposition as anneal_xrj (4 waves per CU, 32 rows of J per
// wave in FP4 registers, groups of 64 replicas): the mean field runs on the mixed-format matrix
// instruction v_mfma_scale_f32_16x16x128_f8f6f4 with the FP4 couplings as A operand and the FP8
// E4M3 spins as B operand, both taken as they are stored (unit scales). The two operands lay out
// k differently (measured on gfx950 with a one-hot probe): lane 16 g + i of the FP4 operand holds
// row i at k = 32 g .. 32 g + 31 of the 128-k step (nibbles low first), which is how the J
// registers are laid out, so J needs no widening; lane 16 g + i of the FP8 operand holds column i
// at k = 16 g .. 16 g + 15 in its first 16 bytes and at k = 64 + 16 g .. 64 + 16 g + 15 in its
// last 16. One 128-k chunk is one MFMA per (row tile, column tile). Spin chunks are 64 replicas x
// 128 bytes (8 KB); unit u (16 k) of replica q is stored at u ^ ((q >> 1) & 7) of its 128-byte
// row, so that the 16 lanes a ds_read_b128 serves hit 16 distinct 16-byte bank groups. The
// epilogue packs each lane's four new spins of a column tile into one 32-bit word.
constexpr int XRJ8_CHB = XRJ_RG * XRJ_KC;  // bytes of one chunk: 64 replicas x 128 k, FP8

typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int NCH>
__global__ __launch_bounds__(256, 1) void anneal_xrj8(AnnealArgs a, XcdArgs x) {
  extern __shared__ __align__(16) unsigned char smem[];  // XRJ_NB chunk buffers
  __shared__ unsigned abort_word;                        // the group barrier's decision
  constexpr int NB = XRJ_NB;
  constexpr int RT = 2;
  constexpr int DPW = 2;  // 1 KB direct-to-LDS loads per wave and chunk (8 KB over 4 waves)
  static_assert(DPW * (XRJ_LA - 1) <= 63, "wait counts fit the vmcnt field");
  static_assert(XRJ_LA <= NB - 1, "a chunk may only be loaded into a buffer that every wave is done with");
  const int N = a.N, ks = x.ks;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g4 = lane >> 4, c = lane & 15;

  const XcdSlot slot = xcd_register(x, tid);
  const unsigned my_group = slot.my_group;
  const int group = (int)my_group + x.group_base;
  const int rb = slot.rb;
  const bool xcd_mode = slot.xcd_mode;
  bool aborted = slot.aborted;

  // J of this wave, as in anneal_xrj: jr[ch][q][rt] = the 8 FP4 couplings of row
  // rb*128 + 32*wave + 16*rt + c at k = 128*ch + 32*g4 + 8*q .. +7
  uint32_t jr[NCH][4][RT];
  {
    const int jrow = 64 * NCH;  // bytes of one FP4 row (Kp / 2)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const unsigned char* p = reinterpret_cast<const unsigned char*>(a.J) +
                               (size_t)(rb * XRJ_ROWS + 16 * RT * wave + 16 * rt + c) * jrow + 16 * g4;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const uint4 v = *reinterpret_cast<const uint4*>(p + 64 * ch);
        jr[ch][0][rt] = v.x;
        jr[ch][1][rt] = v.y;
        jr[ch][2][rt] = v.z;
        jr[ch][3][rt] = v.w;
      }
    }
  }

  const float* inv_g = reinterpret_cast<const float*>(a.inv_norm);
  const float* h_g = reinterpret_cast<const float*>(a.hterm);
  float* state = reinterpret_cast<float*>(a.state);
  float* traj = reinterpret_cast<float*>(a.traj);
  const float* coef = reinterpret_cast<const float*>(a.coef);
  float inv[RT][4], hv[RT][4], s[RT][4][4];
  int row0[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    row0[rt] = rb * XRJ_ROWS + 16 * RT * wave + 16 * rt + 4 * g4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      inv[rt][v] = inv_g[row0[rt] + v];
      hv[rt][v] = h_g[row0[rt] + v];
    }
  }
  const int rgroup0 = group * XRJ_RG;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int r = rgroup0 + 16 * ct + c;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0[rt] + v;
        s[rt][ct][v] = (a.load_state && r < a.R && i < N) ? state[(size_t)r * N + i] : 0.0f;
      }
  }
  const float sg = (float)a.sigma;
  const float neg2ln2_s2 = -2.0f * 0.6931471805599453f * sg * sg;
  const float alpha = (float)a.alpha, oma = (float)(1.0 - a.alpha);
  float zn[RT][4][4];
  auto draw_noise_half = [&](int tt, int ct0) {
#pragma unroll
    for (int ct = ct0; ct < ct0 + 2; ++ct)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        sigma_gauss4_f32(philox4x32_10((uint32_t)(row0[rt] >> 2), (uint32_t)(rgroup0 + 16 * ct + c), (uint32_t)tt, 0u,
                                       a.key0, a.key1),
                         neg2ln2_s2, zn[rt][ct]);
  };
  auto pin_noise_half = [&](int ct0) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = ct0; ct < ct0 + 2; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) asm volatile("" ::"v"(zn[rt][ct][v]));
  };
  draw_noise_half(a.t_begin, 0);
  draw_noise_half(a.t_begin, 2);

  // spin fragments: lane (c, g4) of column tile ct reads units g4 and g4 + 4 of replica 16*ct + c
  // (the FP8 operand's k layout); (q >> 1) & 7 does not depend on ct, and the column tiles are
  // 2 KB apart
  int boff[2];
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) boff[hf] = c * 128 + ((g4 + 4 * hf) ^ ((c >> 1) & 7)) * 16;
  // direct-to-LDS loads: block b (1 KB) holds replicas 8b .. 8b + 7; lane l fills position l % 8
  // of replica 8b + l / 8 with the global unit that the swizzle puts there
  unsigned dma_off[DPW];
#pragma unroll
  for (int u = 0; u < DPW; ++u) {
    const int blk = DPW * wave + u;
    const int q = 8 * blk + (lane >> 3);
    const int pos = lane & 7;
    dma_off[u] = (unsigned)(q * ks + (pos ^ ((q >> 1) & 7)) * 16);  // bytes within the group's block
  }

  const unsigned char* S0 = reinterpret_cast<const unsigned char*>(x.S[0]);
  const unsigned char* S1 = reinterpret_cast<const unsigned char*>(x.S[1]);
  unsigned char* ring = smem;
  unsigned* bar = &x.ctl[CTL_BAR + 16 * (int)my_group];
  int epoch = 0;
  __syncthreads();

  for (int t = a.t_begin; t <= a.t_end && !aborted; ++t) {
    const unsigned char* Sg = ((t & 1) ? S1 : S0) + (size_t)group * XRJ_RG * ks;
    unsigned char* Snext = const_cast<unsigned char*>((t & 1) ? S0 : S1);

    auto issue = [&](int ch, int buf) {
#pragma unroll
      for (int u = 0; u < DPW; ++u)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint32_t*>(Sg + dma_off[u] + ch * XRJ_KC),
                                         ring + buf * XRJ8_CHB + (DPW * wave + u) * 1024, 16, 0, 0);
    };
    i32x8 fb[2][4];  // [register set][column tile]: the spins of one 128-k chunk
    auto load = [&](int ch) {
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const unsigned char* base = smem + (ch % NB) * XRJ8_CHB + 2048 * ct;
        const uint4 lo = *reinterpret_cast<const uint4*>(base + boff[0]);
        const uint4 hi = *reinterpret_cast<const uint4*>(base + boff[1]);
        fb[ch & 1][ct] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
    };
    f32x4 acc[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[rt][ct][v] = 0.0f;

    constexpr int PRO = XRJ_LA < NCH ? XRJ_LA : NCH;
#pragma unroll
    for (int q = 0; q < PRO; ++q) issue(q, q);
    wait_vm<DPW * (PRO - 1)>();
    bare_barrier();
    load(0);
    // chunk ch: chunk ch+1 has landed for every wave once they meet at the barrier (and every
    // wave is done with chunk ch-1); its spins are read into the other register set while the
    // MFMAs of chunk ch run; chunk ch+XRJ_LA goes to buffer (ch+XRJ_LA) % NB, last used by chunk
    // ch+XRJ_LA-NB <= ch-1
    static_for(
        [&](auto chc) {
          constexpr int ch = decltype(chc)::value;
          if constexpr (ch + 1 < NCH) {
            constexpr int last_issued = (ch + XRJ_LA - 1 < NCH - 1) ? ch + XRJ_LA - 1 : NCH - 1;
            wait_vm<DPW * (last_issued - (ch + 1))>();
            __builtin_amdgcn_sched_barrier(0);
            bare_barrier();
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (ch + XRJ_LA < NCH) issue(ch + XRJ_LA, (ch + XRJ_LA) % NB);
          }
          wait_lds();
          if constexpr (ch + 1 < NCH) load(ch + 1);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            const i32x8 af = i32x8{(int)jr[ch][0][rt], (int)jr[ch][1][rt], (int)jr[ch][2][rt], (int)jr[ch][3][rt],
                                   0, 0, 0, 0};
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
              acc[rt][ct] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(af, fb[ch & 1][ct], acc[rt][ct], 4, 0, 0,
                                                                              0x7f7f7f7f, 0, 0x7f7f7f7f);
          }
          // The MFMA builtin has no side effects, so without this the compiler sinks every chunk's
          // MFMAs to the epilogue and keeps all chunks' spin fragments live: an empty volatile
          // statement that takes the accumulators (in the accumulation registers) holds each
          // chunk's MFMAs in its own step.
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) asm volatile("" : "+a"(acc[rt][ct]));
          __builtin_amdgcn_sched_barrier(0);
        },
        std::make_integer_sequence<int, NCH>{});

    // ---- fused epilogue --------------------------------------------------------------------
    const float coef_t = coef[t - 1];
    const int k_rec = t - a.t_begin;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int r = rgroup0 + 16 * ct + c;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float xf = fmaf(acc[rt][ct][v], inv[rt][v], hv[rt][v]);
          const float phi = a.negate_noise ? xf - zn[rt][ct][v] : xf + zn[rt][ct][v];
          const float sh = neg_tanh_from_exp2_arg(phi * coef_t);
          float sv = fmaf(alpha, sh, oma * s[rt][ct][v]);
          if (row0[rt] + v >= N) sv = 0.0f;
          s[rt][ct][v] = sv;
        }
        int w = __builtin_amdgcn_cvt_pk_fp8_f32(s[rt][ct][0], s[rt][ct][1], 0, false);
        w = __builtin_amdgcn_cvt_pk_fp8_f32(s[rt][ct][2], s[rt][ct][3], w, true);
        *reinterpret_cast<int*>(Snext + (size_t)r * ks + row0[rt]) = w;
        if (traj && k_rec < a.record && r < a.R) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (row0[rt] + v < N) traj[((size_t)k_rec * a.R + r) * N + row0[rt] + v] = s[rt][ct][v];
        }
      }
    }

    if (t < a.t_end) {
      xcd_group_arrive(bar, xcd_mode, tid);
      draw_noise_half(t + 1, 0);
      pin_noise_half(0);
      unsigned seen = 0;
      __builtin_amdgcn_sched_barrier(0);
      if (tid == 0) seen = ld_dev(bar);
      __builtin_amdgcn_sched_barrier(0);
      draw_noise_half(t + 1, 2);
      pin_noise_half(2);
      aborted = xrj_group_wait(x, bar, (unsigned)++epoch, xcd_mode, tid, seen, &abort_word);
    }
  }

  // ---- final state and readout ---------------------------------------------------------------
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int r = rgroup0 + 16 * ct + c;
    if (r >= a.R) continue;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0[rt] + v;
        if (i < N) {
          state[(size_t)r * N + i] = s[rt][ct][v];
          if (a.spins) a.spins[(size_t)r * N + i] = (s[rt][ct][v] >= 0.0f) ? (int8_t)1 : (int8_t)-1;
        }
      }
  }
}

size_t xcd_j_lds_bytes(int jfmt, int Kp) {
  return (size_t)XCD_ROWS * (jfmt == 0 ? (size_t)Kp * 2 : (jfmt == 1 ? (size_t)Kp : (size_t)Kp / 2));
}
size_t xcd_chunk_bytes() { return (size_t)XCD_RG * XCD_KC * 2; }

// Row stride of S. Padding the rows (so that the 128 rows of a chunk do not share their low
// address bits) was measured to make no difference on MI355X, so the rows are packed.
int xcd_spin_stride(int Kp) { return Kp; }

int xrj_rows() { return XRJ_ROWS; }
int xrj_group_replicas() { return XRJ_RG; }
int xrj_kp(int n) { return n <= 512 ? 512 : ((n + 255) / 256) * 256; }
bool xrj_fits(int n) { return xrj_kp(n) <= 2048; }

int xcd_ctl_words() { return CTL_WORDS; }
int xcd_rows() { return XCD_ROWS; }
int xcd_group_replicas() { return XCD_RG; }

template <int JFMT>
static const void* xcd_fn(int nbuf) {
  switch (nbuf) {
    case 2: return (const void*)anneal_xcd<JFMT, 2>;
    case 3: return (const void*)anneal_xcd<JFMT, 3>;
    case 4: return (const void*)anneal_xcd<JFMT, 4>;
    case 6: return (const void*)anneal_xcd<JFMT, 6>;
    default: return nullptr;
  }
}

int xcd_pick_buffers(size_t room) {
  const size_t cb = xcd_chunk_bytes();
  if (room >= 6 * cb) return 6;
  if (room >= 4 * cb) return 4;
  if (room >= 3 * cb) return 3;
  if (room >= 2 * cb) return 2;
  return 0;
}

// Every workgroup of a launch must be resident at once (they wait for each other). One
// workgroup fills a CU's LDS, so that holds when the grid does not exceed what the occupancy
// calculator allows; a launch that cannot become resident (a GPU shared with long-running work)
// ends in the bounded registration wait with an error rather than hanging. An ordinary launch is
// used rather than the cooperative-launch API, under which the ROCm profiler cannot trace the
// process.
static hipError_t launch_resident(const void* fn, int grid, int block, size_t lds, const AnnealArgs& a,
                                  const XcdArgs& x, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0, cus = 0, dev = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds);
  if (e != hipSuccess) return e;
  if ((long)per_cu * cus < (long)grid) return hipErrorCooperativeLaunchTooLarge;
  AnnealArgs aa = a;
  XcdArgs xx = x;
  void* args[] = {&aa, &xx};
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, st);
}

static const void* xrj8_fn(int Kp) {
  switch (Kp) {
    case 512: return (const void*)anneal_xrj8<4>;
    case 768: return (const void*)anneal_xrj8<6>;
    case 1024: return (const void*)anneal_xrj8<8>;
    case 1280: return (const void*)anneal_xrj8<10>;
    case 1536: return (const void*)anneal_xrj8<12>;
    case 1792: return (const void*)anneal_xrj8<14>;
    case 2048: return (const void*)anneal_xrj8<16>;
    default: return nullptr;
  }
}

hipError_t launch_anneal_xrj8(const AnnealArgs& a, const XcdArgs& x, int groups, hipStream_t st) {
  const void* fn = xrj8_fn(a.Kp);
  if (!fn) return hipErrorInvalidValue;
  return launch_resident(fn, groups * x.P, 256, (size_t)XRJ_NB * XRJ8_CHB, a, x, st);
}

static const void* xrj_fn(int Kp) {
  switch (Kp) {
    case 512: return (const void*)anneal_xrj<4>;
    case 768: return (const void*)anneal_xrj<6>;
    case 1024: return (const void*)anneal_xrj<8>;
    case 1280: return (const void*)anneal_xrj<10>;
    case 1536: return (const void*)anneal_xrj<12>;
    case 1792: return (const void*)anneal_xrj<14>;
    case 2048: return (const void*)anneal_xrj<16>;
    default: return nullptr;
  }
}

hipError_t launch_anneal_xrj(const AnnealArgs& a, const XcdArgs& x, int groups, hipStream_t st) {
  const void* fn = xrj_fn(a.Kp);
  if (!fn) return hipErrorInvalidValue;
  return launch_resident(fn, groups * x.P, 512, (size_t)XRJ_NB * XRJ_CHB, a, x, st);
}

hipError_t launch_anneal_xcd(int jfmt, const AnnealArgs& a, const XcdArgs& x, int groups, hipStream_t st) {
  const size_t lds = xcd_j_lds_bytes(jfmt, a.Kp) + (size_t)x.nbuf * xcd_chunk_bytes();
  const void* fn = jfmt == 0 ? xcd_fn<0>(x.nbuf) : (jfmt == 1 ? xcd_fn<1>(x.nbuf) : xcd_fn<2>(x.nbuf));
  if (!fn) return hipErrorInvalidValue;
  return launch_resident(fn, groups * x.P, 512, lds, a, x, st);
}

}  // namespace nmfa
