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
//     LDS with the direct-to-LDS loads of gfx950 (buffer_load_dwordx4 ... lds) in chunks of 64 k
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

    // DMA of chunk ch into buffer buf: DPW wave-instructions of 1 KB per wave, through a buffer
    // resource over the group's spin rows (the global form would make the compiler wait for every
    // LDS read before each use of one)
    const __amdgpu_buffer_rsrc_t srs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<__bf16*>(Sgrp), 0, XCD_RG * ks * 2, 0x00020000);
    auto issue_chunk = [&](int ch, int buf) {
#pragma unroll
      for (int u = 0; u < DPW; ++u)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(srs, Sl + (size_t)buf * CHUNK_BYTES + dma_dst[u], 16,
                                                 (unsigned)dma_src[u] * 2u, ch * KC * 2, 0, 0);
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

// ---- register-resident J, BF16 spins -------------------------------------------------------
// For couplings that FP4 E2M1 holds exactly and N <= 2048. A workgroup covers 256 rows x 32
// replicas (groups of 32 replicas over P = Mp / 256 workgroups) with four waves, one per SIMD:
//   * Wave w keeps rows 64 w .. 64 w + 63 of the workgroup's block of J for every k in registers,
//     as FP4 (one 32-bit register per 8 couplings: 256 registers at Kp = 2048), so each output's
//     whole sum stays in one wave. Per 16-k step it widens two J fragments (two 32-row tiles) and
//     runs two v_mfma_f32_32x32x16_bf16 on the step's spin fragment, read from LDS three steps ahead.
//   * The group's BF16 spins stream through LDS in 8 KB chunks (32 replicas x 128 k), one buffer
//     per chunk, by direct-to-LDS buffer loads: a CU receives 128 KB of spins per iteration. The
//     loaded chunks come in batches of XRB_GB: the workgroup meets once per batch, when every load
//     issued so far has landed, and then issues the next batch (fewer barriers, and fewer loads in
//     flight beside the matrix instructions, measured faster than a barrier per chunk with loads
//     four chunks ahead).
//   * The chunks are visited starting at the workgroup's own rows (two chunks) and wrapping around,
//     the same order on every pass. The spins of the own rows are written into the ring by the
//     epilogue, so an iteration starts on them while the loads of the other chunks are in flight.
//   * The Philox noise of the next iteration and its field term (h_i + z) / (T_t norm_i) are
//     computed while the group barrier completes (half before this workgroup's arrival, while its
//     spin stores complete, half after it).
//   * The epilogue (exp2, reciprocal, damped update) runs on the accumulator layout; the FP32 master
//     state stays in registers.
// The k loop is unrolled over all chunks, so every register index, buffer index, wait count and
// load offset is a compile-time constant.
constexpr int XRB_ROWS = 256;                  // rows of J per workgroup (64 per wave)
constexpr int XRB_RG = 32;                     // replicas per group
constexpr int XRB_KC = 128;                    // k per spin chunk
constexpr int XRB_NB = 16;                     // spin chunk buffers in LDS (one per chunk at Kp = 2048)
constexpr int XRB_GB = 3;                      // loaded chunks per workgroup barrier (and per batch of loads)
constexpr int XRB_CHB = XRB_RG * XRB_KC * 2;   // bytes of one chunk: 32 replicas x 128 k, BF16

typedef float f32x16 __attribute__((ext_vector_type(16)));

template <class F, int... I>
__device__ __forceinline__ void static_for(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}

// Output layout of v_mfma_f32_32x32x16_bf16: lane l holds column l % 32 and, in accumulator
// element i, row 8 (i / 4) + 4 (l / 32) + i % 4: four quads of consecutive rows, each the four
// Gaussians of one Philox call.
//
// NCH: number of 128-k chunks (Kp = 128 NCH).
template <int NCH>
__global__ __launch_bounds__(256, 1) void anneal_xrj(AnnealArgs a, XcdArgs x) {
  constexpr int NC = NCH, NST = 8, NSTEP = NC * NST;  // chunks; 16-k steps per chunk
  constexpr int D = 3;                                // spin fragments read D steps ahead
  constexpr int OWN = XRB_ROWS / XRB_KC;              // chunks of the workgroup's own rows (2)
  constexpr int CHB = XRB_CHB, NB = XRB_NB, GB = XRB_GB;
  constexpr int DPW = CHB / 1024 / 4;                 // 1 KB direct-to-LDS loads per wave and chunk (2)
  static_assert(NC >= OWN + 1 && NC <= NB, "own chunks keep buffers 0 and 1 to themselves");
  static_assert(DPW * (OWN + GB) <= 63, "wait counts fit the vmcnt field");
  extern __shared__ __align__(16) unsigned char smem[];  // the chunk ring
  __shared__ unsigned abort_word;                        // the group barrier's decision
  __shared__ f32x4 rowc[2][XRB_ROWS / 4];                // 1 / norm_i and h_i / norm_i of the workgroup's rows
  const int N = a.N, ks = x.ks;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar registers
  const int g = lane >> 5, c = lane & 31;

  const XcdSlot slot = xcd_register(x, tid);
  const unsigned my_group = slot.my_group;
  const int group = (int)my_group + x.group_base;
  const int rb = slot.rb;
  const bool xcd_mode = slot.xcd_mode;
  bool aborted = slot.aborted;

  // J of this wave: jr[i][st][at] = the 8 FP4 couplings of row rb*256 + 64 wave + 32 at + c at
  // k = 128 ch + 16 st + 8 g .. +7 with ch = (2 rb + i) mod NC. Lane group g supplies k octet g of
  // every 16-k step, for J and spins alike (a dot product does not depend on the order of its terms).
  uint32_t jr[NC][NST][2];
  {
    const int jrow = 64 * NC;  // bytes of one FP4 row (Kp / 2)
#pragma unroll
    for (int at = 0; at < 2; ++at) {
      const unsigned char* p = reinterpret_cast<const unsigned char*>(a.J) +
                               (size_t)(rb * XRB_ROWS + 64 * wave + 32 * at + c) * jrow + 4 * g;
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        const int ch = (OWN * rb + i) % NC;
#pragma unroll
        for (int st = 0; st < NST; ++st) jr[i][st][at] = *reinterpret_cast<const uint32_t*>(p + 64 * ch + 8 * st);
      }
    }
  }

  // the per-row constants live in LDS for the whole anneal (the epilogue reads them every iteration)
  if (tid < XRB_ROWS / 4) {
    rowc[0][tid] = reinterpret_cast<const f32x4*>(a.inv_norm)[rb * (XRB_ROWS / 4) + tid];
    rowc[1][tid] = reinterpret_cast<const f32x4*>(a.hterm)[rb * (XRB_ROWS / 4) + tid];
  }
  __syncthreads();
  float* state = reinterpret_cast<float*>(a.state);
  float* traj = reinterpret_cast<float*>(a.traj);
  const float* coef = reinterpret_cast<const float*>(a.coef);
  // outputs of this lane: rows row0 + 32 at + 8 j + v (at = 0, 1; j, v = 0..3), replica rgroup0 + c
  const int row0 = rb * XRB_ROWS + 64 * wave + 4 * g;
  const int rgroup0 = group * XRB_RG;
  float s[2][16];
  {
    const int r = rgroup0 + c;
#pragma unroll
    for (int at = 0; at < 2; ++at)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int row = row0 + 32 * at + 8 * (i / 4) + i % 4;
        s[at][i] = (a.load_state && r < a.R && row < N) ? state[(size_t)r * N + row] : 0.0f;
      }
  }
  const float sg = (float)a.sigma;
  const float neg2ln2_s2 = -2.0f * 0.6931471805599453f * sg * sg;
  const float alpha2 = (float)(2.0 * a.alpha), nalpha = (float)(-a.alpha), oma = (float)(1.0 - a.alpha);

  // Spin chunks: replica rows of 16 units of 16 bytes; unit u of replica q sits at u ^ (q & 15),
  // so the 16 lanes that one ds_read_b128 serves at a time (16 replicas, one unit) hit all 64
  // banks once. Step st reads unit 2 st + g of replica c.
  int boff[NST];
#pragma unroll
  for (int st = 0; st < NST; ++st) boff[st] = c * 256 + (((2 * st + g) ^ (c & 15)) * 16);
  // Direct-to-LDS loads: a chunk is 8 loads of 1 KB (4 replicas each); wave w issues loads
  // DPW w .. DPW w + DPW - 1. Lane l fills position l % 16 of replica 4 blk + l / 16 with the global
  // unit the swizzle puts there.
  unsigned dma_off[DPW];
#pragma unroll
  for (int u = 0; u < DPW; ++u) {
    const int blk = DPW * wave + u;
    const int q = 4 * blk + lane / 16;
    const int pu = lane % 16;
    dma_off[u] = (unsigned)(q * ks + (pu ^ (q & 15)) * 8) * 2u;
  }
  // where this lane's four new spins of row quad (at, j) go in the own chunks (ring buffers 0, 1):
  // workgroup row 64 wave + 32 at + 8 j + 4 g is k = 64 (wave & 1) + 32 at + 8 j + 4 g of own chunk
  // wave / 2, i.e. half g of unit 8 (wave & 1) + 4 at + j
  auto own_off = [&](int at, int j, int ln) {
    const int q = ln & 31;
    return (wave >> 1) * CHB + q * 256 + (((8 * (wave & 1) + 4 * at + j) ^ (q & 15)) * 16) + 8 * (ln >> 5);
  };

  // w = (h_i + sigma z) / (T_t norm_i) for this lane's outputs of iteration tt (exp2 units), with the
  // Philox noise of (row quad, replica, tt). Drawn one iteration ahead, while the group barrier of
  // the previous iteration completes.
  float w[2][16];
  float coef_next = coef[a.t_begin - 1];
  // h_i / norm_i of this lane's rows (quad (at, j) is entry 16 wave + 8 at + 2 j + g of the workgroup's
  // rows), read again in the epilogue for the next draws
  f32x4 hrow[2][4];
#pragma unroll
  for (int at = 0; at < 2; ++at)
#pragma unroll
    for (int j = 0; j < 4; ++j) hrow[at][j] = rowc[1][16 * wave + 8 * at + 2 * j + g];
  auto draw = [&](int tt, int d0, int nd, float coef_tt) {
    const float coef_z = a.negate_noise ? -coef_tt : coef_tt;
#pragma unroll
    for (int d = d0; d < d0 + nd; ++d) {
      const int at = d >> 2, j = d & 3;
      float z[4];
      sigma_gauss4_f32(philox4x32_10((uint32_t)((row0 + 32 * at + 8 * j) >> 2), (uint32_t)(rgroup0 + c),
                                     (uint32_t)tt, 0u, a.key0, a.key1),
                       neg2ln2_s2, z);
      const f32x4 hc = hrow[at][j] * coef_tt;
#pragma unroll
      for (int v = 0; v < 4; ++v) w[at][4 * j + v] = fmaf(z[v], coef_z, hc[v]);
    }
  };
  auto pin_noise = [&](int d0, int nd) {
#pragma unroll
    for (int d = d0; d < d0 + nd; ++d)
#pragma unroll
      for (int v = 0; v < 4; ++v) asm volatile("" ::"v"(w[d >> 2][4 * (d & 3) + v]));
  };
  draw(a.t_begin, 0, 8, coef_next);

  const __bf16* S0 = reinterpret_cast<const __bf16*>(x.S[0]);
  const __bf16* S1 = reinterpret_cast<const __bf16*>(x.S[1]);
  unsigned char* ring = smem;
  unsigned* bar = &x.ctl[CTL_BAR + 16 * (int)my_group];
  int epoch = 0;
  __syncthreads();

  for (int t = a.t_begin; t <= a.t_end && !aborted; ++t) {
    const float coef_t = coef_next;
    const unsigned char* Sg =
        reinterpret_cast<const unsigned char*>(((t & 1) ? S1 : S0) + (size_t)group * XRB_RG * ks);
    __bf16* Snext = const_cast<__bf16*>((t & 1) ? S0 : S1);
    const bool own_in_lds = t > a.t_begin;

    // the chunk offsets are recomputed every iteration from an opaque copy of rb: held across the
    // loop they would occupy scalar registers for every chunk
    int rb_t = rb;
    asm volatile("" : "+s"(rb_t));
    // The direct-to-LDS loads go through a buffer resource over the group's spin rows (reads past
    // it return 0) rather than the global form, which the compiler treats as a flat access to both
    // memory and LDS and then follows with full LDS waits before every use of an LDS read.
    const __amdgpu_buffer_rsrc_t srs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(Sg), 0, XRB_RG * ks * 2, 0x00020000);
    auto issue = [&](int i, int buf) {
      int ch = OWN * rb_t + i;
      if (ch >= NC) ch -= NC;
      // the LDS destination is formed at each issue from an opaque copy of the wave's base: every
      // (buffer, load) address held across the loop would take a scalar register, and the
      // compiler spills scalar registers to vector lanes beyond about a hundred of them
      int wb = DPW * 1024 * wave;
      asm volatile("" : "+s"(wb));
#pragma unroll
      for (int u = 0; u < DPW; ++u)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(srs, ring + wb + buf * CHB + u * 1024, 16, dma_off[u],
                                                 ch * 2 * XRB_KC, 0, 0);
    };
    bf16x8 fb[D + 1];  // [register set]: the spins of one 16-k step
    auto load = [&](int sidx) {
      fb[sidx % (D + 1)] = *reinterpret_cast<const bf16x8*>(smem + ((sidx / NST) % NB) * CHB + boff[sidx % NST]);
    };
    f32x16 acc[2];

    // chunks 0 .. OWN - 1 (the own rows) come from the previous iteration's epilogue, or on the
    // first iteration from memory; the first batch, chunks OWN .. PRO, is loaded while they are
    // multiplied. Chunk ch always goes to buffer ch (NC <= NB): the group barrier at the end of the
    // previous iteration orders every load after every read of the buffer it overwrites.
    if (!own_in_lds) {
#pragma unroll
      for (int p = 0; p < OWN; ++p) issue(p, p);
    }
    constexpr int PRO = OWN + GB - 1 < NC - 1 ? OWN + GB - 1 : NC - 1;
#pragma unroll
    for (int p = OWN; p <= PRO; ++p) issue(p, p);
    wait_vm<DPW * (PRO - OWN + 1)>();
    bare_barrier();
#pragma unroll
    for (int sidx = 0; sidx < D; ++sidx) load(sidx);

    // step sidx (chunk sidx / NST, step sidx % NST): the spins of step sidx + D are read while the
    // MFMAs of step sidx run. Before the first read of the batch that starts at chunk ci (D steps
    // before it starts) every wave waits for all of its loads and the workgroup meets at a
    // barrier: chunks ci .. ci + GB - 1 have landed for every wave. The next batch is issued then.
    static_for(
        [&](auto sc) {
          constexpr int sidx = decltype(sc)::value;
          constexpr int i = sidx / NST, st = sidx % NST;
          constexpr int nxt = sidx + D;
          if constexpr (nxt < NSTEP && nxt % NST == 0 && nxt / NST >= OWN && (nxt / NST - OWN) % GB == 0) {
            constexpr int ci = nxt / NST;  // first chunk of the batch about to be read
            wait_vm<0>();
            __builtin_amdgcn_sched_barrier(0);
            bare_barrier();
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = ci + GB; q < ci + 2 * GB && q < NC; ++q) issue(q, q);
          }
          if constexpr (nxt < NSTEP) load(nxt);
#pragma unroll
          for (int at = 0; at < 2; ++at)
            acc[at] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fp4x8_to_bf16x8(jr[i][st][at]), fb[sidx % (D + 1)],
                                                             sidx == 0 ? f32x16{} : acc[at], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);  // keeps the reads D steps ahead of their use
        },
        std::make_integer_sequence<int, NSTEP>{});

    // Lane-dependent values after the k loop are derived afresh from an opaque copy of the lane
    // index, so that they are not kept live across the k loop.
    int lane_e = lane;
    asm volatile("" : "+v"(lane_e));
    const int c_e = lane_e & 31;
    const int row0e = rb * XRB_ROWS + 64 * wave + 4 * (lane_e >> 5);

    // the next iteration's temperature (read here, not during the k loop: a scalar load in flight
    // there would force every LDS wait to wait for all LDS reads); this iteration's 1 / (T_t norm_i)
    if (t < a.t_end) coef_next = coef[t];
    f32x4 invc[2][4];
#pragma unroll
    for (int at = 0; at < 2; ++at)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = 16 * wave + 8 * at + 2 * j + (lane_e >> 5);
        invc[at][j] = rowc[0][q] * coef_t;
        hrow[at][j] = rowc[1][q];
      }

    // ---- fused epilogue --------------------------------------------------------------------
    // The own chunks (buffers 0, 1) were last read at the start of this iteration, so they may be
    // overwritten without a barrier.
    const int k_rec = t - a.t_begin;
    {
      const int r = rgroup0 + c_e;
#pragma unroll
      for (int at = 0; at < 2; ++at)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          __bf16 outv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = 4 * j + v;
            // -tanh(Phi / T) = 2 / (1 + exp2(arg)) - 1 with arg = 2 log2(e) Phi / T; damped update
            const float e = __builtin_amdgcn_exp2f(fmaf(acc[at][i], invc[at][j][v], w[at][i]));
            const float sv = fmaf(alpha2, __builtin_amdgcn_rcpf(1.0f + e), fmaf(oma, s[at][i], nalpha));
            s[at][i] = sv;
            outv[v] = (__bf16)sv;
          }
          const uint2 pk = *reinterpret_cast<const uint2*>(outv);
          *reinterpret_cast<uint2*>(Snext + (size_t)r * ks + row0e + 32 * at + 8 * j) = pk;
          *reinterpret_cast<uint2*>(ring + own_off(at, j, lane_e)) = pk;
        }
      if (traj && k_rec < a.record) {
#pragma unroll
        for (int at = 0; at < 2; ++at)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int row = row0e + 32 * at + 8 * (i / 4) + i % 4;
            if (r < a.R && row < N) traj[((size_t)k_rec * a.R + r) * N + row] = s[at][i];
          }
      }
    }

    if (t < a.t_end) {
      // half of the next iteration's noise while the spin stores complete, arrive (this
      // workgroup's spins are stored), the other half while the other workgroups arrive, then wait
      // for the group; the wait ends with a workgroup barrier, after which the ring may be
      // overwritten
      draw(t + 1, 0, 4, coef_next);
      pin_noise(0, 4);
      xcd_group_arrive(bar, xcd_mode, tid);
      draw(t + 1, 4, 2, coef_next);
      pin_noise(4, 2);
      unsigned seen = 0;
      __builtin_amdgcn_sched_barrier(0);
      if (tid == 0) seen = ld_dev(bar);  // polled once ahead, read after the last draws
      __builtin_amdgcn_sched_barrier(0);
      draw(t + 1, 6, 2, coef_next);
      pin_noise(6, 2);
      aborted = xrj_group_wait(x, bar, (unsigned)++epoch, xcd_mode, tid, seen, &abort_word);
    }
  }

  // ---- final state and readout ---------------------------------------------------------------
  int lane_f = lane;
  asm volatile("" : "+v"(lane_f));
  const int row0f = rb * XRB_ROWS + 64 * wave + 4 * (lane_f >> 5);
  const int r = rgroup0 + (lane_f & 31);
  if (r < a.R) {
#pragma unroll
    for (int at = 0; at < 2; ++at)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int row = row0f + 32 * at + 8 * (i / 4) + i % 4;
        if (row < N) {
          state[(size_t)r * N + row] = s[at][i];
          if (a.spins) a.spins[(size_t)r * N + row] = (s[at][i] >= 0.0f) ? (int8_t)1 : (int8_t)-1;
        }
      }
  }
}

// ---- register-resident J, FP8 spins ----------------------------------------------------------
// The FP8-spin precision on the decomposition of anneal_xrj (256 rows x 32 replicas per
// workgroup, four waves of 64 rows each with every k of FP4 J in registers, groups of 32
// replicas): the mean field runs on the mixed-format matrix instruction
// v_mfma_scale_f32_16x16x128_f8f6f4 with the FP4 couplings as A operand and the FP8 E4M3 spins as
// B operand, both taken as they are stored (unit scales), so J needs no widening. The two operands
// lay out k differently (measured on gfx950 with a one-hot probe): lane 16 g + i of the FP4
// operand holds row i at k = 32 g .. 32 g + 31 of the 128-k step (nibbles low first), which is how
// the J registers are laid out; lane 16 g + i of the FP8 operand holds column i at
// k = 16 g .. 16 g + 15 in its first 16 bytes and at k = 64 + 16 g .. 64 + 16 g + 15 in its last
// 16. One 128-k chunk is one MFMA per (16-row tile, 16-column tile): 4 x 2 per wave.
//   * Spin chunks are 32 replicas x 128 bytes (4 KB); unit u (16 k) of replica q is stored at
//     u ^ ((q >> 1) & 7) of its 128-byte row, so the 16 lanes a ds_read_b128 serves hit 16
//     distinct 16-byte bank groups. A CU receives 64 KB of spins per iteration, one buffer per
//     chunk, loaded by direct-to-LDS buffer loads in batches of XR8_GB chunks (one workgroup
//     barrier per batch, as in anneal_xrj). With chunks half the size of the BF16 kernel's, one
//     batch of every loaded chunk, issued when the iteration starts, measured fastest (25.0 ms per
//     headline anneal, against 26.1 for batches of seven and 27.4 for batches of three).
//   * The chunks are visited from the workgroup's own rows (two chunks), which the epilogue writes
//     into buffers 0 and 1 as well as to memory; the fragments of the next chunk are read into a
//     second register set while the MFMAs of the current one run.
//   * The Philox noise of the next iteration and its field term are drawn while the group barrier
//     completes; the per-row constants live in LDS; the epilogue (exp2, reciprocal, damped update)
//     packs each lane's four new spins of a (row tile, column tile) into one 32-bit word.
constexpr int XR8_ROWS = 256;                  // rows of J per workgroup (64 per wave)
constexpr int XR8_RG = 32;                     // replicas per group
constexpr int XR8_KC = 128;                    // k per spin chunk
constexpr int XR8_NB = 16;                     // spin chunk buffers in LDS (one per chunk at Kp = 2048)
constexpr int XR8_GB = 14;                     // loaded chunks per batch: all of them at Kp = 2048
constexpr int XR8_CHB = XR8_RG * XR8_KC;       // bytes of one chunk: 32 replicas x 128 k, FP8

typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int NCH>
__global__ __launch_bounds__(256, 1) void anneal_xrj8(AnnealArgs a, XcdArgs x) {
  constexpr int NC = NCH, RT = 4, CT = 2;
  constexpr int OWN = XR8_ROWS / XR8_KC;  // chunks of the workgroup's own rows (2)
  constexpr int CHB = XR8_CHB, NB = XR8_NB, GB = XR8_GB;
  static_assert(NC >= OWN + 1 && NC <= NB, "own chunks keep buffers 0 and 1 to themselves");
  static_assert(OWN + GB <= 63, "wait counts fit the vmcnt field");
  extern __shared__ __align__(16) unsigned char smem[];  // the chunk buffers
  __shared__ unsigned abort_word;                        // the group barrier's decision
  __shared__ f32x4 rowc[2][XR8_ROWS / 4];                // 1 / norm_i and h_i / norm_i of the workgroup's rows
  const int N = a.N, ks = x.ks;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar registers
  const int g = lane >> 4, c = lane & 15;

  const XcdSlot slot = xcd_register(x, tid);
  const unsigned my_group = slot.my_group;
  const int group = (int)my_group + x.group_base;
  const int rb = slot.rb;
  const bool xcd_mode = slot.xcd_mode;
  bool aborted = slot.aborted;

  // J of this wave: jr[i][rt][q] = the 8 FP4 couplings of row rb*256 + 64 wave + 16 rt + c at
  // k = 128 ch + 32 g + 8 q .. +7 with ch = (2 rb + i) mod NC
  uint32_t jr[NC][RT][4];
  {
    const int jrow = 64 * NC;  // bytes of one FP4 row (Kp / 2)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const unsigned char* p = reinterpret_cast<const unsigned char*>(a.J) +
                               (size_t)(rb * XR8_ROWS + 64 * wave + 16 * rt + c) * jrow + 16 * g;
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        const int ch = (OWN * rb + i) % NC;
        const uint4 v = *reinterpret_cast<const uint4*>(p + 64 * ch);
        jr[i][rt][0] = v.x;
        jr[i][rt][1] = v.y;
        jr[i][rt][2] = v.z;
        jr[i][rt][3] = v.w;
      }
    }
  }

  if (tid < XR8_ROWS / 4) {
    rowc[0][tid] = reinterpret_cast<const f32x4*>(a.inv_norm)[rb * (XR8_ROWS / 4) + tid];
    rowc[1][tid] = reinterpret_cast<const f32x4*>(a.hterm)[rb * (XR8_ROWS / 4) + tid];
  }
  __syncthreads();
  float* state = reinterpret_cast<float*>(a.state);
  float* traj = reinterpret_cast<float*>(a.traj);
  const float* coef = reinterpret_cast<const float*>(a.coef);
  // outputs of this lane: rows row0 + 16 rt + v (rt, v = 0..3), replicas rgroup0 + 16 ct + c
  const int row0 = rb * XR8_ROWS + 64 * wave + 4 * g;
  const int rgroup0 = group * XR8_RG;
  float s[RT][CT][4];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int r = rgroup0 + 16 * ct + c;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + 16 * rt + v;
        s[rt][ct][v] = (a.load_state && r < a.R && row < N) ? state[(size_t)r * N + row] : 0.0f;
      }
  }
  const float sg = (float)a.sigma;
  const float neg2ln2_s2 = -2.0f * 0.6931471805599453f * sg * sg;
  const float alpha2 = (float)(2.0 * a.alpha), nalpha = (float)(-a.alpha), oma = (float)(1.0 - a.alpha);

  // spin fragments: lane (c, g) of column tile ct reads units g and g + 4 of replica 16 ct + c
  // (the FP8 operand's k layout); (q >> 1) & 7 does not depend on ct, and the column tiles are
  // 2 KB apart
  int boff[2];
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) boff[hf] = c * 128 + (((g + 4 * hf) ^ ((c >> 1) & 7)) * 16);
  // direct-to-LDS loads: a chunk is 4 loads of 1 KB, wave w fills replicas 8 w .. 8 w + 7; lane l
  // fills position l % 8 of replica 8 w + l / 8 with the global unit the swizzle puts there
  unsigned dma_off;
  {
    const int q = 8 * wave + (lane >> 3);
    const int pos = lane & 7;
    dma_off = (unsigned)(q * ks + (pos ^ ((q >> 1) & 7)) * 16);
  }
  // where this lane's four new spins of tile (rt, ct) go in the own chunks (buffers 0, 1):
  // workgroup row 64 wave + 16 rt + 4 g is k = 64 (wave & 1) + 16 rt + 4 g of own chunk wave / 2,
  // i.e. bytes 4 g .. 4 g + 3 of unit 4 (wave & 1) + rt
  auto own_off = [&](int rt, int ct, int ln) {
    const int q = 16 * ct + (ln & 15);
    return (wave >> 1) * CHB + q * 128 + (((4 * (wave & 1) + rt) ^ ((q >> 1) & 7)) * 16) + 4 * (ln >> 4);
  };

  // w = (h_i + sigma z) / (T_t norm_i) for this lane's outputs of iteration tt (exp2 units), with the
  // Philox noise of (row quad, replica, tt); draw d covers tile (d / 2, d % 2). Drawn one iteration
  // ahead, while the group barrier of the previous iteration completes.
  float w[RT][CT][4];
  float coef_next = coef[a.t_begin - 1];
  f32x4 hrow[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) hrow[rt] = rowc[1][16 * wave + 4 * rt + g];
  auto draw = [&](int tt, int d0, int nd, float coef_tt) {
    const float coef_z = a.negate_noise ? -coef_tt : coef_tt;
#pragma unroll
    for (int d = d0; d < d0 + nd; ++d) {
      const int rt = d >> 1, ct = d & 1;
      float z[4];
      sigma_gauss4_f32(philox4x32_10((uint32_t)((row0 + 16 * rt) >> 2), (uint32_t)(rgroup0 + 16 * ct + c),
                                     (uint32_t)tt, 0u, a.key0, a.key1),
                       neg2ln2_s2, z);
      const f32x4 hc = hrow[rt] * coef_tt;
#pragma unroll
      for (int v = 0; v < 4; ++v) w[rt][ct][v] = fmaf(z[v], coef_z, hc[v]);
    }
  };
  auto pin_noise = [&](int d0, int nd) {
#pragma unroll
    for (int d = d0; d < d0 + nd; ++d)
#pragma unroll
      for (int v = 0; v < 4; ++v) asm volatile("" ::"v"(w[d >> 1][d & 1][v]));
  };
  draw(a.t_begin, 0, 8, coef_next);

  const unsigned char* S0 = reinterpret_cast<const unsigned char*>(x.S[0]);
  const unsigned char* S1 = reinterpret_cast<const unsigned char*>(x.S[1]);
  unsigned char* ring = smem;
  unsigned* bar = &x.ctl[CTL_BAR + 16 * (int)my_group];
  int epoch = 0;
  __syncthreads();

  for (int t = a.t_begin; t <= a.t_end && !aborted; ++t) {
    const float coef_t = coef_next;
    const unsigned char* Sg = ((t & 1) ? S1 : S0) + (size_t)group * XR8_RG * ks;
    unsigned char* Snext = const_cast<unsigned char*>((t & 1) ? S0 : S1);
    const bool own_in_lds = t > a.t_begin;

    int rb_t = rb;
    asm volatile("" : "+s"(rb_t));
    const __amdgpu_buffer_rsrc_t srs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(Sg), 0, XR8_RG * ks, 0x00020000);
    auto issue = [&](int i, int buf) {
      int ch = OWN * rb_t + i;
      if (ch >= NC) ch -= NC;
      int wb = 1024 * wave;  // LDS destination from an opaque per-wave base (no scalar register per address)
      asm volatile("" : "+s"(wb));
      __builtin_amdgcn_raw_ptr_buffer_load_lds(srs, ring + wb + buf * CHB, 16, dma_off, ch * XR8_KC, 0, 0);
    };
    i32x8 fb[2][CT];  // [register set][column tile]: the spins of one 128-k chunk
    auto load = [&](int i) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const unsigned char* base = smem + i * CHB + 2048 * ct;
        const uint4 lo = *reinterpret_cast<const uint4*>(base + boff[0]);
        const uint4 hi = *reinterpret_cast<const uint4*>(base + boff[1]);
        fb[i & 1][ct] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
    };
    f32x4 acc[RT][CT];

    // chunks 0 .. OWN - 1 (the own rows) come from the previous iteration's epilogue, or on the
    // first iteration from memory; the first batch, chunks OWN .. PRO, is loaded while they are
    // multiplied. Chunk i always goes to buffer i (NC <= NB): the group barrier at the end of the
    // previous iteration orders every load after every read of the buffer it overwrites.
    if (!own_in_lds) {
#pragma unroll
      for (int p = 0; p < OWN; ++p) issue(p, p);
    }
    constexpr int PRO = OWN + GB - 1 < NC - 1 ? OWN + GB - 1 : NC - 1;
#pragma unroll
    for (int p = OWN; p <= PRO; ++p) issue(p, p);
    wait_vm<PRO - OWN + 1>();
    bare_barrier();
    load(0);

    // chunk i: the spins of chunk i + 1 are read into the other register set while the MFMAs of
    // chunk i run. Before the first read of the batch that starts at chunk ci (during chunk ci - 1)
    // every wave waits for all of its loads and the workgroup meets at a barrier: chunks
    // ci .. ci + GB - 1 have landed for every wave. The next batch is issued then.
    static_for(
        [&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int ci = i + 1;
          if constexpr (ci < NC && ci >= OWN && (ci - OWN) % GB == 0) {
            wait_vm<0>();
            __builtin_amdgcn_sched_barrier(0);
            bare_barrier();
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = ci + GB; q < ci + 2 * GB && q < NC; ++q) issue(q, q);
          }
          wait_lds();
          if constexpr (i + 1 < NC) load(i + 1);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            const i32x8 af = i32x8{(int)jr[i][rt][0], (int)jr[i][rt][1], (int)jr[i][rt][2], (int)jr[i][rt][3],
                                   0, 0, 0, 0};
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
              acc[rt][ct] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                  af, fb[i & 1][ct], i == 0 ? f32x4{} : acc[rt][ct], 4, 0, 0, 0x7f7f7f7f, 0, 0x7f7f7f7f);
          }
          // The MFMA builtin has no side effects: without this the compiler sinks every chunk's
          // MFMAs to the epilogue and keeps all chunks' spin fragments live.
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) asm volatile("" : "+a"(acc[rt][ct]));
          __builtin_amdgcn_sched_barrier(0);
        },
        std::make_integer_sequence<int, NC>{});

    int lane_e = lane;
    asm volatile("" : "+v"(lane_e));
    const int c_e = lane_e & 15;
    const int row0e = rb * XR8_ROWS + 64 * wave + 4 * (lane_e >> 4);

    if (t < a.t_end) coef_next = coef[t];
    f32x4 invc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int q = 16 * wave + 4 * rt + (lane_e >> 4);
      invc[rt] = rowc[0][q] * coef_t;
      hrow[rt] = rowc[1][q];
    }

    // ---- fused epilogue --------------------------------------------------------------------
    // The own chunks (buffers 0, 1) were last read at the start of this iteration, so they may be
    // overwritten without a barrier.
    const int k_rec = t - a.t_begin;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int r = rgroup0 + 16 * ct + c_e;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // -tanh(Phi / T) = 2 / (1 + exp2(arg)) - 1 with arg = 2 log2(e) Phi / T; damped update
          const float e = __builtin_amdgcn_exp2f(fmaf(acc[rt][ct][v], invc[rt][v], w[rt][ct][v]));
          s[rt][ct][v] = fmaf(alpha2, __builtin_amdgcn_rcpf(1.0f + e), fmaf(oma, s[rt][ct][v], nalpha));
        }
        int pk = __builtin_amdgcn_cvt_pk_fp8_f32(s[rt][ct][0], s[rt][ct][1], 0, false);
        pk = __builtin_amdgcn_cvt_pk_fp8_f32(s[rt][ct][2], s[rt][ct][3], pk, true);
        *reinterpret_cast<int*>(Snext + (size_t)r * ks + row0e + 16 * rt) = pk;
        *reinterpret_cast<int*>(ring + own_off(rt, ct, lane_e)) = pk;
      }
    }
    if (traj && k_rec < a.record) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int r = rgroup0 + 16 * ct + c_e;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = row0e + 16 * rt + v;
            if (r < a.R && row < N) traj[((size_t)k_rec * a.R + r) * N + row] = s[rt][ct][v];
          }
      }
    }

    if (t < a.t_end) {
      // half of the next iteration's noise while the spin stores complete, arrive, the other half
      // while the other workgroups arrive, then wait for the group (the wait ends with a workgroup
      // barrier, after which the buffers may be overwritten)
      draw(t + 1, 0, 4, coef_next);
      pin_noise(0, 4);
      xcd_group_arrive(bar, xcd_mode, tid);
      draw(t + 1, 4, 2, coef_next);
      pin_noise(4, 2);
      unsigned seen = 0;
      __builtin_amdgcn_sched_barrier(0);
      if (tid == 0) seen = ld_dev(bar);  // polled once ahead, read after the last draws
      __builtin_amdgcn_sched_barrier(0);
      draw(t + 1, 6, 2, coef_next);
      pin_noise(6, 2);
      aborted = xrj_group_wait(x, bar, (unsigned)++epoch, xcd_mode, tid, seen, &abort_word);
    }
  }

  // ---- final state and readout ---------------------------------------------------------------
  int lane_f = lane;
  asm volatile("" : "+v"(lane_f));
  const int row0f = rb * XR8_ROWS + 64 * wave + 4 * (lane_f >> 4);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int r = rgroup0 + 16 * ct + (lane_f & 15);
    if (r >= a.R) continue;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0f + 16 * rt + v;
        if (row < N) {
          state[(size_t)r * N + row] = s[rt][ct][v];
          if (a.spins) a.spins[(size_t)r * N + row] = (s[rt][ct][v] >= 0.0f) ? (int8_t)1 : (int8_t)-1;
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

int xrj_rows(int fp8_spins) { return fp8_spins ? XR8_ROWS : XRB_ROWS; }
int xrj_group_replicas(int fp8_spins) { return fp8_spins ? XR8_RG : XRB_RG; }
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
  return launch_resident(fn, groups * x.P, 256, (size_t)XR8_NB * XR8_CHB, a, x, st);
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
  return launch_resident(fn, groups * x.P, 256, (size_t)XRB_NB * XRB_CHB, a, x, st);
}

hipError_t launch_anneal_xcd(int jfmt, const AnnealArgs& a, const XcdArgs& x, int groups, hipStream_t st) {
  const size_t lds = xcd_j_lds_bytes(jfmt, a.Kp) + (size_t)x.nbuf * xcd_chunk_bytes();
  const void* fn = jfmt == 0 ? xcd_fn<0>(x.nbuf) : (jfmt == 1 ? xcd_fn<1>(x.nbuf) : xcd_fn<2>(x.nbuf));
  if (!fn) return hipErrorInvalidValue;
  return launch_resident(fn, groups * x.P, 512, lds, a, x, st);
}

}  // namespace nmfa
