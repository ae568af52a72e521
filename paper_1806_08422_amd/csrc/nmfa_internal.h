// Internal interface between the C-ABI layer (nmfa_api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nmfa {

// Arguments of one anneal launch (passed by value to the kernels).
struct AnnealArgs {
  const void* J;         // couplings, [Mp][Kp] row-major in the operand type (FP8 bytes for J8)
  const void* inv_norm;  // [Mp] 1/sqrt(h_i^2 + sum_j J_ij^2), 0 for padding and zero normalisers
  const void* hterm;     // [Mp] FP64 path: h_i; FP32/BF16 paths: h_i * inv_norm_i
  const void* coef;      // [t_f] FP64 path: 1/T_t; FP32/BF16 paths: 2 log2(e) / T_t
  void* state;           // [R][N] master state (FP64 or FP32), in/out
  int8_t* spins;         // [R][N] sign readout, or null
  void* traj;            // [record][R][N] master-precision trajectory, or null
  int record;            // number of iterations recorded, counted from t_begin
  int N, Mp, Kp, R, Rp;  // spins, padded rows, padded k, replicas, padded replicas
  int lds_stride;        // LDS row stride in elements (persistent kernel)
  int t_begin, t_end;    // iterations run, 1-based, inclusive
  int load_state;        // 1: continue from `state`; 0: start from s = 0
  uint32_t key0, key1;   // Philox key = 64-bit seed
  double alpha, sigma;
  int negate_noise;      // test hook: z -> -z
};

// Persistent large-N kernel (XCD groups): extra arguments.
struct XcdArgs {
  void* S[2];        // operand copies of the spins, BF16 [Rp][ks], double-buffered by parity of t
  int ks;            // row stride of S in elements (>= Kp, a multiple of 8)
  unsigned* ctl;     // control block (xcd_ctl_words() words, zeroed before every launch)
  int P;             // workgroups per replica group = Mp / xcd_rows()
  int group_base;    // first replica group of this launch
  int force_fenced;  // test hook: use device-scope fences even when the groups are XCD-local
  int nbuf;          // spin chunk buffers in LDS: 2, 3, 4 or 6
};

hipError_t launch_anneal_small(int prec, const AnnealArgs& a, hipStream_t st);
// jobs: device array of AnnealArgs (one per job); tasks: device array of (job, replica block).
hipError_t launch_anneal_small_batched(int prec, const AnnealArgs* jobs, const int2* tasks, int n_tasks,
                                       int max_Mp, size_t lds, hipStream_t st);
// jfmt: format of J in global memory and LDS: 0 = BF16, 1 = FP8 E4M3, 2 = FP4 E2M1
hipError_t launch_anneal_xcd(int jfmt, const AnnealArgs& a, const XcdArgs& x, int groups, hipStream_t st);
// Register-resident-J variant (FP4 J), Kp = xrj_kp(n): BF16 spins with 256 rows per workgroup and
// groups of 32 replicas; FP8 spins (launch_anneal_xrj8) with 128 rows and groups of 64 replicas.
hipError_t launch_anneal_xrj(const AnnealArgs& a, const XcdArgs& x, int groups, hipStream_t st);
// The same decomposition with FP8 E4M3 spin operands (FP4 x FP8 scaled MFMA); S holds bytes.
hipError_t launch_anneal_xrj8(const AnnealArgs& a, const XcdArgs& x, int groups, hipStream_t st);
int xrj_rows(int fp8_spins);
int xrj_group_replicas(int fp8_spins);
int xrj_kp(int n);
bool xrj_fits(int n);
size_t xcd_j_lds_bytes(int jfmt, int Kp);
size_t xcd_chunk_bytes();
int xcd_spin_stride(int Kp);  // row stride of S for the XCD kernel
int xcd_pick_buffers(size_t lds_room);  // chunk buffers that fit in lds_room bytes (0 if < 2)
int xcd_ctl_words();
// Zero words [a0, a1) and [b0, b1) of p (device) on st; either range may be empty.
hipError_t launch_zero_words(uint32_t* p, size_t a0, size_t a1, size_t b0, size_t b1, hipStream_t st);
int xcd_rows();
int xcd_group_replicas();
size_t small_lds_bytes(int prec, int Mp, int stride);
// jfmt: storage format of J for the BF16-operand precisions (0 = BF16, 1 = FP8 E4M3, 2 = FP4 E2M1;
// the tiled kernel widens FP8 / FP4 to BF16); 0 for FP32 / FP64
hipError_t launch_anneal_step(int prec, int jfmt, const AnnealArgs& a, const void* S_cur, void* S_next, int t,
                              hipStream_t st);
// Writes rows [0, Rp) x columns [0, Kp) of S (row stride ld) from the master state (zero: all 0).
hipError_t launch_pack_state(int prec, const void* state, void* S, int N, int R, int Kp, int ld, int Rp, int zero,
                             hipStream_t st);
hipError_t launch_readout(int prec, const void* state, int8_t* spins, size_t count, hipStream_t st);
// With J8: h_integral tells whether h is integral (then E_int is exact). With J64 instead: h_integral
// = 1 states that J and h are integral and every sum fits in 2^53, so E_int is exact; else E_int = 0.
hipError_t launch_energy(const int8_t* J8, const double* J64, const double* h, int h_integral,
                         const int8_t* spins, int N, int R, long long* E_int, double* E, hipStream_t st);
// Sparse couplings in ELL form (D entries per row, ascending columns, zero-weight padding; values
// in the accumulation type of prec: FP64 for PREC_FP64, else FP32); RB replicas per workgroup.
// allow_rq: use the register-ELL kernel where it applies; *used_rq (if not null) tells whether it ran.
// sparse_rq_applies: the register-ELL kernel serves (prec, N, D) for any replica count.
size_t sparse_lds_bytes(int prec, int N, int RB);
int sparse_rq_applies(int prec, int N, int D);
hipError_t launch_anneal_sparse(int prec, const AnnealArgs& a, const int* ell_col, const void* ell_val, int D,
                                int RB, int allow_rq, int* used_rq, hipStream_t st);
// Exact energies for integral |J| <= 127 on the int8 matrix cores. J8p: [Np][Np] zero-padded
// (Np a multiple of 64); Sp: scratch of roundup(R, 64) * Np bytes; E2: scratch of R int64.
hipError_t launch_energy_i8(const int8_t* J8p, int Np, const double* h, int h_integral, const int8_t* spins,
                            int N, int R, int8_t* Sp, unsigned long long* E2, long long* E_int, double* E,
                            hipStream_t st);
hipError_t launch_noise_words(uint32_t k0, uint32_t k1, uint32_t t, uint32_t r0, int nrep, int nq,
                              uint32_t* out, hipStream_t st);
hipError_t launch_noise_values(uint32_t k0, uint32_t k1, uint32_t t, uint32_t r0, int nrep, int nq,
                               int fp64, double* out, hipStream_t st);

}  // namespace nmfa
