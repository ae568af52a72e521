// Internal: the solver context behind the opaque nmfa_ctx handle of include/nmfa.h, and the
// pieces of the anneal call that the serving scheduler reuses.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/nmfa.h"
#include "nmfa_internal.h"

struct nmfa_ctx {
  int n = 0;
  int prec = NMFA_BF16;
  int path = 0;  // 0 = persistent small-N kernel, 1 = per-iteration kernel, 2 = XCD-group kernel
  int jfmt = 1;              // path 2: J format in LDS (0 BF16, 1 FP8 E4M3, 2 FP4 E2M1)
  int nbuf = 2;              // path 2: spin chunk buffers in LDS (2, 3, 4 or 6)
  int xvar = 0;              // path 2: 0 = J rows in LDS, 1 = J rows in registers (FP4)
  unsigned* d_ctl = nullptr; // path 2: control block
  bool ctl_pending = false;  // path 2: abort/mode flags not yet read back
  int exchange_mode = 0;     // path 2: 1 = XCD-local, 2 = device-scope fences
  int Mp = 0, Kp = 0, lds_stride = 0;
  int Ks = 0;                 // row stride (elements) of the spin operand copies d_S
  double alpha = 0.15, sigma = 0.15;
  uint32_t flags = 0;
  int record = 0;
  std::vector<double> ku, kT;
  std::vector<double> T_explicit;  // caller's temperatures T_1..T_tf (empty: the knots)
  std::vector<double> h;  // empty if h = 0
  bool has_h = false;
  bool J_integral = false, h_integral = true;
  bool exact_int = false;        // energies are also returned as exact integers (J, h integral)
  bool pairs_exact_f64 = false;  // integral J beyond int8: the FP64 energy kernel's sums are exact
  double w_total = 0.0;  // sum_{i<j} J_ij
  int device = 0;

  // device data of the instance
  void* d_J = nullptr;       // operand layout of the selected path
  void* d_inv = nullptr;     // [Mp] acc_t
  void* d_hterm = nullptr;   // [Mp] acc_t
  int8_t* d_J8 = nullptr;    // [Np8][Np8] zero-padded, for exact energies (integral |J| <= 127)
  int Np8 = 0;               // roundup(n, 64)
  double* d_J64 = nullptr;   // [n][n] otherwise
  int* d_ell_col = nullptr;  // path 3: [n][ell_D] column indices (ascending, padded with i)
  void* d_ell_val = nullptr; // path 3: [n][ell_D] couplings (FP64 for the FP64 precision, else FP32)
  int ell_D = 0;             // path 3: entries per row (maximum degree)
  int sp_RB = 0;             // path 3: replicas per workgroup (generic ELL kernel)
  int sp_rq = 0;             // path 3: the last anneal ran the register-ELL kernel
  double* d_h = nullptr;     // [n] or null

  // per-run buffers
  int cap_R = 0;             // replicas the buffers hold
  int R = 0, t_f = 0;        // current run
  uint64_t seed = 0;
  bool state_valid = false;
  bool result_valid = false;
  int traj_iters = 0;        // iterations recorded by the last call
  void* d_state = nullptr;   // [R][n] acc_t
  int8_t* d_spins = nullptr; // [R][n]
  double* d_E = nullptr;     // [R]
  long long* d_Eint = nullptr;
  int8_t* d_Sp = nullptr;    // energy scratch: padded signs [roundup(R, 64)][Np8]
  unsigned long long* d_E2 = nullptr;  // energy scratch [R]
  void* d_S[2] = {nullptr, nullptr};  // paths 1 and 2: [Rp][Ks] op_t
  int cap_Rp = 0;
  void* d_traj = nullptr;
  size_t traj_cap = 0;
  void* d_coef = nullptr;
  int coef_tf = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evm = nullptr;
  int launches = 0;
  bool timed = false;

  size_t acc_size() const { return prec == NMFA_FP64 ? 8 : 4; }
  size_t op_size() const { return prec == NMFA_FP64 ? 8 : (prec == NMFA_FP32 ? 4 : (prec == NMFA_FP8J_FP8S ? 1 : 2)); }
};

// Validate one anneal call, make its buffers and fill the kernel arguments (no launch).
int ctx_prepare_run(nmfa_ctx* c, int32_t R, int32_t t_f, int32_t t_begin, int32_t t_end, uint64_t seed,
                    hipStream_t st, nmfa::AnnealArgs* out);
// For the persistent XCD-group path (whose workgroups wait for each other, so that all of one
// launch must be resident at once): P workgroups per replica group and G groups for R replicas.
// Returns false for the other paths.
bool ctx_group_shape(const nmfa_ctx* c, int32_t R, int* P, int* G);
// Enqueue iterations t_begin..t_end on the context's kernel path; with finish, also the energies.
// max_workgroups > 0 caps the workgroups of one group-kernel launch (more launches, one after the
// other on st, cover the remaining groups); results do not depend on it.
int ctx_launch_run(nmfa_ctx* c, int32_t R, int32_t t_f, int32_t t_begin, int32_t t_end, uint64_t seed,
                   hipStream_t st, bool finish, int max_workgroups = 0);
// Energies (E_int zero unless exact) and spins of a run whose energies were enqueued by
// ctx_finish_run: waits for that run's own completion event rather than its stream, which may
// already hold later work, then checks the group kernels' abort word. All pointers are host.
int ctx_read_results(nmfa_ctx* c, double* E, int64_t* E_int, int8_t* spins);
// Enqueue the energies of the readout and mark the results valid.
int ctx_finish_run(nmfa_ctx* c, hipStream_t st);
// Record an error message for nmfa_last_error() and return code.
int nmfa_fail(int code, const char* fmt, ...);
