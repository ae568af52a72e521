// C-ABI layer of libnmfa.so: argument validation, host-side setup (normalisers, schedule,
// operand conversion), device buffers and kernel dispatch. Declarations and the contract of
// every entry point are in include/nmfa.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/nmfa.h"
#include "nmfa_ctx.h"
#include "nmfa_internal.h"

using namespace nmfa;

// ------------------------------------------------------------------------------------------
// Error reporting
// ------------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

int nmfa_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
#define fail nmfa_fail

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return fail(_e == hipErrorOutOfMemory ? NMFA_ENOMEM : NMFA_EDEVICE, "%s failed: %s", \
                  #expr, hipGetErrorString(_e));                                            \
  } while (0)

extern "C" const char* nmfa_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------------------------------
// Host helpers
// ------------------------------------------------------------------------------------------
static const double kDefaultKnotU[4] = {0.0, 0.1, 0.6, 1.0};
static const double kDefaultKnotT[4] = {10.0, 2.0, 0.5, 0.05};

static size_t round_up(size_t v, size_t m) { return (v + m - 1) / m * m; }

// Temperature of iteration t (1-based) of a t_f-iteration run: log T is linear in relative time
// between consecutive knots (the paper's three-segment piecewise-exponential schedule, Fig. 2).
static double schedule_T(const std::vector<double>& ku, const std::vector<double>& kT, int t, int t_f) {
  const size_t K = kT.size();
  if (K == 1) return kT[0];
  const double u = (t_f <= 1) ? 0.0 : double(t - 1) / double(t_f - 1);
  size_t seg = 0;
  while (seg + 2 < K && u > ku[seg + 1]) ++seg;
  if (u == ku[seg]) return kT[seg];
  if (u == ku[seg + 1]) return kT[seg + 1];
  const double w = (u - ku[seg]) / (ku[seg + 1] - ku[seg]);
  return std::exp((1.0 - w) * std::log(kT[seg]) + w * std::log(kT[seg + 1]));
}

static uint16_t bf16_bits(double v) {
  float f = (float)v;
  uint32_t b;
  std::memcpy(&b, &f, 4);
  b += 0x7fffu + ((b >> 16) & 1u);  // round to nearest even (finite values)
  return (uint16_t)(b >> 16);
}

// FP8 E4M3 ("fn": bias 7, max 448, no infinities), round to nearest even, saturating.
static uint8_t fp8e4m3_bits(double v) {
  const uint8_t sign = std::signbit(v) ? 0x80 : 0x00;
  double a = std::fabs(v);
  if (a == 0.0) return sign;
  if (a >= 464.0) return sign | 0x7e;
  int e2;
  std::frexp(a, &e2);
  int ex = e2 - 1;  // a = 2^ex * (1 + f)
  if (ex < -6) {
    double k = std::nearbyint(a * 512.0);  // subnormal step 2^-9
    if (k >= 8.0) return sign | 0x08;      // rounds up to the smallest normal 2^-6
    return sign | (uint8_t)k;
  }
  double f = std::nearbyint((a / std::ldexp(1.0, ex) - 1.0) * 8.0);
  if (f >= 8.0) {
    f = 0.0;
    ex += 1;
  }
  if (ex > 8 || (ex == 8 && f > 6.0)) return sign | 0x7e;
  return sign | (uint8_t)((ex + 7) << 3) | (uint8_t)f;
}

static double fp8e4m3_value(uint8_t b) {
  const int e = (b >> 3) & 0xf, m = b & 7;
  double w = (e == 0) ? std::ldexp((double)m, -9) : std::ldexp(1.0 + m / 8.0, e - 7);
  return (b & 0x80) ? -w : w;
}

// FP4 E2M1 code (sign bit 8, magnitudes 0, 1/2, 1, 3/2, 2, 3, 4, 6) of v, or -1 if v is not one.
static int fp4e2m1_code(double v) {
  static const double mags[8] = {0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0};
  const double a = std::fabs(v);
  for (int k = 0; k < 8; ++k)
    if (a == mags[k]) return (v < 0 ? 8 : 0) | k;
  return -1;
}

static bool is_integral(double v) { return std::isfinite(v) && v == std::floor(v) && std::fabs(v) < 9e15; }

// The storage codes of coupling values (FP8 bits and value, FP4 code, BF16 bits), memoised by
// bit pattern: an instance has few distinct couplings (often 0 and +-1), and the rounding
// routines would otherwise run once per matrix element. Values beyond the first CAP distinct
// ones are converted directly.
// Runs f(lo, hi) over [0, n) split into contiguous ranges on up to 16 host threads (one range
// for small n, where starting threads costs more than the pass).
template <class F>
static void parallel_rows(int n, F&& f) {
  int T = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  T = std::min(T, n / 128);
  if (T <= 1) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T);
  for (int t = 0; t < T; ++t) {
    const int lo = (int)((long)n * t / T), hi = (int)((long)n * (t + 1) / T);
    th.emplace_back([&f, lo, hi] { f(lo, hi); });
  }
  for (auto& x : th) x.join();
}

struct CouplingCodes {
  static constexpr int CAP = 16;
  int n = 0;
  uint64_t key[CAP];
  uint8_t f8[CAP];
  double f8v[CAP];
  int f4[CAP];
  uint16_t b16[CAP];
  int slot(double v) {
    uint64_t b;
    std::memcpy(&b, &v, 8);
    for (int k = 0; k < n; ++k)
      if (key[k] == b) return k;
    if (n == CAP) return -1;
    key[n] = b;
    f8[n] = fp8e4m3_bits(v);
    f8v[n] = fp8e4m3_value(f8[n]);
    f4[n] = fp4e2m1_code(v);
    b16[n] = bf16_bits(v);
    return n++;
  }
  uint8_t fp8(double v) {
    const int k = slot(v);
    return k >= 0 ? f8[k] : fp8e4m3_bits(v);
  }
  double fp8_value(double v) {
    const int k = slot(v);
    return k >= 0 ? f8v[k] : fp8e4m3_value(fp8e4m3_bits(v));
  }
  int fp4(double v) {
    const int k = slot(v);
    return k >= 0 ? f4[k] : fp4e2m1_code(v);
  }
  uint16_t bf16(double v) {
    const int k = slot(v);
    return k >= 0 ? b16[k] : bf16_bits(v);
  }
};

// ------------------------------------------------------------------------------------------
// Context
// ------------------------------------------------------------------------------------------

static void free_run_buffers(nmfa_ctx* c) {
  (void)hipFree(c->d_state);
  (void)hipFree(c->d_spins);
  (void)hipFree(c->d_E);
  (void)hipFree(c->d_Eint);
  (void)hipFree(c->d_Sp);
  (void)hipFree(c->d_E2);
  c->d_Sp = nullptr;
  c->d_E2 = nullptr;
  (void)hipFree(c->d_S[0]);
  (void)hipFree(c->d_S[1]);
  c->d_state = nullptr;
  c->d_spins = nullptr;
  c->d_E = nullptr;
  c->d_Eint = nullptr;
  c->d_S[0] = c->d_S[1] = nullptr;
  c->cap_R = 0;
  c->cap_Rp = 0;
}

extern "C" void nmfa_params_default(nmfa_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(nmfa_params);
  p->precision = NMFA_BF16;
  p->alpha = 0.15;
  p->sigma = 0.15;
  p->n_knots = 0;
  p->flags = 0;
  p->record_iters = 0;
}

extern "C" void nmfa_destroy(nmfa_ctx* c) {
  if (!c) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_run_buffers(c);
  (void)hipFree(c->d_J);
  (void)hipFree(c->d_inv);
  (void)hipFree(c->d_hterm);
  (void)hipFree(c->d_J8);
  (void)hipFree(c->d_J64);
  (void)hipFree(c->d_ell_col);
  (void)hipFree(c->d_ell_val);
  (void)hipFree(c->d_h);
  (void)hipFree(c->d_traj);
  (void)hipFree(c->d_coef);
  (void)hipFree(c->d_ctl);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->evm) (void)hipEventDestroy(c->evm);
  (void)hipSetDevice(prev);
  delete c;
}

static int device_max_lds() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
  return v;
}

extern "C" int nmfa_create(int32_t n, const double* J, const double* h, const nmfa_params* p,
                           nmfa_ctx** out) {
  if (!out) return fail(NMFA_EINVAL, "nmfa_create: out is NULL");
  *out = nullptr;
  nmfa_params dp;
  nmfa_params_default(&dp);
  if (!p) p = &dp;
  if (p->struct_size != sizeof(nmfa_params))
    return fail(NMFA_EINVAL, "nmfa_create: params.struct_size %u != %zu", p->struct_size, sizeof(nmfa_params));
  if (n < 1 || n > 16384) return fail(NMFA_EINVAL, "nmfa_create: n = %d outside [1, 16384]", n);
  if (!J) return fail(NMFA_EINVAL, "nmfa_create: J is NULL");
  if (p->precision > NMFA_FP8J_FP8S) return fail(NMFA_EINVAL, "nmfa_create: unknown precision %u", p->precision);
  if (!(p->alpha > 0.0 && p->alpha <= 1.0)) return fail(NMFA_EINVAL, "nmfa_create: alpha must be in (0, 1]");
  if (!(p->sigma >= 0.0) || !std::isfinite(p->sigma)) return fail(NMFA_EINVAL, "nmfa_create: sigma must be >= 0");
  if (p->record_iters < 0) return fail(NMFA_EINVAL, "nmfa_create: record_iters < 0");
  if (p->n_T_explicit < 0 || (p->n_T_explicit > 0 && !p->T_explicit))
    return fail(NMFA_EINVAL, "nmfa_create: invalid explicit temperatures");
  for (int k = 0; k < p->n_T_explicit; ++k)
    if (!(p->T_explicit[k] > 0.0) || !std::isfinite(p->T_explicit[k]))
      return fail(NMFA_EINVAL, "nmfa_create: explicit temperature %d is not a finite value > 0", k);

  // schedule knots
  std::vector<double> ku, kT;
  if (p->n_knots == 0) {
    ku.assign(kDefaultKnotU, kDefaultKnotU + 4);
    kT.assign(kDefaultKnotT, kDefaultKnotT + 4);
  } else {
    if (p->n_knots < 0 || !p->knot_T || (p->n_knots > 1 && !p->knot_u))
      return fail(NMFA_EINVAL, "nmfa_create: invalid schedule knots");
    for (int k = 0; k < p->n_knots; ++k) {
      if (!(p->knot_T[k] > 0.0) || !std::isfinite(p->knot_T[k]))
        return fail(NMFA_EINVAL, "nmfa_create: knot temperature %d is not > 0", k);
      kT.push_back(p->knot_T[k]);
      ku.push_back(p->n_knots > 1 ? p->knot_u[k] : 0.0);
      if (k > 0 && !(ku[k] > ku[k - 1])) return fail(NMFA_EINVAL, "nmfa_create: knot positions must increase");
    }
    if (p->n_knots > 1 && (ku.front() != 0.0 || ku.back() != 1.0))
      return fail(NMFA_EINVAL, "nmfa_create: knot positions must start at 0 and end at 1");
  }

  // couplings: symmetrise if given as an upper triangle (else J is used in place), validate
  const size_t nn = (size_t)n * n;
  const bool upper = (p->flags & NMFA_FLAG_UPPER_TRIANGULAR) != 0;
  std::vector<double> Jmirror;
  if (upper) {
    Jmirror.resize(nn);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        Jmirror[(size_t)i * n + j] = (i < j) ? J[(size_t)i * n + j] : (i > j ? J[(size_t)j * n + i] : 0.0);
  }
  const double* Jf = upper ? Jmirror.data() : J;
  // one pass over the rows (on host threads) gathers what the checks and the set-up need:
  // finiteness, integrality and magnitude, the exact storage formats, nonzeros per row, and
  // h_i^2 + sum_j J_ij^2 summed in column order
  const bool fp8j = p->precision == NMFA_FP8J_BF16S || p->precision == NMFA_FP8J_FP8S;
  struct RowInfo {
    int bad_j = -1, sym_j = -1, deg = 0, jmax = 0;
    bool integral = true, fp8x = true, fp4x = true;
    double sumsq = 0.0;
  };
  std::vector<RowInfo> rows(n);
  parallel_rows(n, [&](int lo, int hi) {
    CouplingCodes cc;
    for (int i = lo; i < hi; ++i) {
      RowInfo& r = rows[i];
      const double* Ji = Jf + (size_t)i * n;
      double acc = h ? h[i] * h[i] : 0.0;
      for (int j = 0; j < n; ++j) {
        const double v = Ji[j];
        if (!std::isfinite(v)) {
          r.bad_j = j;
          break;
        }
        acc += v * v;
        if (v != 0.0) ++r.deg;
        if (r.integral) {
          if (is_integral(v)) r.jmax = std::max(r.jmax, (int)std::min(std::fabs(v), 1e9));
          else r.integral = false;
        }
        if (r.fp8x || r.fp4x) {
          const double w = fp8j ? cc.fp8_value(v) : v;
          if (!fp8j && cc.fp8_value(w) != w) r.fp8x = false;
          if (cc.fp4(w) < 0) r.fp4x = false;
        }
      }
      r.sumsq = acc;
    }
  });
  for (int i = 0; i < n; ++i)
    if (rows[i].bad_j >= 0) return fail(NMFA_EINVAL, "nmfa_create: J[%d][%d] is not finite", i, rows[i].bad_j);
  for (int i = 0; i < n; ++i)
    if (Jf[(size_t)i * n + i] != 0.0) return fail(NMFA_EINVAL, "nmfa_create: J[%d][%d] != 0 (diagonal)", i, i);
  // symmetry in 64 x 64 tiles, so that the transposed reads stay in cache; each row keeps its
  // first violation, so the first one in row-major order is reported
  parallel_rows((n + 63) / 64, [&](int blo, int bhi) {
    for (int ib = 64 * blo; ib < std::min(64 * bhi, n); ib += 64)
      for (int jb = ib; jb < n; jb += 64)
        for (int i = ib; i < std::min(ib + 64, n); ++i)
          for (int j = std::max(jb, i + 1); j < std::min(jb + 64, n); ++j)
            if (rows[i].sym_j < 0 && Jf[(size_t)i * n + j] != Jf[(size_t)j * n + i]) rows[i].sym_j = j;
  });
  for (int i = 0; i < n; ++i)
    if (rows[i].sym_j >= 0)
      return fail(NMFA_EINVAL, "nmfa_create: J is not symmetric at (%d, %d)", i, rows[i].sym_j);
  if (h)
    for (int i = 0; i < n; ++i)
      if (!std::isfinite(h[i])) return fail(NMFA_EINVAL, "nmfa_create: h[%d] is not finite", i);

  nmfa_ctx* c = new nmfa_ctx();
  c->n = n;
  c->prec = (int)p->precision;
  c->alpha = p->alpha;
  c->sigma = p->sigma;
  c->flags = p->flags;
  c->record = p->record_iters;
  c->ku = ku;
  c->kT = kT;
  if (p->n_T_explicit > 0) c->T_explicit.assign(p->T_explicit, p->T_explicit + p->n_T_explicit);
  (void)hipGetDevice(&c->device);
  bool any_h = false;
  if (h) {
    c->h.assign(h, h + n);
    for (int i = 0; i < n; ++i) {
      if (h[i] != 0.0) any_h = true;
      if (!is_integral(h[i])) c->h_integral = false;
    }
  }
  c->has_h = any_h;
  if (!any_h) c->h.clear();
  c->J_integral = true;
  int Jmax = 0;
  for (int i = 0; i < n; ++i) {
    c->J_integral = c->J_integral && rows[i].integral;
    Jmax = std::max(Jmax, rows[i].jmax);
  }
  const bool use_J8 = c->J_integral && Jmax <= 127;
  // integral couplings beyond the int8 range: the FP64 energy kernel's sums are exact integers as
  // long as every |sum_i s_i sum_j J_ij s_j| stays below 2^53
  const bool pairs_exact_f64 = c->J_integral && (double)Jmax * (double)n * (double)n < 4503599627370496.0;
  c->exact_int = c->h_integral && (use_J8 || pairs_exact_f64);
  c->pairs_exact_f64 = pairs_exact_f64 && !use_J8;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) c->w_total += Jf[(size_t)i * n + j];

  // kernel path and padded layout
  const size_t es = c->op_size();
  const bool fp8s = c->prec == NMFA_FP8J_FP8S;
  const bool bf = (c->prec == NMFA_BF16 || c->prec == NMFA_FP8J_BF16S || fp8s);
  // exact formats of the couplings the MFMA consumes (FP8-rounded for the FP8-J precision)
  bool j_fp8_exact = true, j_fp4_exact = true;
  for (int i = 0; i < n; ++i) {
    j_fp8_exact = j_fp8_exact && rows[i].fp8x;
    j_fp4_exact = j_fp4_exact && rows[i].fp4x;
  }
  const int Mp_s = (int)round_up(n, 16);
  const int Kp_s = (int)round_up(n, bf ? 32 : 16);
  const int stride_s = (int)((round_up(Kp_s * es, 256) + 16) / es);
  const bool small_fits = Mp_s <= 256 && small_lds_bytes(c->prec, Mp_s, stride_s) <= (size_t)device_max_lds();
  // persistent XCD-group kernel: BF16 operands; J rows in LDS as FP4 / FP8 when exact, else BF16
  const int Mp_x = (int)round_up(n, xcd_rows());
  const int Kp_x = (int)round_up(n, 128);
  const int x_jfmt = j_fp4_exact ? 2 : (j_fp8_exact ? 1 : 0);
  const size_t x_jlds = xcd_j_lds_bytes(x_jfmt, Kp_x);
  const size_t lds_max = (size_t)device_max_lds();
  const int x_nbuf = x_jlds < lds_max ? xcd_pick_buffers(lds_max - x_jlds) : 0;  // spin chunk ring
  const bool x_ok = bf && Mp_x / xcd_rows() <= 32 && x_nbuf >= 2;
  // register-resident-J variant of the XCD-group kernel: FP4-exact couplings, n <= 2048
  const bool x_rj = x_ok && x_jfmt == 2 && xrj_fits(n) && !(p->flags & NMFA_FLAG_FORCE_LDS_J);
  // sparse (ELL) kernel: maximum degree D <= 64 and the workgroup's state fits in LDS
  int deg_max = 0;
  for (int i = 0; i < n; ++i) deg_max = std::max(deg_max, rows[i].deg);
  const int sp_prec = (c->prec == NMFA_FP64) ? 0 : 1;  // kernel arithmetic: FP64 or FP32
  int sp_rb = 0;
  for (int rb : {8, 4, 2, 1})
    if (sparse_lds_bytes(sp_prec, n, rb) <= (size_t)64 * 1024) { sp_rb = rb; break; }
  if (!sp_rb && sparse_lds_bytes(sp_prec, n, 1) <= (size_t)device_max_lds()) sp_rb = 1;
  const bool sp_ok = deg_max <= 64 && sp_rb > 0;
  // chosen by itself where the register-ELL kernel serves it (2-4x faster than the dense kernels
  // at n = 2000, degree 3-16), or where no persistent dense kernel applies; the generic ELL
  // kernel, which reads J from global memory every iteration, is slower than the XCD kernel
  const bool sp_rq = sp_ok && sparse_rq_applies(sp_prec, n, std::max(deg_max, 1));
  const bool sp_auto = sp_ok && n > 256 && 8 * std::max(deg_max, 1) <= n && (sp_rq || !x_ok);
  if (fp8s) {
    // FP8 spins run on the register-J kernel only
    if (!x_rj || (p->flags & (NMFA_FLAG_FORCE_STEP | NMFA_FLAG_FORCE_SPARSE))) {
      nmfa_destroy(c);
      return fail(NMFA_EINVAL, "nmfa_create: FP8 spins need the register-J kernel: couplings exact in FP4 E2M1 "
                               "(e.g. {0, +-1}), n <= 2048, and none of FORCE_STEP / FORCE_SPARSE / FORCE_LDS_J");
    }
    c->path = 2;
  } else if (p->flags & NMFA_FLAG_FORCE_STEP) {
    c->path = 1;
  } else if (p->flags & NMFA_FLAG_FORCE_SPARSE) {
    if (!sp_ok) {
      nmfa_destroy(c);
      return fail(NMFA_EINVAL, "nmfa_create: the sparse kernel needs at most 64 couplings per row and a state "
                               "that fits in LDS (n = %d, maximum degree %d)", n, deg_max);
    }
    c->path = 3;
  } else if ((p->flags & NMFA_FLAG_FORCE_XCD) && x_ok) {
    c->path = 2;
  } else if ((p->flags & NMFA_FLAG_FORCE_XCD)) {
    return fail(NMFA_EINVAL, "nmfa_create: the XCD-group kernel needs BF16 / FP8-J precision, n <= 2048 and "
                             "couplings that fit its LDS");
  } else if (small_fits) {
    c->path = 0;
  } else if (sp_auto) {
    c->path = 3;
  } else if (x_ok) {
    c->path = 2;
  } else {
    c->path = 1;
  }
  if (c->path == 0) {
    c->Mp = Mp_s;
    c->Kp = Kp_s;
    c->lds_stride = stride_s;
  } else if (c->path == 3) {
    c->Mp = (int)round_up(n, 4);
    c->Kp = c->Mp;
    c->lds_stride = 0;
    c->ell_D = std::max(deg_max, 1);
    c->sp_RB = sp_rb;
  } else if (c->path == 2 && x_rj) {
    c->xvar = fp8s ? 2 : 1;
    c->Mp = (int)round_up(n, xrj_rows(fp8s ? 1 : 0));
    c->Kp = xrj_kp(n);
    c->lds_stride = 0;
    c->jfmt = x_jfmt;
  } else if (c->path == 2) {
    c->Mp = Mp_x;
    c->Kp = Kp_x;
    c->lds_stride = 0;
    c->jfmt = x_jfmt;
    c->nbuf = x_nbuf;
  } else {
    c->Mp = (int)round_up(n, 256);  // the tiled per-iteration kernels work on 256-row (BF16) and 128-row (FP64) tiles
    c->Kp = c->Mp;
    c->lds_stride = 0;
    c->jfmt = bf ? x_jfmt : 0;  // BF16-operand precisions: J streamed as FP4 / FP8 where exact
  }
  c->Ks = c->path == 2 ? xcd_spin_stride(c->Kp) : c->Kp;
  const int Mp = c->Mp, Kp = c->Kp;

  // normalisers sqrt(h_i^2 + sum_j J_ij^2) in FP64; a zero normaliser gives inv = 0
  std::vector<double> inv(Mp, 0.0), hterm(Mp, 0.0);
  for (int i = 0; i < n; ++i) {
    const double hi = any_h ? h[i] : 0.0;
    const double nrm = std::sqrt(rows[i].sumsq);
    inv[i] = nrm > 0.0 ? 1.0 / nrm : 0.0;
    hterm[i] = (c->prec == NMFA_FP64) ? hi : hi * inv[i];
  }

  // operand copy of J: FP8 bytes for the small FP8-J kernel; FP4 / FP8 / BF16 for the XCD-group
  // kernel and the tiled per-iteration kernel of the BF16-operand precisions; else the precision's
  // operand type
  const bool j8_small = (c->prec == NMFA_FP8J_BF16S && c->path == 0);
  const int jfmt2 = (c->path == 2 || (c->path == 1 && bf)) ? c->jfmt : -1;
  size_t jbytes;
  if (c->path == 3) jbytes = 0;  // the sparse kernel reads its ELL copy instead
  else if (j8_small || jfmt2 == 1) jbytes = (size_t)Mp * Kp;
  else if (jfmt2 == 2) jbytes = (size_t)Mp * Kp / 2;
  else jbytes = (size_t)Mp * Kp * (jfmt2 == 0 ? 2 : es);
  std::vector<unsigned char> jbuf(jbytes, 0);
  if (jbytes) parallel_rows(n, [&](int lo, int hi) {
  CouplingCodes codes;
  for (int i = lo; i < hi; ++i) {
    for (int j = 0; j < n; ++j) {
      double v = Jf[(size_t)i * n + j];
      if (c->prec == NMFA_FP8J_BF16S || fp8s) v = codes.fp8_value(v);
      const size_t idx = (size_t)i * Kp + j;
      if (j8_small || jfmt2 == 1) {
        jbuf[idx] = codes.fp8(v);
      } else if (jfmt2 == 2) {
        const uint8_t code = (uint8_t)codes.fp4(v);
        jbuf[idx / 2] |= (uint8_t)((idx & 1) ? (code << 4) : code);
      } else if (c->prec == NMFA_FP64) {
        std::memcpy(&jbuf[idx * 8], &v, 8);
      } else if (c->prec == NMFA_FP32) {
        const float f = (float)v;
        std::memcpy(&jbuf[idx * 4], &f, 4);
      } else {
        const uint16_t bits = codes.bf16(v);
        std::memcpy(&jbuf[idx * 2], &bits, 2);
      }
    }
  }
  });

  auto cleanup_fail = [&](int code) {
    nmfa_destroy(c);
    return code;
  };
#define CREATE_TRY(expr)                                                                            \
  do {                                                                                              \
    hipError_t _e = (expr);                                                                         \
    if (_e != hipSuccess)                                                                           \
      return cleanup_fail(fail(_e == hipErrorOutOfMemory ? NMFA_ENOMEM : NMFA_EDEVICE, "%s failed: %s", \
                               #expr, hipGetErrorString(_e)));                                      \
  } while (0)

  if (jbytes) {
    CREATE_TRY(hipMalloc(&c->d_J, jbytes));
    CREATE_TRY(hipMemcpy(c->d_J, jbuf.data(), jbytes, hipMemcpyHostToDevice));
  }
  if (c->path == 3) {
    // ELL rows: the nonzeros of row i in ascending column order, padded with (i, 0); values
    // rounded as the precision prescribes (FP8 / BF16 / FP32), held in FP32 (FP64 for FP64)
    const int D = c->ell_D;
    std::vector<int> col((size_t)n * D);
    std::vector<double> vd((size_t)n * D, 0.0);
    parallel_rows(n, [&](int lo, int hi) {
    CouplingCodes codes;
    for (int i = lo; i < hi; ++i) {
      int d = 0;
      for (int j = 0; j < n; ++j) {
        double v = Jf[(size_t)i * n + j];
        if (v == 0.0) continue;
        if (c->prec == NMFA_FP8J_BF16S) v = codes.fp8_value(v);
        else if (c->prec == NMFA_BF16) {
          const uint32_t b = (uint32_t)codes.bf16(v) << 16;
          float f;
          std::memcpy(&f, &b, 4);
          v = f;
        } else if (c->prec == NMFA_FP32) v = (float)v;
        col[(size_t)i * D + d] = j;
        vd[(size_t)i * D + d] = v;
        ++d;
      }
      for (; d < D; ++d) col[(size_t)i * D + d] = i;
    }
    });
    CREATE_TRY(hipMalloc(&c->d_ell_col, col.size() * sizeof(int)));
    CREATE_TRY(hipMemcpy(c->d_ell_col, col.data(), col.size() * sizeof(int), hipMemcpyHostToDevice));
    if (c->prec == NMFA_FP64) {
      CREATE_TRY(hipMalloc(&c->d_ell_val, vd.size() * 8));
      CREATE_TRY(hipMemcpy(c->d_ell_val, vd.data(), vd.size() * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> vf(vd.begin(), vd.end());
      CREATE_TRY(hipMalloc(&c->d_ell_val, vf.size() * 4));
      CREATE_TRY(hipMemcpy(c->d_ell_val, vf.data(), vf.size() * 4, hipMemcpyHostToDevice));
    }
  }
  const size_t as = c->acc_size();
  CREATE_TRY(hipMalloc(&c->d_inv, Mp * as));
  CREATE_TRY(hipMalloc(&c->d_hterm, Mp * as));
  if (c->prec == NMFA_FP64) {
    CREATE_TRY(hipMemcpy(c->d_inv, inv.data(), Mp * 8, hipMemcpyHostToDevice));
    CREATE_TRY(hipMemcpy(c->d_hterm, hterm.data(), Mp * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> fi(Mp), fh(Mp);
    for (int i = 0; i < Mp; ++i) {
      fi[i] = (float)inv[i];
      fh[i] = (float)hterm[i];
    }
    CREATE_TRY(hipMemcpy(c->d_inv, fi.data(), Mp * 4, hipMemcpyHostToDevice));
    CREATE_TRY(hipMemcpy(c->d_hterm, fh.data(), Mp * 4, hipMemcpyHostToDevice));
  }
  if (use_J8) {
    c->Np8 = (int)round_up(n, 64);
    const size_t np = (size_t)c->Np8 * c->Np8;
    std::vector<int8_t> j8(np, 0);
    const int np8 = c->Np8;
    parallel_rows(n, [&](int lo, int hi) {
      for (int i = lo; i < hi; ++i)
        for (int j = 0; j < n; ++j) j8[(size_t)i * np8 + j] = (int8_t)Jf[(size_t)i * n + j];
    });
    CREATE_TRY(hipMalloc(&c->d_J8, np));
    CREATE_TRY(hipMemcpy(c->d_J8, j8.data(), np, hipMemcpyHostToDevice));
  } else {
    CREATE_TRY(hipMalloc(&c->d_J64, nn * 8));
    CREATE_TRY(hipMemcpy(c->d_J64, Jf, nn * 8, hipMemcpyHostToDevice));
  }
  if (any_h) {
    CREATE_TRY(hipMalloc(&c->d_h, n * 8));
    CREATE_TRY(hipMemcpy(c->d_h, c->h.data(), n * 8, hipMemcpyHostToDevice));
  }
  CREATE_TRY(hipEventCreate(&c->ev0));
  CREATE_TRY(hipEventCreate(&c->ev1));
  CREATE_TRY(hipEventCreate(&c->evm));
  if (c->path == 2) {
    CREATE_TRY(hipMalloc(&c->d_ctl, (size_t)xcd_ctl_words() * 4));
    CREATE_TRY(hipMemset(c->d_ctl, 0, (size_t)xcd_ctl_words() * 4));
  }
#undef CREATE_TRY
  *out = c;
  return NMFA_OK;
}

// Make sure the per-run buffers hold R replicas (contents are kept only if R is unchanged).
static int ensure_run_buffers(nmfa_ctx* c, int R) {
  const int Rp = (int)round_up(R, 128);
  if (R > c->cap_R) {
    free_run_buffers(c);
    const size_t cnt = (size_t)R * c->n;
    HIP_TRY(hipMalloc(&c->d_state, cnt * c->acc_size()));
    HIP_TRY(hipMalloc(&c->d_spins, cnt));
    HIP_TRY(hipMalloc(&c->d_E, (size_t)R * 8));
    HIP_TRY(hipMalloc(&c->d_Eint, (size_t)R * 8));
    if (c->d_J8) {
      HIP_TRY(hipMalloc(&c->d_Sp, round_up(R, 64) * (size_t)c->Np8));
      HIP_TRY(hipMalloc(&c->d_E2, (size_t)R * 8));
    }
    c->cap_R = R;
    c->state_valid = false;
  }
  if ((c->path == 1 || c->path == 2) && Rp > c->cap_Rp) {
    (void)hipFree(c->d_S[0]);
    (void)hipFree(c->d_S[1]);
    c->d_S[0] = c->d_S[1] = nullptr;
    const size_t sb = (size_t)Rp * c->Ks * c->op_size();
    HIP_TRY(hipMalloc(&c->d_S[0], sb));
    HIP_TRY(hipMalloc(&c->d_S[1], sb));
    // columns beyond the padded rows are read (times zero couplings) but never written
    HIP_TRY(hipMemset(c->d_S[0], 0, sb));
    HIP_TRY(hipMemset(c->d_S[1], 0, sb));
    c->cap_Rp = Rp;
  }
  return NMFA_OK;
}

// Temperature of iteration t of a t_f-iteration run: the caller's own value when the context
// holds explicit temperatures, else the knot schedule.
static double ctx_T(const nmfa_ctx* c, int t, int t_f) {
  return c->T_explicit.empty() ? schedule_T(c->ku, c->kT, t, t_f) : c->T_explicit[t - 1];
}

static int ensure_coef(nmfa_ctx* c, int t_f) {
  if (c->coef_tf == t_f && c->d_coef) return NMFA_OK;
  (void)hipFree(c->d_coef);
  c->d_coef = nullptr;
  c->coef_tf = 0;
  const double two_log2e = 2.0 / std::log(2.0);
  if (c->prec == NMFA_FP64) {
    std::vector<double> v(t_f);
    for (int t = 1; t <= t_f; ++t) v[t - 1] = 1.0 / ctx_T(c, t, t_f);
    HIP_TRY(hipMalloc(&c->d_coef, (size_t)t_f * 8));
    HIP_TRY(hipMemcpy(c->d_coef, v.data(), (size_t)t_f * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> v(t_f);
    for (int t = 1; t <= t_f; ++t) v[t - 1] = (float)(two_log2e / ctx_T(c, t, t_f));
    HIP_TRY(hipMalloc(&c->d_coef, (size_t)t_f * 4));
    HIP_TRY(hipMemcpy(c->d_coef, v.data(), (size_t)t_f * 4, hipMemcpyHostToDevice));
  }
  c->coef_tf = t_f;
  return NMFA_OK;
}

// Validation, buffers and kernel arguments of one anneal call (shared with the serving scheduler).
int ctx_prepare_run(nmfa_ctx* c, int32_t R, int32_t t_f, int32_t t_begin, int32_t t_end, uint64_t seed,
                    hipStream_t st, nmfa::AnnealArgs* out) {
  if (!c) return fail(NMFA_EINVAL, "nmfa_anneal: context is NULL");
  if (R < 1 || R > (1 << 24)) return fail(NMFA_EINVAL, "nmfa_anneal: R = %d outside [1, 2^24]", R);
  if (t_f < 1) return fail(NMFA_EINVAL, "nmfa_anneal: t_f = %d < 1", t_f);
  if (t_begin < 1 || t_end < t_begin || t_end > t_f)
    return fail(NMFA_EINVAL, "nmfa_anneal: need 1 <= t_begin (%d) <= t_end (%d) <= t_f (%d)", t_begin, t_end, t_f);
  if (!c->T_explicit.empty() && (size_t)t_f != c->T_explicit.size())
    return fail(NMFA_EINVAL, "nmfa_anneal: t_f = %d but the context holds %zu explicit temperatures", t_f,
                c->T_explicit.size());
  if (t_begin > 1 && !(c->state_valid && c->R == R))
    return fail(NMFA_ESTATE, "nmfa_anneal: t_begin > 1 needs the state of a previous call with R = %d", R);
  HIP_TRY(hipSetDevice(c->device));
  int rc;
  if (c->R != R && c->cap_R >= R && t_begin == 1) c->state_valid = false;
  if ((rc = ensure_run_buffers(c, R)) != NMFA_OK) return rc;
  if ((rc = ensure_coef(c, t_f)) != NMFA_OK) return rc;
  const int iters = t_end - t_begin + 1;
  const int rec = std::min(c->record, iters);
  if (rec > 0) {
    const size_t need = (size_t)rec * R * c->n * c->acc_size();
    if (need > c->traj_cap) {
      (void)hipFree(c->d_traj);
      c->d_traj = nullptr;
      c->traj_cap = 0;
      HIP_TRY(hipMalloc(&c->d_traj, need));
      c->traj_cap = need;
    }
  }
  c->R = R;
  c->t_f = t_f;
  c->seed = seed;
  c->stream = st;
  c->result_valid = false;

  AnnealArgs a{};
  a.J = c->d_J;
  a.inv_norm = c->d_inv;
  a.hterm = c->d_hterm;
  a.coef = c->d_coef;
  a.state = c->d_state;
  a.spins = c->d_spins;
  a.traj = rec > 0 ? c->d_traj : nullptr;
  a.record = rec;
  a.N = c->n;
  a.Mp = c->Mp;
  a.Kp = c->Kp;
  a.R = R;
  a.Rp = (int)round_up(R, 64);
  a.lds_stride = c->lds_stride;
  a.t_begin = t_begin;
  a.t_end = t_end;
  a.load_state = (t_begin > 1) ? 1 : 0;
  a.key0 = (uint32_t)(seed & 0xffffffffu);
  a.key1 = (uint32_t)(seed >> 32);
  a.alpha = c->alpha;
  a.sigma = c->sigma;
  a.negate_noise = (c->flags & NMFA_FLAG_NEGATE_NOISE) ? 1 : 0;
  c->traj_iters = rec;
  *out = a;
  return NMFA_OK;
}

// Energies of the readout and the completion bookkeeping of one anneal call.
int ctx_finish_run(nmfa_ctx* c, hipStream_t st) {
  if (c->d_J8)
    HIP_TRY(launch_energy_i8(c->d_J8, c->Np8, c->d_h, c->h_integral ? 1 : 0, c->d_spins, c->n, c->R, c->d_Sp,
                             c->d_E2, c->d_Eint, c->d_E, st));
  else
    HIP_TRY(launch_energy(nullptr, c->d_J64, c->d_h, c->exact_int ? 1 : 0, c->d_spins, c->n, c->R, c->d_Eint, c->d_E,
                          st));
  HIP_TRY(hipEventRecord(c->ev1, st));
  c->timed = true;
  c->state_valid = true;
  c->result_valid = true;
  return NMFA_OK;
}

extern "C" int nmfa_anneal_range(nmfa_ctx* c, int32_t R, int32_t t_f, int32_t t_begin, int32_t t_end,
                                 uint64_t seed, void* hip_stream) {
  return ctx_launch_run(c, R, t_f, t_begin, t_end, seed, (hipStream_t)hip_stream, true);
}

bool ctx_group_shape(const nmfa_ctx* c, int32_t R, int* P, int* G) {
  if (c->path != 2) return false;
  const int Rg = c->xvar ? xrj_group_replicas(c->xvar == 2) : xcd_group_replicas();
  *G = (R + Rg - 1) / Rg;
  *P = c->Mp / (c->xvar ? xrj_rows(c->xvar == 2) : xcd_rows());
  return true;
}

int ctx_launch_run(nmfa_ctx* c, int32_t R, int32_t t_f, int32_t t_begin, int32_t t_end, uint64_t seed,
                   hipStream_t st, bool finish, int max_workgroups) {
  AnnealArgs a{};
  int rc = ctx_prepare_run(c, R, t_f, t_begin, t_end, seed, st, &a);
  if (rc != NMFA_OK) return rc;

  HIP_TRY(hipEventRecord(c->ev0, st));
  if (c->path == 0) {
    HIP_TRY(launch_anneal_small(c->prec, a, st));
    c->launches = 1;
    HIP_TRY(hipEventRecord(c->evm, st));
  } else if (c->path == 3) {
    HIP_TRY(launch_anneal_sparse(c->prec == NMFA_FP64 ? 0 : 1, a, c->d_ell_col, c->d_ell_val, c->ell_D, c->sp_RB,
                                 (c->flags & NMFA_FLAG_SPARSE_GENERIC) ? 0 : 1, &c->sp_rq, st));
    c->launches = 1;
    HIP_TRY(hipEventRecord(c->evm, st));
  } else if (c->path == 2) {
    const int Rg = c->xvar ? xrj_group_replicas(c->xvar == 2) : xcd_group_replicas();
    const int G = (R + Rg - 1) / Rg;
    const int P = c->Mp / (c->xvar ? xrj_rows(c->xvar == 2) : xcd_rows());
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    int width = std::min(cus, 256);  // the control block serves 256 workgroups
    if (max_workgroups > 0) width = std::min(width, max_workgroups);
    const int per_launch = std::max(1, width / P);
    HIP_TRY(launch_pack_state(c->prec, c->d_state, c->d_S[t_begin & 1], c->n, R, c->Kp, c->Ks, G * Rg,
                              t_begin == 1 ? 1 : 0, st));
    // A new run clears the whole control block; a continued one (and every launch after the
    // first) only the registration and barrier counters, so that an abort in an earlier chunk of
    // the run stays raised, ends the later ones at once, and is reported when the run is read.
    const size_t ctl_words = (size_t)xcd_ctl_words();
    uint32_t* ctl = reinterpret_cast<uint32_t*>(c->d_ctl);
    if (t_begin == 1) HIP_TRY(launch_zero_words(ctl, 0, ctl_words, 0, 0, st));
    HIP_TRY(hipEventRecord(c->ev0, st));
    c->launches = 0;
    for (int gb = 0; gb < G; gb += per_launch) {
      const int ng = std::min(per_launch, G - gb);
      if (gb > 0 || t_begin > 1) {  // fresh registration and barrier counters; abort and mode persist
        HIP_TRY(launch_zero_words(ctl, 0, 17, 64, ctl_words, st));
      }
      XcdArgs x{};
      x.S[0] = c->d_S[0];
      x.S[1] = c->d_S[1];
      x.ks = c->Ks;
      x.ctl = c->d_ctl;
      x.P = P;
      x.group_base = gb;
      x.force_fenced = (c->flags & NMFA_FLAG_FORCE_FENCED) ? 1 : 0;
      x.nbuf = c->nbuf;
      if (c->xvar == 2) HIP_TRY(launch_anneal_xrj8(a, x, ng, st));
      else if (c->xvar) HIP_TRY(launch_anneal_xrj(a, x, ng, st));
      else HIP_TRY(launch_anneal_xcd(c->jfmt, a, x, ng, st));
      ++c->launches;
    }
    HIP_TRY(hipEventRecord(c->evm, st));
    c->ctl_pending = true;
  } else {
    if (t_begin == 1)
      HIP_TRY(launch_zero_words(reinterpret_cast<uint32_t*>(c->d_state), 0, (size_t)R * c->n * c->acc_size() / 4, 0, 0,
                                st));
    HIP_TRY(launch_pack_state(c->prec, c->d_state, c->d_S[0], c->n, R, c->Kp, c->Kp, a.Rp, t_begin == 1 ? 1 : 0, st));
    HIP_TRY(hipEventRecord(c->ev0, st));
    int cur = 0;
    for (int t = t_begin; t <= t_end; ++t) {
      HIP_TRY(launch_anneal_step(c->prec, c->path == 1 ? c->jfmt : 0, a, c->d_S[cur], c->d_S[cur ^ 1], t, st));
      cur ^= 1;
    }
    c->launches = t_end - t_begin + 1;
    HIP_TRY(hipEventRecord(c->evm, st));
    HIP_TRY(launch_readout(c->prec, c->d_state, c->d_spins, (size_t)R * c->n, st));
  }
  if (!finish) {
    c->state_valid = true;
    return NMFA_OK;
  }
  return ctx_finish_run(c, st);
}

extern "C" int nmfa_anneal(nmfa_ctx* c, int32_t R, int32_t t_f, uint64_t seed, void* hip_stream) {
  return nmfa_anneal_range(c, R, t_f, 1, t_f, seed, hip_stream);
}

static int check_ctl(nmfa_ctx* c);

static int sync_ctx(nmfa_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  if (c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
  else HIP_TRY(hipDeviceSynchronize());
  return check_ctl(c);
}

// After the work of a run has completed: the XCD-group kernels' abort and exchange-mode words.
// They are read on every access to results or state, not only after an anneal enqueued through
// this library, so that a run replayed from a recorded HIP graph is checked as well.
static int check_ctl(nmfa_ctx* c) {
  if (c->path != 2 || !c->d_ctl) return NMFA_OK;
  unsigned flags[3] = {0, 0, 0};
  HIP_TRY(hipMemcpy(flags, c->d_ctl + 16, sizeof(flags), hipMemcpyDeviceToHost));
  c->ctl_pending = false;
  if (flags[2]) c->exchange_mode = (int)flags[2];
  if (flags[1]) {
    c->result_valid = false;
    c->state_valid = false;
    return fail(NMFA_EDEVICE, "XCD-group kernel: a group barrier or the start-up registration timed out");
  }
  return NMFA_OK;
}

extern "C" int nmfa_debug_raise_abort(nmfa_ctx* c) {
  if (!c || c->path != 2 || !c->d_ctl) return fail(NMFA_EINVAL, "nmfa_debug_raise_abort: not a group-kernel context");
  HIP_TRY(hipSetDevice(c->device));
  const unsigned one = 1u;
  HIP_TRY(hipMemcpy(c->d_ctl + 17, &one, sizeof(one), hipMemcpyHostToDevice));
  return NMFA_OK;
}

int ctx_read_results(nmfa_ctx* c, double* E, int64_t* E_int, int8_t* spins) {
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipEventSynchronize(c->ev1));
  int rc = check_ctl(c);
  if (rc) return rc;
  HIP_TRY(hipMemcpy(E, c->d_E, (size_t)c->R * 8, hipMemcpyDeviceToHost));
  if (c->exact_int)
    HIP_TRY(hipMemcpy(E_int, c->d_Eint, (size_t)c->R * 8, hipMemcpyDeviceToHost));
  else
    std::memset(E_int, 0, (size_t)c->R * 8);
  HIP_TRY(hipMemcpy(spins, c->d_spins, (size_t)c->R * c->n, hipMemcpyDeviceToHost));
  return NMFA_OK;
}

extern "C" int nmfa_spins(nmfa_ctx* c, int8_t* out, int32_t on_device) {
  if (!c || !out) return fail(NMFA_EINVAL, "nmfa_spins: NULL argument");
  if (!c->result_valid) return fail(NMFA_ESTATE, "nmfa_spins: no anneal has run");
  int rc = sync_ctx(c);
  if (rc) return rc;
  HIP_TRY(hipMemcpy(out, c->d_spins, (size_t)c->R * c->n,
                    on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return NMFA_OK;
}

extern "C" int nmfa_energies(nmfa_ctx* c, double* E, int64_t* E_int) {
  if (!c || !E) return fail(NMFA_EINVAL, "nmfa_energies: NULL argument");
  if (!c->result_valid) return fail(NMFA_ESTATE, "nmfa_energies: no anneal has run");
  int rc = sync_ctx(c);
  if (rc) return rc;
  HIP_TRY(hipMemcpy(E, c->d_E, (size_t)c->R * 8, hipMemcpyDeviceToHost));
  if (E_int) {
    if (c->exact_int) {
      HIP_TRY(hipMemcpy(E_int, c->d_Eint, (size_t)c->R * 8, hipMemcpyDeviceToHost));
    } else {
      std::memset(E_int, 0, (size_t)c->R * 8);
    }
  }
  return NMFA_OK;
}

extern "C" int nmfa_cuts(nmfa_ctx* c, double* cut) {
  if (!c || !cut) return fail(NMFA_EINVAL, "nmfa_cuts: NULL argument");
  std::vector<double> E(c->R > 0 ? c->R : 1);
  int rc = nmfa_energies(c, E.data(), nullptr);
  if (rc) return rc;
  for (int r = 0; r < c->R; ++r) cut[r] = (c->w_total - E[r]) / 2.0;
  return NMFA_OK;
}

extern "C" int nmfa_energies_of(nmfa_ctx* c, int32_t R, const int8_t* spins, double* E, int64_t* E_int) {
  if (!c || !spins || !E || R < 1) return fail(NMFA_EINVAL, "nmfa_energies_of: invalid argument");
  for (size_t k = 0; k < (size_t)R * c->n; ++k)
    if (spins[k] != 1 && spins[k] != -1) return fail(NMFA_EINVAL, "nmfa_energies_of: spins must be +1/-1");
  HIP_TRY(hipSetDevice(c->device));
  int8_t* d_s = nullptr;
  double* d_E = nullptr;
  long long* d_Ei = nullptr;
  int8_t* d_Sp = nullptr;
  unsigned long long* d_E2 = nullptr;
  const size_t cnt = (size_t)R * c->n;
  hipError_t e = hipMalloc(&d_s, cnt);
  if (e == hipSuccess) e = hipMalloc(&d_E, (size_t)R * 8);
  if (e == hipSuccess) e = hipMalloc(&d_Ei, (size_t)R * 8);
  if (e == hipSuccess && c->d_J8) e = hipMalloc(&d_Sp, round_up(R, 64) * (size_t)c->Np8);
  if (e == hipSuccess && c->d_J8) e = hipMalloc(&d_E2, (size_t)R * 8);
  if (e == hipSuccess) e = hipMemcpy(d_s, spins, cnt, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    if (c->d_J8)
      e = launch_energy_i8(c->d_J8, c->Np8, c->d_h, c->h_integral ? 1 : 0, d_s, c->n, R, d_Sp, d_E2, d_Ei, d_E, 0);
    else
      e = launch_energy(nullptr, c->d_J64, c->d_h, c->exact_int ? 1 : 0, d_s, c->n, R, d_Ei, d_E, 0);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(E, d_E, (size_t)R * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess && E_int) {
    if (c->exact_int) e = hipMemcpy(E_int, d_Ei, (size_t)R * 8, hipMemcpyDeviceToHost);
    else std::memset(E_int, 0, (size_t)R * 8);
  }
  (void)hipFree(d_s);
  (void)hipFree(d_E);
  (void)hipFree(d_Ei);
  (void)hipFree(d_Sp);
  (void)hipFree(d_E2);
  if (e != hipSuccess) return fail(NMFA_EDEVICE, "nmfa_energies_of: %s", hipGetErrorString(e));
  return NMFA_OK;
}

extern "C" int nmfa_get_state(nmfa_ctx* c, double* out) {
  if (!c || !out) return fail(NMFA_EINVAL, "nmfa_get_state: NULL argument");
  if (!c->state_valid) return fail(NMFA_ESTATE, "nmfa_get_state: no state");
  int rc = sync_ctx(c);
  if (rc) return rc;
  const size_t cnt = (size_t)c->R * c->n;
  if (c->prec == NMFA_FP64) {
    HIP_TRY(hipMemcpy(out, c->d_state, cnt * 8, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(cnt);
    HIP_TRY(hipMemcpy(f.data(), c->d_state, cnt * 4, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < cnt; ++k) out[k] = f[k];
  }
  return NMFA_OK;
}

extern "C" int nmfa_set_state(nmfa_ctx* c, int32_t R, const double* in) {
  if (!c || !in || R < 1) return fail(NMFA_EINVAL, "nmfa_set_state: invalid argument");
  const size_t cnt = (size_t)R * c->n;
  for (size_t k = 0; k < cnt; ++k)
    if (!(std::fabs(in[k]) <= 1.0)) return fail(NMFA_EINVAL, "nmfa_set_state: state values must lie in [-1, 1]");
  HIP_TRY(hipSetDevice(c->device));
  if (c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
  else HIP_TRY(hipDeviceSynchronize());
  // a new state replaces whatever an aborted group-kernel run left: clear its abort word
  if (c->path == 2 && c->d_ctl) HIP_TRY(hipMemset(c->d_ctl + 17, 0, sizeof(unsigned)));
  int rc;
  if ((rc = ensure_run_buffers(c, R)) != NMFA_OK) return rc;
  if (c->prec == NMFA_FP64) {
    HIP_TRY(hipMemcpy(c->d_state, in, cnt * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(cnt);
    for (size_t k = 0; k < cnt; ++k) f[k] = (float)in[k];
    HIP_TRY(hipMemcpy(c->d_state, f.data(), cnt * 4, hipMemcpyHostToDevice));
  }
  c->R = R;
  c->state_valid = true;
  c->result_valid = false;
  return NMFA_OK;
}

extern "C" int nmfa_trajectory(nmfa_ctx* c, double* out) {
  if (!c || !out) return fail(NMFA_EINVAL, "nmfa_trajectory: NULL argument");
  if (!c->result_valid || c->traj_iters <= 0) return fail(NMFA_ESTATE, "nmfa_trajectory: nothing recorded");
  int rc = sync_ctx(c);
  if (rc) return rc;
  const size_t cnt = (size_t)c->traj_iters * c->R * c->n;
  if (c->prec == NMFA_FP64) {
    HIP_TRY(hipMemcpy(out, c->d_traj, cnt * 8, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(cnt);
    HIP_TRY(hipMemcpy(f.data(), c->d_traj, cnt * 4, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < cnt; ++k) out[k] = f[k];
  }
  return NMFA_OK;
}

extern "C" int nmfa_info(nmfa_ctx* c, int32_t* n, int32_t* precision, int32_t* path) {
  if (!c) return fail(NMFA_EINVAL, "nmfa_info: context is NULL");
  if (n) *n = c->n;
  if (precision) *precision = c->prec;
  if (path) {
    if (c->path == 2) {
      if (c->ctl_pending) {
        int rc = sync_ctx(c);
        if (rc) return rc;
      }
      *path = ((c->exchange_mode == 2) ? 3 : 2) + (c->xvar ? 2 : 0);
    } else {
      *path = (c->path == 3) ? 6 + c->sp_rq : c->path;
    }
  }
  return NMFA_OK;
}

extern "C" int nmfa_j_format(nmfa_ctx* c, int32_t* fmt) {
  if (!c || !fmt) return fail(NMFA_EINVAL, "nmfa_j_format: NULL argument");
  if (c->path == 2) *fmt = c->jfmt;
  else if (c->path == 1 && c->prec != NMFA_FP64 && c->prec != NMFA_FP32) *fmt = c->jfmt;
  else if (c->path == 3) *fmt = NMFA_JFMT_ELL;
  else if (c->prec == NMFA_FP64 || c->prec == NMFA_FP32) *fmt = NMFA_JFMT_NATIVE;
  else if (c->prec == NMFA_FP8J_BF16S && c->path == 0) *fmt = NMFA_JFMT_FP8;
  else *fmt = NMFA_JFMT_BF16;
  return NMFA_OK;
}

extern "C" int nmfa_last_timing(nmfa_ctx* c, double* anneal_ms, double* total_ms, int32_t* launches) {
  if (!c) return fail(NMFA_EINVAL, "nmfa_last_timing: context is NULL");
  if (!c->timed) return fail(NMFA_ESTATE, "nmfa_last_timing: no anneal has run");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipEventSynchronize(c->ev1));
  float fa = 0.f, ft = 0.f;
  HIP_TRY(hipEventElapsedTime(&fa, c->ev0, c->evm));
  HIP_TRY(hipEventElapsedTime(&ft, c->ev0, c->ev1));
  if (anneal_ms) *anneal_ms = fa;
  if (total_ms) *total_ms = ft;
  if (launches) *launches = c->launches;
  return NMFA_OK;
}

// ------------------------------------------------------------------------------------------
// Noise utilities
// ------------------------------------------------------------------------------------------
extern "C" int nmfa_noise_words(uint64_t seed, int32_t t, int32_t r0, int32_t n_rep, int32_t n_quads, uint32_t* out) {
  if (!out || t < 0 || r0 < 0 || n_rep < 1 || n_quads < 1 || (int64_t)n_rep * n_quads > (1 << 26))
    return fail(NMFA_EINVAL, "nmfa_noise_words: invalid argument");
  const size_t cnt = (size_t)n_rep * n_quads * 4;
  uint32_t* d = nullptr;
  HIP_TRY(hipMalloc(&d, cnt * 4));
  hipError_t e = launch_noise_words((uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)t, (uint32_t)r0, n_rep, n_quads, d, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(out, d, cnt * 4, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(NMFA_EDEVICE, "nmfa_noise_words: %s", hipGetErrorString(e));
  return NMFA_OK;
}

extern "C" int nmfa_noise_values(uint64_t seed, int32_t t, int32_t r0, int32_t n_rep, int32_t n_quads, int32_t fp64,
                                 double* out) {
  if (!out || t < 0 || r0 < 0 || n_rep < 1 || n_quads < 1 || (int64_t)n_rep * n_quads > (1 << 26))
    return fail(NMFA_EINVAL, "nmfa_noise_values: invalid argument");
  const size_t cnt = (size_t)n_rep * n_quads * 4;
  double* d = nullptr;
  HIP_TRY(hipMalloc(&d, cnt * 8));
  hipError_t e = launch_noise_values((uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)t, (uint32_t)r0, n_rep, n_quads,
                                     fp64 ? 1 : 0, d, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(out, d, cnt * 8, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(NMFA_EDEVICE, "nmfa_noise_values: %s", hipGetErrorString(e));
  return NMFA_OK;
}
