// Persistent adaptive Runge--Kutta--Cash--Karp 5(4) integrator: one system per
// lane, state in VGPRs, each lane on its own clock and step size (the
// asynchronous per-system time stepping of Sec. 4.2 and Sec. 4.3 of
// arXiv:2011.01740), with a device work queue that refills a lane as soon as
// its system is finished.
//
// Work distribution.  The grid is the resident capacity of the chip.  A wave
// keeps stepping its active lanes; when at least `refill` of its lanes are
// idle (or all are), the lowest idle lane claims that many consecutive system
// indices with one atomic add on the queue head, and the idle lanes take
// base + (number of idle lanes below them).  A wave whose claim reaches n
// stops refilling and retires when its last lane finishes.  Systems are
// handed out in index order, so neighbouring lanes integrate neighbouring
// parameters (the paper's advice against divergence, Sec. 3.2.1) and
// sub-ensembles are started in the order they are given.
//
// Per step, per lane: six stages, the embedded error estimate, the max-norm
// error ratio, accept/reject, step-size update, phase bookkeeping, and for
// the relief valve event detection, secant retry and the impact law.  Only
// the bookkeeping branches diverge; the stages are the same instruction
// stream for every lane.  Sub-ensemble descriptors (shared parameters and
// budgets) sit in LDS.
#include <cmath>

#include "ens_internal.h"

namespace ens {
namespace {

constexpr int kMaxBlock = 256;

// Cash--Karp 5(4) tableau (Cash and Karp, ACM TOMS 16, 1990).
constexpr double A21 = 1.0 / 5.0;
constexpr double A31 = 3.0 / 40.0, A32 = 9.0 / 40.0;
constexpr double A41 = 3.0 / 10.0, A42 = -9.0 / 10.0, A43 = 6.0 / 5.0;
constexpr double A51 = -11.0 / 54.0, A52 = 5.0 / 2.0, A53 = -70.0 / 27.0, A54 = 35.0 / 27.0;
constexpr double A61 = 1631.0 / 55296.0, A62 = 175.0 / 512.0, A63 = 575.0 / 13824.0,
                 A64 = 44275.0 / 110592.0, A65 = 253.0 / 4096.0;
constexpr double C2 = 1.0 / 5.0, C3 = 3.0 / 10.0, C4 = 3.0 / 5.0, C5 = 1.0, C6 = 7.0 / 8.0;
constexpr double B1 = 37.0 / 378.0, B3 = 250.0 / 621.0, B4 = 125.0 / 594.0,
                 B6 = 512.0 / 1771.0;
// fifth- minus fourth-order weights
constexpr double E1 = B1 - 2825.0 / 27648.0, E3 = B3 - 18575.0 / 48384.0,
                 E4 = B4 - 13525.0 / 55296.0, E5 = -277.0 / 14336.0, E6 = B6 - 1.0 / 4.0;

// Schemes of the persistent kernel.
constexpr int kCK = 0;  // Cash--Karp 5(4), six stages
constexpr int kDP = 1;  // Dormand--Prince 5(4), seven stages, first same as last

// Dormand--Prince 5(4) tableau (Dormand and Prince, J. Comput. Appl. Math. 6,
// 1980).  Its last row is the fifth-order weights: stage 7 is f at y5.
constexpr double D21 = 1.0 / 5.0;
constexpr double D31 = 3.0 / 40.0, D32 = 9.0 / 40.0;
constexpr double D41 = 44.0 / 45.0, D42 = -56.0 / 15.0, D43 = 32.0 / 9.0;
constexpr double D51 = 19372.0 / 6561.0, D52 = -25360.0 / 2187.0, D53 = 64448.0 / 6561.0,
                 D54 = -212.0 / 729.0;
constexpr double D61 = 9017.0 / 3168.0, D62 = -355.0 / 33.0, D63 = 46732.0 / 5247.0,
                 D64 = 49.0 / 176.0, D65 = -5103.0 / 18656.0;
constexpr double D71 = 35.0 / 384.0, D73 = 500.0 / 1113.0, D74 = 125.0 / 192.0,
                 D75 = -2187.0 / 6784.0, D76 = 11.0 / 84.0;
constexpr double DC2 = 1.0 / 5.0, DC3 = 3.0 / 10.0, DC4 = 4.0 / 5.0, DC5 = 8.0 / 9.0;
// fifth- minus fourth-order weights (the fourth-order ones: 5179/57600, 0,
// 7571/16695, 393/640, -92097/339200, 187/2100, 1/40)
constexpr double DE1 = D71 - 5179.0 / 57600.0, DE3 = D73 - 7571.0 / 16695.0,
                 DE4 = D74 - 393.0 / 640.0, DE5 = D75 + 92097.0 / 339200.0,
                 DE6 = D76 - 187.0 / 2100.0, DE7 = -1.0 / 40.0;

// Both tableaux again as tables in constant memory.  An attempt reads its
// coefficients through scalar_table(): a handful of wide scalar loads per
// attempt instead of two 32-bit immediates per double, which also leaves the
// scalar registers that the immediates took to the rest of the loop.
struct CkTab {
  double a21, a31, a32, a41, a42, a43, a51, a52, a53, a54, a61, a62, a63, a64, a65;
  double b1, b3, b4, b6, e1, e3, e4, e5, e6;
};
__constant__ CkTab kCkTab = {A21, A31, A32, A41, A42, A43, A51, A52, A53, A54,
                             A61, A62, A63, A64, A65, B1,  B3,  B4,  B6,  E1,
                             E3,  E4,  E5,  E6};
struct DpTab {
  double a21, a31, a32, a41, a42, a43, a51, a52, a53, a54, a61, a62, a63, a64, a65;
  double b1, b3, b4, b5, b6, e1, e3, e4, e5, e6, e7;
};
__constant__ DpTab kDpTab = {D21, D31, D32, D41, D42, D43, D51, D52, D53, D54,
                             D61, D62, D63, D64, D65, D71, D73, D74, D75, D76,
                             DE1, DE3, DE4, DE5, DE6, DE7};

// A table in constant memory as the attempt sees it.  The pointer passes
// through an empty asm in scalar registers, so the compiler cannot hoist the
// loads out of the step loop (which would pin the values in scalar registers
// for the whole loop and spill others); the constant address space lets it
// use scalar loads.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T &scalar_table(const T &t) {
  const T *p = &t;
  asm volatile("" : "+s"(p));
  return *(const __attribute__((address_space(4))) T *)p;
}

// Occupancy floor per (model, scheme, located maxima): the seventh stage and
// the carried k1 of Dormand--Prince, or Cash--Karp's end-point evaluations
// for located maxima, cost one wave per SIMD.
constexpr int min_waves(int base, int sc, bool loc) {
  return (sc == kDP || loc) ? base - 1 : base;
}

// 1/d from the hardware reciprocal estimate r (relative error e = 1 - d r
// below 2^-22) and one third-order correction r (1 + e + e^2), which leaves
// e^3 < 2^-66 before the final rounding: within an ulp of the correctly
// rounded quotient for the normal, finite d used here, in three dependent
// instructions where two Newton steps take four (d = 0 or non-finite gives
// a non-finite result).
__device__ __forceinline__ double rcp_nr(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// sqrt(x) for the valve's chamber pressure: r = v_rsq_f64 (relative error
// ~2^-23), one coupled Newton step on g = x r and h = r/2 (~2^-46), one
// residual correction g + (x - g^2) h: within an ulp of the correctly
// rounded root for normal x, in 8 dependent VALU against 17 for the library
// sqrt, which also rescales tiny and huge arguments (not needed here: the
// pressure stays O(1..10)).  The estimate is taken of x + 1e-300, which is
// x itself for every x above 1e-284 and keeps r finite at x = 0, where
// g = 0 x r = 0 then gives the root 0 without a select; x < 0 gives NaN like
// sqrt.
__device__ __forceinline__ double sqrt_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x + 1e-300);
  double g = x * r, h = 0.5 * r;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  return fma(fma(-g, g, x), h, g);
}

// max / min as one v_max_f64 / v_min_f64.  fmax() and fmin() make the
// compiler first quiet every operand it cannot prove canonical (a loop-
// carried state, a kernel argument) with an extra v_max of the value with
// itself, in case it is a signalling NaN; the operands here are arithmetic
// results or host-checked step bounds, never signalling NaNs (a quiet NaN
// in the error norm is caught by its finite test).  The bound of a clamp is
// a scalar operand (an SGPR pair), as the kernel arguments already are.
__device__ __forceinline__ double vmax_abs(double a, double b) {   // max(|a|, |b|)
  double r;
  asm("v_max_f64 %0, |%1|, |%2|" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double vmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double vmax_s(double a, double b) {     // b uniform
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(b));
  return r;
}
__device__ __forceinline__ double vmin_s(double a, double b) {     // b uniform
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(b));
  return r;
}

// x^(-1/5) for x in [1e-30, 1e30]: an FP32 estimate r0 from the hardware
// base-2 logarithm and exponential (relative error ~1e-7), then in FP64 with
// e = 1 - x r0^5 the series r = r0 (1 - e)^(-1/5) = r0 (1 + e/5 + 3 e^2/25
// + O(e^3)): the truncation is ~1e-20, below rounding.  ~12 VALU instead of
// the ~200 of a general pow.
// (c12 = 3/25 and c2 = 1/5 are the series coefficients; rfifth_c takes them as
// arguments so that a caller can supply them from scalar registers.)
__device__ __forceinline__ double rfifth_c(double x, double c12, double c2) {
  const double r0 =
      (double)__builtin_amdgcn_exp2f(-0.2f * __builtin_amdgcn_logf((float)x));
  const double r2 = r0 * r0;
  const double e = fma(-x, r2 * r2 * r0, 1.0);
  return fma(r0, e * fma(c12, e, c2), r0);
}
__device__ __forceinline__ double rfifth(double x) { return rfifth_c(x, 0.12, 0.2); }

// The step-size controller's constants as a table in constant memory, read
// with one scalar load per attempt (scalar_table).  The valve's step takes
// them from there (its scalar registers are short, and the compiler would
// rebuild each double from two 32-bit immediates in every attempt); the
// Keller--Miksis steps keep them as immediates, which its kernel holds.
struct CtlTab {
  double e_lo, e_hi, safety, f_lo, f_hi, c12, c2;
};
__constant__ CtlTab kCtlTab = {1e-4, 4e3, 0.9, 0.2, 5.0, 0.12, 0.2};
constexpr CtlTab kCtlImm = {1e-4, 4e3, 0.9, 0.2, 5.0, 0.12, 0.2};

// Step-size factor 0.9 E^(-1/5), clamped to [0.2, 5] (E = 0 gives 5), for a
// finite E >= 0.  The root is taken of E limited to [1e-4, 4e3], where FP32
// holds it: below, 0.9 (1e-4)^(-1/5) = 5.68 clamps to 5, and above,
// 0.9 (4e3)^(-1/5) = 0.171 clamps to 0.2, the factors of the unlimited E.
template <class T>
__device__ __forceinline__ double step_factor_with(const T &c, double E) {
  const double f = c.safety * rfifth_c(vmin_s(vmax_s(E, c.e_lo), c.e_hi), c.c12, c.c2);
  return vmin_s(vmax_s(f, c.f_lo), c.f_hi);
}
template <bool TABLE>
__device__ __forceinline__ double step_factor(double E) {
  if constexpr (TABLE)
    return step_factor_with(scalar_table(kCtlTab), E);
  else
    return step_factor_with(kCtlImm, E);
}

// Scaled error of an attempt, E = max_c |err_c| / (rtol max(|y_c|, |y5_c|) +
// atol), and whether every new component and ratio is finite: 0 v is 0 for a
// finite v and NaN otherwise, so one compare of the sum of those products
// decides.
template <int D>
__device__ __forceinline__ bool error_ratio(double rtol, double atol, const double *y,
                                            const double *y5, const double *err, double &E) {
  double z = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double sc = fma(rtol, vmax_abs(y[c], y5[c]), atol);
    const double r = fabs(err[c]) * rcp_nr(sc);
    z = fma(0.0, y5[c], z);
    z = fma(0.0, r, z);
    E = c == 0 ? r : vmax(E, r);
  }
  return z == 0.0;
}

// ------------------------------------------------------------------ models
// Each model: D, lane constants set at refill, rhs(t, y, f).

struct MQuad {  // dx/dt = x^2 - p (Sec. 3)
  static constexpr int D = 1;
  static constexpr bool kEvents = false;
  static constexpr int kMinWaves = 5;
  static constexpr bool kPrio = false;  // issue priority by remaining work
  static constexpr bool kLocate = false;
  static constexpr bool kDrive2 = false;
  static constexpr int kF = 1;           // record fields
  static constexpr bool kTangent = false;
  static constexpr int kNCoef = 0;  // no precomputed coefficients
  double p;
  __device__ void init(const double *P, int64_t n, int64_t i, const double *sh) { p = P[i]; }
  __device__ void begin(double) {}
  template <int SC, int S>
  __device__ void rhs(double, double, const double *y, double *f) const {
    f[0] = fma(y[0], y[0], -p);
  }
  // with K tangents of the variational equation: df_v = J dy_v, J = 2x
  template <int SC, int S, int K>
  __device__ void rhs_tan(double t, double h, const double *y, const double *dy, double *f,
                          double *df) const {
    rhs<SC, S>(t, h, y, f);
    const double j = 2.0 * y[0];
#pragma unroll
    for (int v = 0; v < K; ++v) df[v] = j * dy[v];
  }
};

struct MLorenz {  // Sec. 4.1
  static constexpr int D = 3;
  static constexpr bool kEvents = false;
  static constexpr int kMinWaves = 5;
  static constexpr bool kPrio = false;  // issue priority by remaining work
  static constexpr bool kLocate = false;
  static constexpr bool kDrive2 = false;
  static constexpr int kF = 1;
  static constexpr bool kTangent = false;
  static constexpr int kNCoef = 0;  // no precomputed coefficients
  double rho, sigma, beta;
  __device__ void init(const double *P, int64_t n, int64_t i, const double *sh) {
    rho = P[i];
    sigma = sh[0];
    beta = sh[1];
  }
  __device__ void begin(double) {}
  template <int SC, int S>
  __device__ void rhs(double, double, const double *y, double *f) const {
    f[0] = sigma * (y[1] - y[0]);
    f[1] = fma(-y[0], y[2], fma(rho, y[0], -y[1]));
    f[2] = fma(y[0], y[1], -beta * y[2]);
  }
  // J = [[-sigma, sigma, 0], [rho - z, -1, -x], [y, x, -beta]], applied to
  // each of the K tangents
  template <int SC, int S, int K>
  __device__ void rhs_tan(double t, double h, const double *y, const double *dy, double *f,
                          double *df) const {
    rhs<SC, S>(t, h, y, f);
    const double rz = rho - y[2];
#pragma unroll
    for (int v = 0; v < K; ++v) {
      const double *d = dy + 3 * v;
      double *g = df + 3 * v;
      g[0] = sigma * (d[1] - d[0]);
      g[1] = fma(rz, d[0], fma(-y[0], d[2], -d[1]));
      g[2] = fma(y[1], d[0], fma(y[0], d[1], -beta * d[2]));
    }
  }
};

// sin x and cos x from their Taylor series, sin through x^(2 NS - 1) and cos
// through x^(2 NC - 2), Horner in x^2.  The callers size NS, NC for the
// largest |x| they pass so that the first omitted term is below 1e-17 of the
// value (a tenth of its rounding unit).
constexpr double kInvFact[20] = {
    1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040, 1.0 / 40320,
    1.0 / 362880, 1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600, 1.0 / 6227020800.0,
    1.0 / 87178291200.0, 1.0 / 1307674368000.0, 1.0 / 20922789888000.0,
    1.0 / 355687428096000.0, 1.0 / 6402373705728000.0, 1.0 / 121645100408832000.0};

template <int NS, int NC>
__device__ __forceinline__ void sincos_taylor(double x, double *s, double *c) {
  static_assert(NS >= 2 && NC >= 2 && 2 * NS - 1 < 20 && 2 * NC - 2 < 20, "series length");
  const double x2 = x * x;
  // sin x = x (1 - x^2/3! + ...): coefficients of x^(2k+1), k = 0 .. NS-1
  double ps = ((NS - 1) % 2 ? -1.0 : 1.0) * kInvFact[2 * NS - 1];
#pragma unroll
  for (int k = NS - 2; k >= 1; --k) ps = fma(ps, x2, (k % 2 ? -1.0 : 1.0) * kInvFact[2 * k + 1]);
  *s = fma(ps * x2, x, x);
  // cos x = 1 - x^2 (1/2! - x^2/4! + ...): coefficients of x^(2k), k = 1 .. NC-1
  double pc = ((NC - 1) % 2 ? 1.0 : -1.0) * kInvFact[2 * NC - 2];
#pragma unroll
  for (int k = NC - 2; k >= 1; --k) pc = fma(pc, x2, (k % 2 ? 1.0 : -1.0) * kInvFact[2 * k]);
  *c = fma(-pc, x2, 1.0);
}

// sin(pi x) and cos(pi x), |x| < 2^50: x minus the nearest multiple of 1/2
// (exact) leaves |r| <= 1/4; pi r is formed as a rounded product plus its
// error (FMA) and the error of pi's double, the series above gives sin and
// cos of the rounded part, a first-order term adds the rest, and the quarter
// turns swap and negate.  Within an ulp of the correctly rounded values;
// about half the instructions of the general library routine, which
// reduces any argument.
__device__ __forceinline__ void sincospi_quarter(double x, double *s, double *c) {
  constexpr double kPiLo = 1.2246467991473532e-16;  // pi - (double)pi
  const double q = rint(2.0 * x);
  const double r = fma(q, -0.5, x);
  const double t = M_PI * r;
  const double tl = fma(M_PI, r, -t) + kPiLo * r;
  double sr, cr;
  sincos_taylor<9, 10>(t, &sr, &cr);
  const double sr1 = fma(tl, cr, sr), cr1 = fma(-tl, sr, cr);
  sr = sr1;
  cr = cr1;
  const int k = (int)(q - 4.0 * floor(0.25 * q));  // quarter turns modulo 4 (exact)
  const double ss = (k & 1) ? cr : sr;
  const double cc = (k & 1) ? sr : cr;
  *s = (k & 2) ? -ss : ss;            // k = 2, 3
  *c = ((k + 1) & 2) ? -cc : cc;      // k = 1, 2
}

// Dimensionless Keller--Miksis equation (Sec. 4.2), single-frequency drive.
// The lane derives its coefficients from (P_A1, f1) and the shared material
// constants when it picks the system up; only the nine that are non-zero for
// a single-frequency drive are kept.  Terms are grouped so that each
// coefficient multiplies once:
//   N = (K0 + K1 y2) y1^-K10 - (K2 + K5 s)(1 + K9 y2) - (K3 + K4 y2)/y1
//       - (1 - K9 y2 / 3) 1.5 y2^2 - K7 c y1,       s, c = sin, cos(2 pi tau)
//   D = y1 (1 - K9 y2) + K4 K9.
// One division serves both 1/y1 and 1/D: q = 1 / (y1 D), 1/y1 = D q,
// N / D = N y1 q.
// FAST (chosen by the host when 3 gamma = 21/5, the polytropic exponent of
// air, and dt_max <= 1/8): the gas term is (1/y1)^4 y1^(-1/5) with the Newton
// fifth root, and the forcing phase of each stage, 2 pi (t + c_i h), comes
// from sin/cos of 2 pi t (once per attempted step, by quarter-turn reduction
// and a series) by angle addition with the
// small offset 2 pi c_i h <= pi/4.  Otherwise exp(-K10 log y1) and sincospi
// per stage.
// DUAL (chosen when a sub-ensemble has P_A2 != 0): the second drive
// -(K6 sin a2 (1 + K9 y2) + K8 y1 cos a2), a2 = 2 pi (phi + K11 tau) + theta,
// with phi the drive's phase when the integration phase began, carried
// across phases and stored per system (Sec. 4.2: the drive is a function of
// the absolute time, while tau restarts with each phase).  Its stage angles
// 2 pi K11 c_i h need not be small, so each stage reduces its own angle.
// PSYS: (P_A2, f2, theta, R_E) are per-system parameters 2..5 instead of
// shared ones (the six control parameters of Sec. 4.2 swept together).
template <bool FAST, bool DUAL = false, bool PSYS = false>
struct MKM {
  static_assert(DUAL || !PSYS, "per-system second-drive parameters imply the second drive");
  static constexpr int D = 2;
  static constexpr bool kEvents = false;
  // the second drive's sin/cos needs registers beyond the 4-wave budget
  static constexpr int kMinWaves = DUAL ? 3 : 4;
  static constexpr bool kPrio = true;  // issue priority by remaining work
  static constexpr bool kLocate = true;  // y2 = y1': maxima can be located
  static constexpr bool kDrive2 = DUAL;
  static constexpr int kF = 1;
  static constexpr bool kTangent = false;
  double K0, K1, K2, K3, K4, K5, K7, K9, K10, K49, K9h;  // K9h = K9 / 2
  // FAST: K5 and K7 times sin, cos (2 pi t) at the start of the attempted
  // step, so that each stage forms its forcing terms from its angle offset
  // directly: K5 sin(a + b) = K5 s0 cos b + K5 c0 sin b, and the same for cos
  double k5s, k5c, k7s, k7c;
  __device__ void init(const double *P, int64_t n, int64_t i, const double *sh) {
    const double pa = P[i], f = P[n + i];
    const double rhoL = sh[0], cL = sh[1], pV = sh[2], sig = sh[3], mu = sh[4];
    const double gam = sh[5], pinf = sh[6];
    const double re = PSYS ? P[5 * n + i] : sh[7];
    const double w = 2.0 * M_PI * f;              // omega1
    const double q = 2.0 * M_PI / (re * w);       // 2 pi / (R_E omega1)
    const double q2 = q * q;
    const double g0 = pinf - pV + 2.0 * sig / re; // gas pressure at rest
    K0 = g0 * q2 / rhoL;
    K1 = (1.0 - 3.0 * gam) * g0 * q / (rhoL * cL);
    K2 = (pinf - pV) * q2 / rhoL;
    K3 = 2.0 * sig * q2 / (rhoL * re);
    K4 = 4.0 * mu * (2.0 * M_PI / w) / (rhoL * re * re);
    K5 = pa * q2 / rhoL;
    K7 = re * w * pa * q2 / (rhoL * cL);
    K9 = re * w / (2.0 * M_PI * cL);
    K10 = 3.0 * gam;
    K49 = K4 * K9;
    K9h = 0.5 * K9;    // exact; once per system, not per attempt
    if constexpr (DUAL) {
      const double pa2 = PSYS ? P[2 * n + i] : sh[8];
      const double w2 = 2.0 * M_PI * (PSYS ? P[3 * n + i] : sh[9]);
      const double th = PSYS ? P[4 * n + i] : sh[10];
      dual = pa2 != 0.0;
      K6 = pa2 * q2 / rhoL;
      K8 = re * w2 * pa2 * q2 / (rhoL * cL);
      K11 = w2 / w;                 // omega2 / omega1, correctly rounded
      thpi = th * M_1_PI;           // theta / pi
    }
  }
  // The coefficients init derives, as a solve precomputes them for every
  // system (k_model_coef: the divisions run once per system, fully
  // parallel) and a lane loads them when it takes the system up, instead of
  // deriving them there for the whole wave: [kNCoef][n], the same doubles.
  static constexpr int kNCoef = DUAL ? 16 : 11;
  __device__ void store_coef(double *c, int64_t n, int64_t i) const {
    c[0 * n + i] = K0;
    c[1 * n + i] = K1;
    c[2 * n + i] = K2;
    c[3 * n + i] = K3;
    c[4 * n + i] = K4;
    c[5 * n + i] = K5;
    c[6 * n + i] = K7;
    c[7 * n + i] = K9;
    c[8 * n + i] = K10;
    c[9 * n + i] = K49;
    c[10 * n + i] = K9h;
    if constexpr (DUAL) {
      c[11 * n + i] = K6;
      c[12 * n + i] = K8;
      c[13 * n + i] = K11;
      c[14 * n + i] = thpi;
      c[15 * n + i] = dual ? 1.0 : 0.0;
    }
  }
  __device__ void load_coef(const double *c, int64_t n, int64_t i) {
    K0 = c[0 * n + i];
    K1 = c[1 * n + i];
    K2 = c[2 * n + i];
    K3 = c[3 * n + i];
    K4 = c[4 * n + i];
    K5 = c[5 * n + i];
    K7 = c[6 * n + i];
    K9 = c[7 * n + i];
    K10 = c[8 * n + i];
    K49 = c[9 * n + i];
    K9h = c[10 * n + i];
    if constexpr (DUAL) {
      K6 = c[11 * n + i];
      K8 = c[12 * n + i];
      K11 = c[13 * n + i];
      thpi = c[14 * n + i];
      dual = c[15 * n + i] != 0.0;
    }
  }
  // Second drive: phi = its phase in cycles when the current phase began;
  // within the phase its angle is 2 pi (phi + K11 tau) + theta.
  double K6, K8, K11, thpi, phi;
  bool dual;
  // A phase of length tp ended: the drive went through K11 tp cycles
  // (multiply and add rounded separately, then reduced modulo 1).
  __device__ void next_phase(double tp) {
    const double v = __dadd_rn(phi, __dmul_rn(K11, tp));
    phi = v - floor(v);
  }
  // FAST: sin/cos of the stage offsets 2 pi c_i h.  Cash--Karp, c = (0, 1/5,
  // 3/10, 3/5, 1, 7/8): stages 2, 3 and 6 from the series, stage 4 by
  // doubling stage 3's angle and stage 5 as stage 4's plus twice stage 2's.
  // Dormand--Prince, c = (0, 1/5, 3/10, 4/5, 8/9, 1, 1): stages 2, 3 and 5
  // from the series, stage 4 by doubling stage 2's angle twice, stage 6 as
  // stage 4's plus stage 2's, stage 7 the same angle as stage 6.
  double so2, co2, so4, co4, so1, co1;
  __device__ void begin(double t) {
    if constexpr (FAST) {
      double s0, c0;
      sincospi_quarter(2.0 * t, &s0, &c0);
      k5s = K5 * s0;
      k5c = K5 * c0;
      k7s = K7 * s0;
      k7c = K7 * c0;
    }
  }
  // SC: the scheme; S: the stage (1..7); tau: its time; h: the attempted step.
  template <int SC, int S>
  __device__ void rhs(double tau, double h, const double *y, double *f) {
    eval<SC, S, 0>(tau, h, y, nullptr, f, nullptr);
  }
  // With the variational equation: df = J dy from the same intermediates.
  template <int SC, int S, int K>
  __device__ void rhs_tan(double tau, double h, const double *y, const double *dy, double *f,
                          double *df) {
    eval<SC, S, K>(tau, h, y, dy, f, df);
  }
  template <int SC, int S, int K>
  __device__ __forceinline__ void eval(double tau, double h, const double *y, const double *dy,
                                       double *f, double *df) {
    const double y1 = y[0], y2 = y[1];
    const double Dn = fma(y1, fma(-K9, y2, 1.0), K49);
    const double qd = rcp_nr(y1 * Dn);
    const double r1 = Dn * qd;                    // 1 / y1
    double gas, s, c;     // (1/y1)^K10; sin, cos (2 pi tau) (not FAST)
    double so, co;        // FAST: sin, cos of the stage's offset 2 pi c_i h
    if constexpr (FAST) {
      const double r2 = r1 * r1;
      gas = (r2 * r2) * rfifth(y1);
      if constexpr (S == 1) {
        so = 0.0;
        co = 1.0;
      } else if constexpr (SC == kDP) {
        if constexpr (S == 2) {
          sincos_taylor<6, 6>((2.0 * M_PI / 5.0) * h, &so2, &co2);      // |x| <= 0.16
          so = so2;
          co = co2;
        } else if constexpr (S == 3) {
          sincos_taylor<6, 7>((2.0 * M_PI * 3.0 / 10.0) * h, &so, &co);  // |x| <= 0.24
        } else if constexpr (S == 4) {
          const double sd = 2.0 * so2 * co2, cd = fma(-2.0 * so2, so2, 1.0);  // 2/5
          so4 = 2.0 * sd * cd;                                                // 4/5
          co4 = fma(-2.0 * sd, sd, 1.0);
          so = so4;
          co = co4;
        } else if constexpr (S == 5) {
          sincos_taylor<8, 9>((2.0 * M_PI * 8.0 / 9.0) * h, &so, &co);   // |x| <= 0.70
        } else if constexpr (S == 6) {
          so1 = fma(so4, co2, co4 * so2);                                 // 4/5 + 1/5
          co1 = fma(co4, co2, -(so4 * so2));
          so = so1;
          co = co1;
        } else {
          so = so1;
          co = co1;
        }
      } else if constexpr (S == 2) {
        sincos_taylor<6, 6>((2.0 * M_PI / 5.0) * h, &so2, &co2);        // |x| <= 0.16
        so = so2;
        co = co2;
      } else if constexpr (S == 3) {
        double so3, co3;
        sincos_taylor<6, 7>((2.0 * M_PI * 3.0 / 10.0) * h, &so3, &co3);  // |x| <= 0.24
        so4 = 2.0 * so3 * co3;             // doubled angle, for stage 4
        co4 = fma(-2.0 * so3, so3, 1.0);
        so = so3;
        co = co3;
      } else if constexpr (S == 4) {
        so = so4;
        co = co4;
      } else if constexpr (S == 5) {
        const double sd = 2.0 * so2 * co2, cd = fma(-2.0 * so2, so2, 1.0);
        so = fma(so4, cd, co4 * sd);
        co = fma(co4, cd, -(so4 * sd));
      } else {
        sincos_taylor<8, 9>((2.0 * M_PI * 7.0 / 8.0) * h, &so, &co);      // |x| <= 0.69
      }
    } else {
      gas = exp(-K10 * log(y1));
      sincospi(2.0 * tau, &s, &c);
    }
    // forcing terms of N: fs = K2 + K5 sin, fc = K7 cos (2 pi tau)
    double fs, fc;
    if constexpr (!FAST) {
      fs = fma(K5, s, K2);
      fc = K7 * c;
    } else if constexpr (S == 1) {
      fs = k5s + K2;
      fc = k7c;
    } else {
      fs = fma(k5s, co, fma(k5c, so, K2));
      fc = fma(k7c, co, -(k7s * so));
    }
    if constexpr (DUAL) {
      if (dual) {
        double s2, c2;
        sincospi_quarter(fma(2.0, fma(K11, tau, phi), thpi), &s2, &c2);
        fs = fma(K6, s2, fs);
        fc = fma(K8, c2, fc);
      }
    }
    const double u = fma(K9, y2, 1.0);
    double N = fma(K1, y2, K0) * gas;
    N = fma(-fs, u, N);
    N = fma(-fma(K4, y2, K3), r1, N);
    N = fma(-fma(-K9h, y2, 1.5) * y2, y2, N);
    N = fma(-fc, y1, N);
    f[0] = y2;
    f[1] = N * (y1 * qd);
    if constexpr (K > 0) {
      // f2 = N / D: d f2 / d y_j = (dN/dy_j - f2 dD/dy_j) / D, 1/D = y1 qd
      const double f2 = f[1], iD = y1 * qd;
      const double dN1 = fma(-K10 * fma(K1, y2, K0) * gas, r1, fma(fma(K4, y2, K3), r1 * r1, -fc));
      const double dN2 = fma(K1, gas, -K9 * fs) - K4 * r1 + y2 * fma(1.5 * K9, y2, -3.0);
      const double J21 = fma(-f2, fma(-K9, y2, 1.0), dN1) * iD;
      const double J22 = fma(f2 * K9, y1, dN2) * iD;
#pragma unroll
      for (int v = 0; v < K; ++v) {
        df[2 * v] = dy[2 * v + 1];
        df[2 * v + 1] = fma(J21, dy[2 * v], J22 * dy[2 * v + 1]);
      }
    }
  }
};

// Pressure-relief valve (Sec. 4.3), shared (kappa, delta, beta, r).  While
// seated (sticking guard) the body is held and the chamber fills.
struct MPRV {
  static constexpr int D = 3;
  static constexpr bool kEvents = true;
  static constexpr int kMinWaves = 5;
  static constexpr bool kPrio = false;  // issue priority by remaining work
  static constexpr bool kLocate = false;
  static constexpr bool kDrive2 = false;
  static constexpr int kF = 2;           // (y1 at the Poincare point, y1min)
  static constexpr bool kTangent = false;
  static constexpr int kNCoef = 0;  // no precomputed coefficients
  double q, kappa, delta, beta, r;
  bool seated;
  __device__ void init(const double *P, int64_t n, int64_t i, const double *sh) {
    q = P[i];
    kappa = sh[0];
    delta = sh[1];
    beta = sh[2];
    r = sh[3];
    seated = false;
  }
  __device__ void begin(double) {}
  template <int SC, int S>
  // Seated, the body rests with y1 = y2 = +0 (the seating sets both and
  // every stage keeps them), so the free-flight expressions give dy1/dt = 0
  // and dy3/dt = beta q exactly; only the acceleration is held at 0.  No
  // branch: the attempt stays one basic block.
  __device__ void rhs(double, double, const double *y, double *f) const {
    const double acc = fma(-kappa, y[1], y[2] - (y[0] + delta));
    f[0] = y[1];
    f[1] = seated ? 0.0 : acc;
    f[2] = beta * fma(-y[0], sqrt_nr(y[2]), q);
  }
};

// One attempted Cash--Karp step: y5 and err = h sum (b5 - b4) k.
template <class M>
__device__ __forceinline__ void ck_attempt(M &m, double t, const double *y, double h,
                                           double *y5, double *err) {
  constexpr int D = M::D;
  double k1[D], k2[D], k3[D], k4[D], k5[D], k6[D], yt[D];
  const auto &T = scalar_table(kCkTab);
  m.begin(t);
  m.template rhs<kCK, 1>(t, h, y, k1);
#pragma unroll
  for (int c = 0; c < D; ++c) yt[c] = fma(h, T.a21 * k1[c], y[c]);
  m.template rhs<kCK, 2>(fma(C2, h, t), h, yt, k2);
#pragma unroll
  for (int c = 0; c < D; ++c) yt[c] = fma(h, fma(T.a32, k2[c], T.a31 * k1[c]), y[c]);
  m.template rhs<kCK, 3>(fma(C3, h, t), h, yt, k3);
#pragma unroll
  for (int c = 0; c < D; ++c)
    yt[c] = fma(h, fma(T.a43, k3[c], fma(T.a42, k2[c], T.a41 * k1[c])), y[c]);
  m.template rhs<kCK, 4>(fma(C4, h, t), h, yt, k4);
#pragma unroll
  for (int c = 0; c < D; ++c)
    yt[c] = fma(h, fma(T.a54, k4[c], fma(T.a53, k3[c], fma(T.a52, k2[c], T.a51 * k1[c]))), y[c]);
  m.template rhs<kCK, 5>(t + C5 * h, h, yt, k5);
#pragma unroll
  for (int c = 0; c < D; ++c)
    yt[c] = fma(h, fma(T.a65, k5[c], fma(T.a64, k4[c], fma(T.a63, k3[c], fma(T.a62, k2[c], T.a61 * k1[c])))),
                y[c]);
  m.template rhs<kCK, 6>(fma(C6, h, t), h, yt, k6);
#pragma unroll
  for (int c = 0; c < D; ++c) {
    y5[c] = fma(h, fma(T.b6, k6[c], fma(T.b4, k4[c], fma(T.b3, k3[c], T.b1 * k1[c]))), y[c]);
    err[c] = h * fma(T.e6, k6[c], fma(T.e5, k5[c], fma(T.e4, k4[c], fma(T.e3, k3[c], T.e1 * k1[c]))));
  }
}

// One attempted Dormand--Prince step from (t, y): k1 = f(t, y) is taken from
// kf when have_k1 (first same as last), else evaluated and left in kf; k7
// receives f(t + h, y5).  Returns the number of RHS evaluations.
template <class M>
__device__ __forceinline__ int dp_attempt(M &m, double t, const double *y, double h,
                                          double *kf, bool have_k1, double *y5, double *err,
                                          double *k7) {
  constexpr int D = M::D;
  double k2[D], k3[D], k4[D], k5[D], k6[D], yt[D];
  const auto &T = scalar_table(kDpTab);
  m.begin(t);
  if (!have_k1) m.template rhs<kDP, 1>(t, h, y, kf);
  const double *k1 = kf;
#pragma unroll
  for (int c = 0; c < D; ++c) yt[c] = fma(h, T.a21 * k1[c], y[c]);
  m.template rhs<kDP, 2>(fma(DC2, h, t), h, yt, k2);
#pragma unroll
  for (int c = 0; c < D; ++c) yt[c] = fma(h, fma(T.a32, k2[c], T.a31 * k1[c]), y[c]);
  m.template rhs<kDP, 3>(fma(DC3, h, t), h, yt, k3);
#pragma unroll
  for (int c = 0; c < D; ++c)
    yt[c] = fma(h, fma(T.a43, k3[c], fma(T.a42, k2[c], T.a41 * k1[c])), y[c]);
  m.template rhs<kDP, 4>(fma(DC4, h, t), h, yt, k4);
#pragma unroll
  for (int c = 0; c < D; ++c)
    yt[c] = fma(h, fma(T.a54, k4[c], fma(T.a53, k3[c], fma(T.a52, k2[c], T.a51 * k1[c]))), y[c]);
  m.template rhs<kDP, 5>(fma(DC5, h, t), h, yt, k5);
#pragma unroll
  for (int c = 0; c < D; ++c)
    yt[c] = fma(h, fma(T.a65, k5[c], fma(T.a64, k4[c], fma(T.a63, k3[c], fma(T.a62, k2[c], T.a61 * k1[c])))),
                y[c]);
  m.template rhs<kDP, 6>(t + h, h, yt, k6);
#pragma unroll
  for (int c = 0; c < D; ++c)
    y5[c] = fma(h, fma(T.b6, k6[c], fma(T.b5, k5[c], fma(T.b4, k4[c], fma(T.b3, k3[c], T.b1 * k1[c])))),
                y[c]);
  m.template rhs<kDP, 7>(t + h, h, y5, k7);
#pragma unroll
  for (int c = 0; c < D; ++c)
    err[c] = h * fma(T.e7, k7[c], fma(T.e6, k6[c], fma(T.e5, k5[c], fma(T.e4, k4[c],
                                                      fma(T.e3, k3[c], T.e1 * k1[c])))));
  return have_k1 ? 6 : 7;
}

// x limited to [lo, hi] for a finite x and lo <= hi (the host checks
// dt_min <= dt_max), as two min/max instructions.
__device__ __forceinline__ double clampd(double x, double lo, double hi) {
  return vmin_s(vmax_s(x, lo), hi);
}

// Lane-private progress of one system.
// A fixed-length-phase model with its variational equation d(dy)/dt =
// J(t, y) dy riding along (the paper's introduction: trajectory manipulation
// between integration phases, here Benettin's renormalisation for the
// largest Lyapunov exponent, done in the kernel).  The lane state is [y; dy]
// (2 M::D components, all under error control); at a phase end dy is
// rescaled to unit length and log |dy| becomes the phase's second record.
template <class M, int K>
struct MTan : M {
  static_assert(!M::kEvents, "the tangent is built for fixed-length phases");
  static_assert(K >= 1 && K <= M::D, "1 .. D tangents");
  static constexpr int D = M::D * (1 + K);
  static constexpr int kMinWaves = M::kMinWaves > K + 1 ? M::kMinWaves - K : 2;
  static constexpr bool kLocate = false;
  static constexpr int kF = 1 + K;       // (y1max, log growth of each tangent)
  static constexpr bool kTangent = true;
  static constexpr int kK = K;
  template <int SC, int S>
  __device__ void rhs(double tau, double h, const double *y, double *f) {
    M::template rhs_tan<SC, S, K>(tau, h, y, y + M::D, f, f + M::D);
  }
  // Renormalisation at a phase end (Gram--Schmidt in order): tangent v is
  // made orthogonal to those before it, g[v] receives its log length, and
  // it is scaled to unit length.
  __device__ void renormalise(double *y, double *g) const {
    constexpr int B = M::D;
#pragma unroll
    for (int v = 0; v < K; ++v) {
      double *w = y + B * (1 + v);
#pragma unroll
      for (int u = 0; u < v; ++u) {
        const double *q = y + B * (1 + u);
        double dot = 0.0;
#pragma unroll
        for (int c = 0; c < B; ++c) dot = fma(q[c], w[c], dot);
#pragma unroll
        for (int c = 0; c < B; ++c) w[c] = fma(-dot, q[c], w[c]);
      }
      double s2 = 0.0;
#pragma unroll
      for (int c = 0; c < B; ++c) s2 = fma(w[c], w[c], s2);
      const double nrm = sqrt(s2);
      const double inv = 1.0 / nrm;
#pragma unroll
      for (int c = 0; c < B; ++c) w[c] *= inv;
      g[v] = log(nrm);
    }
  }
};

struct Lane {
  int64_t sys;
  double t, h, t_ps, ymax, ymin;
  int64_t n_phases, max_impacts;
  uint32_t phase, accepted, rejected, evretry, impacts, attempts;
  uint32_t phase_att;  // attempts when the current phase began
  float rem;           // estimated attempts left: last phase's x phases left
  uint32_t nrhs;       // Dormand--Prince: RHS evaluations (6 or 7 per attempt)
  int32_t status, ev_iter;
  bool head;           // taken from the spread head of the queue
};

// Dormand--Prince: k1 = f(t, y) of the next attempt, valid when `have`.  An
// attempt leaves its k1 here (a rejected step retries from the same point);
// an accepted one replaces it by its k7 (first same as last); a phase end, an
// impact or a lift-off clears it, so that every phase starts by evaluating k1.
template <int D>
struct Fsal {
  double k[D];
  bool have;
};

// Estimated work left after a completed phase.
__device__ __forceinline__ void note_phase_end(Lane &L) {
  const float per = (float)(L.attempts - L.phase_att);
  // phases left, below 2^32 (the phase count is limited to it)
  const uint32_t left =
      L.n_phases > (int64_t)L.phase ? (uint32_t)(L.n_phases - (int64_t)L.phase) : 0u;
  L.rem = per * (float)left;
  L.phase_att = L.attempts;
}

// The cold pointers, read from device memory where they are used (the
// empty asm hides that the address is the same on every iteration, so the
// loads are not hoisted out of the step loop into scalar registers).
__device__ __forceinline__ const RkckCold *cold(const RkckArgs &a) {
  const RkckCold *c = a.cold;
  asm volatile("" : "+s"(c));
  return c;
}

// Ring slot of the current phase: phase mod R in 32 bits (phases are
// counted below 2^32; a ring that long never wraps).
__device__ __forceinline__ int64_t ring_slot(const RkckArgs &a, const Lane &L) {
  return a.R > (int64_t)UINT32_MAX ? (int64_t)L.phase
                                   : (int64_t)(L.phase % (uint32_t)a.R);
}

template <class M>
__device__ __forceinline__ void store_record(const RkckArgs &a, const Lane &L, double v0,
                                             double v1) {
  if (a.R <= 0) return;
  constexpr int F = M::kF;
  const int64_t slot = ring_slot(a, L);
  double *rec = cold(a)->rec;
  rec[(slot * F) * a.n + L.sys] = v0;
  if (F > 1) rec[(slot * F + 1) * a.n + L.sys] = v1;
}

// Record fields 1 .. K of a phase with tangents: their log growths.
template <class M, int K>
__device__ __forceinline__ void store_growth(const RkckArgs &a, const Lane &L, const double *g) {
  if (a.R <= 0) return;
  const int64_t slot = ring_slot(a, L);
  double *rec = cold(a)->rec;
#pragma unroll
  for (int v = 0; v < K; ++v) rec[(slot * M::kF + 1 + v) * a.n + L.sys] = g[v];
}

template <class M, int SC>
__device__ __forceinline__ void store_lane(const RkckArgs &a, const Lane &L, const double *y,
                                           bool seated) {
  constexpr int D = M::D;
  const int64_t n = a.n, i = L.sys;
  const RkckCold *cp = cold(a);
#pragma unroll
  for (int c = 0; c < D; ++c) cp->y[c * n + i] = y[c];
  cp->t[i] = L.t;
  cp->h[i] = L.h;
  const int64_t att = (int64_t)L.accepted + L.rejected + L.evretry;
  int64_t *stats = cp->stats;
  stats[ENS_ST_ACCEPTED * n + i] = L.accepted;
  stats[ENS_ST_REJECTED * n + i] = L.rejected;
  // Cash--Karp: 6 per attempt plus the evaluations of located maxima
  stats[ENS_ST_NRHS * n + i] = SC == kDP ? (int64_t)L.nrhs : 6 * att + (int64_t)L.nrhs;
  stats[ENS_ST_IMPACTS * n + i] = L.impacts;
  stats[ENS_ST_PHASES * n + i] = L.phase;
  stats[ENS_ST_EVRETRY * n + i] = L.evretry;
  cp->status[i] = L.status;
  double *cy = cp->carry;
  cy[ENS_CARRY_YMAX * n + i] = L.ymax;
  cy[ENS_CARRY_YMIN * n + i] = L.ymin;
  cy[ENS_CARRY_TPS * n + i] = L.t_ps;
  cy[ENS_CARRY_SEATED * n + i] = seated ? 1.0 : 0.0;
}

// The valve's seated state (false for the models without a seat).
template <class M>
__device__ __forceinline__ bool seated_of(const M &m) {
  if constexpr (M::kEvents)
    return m.seated;
  else
    return false;
}

// Dense output of a step from y0 to y1 with end derivatives f0, f1 and step
// h: the cubic Hermite interpolant, component c at theta in [0, 1].
template <int D>
__device__ __forceinline__ double hermite(const double *y0, const double *y1, const double *f0,
                                          const double *f1, double h, int c, double th) {
  const double t2 = th * th, t3 = t2 * th;
  return (2.0 * t3 - 3.0 * t2 + 1.0) * y0[c] + (t3 - 2.0 * t2 + th) * h * f0[c] +
         (-2.0 * t3 + 3.0 * t2) * y1[c] + (t3 - t2) * h * f1[c];
}

// y1 at the zero of the interpolant's y2 = y1' inside the step (y2 > 0 at
// its start, <= 0 at its end), by 60 bisections of theta.
template <int D>
__device__ __noinline__ double located_max(const double *y0, const double *y1, const double *f0,
                                           const double *f1, double h) {
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hermite<D>(y0, y1, f0, f1, h, 1, mid) > 0.0)
      lo = mid;
    else
      hi = mid;
  }
  return hermite<D>(y0, y1, f0, f1, h, 0, 0.5 * (lo + hi));
}

// One attempted step of a fixed-length-phase model; returns true when the
// system is finished.
template <class M, int SC, bool LOC>
__device__ __forceinline__ bool step_fixed(const RkckArgs &a, M &m, Lane &L, double *y,
                                           Fsal<M::D> &fs) {
  constexpr int D = M::D;
  double y5[D], err[D], k7[D];
  double h_try = L.h;
  const bool trunc = L.t + h_try >= a.t_phase;
  if (trunc) h_try = a.t_phase - L.t;
  if constexpr (SC == kDP) {
    L.nrhs += dp_attempt(m, L.t, y, h_try, fs.k, fs.have, y5, err, k7);
    fs.have = true;
  } else {
    ck_attempt(m, L.t, y, h_try, y5, err);
  }
  L.attempts++;
  double E;
  const bool finite = error_ratio<D>(a.rtol, a.atol, y, y5, err, E);
  if (!finite) {
    L.status |= ENS_SYS_NONFINITE;
    return true;
  }
  const double fac = step_factor<false>(E);
  // Accept (E <= 1, or at the step-size floor) or reject, by selects: only
  // the rare phase end and located maximum branch.  After a rejection the
  // step only shrinks.
  const bool acc = !(E > 1.0 && h_try > a.dt_min);
  const double h_new = clampd(h_try * (acc ? fac : fmin(fac, 1.0)), a.dt_min, a.dt_max);
  L.status |= (acc && E > 1.0) ? ENS_SYS_DT_MIN : 0;
  L.accepted += acc ? 1 : 0;
  L.rejected += acc ? 0 : 1;
  if constexpr (LOC) {
    if (acc && y[1] > 0.0 && y5[1] <= 0.0) {
      // the maximum of y1 between the step points, on the interpolant
      // (Dormand--Prince has f at both ends; Cash--Karp evaluates them)
      double f0[D], f1[D];
      if constexpr (SC == kDP) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
          f0[c] = fs.k[c];
          f1[c] = k7[c];
        }
      } else {
        m.begin(L.t);
        m.template rhs<SC, 1>(L.t, h_try, y, f0);
        m.begin(L.t + h_try);
        m.template rhs<SC, 1>(L.t + h_try, h_try, y5, f1);
        L.nrhs += 2;
      }
      const double ym = located_max<D>(y, y5, f0, f1, h_try);
      L.ymax = ym > L.ymax ? ym : L.ymax;
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = acc ? y5[c] : y[c];
  if constexpr (SC == kDP) {
#pragma unroll
    for (int c = 0; c < D; ++c) fs.k[c] = acc ? k7[c] : fs.k[c];
  }
  L.ymax = (acc && y[0] > L.ymax) ? y[0] : L.ymax;
  if (acc && trunc) {
    // phase end: the next phase starts with the step proposed before the
    // truncation (L.h is left as it was)
    fs.have = false;
    if constexpr (M::kTangent) {
      double g[M::kK];
      m.renormalise(y, g);
      store_record<M>(a, L, L.ymax, g[0]);
      store_growth<M, M::kK>(a, L, g);
    } else {
      store_record<M>(a, L, L.ymax, 0.0);
    }
    L.phase++;
    if constexpr (M::kPrio) note_phase_end(L);
    if constexpr (M::kDrive2) m.next_phase(a.t_phase);
    L.t = 0.0;
    L.t_ps = 0.0;
    L.ymax = -INFINITY;
    if (L.phase >= L.n_phases) return true;
  } else {
    L.t += acc ? h_try : 0.0;
    L.h = h_new;
  }
  if (a.max_steps > 0 && L.attempts >= a.max_steps) {
    L.status |= ENS_SYS_MAX_STEPS;
    return true;
  }
  return false;
}

// One attempted step of the relief valve with events; true when finished.
template <int SC>
__device__ __forceinline__ bool step_valve(const RkckArgs &a, MPRV &m, Lane &L, double *y,
                                           Fsal<3> &fs) {
  constexpr int D = 3;
  double y5[D], err[D], k7[D];
  const double h_try = L.h;
  if constexpr (SC == kDP) {
    L.nrhs += dp_attempt(m, L.t, y, h_try, fs.k, fs.have, y5, err, k7);
    fs.have = true;
  } else {
    ck_attempt(m, L.t, y, h_try, y5, err);
  }
  L.attempts++;
  double E;
  const bool finite = error_ratio<D>(a.rtol, a.atol, y, y5, err, E);
  if (!finite) {
    L.status |= ENS_SYS_NONFINITE;
    return true;
  }
  const double fac = step_factor<true>(E);
  // The common outcomes (rejection, event retry, plain acceptance) by
  // selects; only the rare ones branch: an event's secant step, a seat
  // change or impact, a Poincare point, settling.
  const bool rej = E > 1.0 && h_try > a.dt_min;
  // after a rejection the step only shrinks
  const double h_next = clampd(h_try * (rej ? fmin(fac, 1.0) : fac), a.dt_min, a.dt_max);
  const double tol = a.event_tol;
  // event detection: overshoot -> secant retry from the same point.  The
  // tests are plain compares; the secant steps (divisions) are formed only
  // when one of them fired, which few steps do.
  const double g3o = y[2] - m.delta, g3n = y5[2] - m.delta;  // lift-off
  const bool free = !m.seated;
  // y1 crossing below the seat: an impact (y1 > 0 before), or a rebound
  // swallowed by one step (y1 = 0 before)
  const bool ev_y1 = free && y[0] >= 0.0 && y5[0] < -tol;
  const bool ev_max = free && y[1] > 0.0 && y5[1] < -tol;   // local maximum, y2 decreasing
  const bool ev_lift = !free && g3o < 0.0 && g3n > tol;
  const bool over = !rej && (ev_y1 || ev_max || ev_lift);
  double hs = INFINITY;
  if (over) {
    if (ev_y1) hs = fmin(hs, y[0] > 0.0 ? h_try * y[0] / (y[0] - y5[0]) : 0.5 * h_try);
    if (ev_max) hs = fmin(hs, h_try * y[1] / (y[1] - y5[1]));
    if (ev_lift) hs = fmin(hs, h_try * (-g3o) / (g3n - g3o));
  }
  const bool retry = over && L.ev_iter < a.max_event_iter;
  const bool take = !rej && !retry;   // the step is accepted
  L.rejected += rej ? 1 : 0;
  L.evretry += retry ? 1 : 0;
  L.accepted += take ? 1 : 0;
  L.status |= (!rej && E > 1.0) ? ENS_SYS_DT_MIN : 0;   // at the step-size floor
  L.status |= (take && over) ? ENS_SYS_EVENT_ITER : 0;  // secant retries exhausted
  L.ev_iter = retry ? L.ev_iter + 1 : (take ? 0 : L.ev_iter);
  L.h = retry ? hs : h_next;
  const double y2o = y[1];
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = take ? y5[c] : y[c];
  if constexpr (SC == kDP) {
#pragma unroll
    for (int c = 0; c < D; ++c) fs.k[c] = take ? k7[c] : fs.k[c];
  }
  L.t += take ? h_try : 0.0;
  // an accepted step may lift the body off its seat, or end in a located
  // impact (Newtonian restitution, Sec. 4.3), or at a located local maximum
  // of the free flight (the Poincare point)
  const bool lift = take && !free && y[2] - m.delta >= 0.0;
  const bool impact = take && free && y[0] <= 0.0 && y[1] < 0.0;
  const bool pmax = take && free && !impact && y2o > 0.0 && y[1] <= 0.0;
  bool done = false;
  // The rare outcomes (a seat change or impact, a Poincare point, settling)
  // behind one wave-uniform test: most attempts of most waves have none, and
  // then skip their exec-mask bookkeeping altogether.
  const bool cap = take && L.t - L.t_ps >= a.t_cap;
  if (__ballot(lift || impact || pmax || cap) == 0ull) {
    L.ymax = take ? fmax(L.ymax, y[0]) : L.ymax;
    L.ymin = take ? fmin(L.ymin, y[0]) : L.ymin;
  } else {
    if (lift || impact) {
      fs.have = false;
      if (lift) {
        m.seated = false;
      } else {
        const double v_in = y[1];
        y[0] = 0.0;
        y[1] = -m.r * v_in;
        L.impacts++;
        if (fabs(v_in) < a.v_stick && y[2] < m.delta) {
          m.seated = true;
          y[1] = 0.0;
          L.status |= ENS_SYS_SEATED;
        }
        if (L.max_impacts > 0 && (int64_t)L.impacts >= L.max_impacts) done = true;
      }
    }
    L.ymax = take ? fmax(L.ymax, y[0]) : L.ymax;
    L.ymin = take ? fmin(L.ymin, y[0]) : L.ymin;
    if (pmax) {
      fs.have = false;
      store_record<MPRV>(a, L, y[0], L.ymin);
      L.phase++;
      if constexpr (MPRV::kPrio) note_phase_end(L);
      L.ymax = -INFINITY;
      L.ymin = INFINITY;
      L.t_ps = L.t;
      if (L.phase >= L.n_phases) done = true;
    } else if (take && L.t - L.t_ps >= a.t_cap) {
      store_record<MPRV>(a, L, L.ymax, L.ymin);
      L.phase++;
      L.status |= ENS_SYS_SETTLED;
      done = true;
    }
  }
  if (!done && a.max_steps > 0 && L.attempts >= a.max_steps) {
    L.status |= ENS_SYS_MAX_STEPS;
    done = true;
  }
  return done;
}

// Each model states the occupancy floor the register allocator must respect
// (kMinWaves waves per SIMD): 5 for the light models, 4 for the fast
// Keller--Miksis variant, whose stage trigonometry needs the extra registers.
// LOC: Keller--Miksis maxima located on the step interpolant (an instantiation
// of its own, so that the plain kernels carry none of its registers).
template <class M, int SC, bool LOC>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(min_waves(M::kMinWaves, SC, LOC), 8))) void k_rkck(RkckArgs a) {
  constexpr int D = M::D;
  __shared__ EnsDesc sdesc[ENS_MAX_ENSEMBLES];
  for (int e = threadIdx.x; e < a.n_ens; e += blockDim.x) sdesc[e] = a.desc[e];
  __syncthreads();

  const int lane = __lane_id();
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (M::kPrio && a.prioritize) __builtin_amdgcn_s_setprio(3);
  M m;
  Lane L;
  Fsal<D> fs;
  double y[D];
  bool active = false;
  bool drained = false;
  // Two queues over the positions of the queue order: the head [0, spread)
  // and the rest [spread, n), each with its own counter.  The wave in slot 0
  // of its SIMD (one per SIMD, from the hardware id) prefers the head, all
  // others the rest; a wave takes from the other queue once its own is
  // empty.  Systems at the head (the longest) thus start one wave per SIMD
  // instead of sharing a SIMD with each other.
  const uint64_t spread = (uint64_t)a.spread, nsys = (uint64_t)a.n;
  const bool slot0 = (__builtin_amdgcn_s_getreg((3 << 11) | 4) & 0xF) == 0;  // HW_ID.WAVE_ID
  bool head_done = spread == 0, rest_done = spread >= nsys;
  bool head_prio = false;  // the wave raised its issue priority for head systems

  while (true) {
    const unsigned long long idle = __ballot(!active);
    const int n_idle = __popcll(idle);
    if (!drained && n_idle > 0 && (n_idle >= a.refill || idle == ~0ull)) {
      const bool use_head = !head_done && (slot0 || rest_done);
      const int leader = __ffsll((long long)idle) - 1;
      unsigned long long base = 0;
      if (lane == leader)
        base = atomicAdd(cold(a)->queue + (use_head ? 1 : 0), (unsigned long long)n_idle);
      // the leader's value to the whole wave as a scalar (so that the queue
      // flags below are wave-uniform values in scalar registers)
      base = ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(base >> 32), leader)
              << 32) |
             (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)base, leader);
      const uint64_t first = use_head ? 0 : spread, limit = use_head ? spread : nsys - spread;
      if (base + (unsigned long long)n_idle >= limit) {
        if (use_head)
          head_done = true;
        else
          rest_done = true;
      }
      drained = head_done && rest_done;
      if (!active) {
        const unsigned long long k = base + (unsigned long long)__popcll(idle & below);
        const unsigned long long me = first + k;
        if (k < limit) {
          const RkckCold *cp = cold(a);
          const int64_t *order = cp->order;
          const int64_t i = order ? order[me] : (int64_t)me;
          int e = 0;
          while (e + 1 < a.n_ens && i >= sdesc[e].last) ++e;
          if constexpr (M::kNCoef > 0) {
            if (cp->coef)
              m.load_coef(cp->coef, a.n, i);
            else
              m.init(cp->p, a.n, i, sdesc[e].shared);
          } else {
            m.init(cp->p, a.n, i, sdesc[e].shared);
          }
          if constexpr (M::kDrive2) m.phi = cp->phi2[i];
#pragma unroll
          for (int c = 0; c < D; ++c) y[c] = cp->y[c * a.n + i];
          L.sys = i;
          L.t = cp->t[i];
          L.h = cp->h[i];
          // the running phase as the previous solve left it (a fresh state
          // carries no maximum or minimum, its phase starting at t0)
          const double *cy = cp->carry;
          L.ymax = cy[ENS_CARRY_YMAX * a.n + i];
          L.ymin = cy[ENS_CARRY_YMIN * a.n + i];
          L.t_ps = cy[ENS_CARRY_TPS * a.n + i];
          if constexpr (M::kEvents) m.seated = cy[ENS_CARRY_SEATED * a.n + i] != 0.0;
          L.n_phases = sdesc[e].n_phases;
          L.max_impacts = sdesc[e].max_impacts;
          L.phase = L.accepted = L.rejected = L.evretry = L.impacts = L.attempts = 0;
          if constexpr (M::kPrio) {
            L.phase_att = 0;
            L.rem = 3.0e38f;  // unknown until the first phase ends: treat as long
          }
          L.status = 0;
          L.ev_iter = 0;
          L.nrhs = 0;
          L.head = use_head;
          fs.have = false;
          active = true;
          if (L.n_phases <= 0) {
            store_lane<M, SC>(a, L, y, seated_of(m));
            if constexpr (M::kDrive2) cold(a)->phi2[i] = m.phi;
            active = false;
          }
        }
      }
      // A wave that carries head systems raises its issue priority, so that
      // the long systems are not slowed by short ones sharing the SIMD (models
      // without their own remaining-work priority; results do not change).
      if constexpr (!M::kPrio) {
        const bool want = spread > 0 && __ballot(active && L.head) != 0ull;
        if (want != head_prio) {
          head_prio = want;
          if (want)
            __builtin_amdgcn_s_setprio(3);
          else
            __builtin_amdgcn_s_setprio(0);
        }
      }
    }
    if (__ballot(active) == 0ull) {
      if (drained) break;
      continue;
    }
    // Attempts until a lane finishes its system: only then can the refill
    // rule above fire or the wave run out of work, so the refill bookkeeping
    // is skipped on the other attempts (one ballot each).
    while (true) {
      const uint32_t ph_before = M::kPrio ? L.phase : 0u;
      bool fin = false;
      if (active) {
        bool done;
        if constexpr (M::kEvents)
          done = step_valve<SC>(a, m, L, y, fs);
        else
          done = step_fixed<M, SC, LOC>(a, m, L, y, fs);
        if (done) {
          store_lane<M, SC>(a, L, y, seated_of(m));
          if constexpr (M::kDrive2) cold(a)->phi2[L.sys] = m.phi;
          active = false;
          fin = true;
        }
      }
      // Issue priority follows the wave's longest remaining work, so that the
      // systems that will finish last are not slowed by short ones sharing the
      // SIMD (a wave's own priority; results do not depend on it).
      // (the wave's largest estimate against each level, by ballots)
      if (M::kPrio && a.prioritize && __ballot(active && L.phase != ph_before) != 0ull) {
        const float r = active ? L.rem : 0.0f;
        if (__ballot(r > 1.0e6f) != 0ull)
          __builtin_amdgcn_s_setprio(3);
        else if (__ballot(r > 2.5e5f) != 0ull)
          __builtin_amdgcn_s_setprio(2);
        else if (__ballot(r > 6.0e4f) != 0ull)
          __builtin_amdgcn_s_setprio(1);
        else
          __builtin_amdgcn_s_setprio(0);
      }
      if (__ballot(fin) != 0ull) break;
    }
  }
}

template <class M, int SC, bool LOC>
hipError_t launch_model(int block, int grid, const RkckArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((k_rkck<M, SC, LOC>), dim3(grid), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <class M, int SC, bool LOC>
int max_blocks_model(int block) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rkck<M, SC, LOC>, block, 0) !=
      hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// The kernel instantiation behind a host model id: calls fn(Pick<M, LOC>{})
// and returns its result, or `none` for an id without a kernel.
template <class Mo, bool L>
struct Pick {
  using M = Mo;
  static constexpr bool loc = L;
};

template <class R, class Fn>
R visit_model(int model, bool loc, R none, Fn &&fn) {
  if (model >= kTangentModel) {
    const int K = model / kTangentModel, base = model % kTangentModel;
    if (K == 1) {
      switch (base) {
        case ENS_QUAD: return fn(Pick<MTan<MQuad, 1>, false>{});
        case ENS_LORENZ: return fn(Pick<MTan<MLorenz, 1>, false>{});
        case ENS_KM: return fn(Pick<MTan<MKM<true>, 1>, false>{});
        case ENS_KM_GENERAL: return fn(Pick<MTan<MKM<false>, 1>, false>{});
        case ENS_KM_DUAL: return fn(Pick<MTan<MKM<false, true>, 1>, false>{});
        case ENS_KM_DUAL_FAST: return fn(Pick<MTan<MKM<true, true>, 1>, false>{});
        case ENS_KM6: return fn(Pick<MTan<MKM<true, true, true>, 1>, false>{});
        case ENS_KM6_GENERAL: return fn(Pick<MTan<MKM<false, true, true>, 1>, false>{});
      }
    } else if (K == 2) {
      switch (base) {
        case ENS_LORENZ: return fn(Pick<MTan<MLorenz, 2>, false>{});
        case ENS_KM: return fn(Pick<MTan<MKM<true>, 2>, false>{});
        case ENS_KM_GENERAL: return fn(Pick<MTan<MKM<false>, 2>, false>{});
        case ENS_KM_DUAL: return fn(Pick<MTan<MKM<false, true>, 2>, false>{});
        case ENS_KM_DUAL_FAST: return fn(Pick<MTan<MKM<true, true>, 2>, false>{});
        case ENS_KM6: return fn(Pick<MTan<MKM<true, true, true>, 2>, false>{});
        case ENS_KM6_GENERAL: return fn(Pick<MTan<MKM<false, true, true>, 2>, false>{});
      }
    } else if (K == 3 && base == ENS_LORENZ) {
      return fn(Pick<MTan<MLorenz, 3>, false>{});
    }
    return none;
  }
  switch (model) {
    case ENS_QUAD: return fn(Pick<MQuad, false>{});
    case ENS_LORENZ: return fn(Pick<MLorenz, false>{});
    case ENS_KM:
      return loc ? fn(Pick<MKM<true>, true>{}) : fn(Pick<MKM<true>, false>{});
    case ENS_KM_GENERAL:
      return loc ? fn(Pick<MKM<false>, true>{}) : fn(Pick<MKM<false>, false>{});
    case ENS_KM_DUAL:
      return loc ? fn(Pick<MKM<false, true>, true>{}) : fn(Pick<MKM<false, true>, false>{});
    case ENS_KM_DUAL_FAST:
      return loc ? fn(Pick<MKM<true, true>, true>{}) : fn(Pick<MKM<true, true>, false>{});
    case ENS_KM6:
      return loc ? fn(Pick<MKM<true, true, true>, true>{})
                 : fn(Pick<MKM<true, true, true>, false>{});
    case ENS_KM6_GENERAL:
      return loc ? fn(Pick<MKM<false, true, true>, true>{})
                 : fn(Pick<MKM<false, true, true>, false>{});
    case ENS_PRV: return fn(Pick<MPRV, false>{});
  }
  return none;
}

// Each system's model coefficients, from its parameters and its ensemble's
// shared constants, into the cold pointers' coef array (one system per
// thread, grid-stride).
template <class M>
__global__ __launch_bounds__(256) void k_model_coef(RkckArgs a) {
  const RkckCold *cp = a.cold;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    int e = 0;
    while (e + 1 < a.n_ens && i >= a.desc[e].last) ++e;
    M m;
    m.init(cp->p, a.n, i, a.desc[e].shared);
    m.store_coef(cp->coef, a.n, i);
  }
}

template <int SC>
hipError_t launch_scheme(int model, bool loc, int block, int grid, const RkckArgs &a,
                         hipStream_t s) {
  return visit_model(model, loc, hipErrorInvalidValue, [&](auto pick) {
    using P = decltype(pick);
    return launch_model<typename P::M, SC, P::loc>(block, grid, a, s);
  });
}

template <int SC>
int max_blocks_scheme(int model, bool loc, int block) {
  return visit_model(model, loc, 0, [&](auto pick) {
    using P = decltype(pick);
    return max_blocks_model<typename P::M, SC, P::loc>(block);
  });
}

}  // namespace

namespace {
// Writes the cold pointers to device memory, stream-ordered (one lane).
__global__ void k_set_cold(RkckCold *dst, RkckCold c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = c;
}
}  // namespace

hipError_t launch_set_cold(RkckCold *dst, const RkckCold &c, hipStream_t s) {
  hipLaunchKernelGGL(k_set_cold, dim3(1), dim3(64), 0, s, dst, c);
  return hipGetLastError();
}

hipError_t launch_rkck_coef(int model, const RkckArgs &a, hipStream_t s) {
  return visit_model(model, false, hipSuccess, [&](auto pick) -> hipError_t {
    using M = typename decltype(pick)::M;
    if constexpr (M::kNCoef > 0) {
      static_assert(M::kNCoef <= ENS_MAX_COEF, "coefficient array");
      const int64_t blocks = (a.n + 255) / 256;
      hipLaunchKernelGGL(k_model_coef<M>, dim3((unsigned)(blocks < 4096 ? blocks : 4096)),
                         dim3(256), 0, s, a);
      return hipGetLastError();
    } else {
      return hipSuccess;
    }
  });
}

hipError_t launch_rkck(int model, int solver, int block, int grid, const RkckArgs &a,
                       hipStream_t s) {
  if (block <= 0 || block > kMaxBlock || block % 64 != 0 || grid <= 0)
    return hipErrorInvalidConfiguration;
  const bool loc = a.locate_max != 0;
  if (solver == ENS_RKDP45) return launch_scheme<kDP>(model, loc, block, grid, a, s);
  if (solver == ENS_RKCK45) return launch_scheme<kCK>(model, loc, block, grid, a, s);
  return hipErrorInvalidValue;
}

int rkck_max_blocks(int model, int solver, bool locate_max, int block) {
  if (block <= 0 || block > kMaxBlock || block % 64 != 0) return 0;
  if (solver == ENS_RKDP45) return max_blocks_scheme<kDP>(model, locate_max, block);
  if (solver == ENS_RKCK45) return max_blocks_scheme<kCK>(model, locate_max, block);
  return 0;
}

}  // namespace ens
