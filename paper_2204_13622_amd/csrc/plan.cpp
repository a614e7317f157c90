// Host planner: validation, geometry, FP64 even/odd basis (Sec. 4) and the
// packed device image.  Everything here runs once per array geometry.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace fcc {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kGapTol = 1e-9;     // relative gap a rank cut must leave

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// ---- scalar format conversions (round to nearest, ties to even) ---------

uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

uint16_t to_fp16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t sign = (u >> 16) & 0x8000u;
  const uint32_t a = u & 0x7fffffffu;
  if (a >= 0x7f800000u) return uint16_t(sign | (a > 0x7f800000u ? 0x7e00u : 0x7c00u));
  if (a >= 0x477ff000u) return uint16_t(sign | 0x7c00u);           // overflow
  if (a < 0x38800000u) {                                           // subnormal half
    if (a < 0x33000000u) return uint16_t(sign);
    const int e = int(a >> 23);
    const uint32_t mant = (a & 0x7fffffu) | 0x800000u;
    const int shift = 126 - e;                                     // 14 .. 24
    uint32_t q = mant >> shift;
    const uint32_t rem = mant & ((1u << shift) - 1u);
    const uint32_t half = 1u << (shift - 1);
    if (rem > half || (rem == half && (q & 1u))) ++q;
    return uint16_t(sign | q);
  }
  uint32_t v = a - 0x38000000u;                                    // rebias 127 -> 15
  uint32_t q = v >> 13;
  const uint32_t rem = v & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (q & 1u))) ++q;
  return uint16_t(sign | q);
}

// OCP FP8 e4m3 (bias 7, largest finite 448, no infinities); saturating.
uint8_t to_e4m3(float f) {
  if (std::isnan(f)) return 0x7f;
  const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
  double a = std::fabs(double(f));
  if (a >= 464.0) return uint8_t(sign | 0x7e);                     // saturate to 448
  if (a < std::ldexp(1.0, -10)) {                                  // below half the min subnormal
    return sign;
  }
  int e;
  std::frexp(a, &e);                                               // a = m 2^e, m in [0.5, 1)
  int exp_unb = e - 1;                                             // a = 1.x 2^exp_unb
  if (exp_unb < -6) exp_unb = -6;                                  // subnormal range
  const double scale = std::ldexp(1.0, 3 - exp_unb);               // 3 mantissa bits
  double q = a * scale;                                            // in [8, 16) or subnormal
  double fl = std::floor(q);
  double rem = q - fl;
  if (rem > 0.5 || (rem == 0.5 && std::fmod(fl, 2.0) != 0.0)) fl += 1.0;
  if (fl >= 16.0) { fl = 8.0; ++exp_unb; }
  if (exp_unb > 8 || (exp_unb == 8 && fl > 14.0)) return uint8_t(sign | 0x7e);
  if (fl < 8.0) return uint8_t(sign | uint8_t(fl));                // subnormal: exponent field 0
  return uint8_t(sign | uint8_t((exp_unb + 7) << 3) | uint8_t(int(fl) - 8));
}

// cos and sin of 2 pi f / N, reduced to the first octant so that the values
// at multiples of N/8 and the symmetries of the circle hold exactly.
void unit_circle(int f, int N, double& cs, double& sn) {
  f %= N;
  if (f < 0) f += N;
  const int q = (4 * f) / N;                  // quadrant
  const int fr = f - q * (N / 4);             // 0 <= fr < N/4
  double c, s;
  if (2 * fr <= N / 4) {
    const double a = 2.0 * kPi * fr / N;
    c = std::cos(a);
    s = std::sin(a);
  } else {                                    // reflect about pi/4
    const double a = 2.0 * kPi * (N / 4 - fr) / N;
    c = std::sin(a);
    s = std::cos(a);
  }
  if (fr == 0) { c = 1.0; s = 0.0; }
  switch (q) {
    case 0: cs = c; sn = s; break;
    case 1: cs = -s; sn = c; break;
    case 2: cs = -c; sn = -s; break;
    default: cs = s; sn = -c; break;
  }
}

}  // namespace

void jacobi_one_sided(std::vector<double>& B, int n, int q, std::vector<double>& J) {
  J.assign(size_t(q) * q, 0.0);
  for (int i = 0; i < q; ++i) J[size_t(i) * q + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < q - 1; ++p) {
      for (int s = p + 1; s < q; ++s) {
        double* bp = &B[size_t(p) * n];
        double* bs = &B[size_t(s) * n];
        double alpha = 0, beta = 0, gamma = 0;
        for (int i = 0; i < n; ++i) {
          alpha += bp[i] * bp[i];
          beta += bs[i] * bs[i];
          gamma += bp[i] * bs[i];
        }
        if (gamma == 0.0 || std::fabs(gamma) <= 1e-15 * std::sqrt(alpha * beta)) continue;
        rotated = true;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t);
        const double sn = cs * t;
        for (int i = 0; i < n; ++i) {
          const double a = bp[i], b = bs[i];
          bp[i] = cs * a - sn * b;
          bs[i] = sn * a + cs * b;
        }
        double* jp = &J[size_t(p) * q];
        double* js = &J[size_t(s) * q];
        for (int i = 0; i < q; ++i) {
          const double a = jp[i], b = js[i];
          jp[i] = cs * a - sn * b;
          js[i] = sn * a + cs * b;
        }
      }
    }
    if (!rotated) break;
  }
}

namespace {

// Singular triplets of one parity block, sorted by decreasing sigma.
struct Parity {
  int n = 0, q = 0;
  std::vector<double> sigma;        // [q]
  std::vector<double> e_scaled;     // [q][n]  sigma_k e_k  (rows of S V^T, centred coords)
  std::vector<double> Ured;         // [q][q]  left vectors on the reduced lag set
};

// The reduced matrices: rows of W (eq. 3) times exp(-j pi tau / 2), restricted to
// real vectors symmetric (cosine) or antisymmetric (sine) about f = N/4.  Rows
// tau and -tau coincide (cosine) or are opposite (sine), so each distinct |tau|
// appears once, scaled by sqrt(2) when it stands for two rows.
Parity solve_parity(const Plan& pl, bool sym) {
  Parity out;
  const int m = pl.m;
  const int rt = pl.r * pl.tau_max;            // lags j / r, j = 0 .. rt
  std::vector<int> rows;
  for (int j = sym ? 0 : 1; j <= rt; ++j) rows.push_back(j);
  out.q = int(rows.size());
  out.n = sym ? m + 1 : m;
  const int n = out.n, q = out.q;
  if (q == 0) return out;
  std::vector<double> B(size_t(q) * n);        // column k = reduced row k, transposed
  for (int k = 0; k < q; ++k) {
    const double tau = double(rows[k]) / pl.r;
    const double w = (rows[k] == 0) ? 1.0 : std::sqrt(2.0);
    for (int f = 0; f < m; ++f) {
      const double ang = 2.0 * kPi * double(f - m) * tau / pl.N;
      B[size_t(k) * n + f] = w * std::sqrt(2.0) * (sym ? std::cos(ang) : std::sin(ang));
    }
    if (sym) B[size_t(k) * n + m] = w * 1.0;
  }
  std::vector<double> J;
  jacobi_one_sided(B, n, q, J);
  std::vector<double> nrm(q);
  for (int k = 0; k < q; ++k) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += B[size_t(k) * n + i] * B[size_t(k) * n + i];
    nrm[k] = std::sqrt(s);
  }
  std::vector<int> order(q);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  out.sigma.resize(q);
  out.e_scaled.resize(size_t(q) * n);
  out.Ured.resize(size_t(q) * q);
  for (int kk = 0; kk < q; ++kk) {
    const int k = order[kk];
    const double* col = &B[size_t(k) * n];
    double mx = 0;
    for (int i = 0; i < n; ++i) mx = std::max(mx, std::fabs(col[i]));
    double sgn = 1.0;
    for (int i = 0; i < n; ++i) {
      if (std::fabs(col[i]) > 1e-6 * mx) { sgn = col[i] > 0 ? 1.0 : -1.0; break; }
    }
    out.sigma[kk] = nrm[k];
    for (int i = 0; i < n; ++i) out.e_scaled[size_t(kk) * n + i] = sgn * col[i];
    for (int i = 0; i < q; ++i) out.Ured[size_t(kk) * q + i] = sgn * J[size_t(k) * q + i];
  }
  return out;
}

fcc_status fail(std::string& err, fcc_status st, const std::string& msg) {
  err = msg;
  return st;
}

}  // namespace

// An enum field of the C configuration as the integer the caller stored: a C
// caller may store any int there, and reading it as the C++ enum type would
// be undefined outside the enumerators' range.
static int32_t enum_bits(const void* field) {
  int32_t v;
  std::memcpy(&v, field, sizeof v);
  return v;
}

fcc_status build_plan(const fcc_config& cfg, Plan& pl, std::string& err) {
  static_assert(sizeof(fcc_precision) == 4 && sizeof(fcc_method) == 4 && sizeof(fcc_operands) == 4,
                "C enums are int-sized");
  const int32_t precision = enum_bits(&cfg.precision), method = enum_bits(&cfg.method),
                operands = enum_bits(&cfg.operands);
  if (precision < FCC_FP32 || precision > FCC_FP8_E4M3) return fail(err, FCC_ERR_INVALID_ARG, "unknown precision");
  if (method != FCC_METHOD_FCC && method != FCC_METHOD_GCC) return fail(err, FCC_ERR_INVALID_ARG, "unknown method");
  if (operands != FCC_OPERANDS_FP16 && operands != FCC_OPERANDS_STORAGE)
    return fail(err, FCC_ERR_INVALID_ARG, "unknown operand type");
  if (cfg.num_mics < 2) return fail(err, FCC_ERR_INVALID_ARG, "num_mics must be >= 2");
  if (cfg.num_mics > 32) return fail(err, FCC_ERR_UNSUPPORTED, "num_mics > 32 is not built");
  if (!cfg.mic_xyz) return fail(err, FCC_ERR_INVALID_ARG, "mic_xyz is NULL");
  if (!is_pow2(cfg.frame_size) || cfg.frame_size < 16 || cfg.frame_size > 2048)
    return fail(err, FCC_ERR_INVALID_ARG, "frame_size must be a power of two in [16, 2048]");
  if (cfg.hop <= 0) return fail(err, FCC_ERR_INVALID_ARG, "hop must be > 0");
  if (!(cfg.fs > 0) || !std::isfinite(cfg.fs)) return fail(err, FCC_ERR_INVALID_ARG, "fs must be > 0");
  if (!(cfg.c > 0) || !std::isfinite(cfg.c)) return fail(err, FCC_ERR_INVALID_ARG, "c must be > 0");
  if (cfg.interp != 1 && cfg.interp != 2 && cfg.interp != 4)
    return fail(err, FCC_ERR_INVALID_ARG, "interp must be 1, 2 or 4");
  if (cfg.method == FCC_METHOD_GCC && cfg.interp * cfg.frame_size > 4096)
    return fail(err, FCC_ERR_UNSUPPORTED, "GCC inverse transforms above 4096 points are not built");
  if (!(cfg.alpha > 0.0f && cfg.alpha <= 1.0f)) return fail(err, FCC_ERR_INVALID_ARG, "alpha must be in (0, 1]");
  if (cfg.alpha < 1.0f && cfg.precision != FCC_FP32)
    return fail(err, FCC_ERR_UNSUPPORTED, "alpha < 1 is built for FP32 spectra only");
  if (cfg.alpha < 1.0f && cfg.method != FCC_METHOD_FCC)
    return fail(err, FCC_ERR_UNSUPPORTED, "alpha < 1 is built for the FCC method only");
  if (cfg.tau_max < 0) return fail(err, FCC_ERR_INVALID_ARG, "tau_max must be >= 0");
  if (cfg.rank < 0) return fail(err, FCC_ERR_INVALID_ARG, "rank must be >= 0");

  pl.M = cfg.num_mics;
  pl.P = pl.M * (pl.M - 1) / 2;
  pl.N = cfg.frame_size;
  pl.hop = cfg.hop;
  pl.F = pl.N / 2 + 1;
  pl.m = pl.N / 4;
  pl.fs = cfg.fs;
  pl.c = cfg.c;
  pl.r = cfg.interp;
  pl.alpha = cfg.alpha;
  pl.precision = cfg.precision;
  pl.method = cfg.method;
  pl.operands = cfg.operands;
  pl.xyz.assign(cfg.mic_xyz, cfg.mic_xyz + 3 * size_t(pl.M));
  for (double v : pl.xyz)
    if (!std::isfinite(v)) return fail(err, FCC_ERR_INVALID_ARG, "mic_xyz has a non-finite entry");

  // Sec. 2: tau = f_S (d / c) cos(theta); the window must hold the largest pair.
  if (cfg.tau_max > 0) {
    pl.tau_max = cfg.tau_max;
  } else {
    double dmax = 0;
    for (int i = 0; i < pl.M; ++i)
      for (int j = i + 1; j < pl.M; ++j) {
        const double dx = pl.xyz[3 * i] - pl.xyz[3 * j];
        const double dy = pl.xyz[3 * i + 1] - pl.xyz[3 * j + 1];
        const double dz = pl.xyz[3 * i + 2] - pl.xyz[3 * j + 2];
        dmax = std::max(dmax, std::sqrt(dx * dx + dy * dy + dz * dz));
      }
    pl.tau_max = int(std::ceil(dmax * pl.fs / pl.c));
  }
  if (pl.r * pl.tau_max >= pl.m)
    return fail(err, FCC_ERR_INVALID_ARG, "r tau_max must be < N/4 (lag window inside the frame)");
  pl.I = 2 * pl.r * pl.tau_max + 1;
  if (pl.method == FCC_METHOD_GCC) {
    pl.D = pl.I;
  } else {
    pl.D = cfg.rank == 0 ? pl.I : cfg.rank;
    if (pl.D > pl.I) return fail(err, FCC_ERR_INVALID_ARG, "rank must be <= I = 2 r tau_max + 1");
    if (pl.D > 64) return fail(err, FCC_ERR_UNSUPPORTED, "rank above 64 is not built");
  }
  pl.Ds = (pl.D + 1) / 2;
  pl.Da = pl.D / 2;

  // ---- basis (Sec. 4): SVD per parity, alternating order of eq. (6) ------
  const Parity S = solve_parity(pl, true);
  const Parity A = solve_parity(pl, false);
  const double smax = std::max(S.q ? S.sigma[0] : 0.0, A.q ? A.sigma[0] : 0.0);
  if (pl.D < pl.I) {
    if (pl.Ds > 0 && pl.Ds < S.q && S.sigma[pl.Ds - 1] - S.sigma[pl.Ds] <= kGapTol * smax)
      return fail(err, FCC_ERR_BASIS_AMBIGUOUS, "rank cuts a cluster of symmetric singular values");
    if (pl.Da > 0 && pl.Da < A.q && A.sigma[pl.Da - 1] - A.sigma[pl.Da] <= kGapTol * smax)
      return fail(err, FCC_ERR_BASIS_AMBIGUOUS, "rank cuts a cluster of antisymmetric singular values");
  }
  const int D = pl.D, I = pl.I, m = pl.m;
  const double inv_r2 = 1.0 / std::sqrt(2.0);
  pl.sigma.assign(D, 0.0);
  pl.is_sym.assign(D, 0);
  pl.p_hat.assign(size_t(D) * (m + 1), 0.0);
  pl.dc.assign(size_t(I) * D, 0.0);
  pl.ds.assign(size_t(I) * D, 0.0);
  const int rt = pl.r * pl.tau_max;
  for (int k = 0; k < D; ++k) {
    const bool sym = (k % 2 == 0);
    const Parity& B = sym ? S : A;
    const int idx = k / 2;
    pl.sigma[k] = B.sigma[idx];
    pl.is_sym[k] = sym ? 1 : 0;
    const double* e = &B.e_scaled[size_t(idx) * B.n];
    for (int f = 0; f < m; ++f) pl.p_hat[size_t(k) * (m + 1) + f] = e[f] * inv_r2;
    pl.p_hat[size_t(k) * (m + 1) + m] = sym ? e[m] : 0.0;
    const double* u = &B.Ured[size_t(idx) * B.q];
    for (int i = 0; i < I; ++i) {
      const int j = i - rt;                      // tau_i = j / r
      const int aj = j < 0 ? -j : j;
      double ured;                               // left vector on the full lag grid
      if (sym) ured = (aj == 0) ? u[0] : u[aj] * inv_r2;
      else ured = (aj == 0) ? 0.0 : (j > 0 ? 1.0 : -1.0) * u[aj - 1] * inv_r2;
      // exp(j pi tau / 2); quarter turns are exact when r = 1
      double ph_re, ph_im;
      if (pl.r == 1) {
        const int q4 = ((j % 4) + 4) % 4;
        ph_re = (q4 == 0) ? 1.0 : (q4 == 2 ? -1.0 : 0.0);
        ph_im = (q4 == 1) ? 1.0 : (q4 == 3 ? -1.0 : 0.0);
      } else {
        const double a = kPi * double(j) / (2.0 * pl.r);
        ph_re = std::cos(a);
        ph_im = std::sin(a);
      }
      // symmetric: u = exp(j pi tau/2) U ; antisymmetric: u = j exp(j pi tau/2) U
      const double re = sym ? ph_re * ured : -ph_im * ured;
      const double im = sym ? ph_im * ured : ph_re * ured;
      pl.dc[size_t(i) * D + k] = re;
      pl.ds[size_t(i) * D + k] = im;
    }
  }

  // ---- device image --------------------------------------------------------
  pl.spec_elem = pl.precision == FCC_FP32 ? 8 : (pl.precision == FCC_FP8_E4M3 ? 2 : 4);
  ImageLayout& L = pl.layout;
  size_t off = 0;
  L.twiddle = off; off = align256(off + 2 * sizeof(float) * pl.N);
  L.twiddle_r = off; off = align256(off + 2 * sizeof(float) * size_t(pl.r) * pl.N);
  L.pairs = off;   off = align256(off + 2 * size_t(pl.P));
  L.basis32 = off; off = align256(off + sizeof(float) * size_t(D) * (m + 1));
  L.dict = off;    off = align256(off + sizeof(float) * size_t(I) * 2 * D);
  L.lagw = off;    off = align256(off + 2 * sizeof(float) * size_t(I) * pl.F);
  const int NH = pl.N / 2;
  {
    // the matrix-core pair kernel is instantiated for 1, 2, 3, 4, 6 or 8
    // blocks of four components; pad D to one of those
    int kb = (D + 3) / 4;
    if (kb == 5) kb = 6;
    if (kb == 7) kb = 8;
    pl.Dpad = 4 * kb;
  }
  pl.Ipad = (I + 15) / 16 * 16;
  L.prow32 = off;  off = align256(off + 2 * sizeof(float) * size_t(pl.Dpad) * NH);
  L.prow16 = off;  off = align256(off + 2 * sizeof(uint16_t) * size_t(pl.Dpad) * NH);
  L.gexp = off;    off = align256(off + sizeof(float) * size_t(pl.Ipad) * pl.Dpad);
  L.prow_op = off; off = align256(off + 2 * sizeof(uint16_t) * size_t(pl.Dpad) * NH);
  L.gexp_op = off; off = align256(off + sizeof(float) * size_t(pl.Ipad) * pl.Dpad);
  pl.Dfold = 0;
  for (int c : {4, 8, 12, 16, 24, 32, 48, 64})
    if (D <= c) { pl.Dfold = c; break; }
  L.pfold = off;   off = align256(off + sizeof(float) * size_t(pl.Dfold) * (m + 1));
  L.total = off;
  pl.image.assign(L.total, 0);
  unsigned char* img = pl.image.data();
  auto fput = [&](size_t base, size_t i, double v) {
    const float f = float(v);
    std::memcpy(img + base + 4 * i, &f, 4);
  };
  for (int f = 0; f < pl.N; ++f) {
    // exp(-j 2 pi f / N) from the first octant, so the quarter points are exact
    double cs, sn;
    unit_circle(f, pl.N, cs, sn);
    fput(L.twiddle, 2 * f, cs);
    fput(L.twiddle, 2 * f + 1, -sn);
  }
  for (int f = 0; f < pl.r * pl.N; ++f) {
    double cs, sn;
    unit_circle(f, pl.r * pl.N, cs, sn);
    fput(L.twiddle_r, 2 * f, cs);
    fput(L.twiddle_r, 2 * f + 1, -sn);
  }
  {
    int p = 0;
    for (int i = 0; i < pl.M; ++i)
      for (int j = i + 1; j < pl.M; ++j, ++p) {
        img[L.pairs + 2 * p] = uint8_t(i);
        img[L.pairs + 2 * p + 1] = uint8_t(j);
      }
  }
  for (size_t i = 0; i < size_t(D) * (m + 1); ++i) fput(L.basis32, i, pl.p_hat[i]);
  for (int i = 0; i < I; ++i)
    for (int k = 0; k < D; ++k) {
      fput(L.dict, size_t(i) * 2 * D + 2 * k, 2.0 * pl.dc[size_t(i) * D + k]);
      fput(L.dict, size_t(i) * 2 * D + 2 * k + 1, -2.0 * pl.ds[size_t(i) * D + k]);
    }
  // full-length rows: p_k(f) = p_hat_k(f) for f <= N/4, +-p_hat_k(N/2 - f) above
  auto prow = [&](int k, int f) {
    const double* ph = &pl.p_hat[size_t(k) * (m + 1)];
    if (f <= m) return ph[f];
    return (pl.is_sym[k] ? 1.0 : -1.0) * ph[pl.N / 2 - f];
  };
  for (int k = 0; k < D; ++k)
    for (int f = 0; f < NH; ++f) {
      const double lo = prow(k, f), hi = (f == 0) ? prow(k, NH) : lo;
      fput(L.prow32, 2 * (size_t(k) * NH + f), lo);
      fput(L.prow32, 2 * (size_t(k) * NH + f) + 1, hi);
      const uint16_t hlo = to_fp16(float(lo)), hhi = to_fp16(float(hi));
      std::memcpy(img + L.prow16 + 4 * (size_t(k) * NH + f), &hlo, 2);
      std::memcpy(img + L.prow16 + 4 * (size_t(k) * NH + f) + 2, &hhi, 2);
    }
  for (int i = 0; i < I; ++i)
    for (int k = 0; k < D; ++k)
      fput(L.gexp, size_t(i) * pl.Dpad + k, pl.dc[size_t(i) * D + k] - pl.ds[size_t(i) * D + k]);
  // operands in the storage type: BF16 rows as they are; e4m3 products need
  // the rows scaled into e4m3's range, by a power of two per component
  // (exact), which the dictionary takes back
  for (int k = 0; k < D; ++k) {
    double pmax = 0.0;
    for (int f = 0; f <= m; ++f) pmax = std::max(pmax, std::fabs(pl.p_hat[size_t(k) * (m + 1) + f]));
    int e = 0;
    if (pl.precision == FCC_FP8_E4M3 && pmax > 0.0) {
      e = int(std::floor(std::log2(240.0 / pmax)));
      while (std::ldexp(pmax, e) > 240.0) --e;
      while (std::ldexp(pmax, e + 1) <= 240.0) ++e;
    }
    for (int f = 0; f < NH; ++f) {
      const double lo = std::ldexp(prow(k, f), e), hi = std::ldexp((f == 0) ? prow(k, NH) : prow(k, f), e);
      uint16_t wlo, whi;
      if (pl.precision == FCC_BF16) {
        wlo = to_bf16(float(lo));
        whi = to_bf16(float(hi));
      } else {
        wlo = to_fp16(float(lo));
        whi = to_fp16(float(hi));
      }
      std::memcpy(img + L.prow_op + 4 * (size_t(k) * NH + f), &wlo, 2);
      std::memcpy(img + L.prow_op + 4 * (size_t(k) * NH + f) + 2, &whi, 2);
    }
    for (int i = 0; i < I; ++i)
      fput(L.gexp_op, size_t(i) * pl.Dpad + k,
           std::ldexp(pl.dc[size_t(i) * D + k] - pl.ds[size_t(i) * D + k], -e));
  }
  for (int k = 0; k < D && k < pl.Dfold; ++k)      // transposed: row f holds p_hat_k(f) for all k
    for (int f = 0; f <= m; ++f) fput(L.pfold, size_t(f) * pl.Dfold + k, pl.p_hat[size_t(k) * (m + 1) + f]);
  for (int i = 0; i < I; ++i) {
    const double tau = double(i) / pl.r - pl.tau_max;
    for (int f = 0; f < pl.F; ++f) {
      const double a = 2.0 * kPi * f * tau / pl.N;
      fput(L.lagw, 2 * (size_t(i) * pl.F + f), std::cos(a));
      fput(L.lagw, 2 * (size_t(i) * pl.F + f) + 1, std::sin(a));
    }
  }
  return FCC_OK;
}

}  // namespace fcc
