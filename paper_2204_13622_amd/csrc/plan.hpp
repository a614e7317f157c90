// Host-side plan of the FCC library: configuration, FP64 basis and the packed
// device image.  Pure C++17; no HIP calls.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "fcc.h"

namespace fcc {

// Offsets (bytes) of the tables inside the device image; each is 256-aligned.
struct ImageLayout {
  size_t twiddle = 0;     // float2 [N]          exp(-j 2 pi f / N), full circle
  size_t twiddle_r = 0;   // float2 [r N]        exp(-j 2 pi f / (r N)) (GCC inverse transform)
  size_t pairs = 0;       // uint8 [P][2]        (i, j), lexicographic
  size_t basis32 = 0;     // float [D][Bs]       p_hat rows, Bs = N/4 + 1
  size_t dict = 0;        // float [I][2D]       (2 Dc, -2 Ds) interleaved per k
  size_t lagw = 0;        // float2 [I][F]       exp(j 2 pi f tau_i / N) (GCC)
  // matrix-core pair stage: full-length rows p_k(f), f = 0 .. N/2, as pairs
  // matching the packed spectrum slots: slot 0 -> (p_k(0), p_k(N/2)),
  // slot f -> (p_k(f), p_k(f)); rows k >= D are zero.
  size_t prow32 = 0;      // float2 [Dpad][N/2]
  size_t prow16 = 0;      // half2  [Dpad][N/2]
  size_t gexp = 0;        // float [Ipad][Dpad]  G(tau_i, k) = Dc - Ds; zero padded
  // operands in the storage type: BF16 pairs (bf16 plans) or FP16 pairs of
  // 2^e_k p_k (e4m3 plans, e_k putting max |2^e_k p_k| in (120, 240]), and G
  // with column k divided by 2^e_k
  size_t prow_op = 0;     // [Dpad][N/2] 4 bytes per slot
  size_t gexp_op = 0;     // float [Ipad][Dpad]
  size_t pfold = 0;       // float [N/4 + 1][Dfold] p_hat, transposed, for the FP32 fold kernel
  size_t total = 0;
};

struct Plan {
  // configuration
  int M = 0, P = 0, N = 0, hop = 0, F = 0, m = 0;
  int tau_max = 0, r = 1, I = 0, D = 0, Ds = 0, Da = 0;
  double fs = 0, c = 0;
  float alpha = 1.0f;
  fcc_precision precision = FCC_FP32;
  fcc_method method = FCC_METHOD_FCC;
  fcc_operands operands = FCC_OPERANDS_FP16;
  std::vector<double> xyz;          // [M][3]

  // FP64 basis in component order S, A, S, A, ... (eq. 6)
  std::vector<double> sigma;        // [D]
  std::vector<int32_t> is_sym;      // [D]
  std::vector<double> p_hat;        // [D][m + 1]
  std::vector<double> dc, ds;       // [I][D]

  // packed device image
  ImageLayout layout;
  std::vector<unsigned char> image;
  int Dpad = 0, Ipad = 0;           // D and I rounded up to the MFMA tiles (4, 16)
  int Dfold = 0;                    // D rounded up to 4, 8, 12, 16, 24, 32, 48 or 64
  int spec_elem = 8;                // bytes per complex spectrum element
};

// Builds a plan; on error returns the status and fills `err`.
fcc_status build_plan(const fcc_config& cfg, Plan& plan, std::string& err);

// One-sided (Hestenes) Jacobi SVD of B given as q columns of length n
// (column-major, n >= q).  On return the columns of B are B0 J with mutually
// orthogonal columns and J (q x q, column-major) is orthogonal.
void jacobi_one_sided(std::vector<double>& B, int n, int q, std::vector<double>& J);

}  // namespace fcc
