// d3q19.h -- D3Q19 velocity set of the GPU path.
//
// The paper's lattice is D2Q9 (Sec. II.A); this is its three-dimensional
// generalisation: the rest link, the 6 axis links and the 12 face diagonals,
// weights 1/3, 1/18, 1/36, c_s^2 = 1/3.  Opposite links are adjacent
// (opp(i) = i + 1 for odd i), so bounce-back is an index flip.
//
// Derived constants, one value per shell (rest, axis, diagonal):
//   phi_i(alpha) = alpha (rest), (1 - alpha) / 12 (axis), (1 - alpha) / 24
//     (diagonal): the modified equilibrium's rest-frame weights; the paper's
//     D2Q9 table alpha, (1-alpha)/5, (1-alpha)/20 follows the same rule
//     phi_i = (1 - alpha) w_i / (1 - w_0).
//   B_i = -2/9, 1/54, 1/27: the perturbation operator's coefficients, from
//     B_i = w_i (|c_i|^2 - 2/3), the rule that gives the paper's printed D2Q9
//     values -4/27, 2/27, 5/108 with (D-1)/3 = 1/3.
#pragma once

namespace lbq {

constexpr int Q = 19;

__host__ __device__ constexpr int cx(int i)
{
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cy(int i)
{
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz(int i)
{
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
}
// 0 = rest, 1 = axis, 2 = face diagonal
__host__ __device__ constexpr int shell(int i) { return i == 0 ? 0 : (i <= 6 ? 1 : 2); }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

__host__ __device__ constexpr double w_of_shell(int s) { return s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr double w(int i) { return w_of_shell(shell(i)); }
__host__ __device__ constexpr double B_of_shell(int s) { return s == 0 ? -2.0 / 9.0 : (s == 1 ? 1.0 / 54.0 : 1.0 / 27.0); }
// 1 / |c_i| for i > 0
__host__ __device__ constexpr double inv_len(int i) { return shell(i) == 1 ? 1.0 : 0.70710678118654752440; }

constexpr double CS2 = 1.0 / 3.0;

}  // namespace lbq
