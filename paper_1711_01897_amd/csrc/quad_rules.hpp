// Symmetric Gauss rules on the reference triangle {(0,0),(1,0),(0,1)}, used by
// the device kernels.  Weights sum to 1/2 (the reference area); point k has
// barycentric coordinates (l0, l1, l2) with xi = l1, eta = l2.
//
// 6 points, degree 4 (Section 3.2.1: the symmetric rule of order 4 with six
// weights): two orbits (1-2a, a, a) of three points each, with the published
// values (Strang & Fix; Dunavant 1985, degree-4 table)
//   a1 = 0.445948490915965, w1 = 0.223381589678011 (weights summing to one)
//   a2 = 0.091576213509771, w2 = 0.109951743655322
// 4 points, degree 3: the centroid with weight -27/48 and the orbit
// (3/5, 1/5, 1/5) with weight 25/48 each (Strang & Fix).
#pragma once

namespace bem {
namespace rule {

constexpr double kA1 = 0.44594849091596488632;
constexpr double kA2 = 0.091576213509770743460;
constexpr double kW1 = 0.22338158967801146570 * 0.5;
constexpr double kW2 = 0.10995174365532186764 * 0.5;

template <int Q>
struct Rule;

template <>
struct Rule<6> {
    static constexpr double w[6] = {kW1, kW1, kW1, kW2, kW2, kW2};
    static constexpr double l0[6] = {1.0 - 2.0 * kA1, kA1, kA1, 1.0 - 2.0 * kA2, kA2, kA2};
    static constexpr double l1[6] = {kA1, 1.0 - 2.0 * kA1, kA1, kA2, 1.0 - 2.0 * kA2, kA2};
    static constexpr double l2[6] = {kA1, kA1, 1.0 - 2.0 * kA1, kA2, kA2, 1.0 - 2.0 * kA2};
};

template <>
struct Rule<4> {
    static constexpr double w[4] = {-27.0 / 96.0, 25.0 / 96.0, 25.0 / 96.0, 25.0 / 96.0};
    static constexpr double l0[4] = {1.0 / 3.0, 0.6, 0.2, 0.2};
    static constexpr double l1[4] = {1.0 / 3.0, 0.2, 0.6, 0.2};
    static constexpr double l2[4] = {1.0 / 3.0, 0.2, 0.2, 0.6};
};

// Barycentric basis value of local vertex e at point p.
template <int Q>
constexpr double lam(int e, int p) {
    return e == 0 ? Rule<Q>::l0[p] : (e == 1 ? Rule<Q>::l1[p] : Rule<Q>::l2[p]);
}

}  // namespace rule
}  // namespace bem
