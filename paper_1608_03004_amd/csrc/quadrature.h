// Host-side Gauss rules for the momentum quadrature (see quadrature.cpp).
#pragma once
#include <vector>

namespace rlb {

// Gauss-Legendre rule of order q on [-1, 1], ascending nodes, exactly symmetric.
bool gauss_legendre_rule(int q, std::vector<double>& x, std::vector<double>& w);
// Gauss-Laguerre rule of order q for the weight p e^{-p} on [0, inf), ascending.
bool gauss_laguerre1_rule(int q, std::vector<double>& x, std::vector<double>& w);
// Legendre P_n(x) and generalised Laguerre L^{(1)}_n(x) (extended precision, rounded).
double legendre_value(int n, double x);
double laguerre1_value(int n, double x);

}  // namespace rlb
