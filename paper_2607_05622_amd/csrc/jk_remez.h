// Minimax exponential-sum approximation of 1/x (host code).
//
// The Laplace identity 1/x = integral_0^inf exp(-x t) dt is replaced by a
// short sum over a grid {t_k, w_k}, chosen so that the largest absolute
// error of 1/x - sum_k w_k exp(-t_k x) over the denominator range
// [xmin, xmax] is as small as possible (best uniform approximation by an
// exponential sum, Sect. 2, Eq. (laplace) and the minimax-grid paragraph
// around it).  The problem is solved on [1, R], R = xmax / xmin, and
// scaled: t = t'/xmin, w = w'/xmin, error = error'/xmin.
//
// The best approximation is characterized by an error curve that
// equioscillates: it takes its extreme magnitude E with alternating signs
// at 2n + 1 points of [1, R], the two ends included.  The Remez exchange
// finds it: locate the extrema of the current error curve, then solve the
// 2n + 1 equations error(x_i) = (-1)^i E for the n nodes, n weights and E
// by Newton's method (nodes and weights kept positive through their
// logarithms), and repeat until the extrema are level.  The start is a
// sinc (trapezoid in log t) quadrature of the Laplace integral refined by
// damped Gauss-Newton least squares.
#pragma once

#include <vector>

namespace jk {

struct RemezResult {
    std::vector<double> t, w;   // nodes and weights on [1, R]
    double err = 0.0;           // max |1/x - sum w exp(-t x)| on [1, R]
    int iterations = 0;
    bool ok = false;
    bool precision_limited = false;   // fewer terms already reach the FP64 rounding floor
};

RemezResult remez_inverse(int n, double R);

}  // namespace jk
