// Host FP64 finite-difference weights by Fornberg's recursion.
//
// B. Fornberg, "Generation of finite difference formulas on arbitrarily
// spaced grids", Math. Comp. 51 (1988) 699-706.  The recursion builds, node
// by node, the weights of every derivative order m <= M on the first n+1
// nodes from those on the first n nodes; it is the numerically stable way to
// obtain the polynomial-interpolation stencils the paper derives at compile
// time (Sec. "Compile-Time Stencil Generation").
#include <cmath>

namespace pf {

// Largest node set and derivative order the library asks for: the fourth
// derivative at accuracy 16 spans 2 (16/2 + 1) + 1 = 19 nodes.  Fixed-size
// arrays keep the generator free of heap allocation (the allocation-free
// step entry point computes its weights on every call).
constexpr int kNodesMax = 19;
constexpr int kDerivMax = 4;

struct FdTable {
    double d[kDerivMax + 1][kNodesMax];  // d[m][k]: m-th derivative weight of node k
};

// Weights of the m-th derivative at x0 on nodes alpha[0..n-1], m = 0..M.
static void fornberg(double x0, const double *alpha, int n, int M, FdTable &cur)
{
    FdTable prev{};
    cur = FdTable{};
    cur.d[0][0] = 1.0;
    double c1 = 1.0;
    for (int i = 1; i < n; ++i) {
        prev = cur;
        double c2 = 1.0;
        const int mmax = i < M ? i : M;
        for (int k = 0; k < i; ++k) {
            const double c3 = alpha[i] - alpha[k];
            c2 *= c3;
            for (int m = mmax; m >= 0; --m) {
                const double lower = m > 0 ? prev.d[m - 1][k] : 0.0;
                cur.d[m][k] = ((alpha[i] - x0) * prev.d[m][k] - m * lower) / c3;
            }
        }
        for (int m = mmax; m >= 0; --m) {
            const double lower = m > 0 ? prev.d[m - 1][i - 1] : 0.0;
            cur.d[m][i] = c1 / c2 * (m * lower - (alpha[i - 1] - x0) * prev.d[m][i - 1]);
        }
        c1 = c2;
    }
}

// Nodes 0, 1, -1, 2, -2, .., rr, -rr (every partial stencil is centred);
// returns the node count.
static int centred_nodes(int rr, double *alpha)
{
    int n = 0;
    alpha[n++] = 0.0;
    for (int j = 1; j <= rr; ++j) {
        alpha[n++] = (double)j;
        alpha[n++] = (double)-j;
    }
    return n;
}

// Centred second-derivative weights w[0..r] (w_{-j} = w_j) for accuracy
// order p = 2r at unit spacing.  The two weights of +j and -j are averaged
// (they agree to rounding).
bool centered_d2_weights(int order, double *w)
{
    if (order < 2 || order % 2 != 0 || order > 16) return false;
    const int r = order / 2;
    double alpha[kNodesMax];
    FdTable t;
    fornberg(0.0, alpha, centred_nodes(r, alpha), 2, t);
    w[0] = t.d[2][0];
    for (int j = 1; j <= r; ++j) w[j] = 0.5 * (t.d[2][2 * j - 1] + t.d[2][2 * j]);
    return true;
}

// Centred first-derivative weights w1[0..r] (w1_{-j} = -w1_j, w1_0 = 0) for
// accuracy order p = 2r at unit spacing (Model H's gradient and divergence);
// the weights of +j and -j are averaged with the sign flipped.
bool centered_d1_weights(int order, double *w1)
{
    if (order < 2 || order % 2 != 0 || order > 16) return false;
    const int r = order / 2;
    double alpha[kNodesMax];
    FdTable t;
    fornberg(0.0, alpha, centred_nodes(r, alpha), 1, t);
    w1[0] = 0.0;
    for (int j = 1; j <= r; ++j) w1[j] = 0.5 * (t.d[1][2 * j - 1] - t.d[1][2 * j]);
    return true;
}

// Centred fourth-derivative weights w4[0..r+1] for accuracy order p = 2r at
// unit spacing (the stencil of the direct biharmonic): 2(r+1)+1 = p+3 nodes,
// the same node order and averaging.
bool centered_d4_weights(int order, double *w4)
{
    if (order < 2 || order % 2 != 0 || order > 16) return false;
    const int r4 = order / 2 + 1;
    double alpha[kNodesMax];
    FdTable t;
    fornberg(0.0, alpha, centred_nodes(r4, alpha), 4, t);
    w4[0] = t.d[4][0];
    for (int j = 1; j <= r4; ++j) w4[j] = 0.5 * (t.d[4][2 * j - 1] + t.d[4][2 * j]);
    return true;
}

}  // namespace pf
