// Host-side least-misfit kernel design and planner (float64).
#pragma once
#include <string>
#include <vector>

namespace wsg {

// Least-misfit gridding function C and correction h for width W and cropping
// parameter x0 (Sec. 3.3): minimises E of eq. norm_bound built from the
// residual L of eq. csum2.  Segments a = 0..W-1 carry c_a(nu) = C(s_a - nu),
// s_a = a - (W-1)/2, nu in [-1/2, 1/2].
struct KernelDesign {
    int W = 0;
    double x0 = 0;
    std::vector<double> xn, wx;      // Gauss-Legendre nodes/weights on [0, x0]
    std::vector<double> nun, wn;     // Gauss-Legendre nodes/weights on [-1/2, 1/2]
    std::vector<double> h;           // h at xn, scaled so that h(0) = 1
    std::vector<double> A;           // W x W normal matrix for h
    std::vector<double> c_nodes;     // [nun.size()][W] c at the nu nodes
    int degree = 0;                  // per-segment polynomial degree in nu (float64 path)
    std::vector<double> poly;        // [W][degree+1] monomial coefficients in nu
    int degree_lo = 0;               // lower degree for the float32 path
    std::vector<double> poly_lo;     // [W][degree_lo+1]
    double E = 0;                    // error bound, evaluated on a finer grid
    int iterations = 0;

    void c_exact(double nu, double* c) const;       // normal equations, W values
    double c_poly(int a, double nu) const;          // fitted polynomial (float64 path)
    double c_poly_lo(int a, double nu) const;       // fitted polynomial (float32 path)
    double h_at(double x) const;                    // pointwise optimality formula
};

// Throws std::runtime_error on a bad argument.
KernelDesign design_kernel(int W, double x0);

struct PlanParams {
    int N = 0, W = 0, Nprime = 0, t_lo = 0, t_hi = 0;
    double L = 0, x0 = 0, wmax = 0, l_max = 0, n_min = 0, n_scale = 0, n0 = 0;
    bool z_offset = true;
    double z_shift = 0;     // (1 - n0) / n_scale: z = (n - 1) / n_scale + z_shift
    int n_layers() const { return t_hi - t_lo + 1; }
};

// Validates and fills the plan parameters; returns an empty string on success,
// else the reason.
// z_offset selects eq. n_params (z in [-z0, z0]) or, when false, the variant
// without z offset, eq. n_params_no_offset (n0 = 1, z in [-z0, 0]; Sec. 5.3).
std::string make_plan_params(int N, double L, int W, double x0, double wmax, PlanParams* p, bool z_offset = true);

}  // namespace wsg
