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

// The top hat of the original W-stacking (Sec. 6.2): W = 1, C = 1 on the
// unit interval (every polynomial coefficient but the constant is zero), no
// correction (h = 1).
KernelDesign top_hat_design();

// w-layer methods: the improved W-stacking with (eq. n_params) or without
// (eq. n_params_no_offset) the z offset, and the original W-stacking of
// Algorithms 3 and 4 (nearest-midpoint w bins).
enum PlanMethod { kImproved = 0, kImprovedNoOffset = 1, kOriginal = 2 };

struct PlanParams {
    int N = 0, W = 0, Nprime = 0, t_lo = 0, t_hi = 0;
    int Wz = 0;             // width of the w-axis gridding function
    double L = 0, x0 = 0, wmax = 0, l_max = 0, n_min = 0, n_scale = 0, n0 = 0;
    double z0 = 0;          // w-axis cropping (improved methods)
    int method = kImproved;
    int n_bins = 0;         // original W-stacking: N_w
    bool z_offset = true;
    double z_shift = 0;     // (1 - n0) / n_scale: z = (n - 1) / n_scale + z_shift
    double w_shift = 0;     // w' = n_scale w + w_shift (original: -1/2, so layer t holds t <= w / dw < t + 1)
    double t_phase = 0;     // layer t's w-screen uses t + t_phase (original: 1/2, the bin midpoints)
    int n_layers() const { return t_hi - t_lo + 1; }
};

// Validates and fills the plan parameters; returns an empty string on success,
// else the reason.
//   improved methods: w axis of width Wz and cropping z0 (Sec. 5.2 allows a
//     C_z of its own), n_scale and n0 from eq. n_params (z in [-z0, z0]) or eq.
//     n_params_no_offset (n0 = 1, z in [-z0, 0]), layers t_lo = floor(Wz/2) -
//     Wz + 1 .. floor(n_scale wmax + Wz/2);
//   original W-stacking: Wz = 1 (top hat), n_bins bins over [0, wmax] (0: the
//     smallest count of eq. N_w), n_scale = n_bins / wmax, n0 = 1, layers
//     0 .. n_bins - 1 at the midpoints (t + 1/2) / n_scale.
std::string make_plan_params_ext(int N, double L, int W, double x0, int Wz, double z0, double wmax, int method,
                                 int n_bins, PlanParams* p);
// Improved method with the same (W, x0) on all axes; z_offset selects eq.
// n_params or eq. n_params_no_offset.
std::string make_plan_params(int N, double L, int W, double x0, double wmax, PlanParams* p, bool z_offset = true);

}  // namespace wsg
