// Valid-subaperture rule of the aperture masks (§2.F): a subaperture of the
// n x n grid laid over the square [-D/2, D/2]^2 is kept when at least half of
// its area lies inside the annular pupil (outer diameter D, inner diameter
// obstruction * D).  Host code only; the areas are exact.
//
// Area of an axis-aligned rectangle inside a disk of radius R centred at the
// origin, by inclusion-exclusion over the corner quadrant areas
//   Q(a, b) = | [0, a] x [0, b]  intersected with the disk |,  a, b >= 0,
// extended to signed corners by the symmetry of the disk.  With a' = min(a, R),
// b' = min(b, R) and x_c = sqrt(R^2 - b'^2) (the abscissa where the circle
// crosses y = b'):
//   Q = b' min(x_c, a') + F(a') - F(min(x_c, a')),
//   F(x) = (x sqrt(R^2 - x^2) + R^2 asin(x / R)) / 2   (the integral of sqrt(R^2 - x^2)).
#include <algorithm>
#include <cmath>

#include "tt_internal.h"

namespace {

double quad_area(double a, double b, double R) {
    if (a <= 0.0 || b <= 0.0 || R <= 0.0) return 0.0;
    a = std::min(a, R);
    b = std::min(b, R);
    if (a * a + b * b <= R * R) return a * b;
    const double xc = std::sqrt(std::max(R * R - b * b, 0.0));
    auto F = [R](double x) { return 0.5 * (x * std::sqrt(std::max(R * R - x * x, 0.0)) + R * R * std::asin(std::min(x / R, 1.0))); };
    const double x0 = std::min(xc, a);
    return b * x0 + F(a) - F(x0);
}

double corner(double x, double y, double R) {
    const double sx = x < 0 ? -1.0 : 1.0, sy = y < 0 ? -1.0 : 1.0;
    return sx * sy * quad_area(std::fabs(x), std::fabs(y), R);
}

double rect_disk(double x0, double x1, double y0, double y1, double R) {
    return corner(x1, y1, R) - corner(x0, y1, R) - corner(x1, y0, R) + corner(x0, y0, R);
}

}  // namespace

tt_status pupil_rule(int n, double D, double obstruction, unsigned char* out, int* n_valid) {
    TT_REQUIRE(out != nullptr, "out is NULL");
    TT_REQUIRE(n >= 1 && n <= 512, "n must be in [1, 512]");
    TT_REQUIRE(std::isfinite(D) && D > 0, "D must be positive");
    TT_REQUIRE(std::isfinite(obstruction) && obstruction >= 0 && obstruction < 1, "obstruction must be in [0, 1)");
    const double d = D / n, Ro = 0.5 * D, Ri = 0.5 * obstruction * D;
    int cnt = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const double x0 = (j - 0.5 * n) * d, y0 = (i - 0.5 * n) * d;
            const double a = rect_disk(x0, x0 + d, y0, y0 + d, Ro) - rect_disk(x0, x0 + d, y0, y0 + d, Ri);
            const bool keep = a >= 0.5 * d * d;
            out[(size_t)i * n + j] = keep ? 1 : 0;
            cnt += keep;
        }
    if (n_valid) *n_valid = cnt;
    return TT_OK;
}

extern "C" tt_status tt_pupil_mask(int n, double D, double obstruction, unsigned char* out, int* n_valid) {
    try {
        return pupil_rule(n, D, obstruction, out, n_valid);
    } catch (...) {
        tt_set_error("tt_pupil_mask: exception");
        return TT_HIP_ERROR;
    }
}
