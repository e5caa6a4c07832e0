// Test harness: the device generator's quadrature on the host (through gen_host.cpp) for cubic
// and unequal voxel edges and short steps, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side by tests/test_sanitizers.py.
#include "gen_host.cpp"

#include <cmath>
#include <cstdio>

int main()
{
    const double cases[][6] = {
        // Dx, Dy, Dz, r, hy, hz
        {0, 0, 0, 1.0, 1.0, 1.0}, {2, -1, 3, 1.0, 1.0, 1.0}, {1.3, -0.7, 0.45, 1.0, 1.0, 1.0},
        {1, 1, 1, 0.3, 1.0, 1.0}, {0, 1, 1, 0.7, 0.7, 1.3},    {-3, 2, 1, 0.6, 1.5, 2.0},
    };
    double sum = 0.0;
    for (const auto &c : cases) {
        const double b = std::sqrt(std::pow((std::fabs(c[0]) + 1), 2) + std::pow((std::fabs(c[1]) + 1) * c[4], 2) +
                                   std::pow((std::fabs(c[2]) + 1) * c[5], 2));
        const int kmax = (int)(b / c[3]) + 3;
        double out[6 * 64];
        if (kmax >= 64) return 2;
        mj::host_kernels(c[0], c[1], c[2], c[3], c[4], c[5], 8, kmax, out);
        for (int i = 0; i < 6 * (kmax + 1); i++) sum += out[i];
    }
    std::printf("checksum %.17g\n", sum);
    return 0;
}
