// Test harness: the device kernel generator's quadrature (mj_gen.hip, __host__ __device__
// functions) executed serially on the host, so that its logic can be checked against the
// oracle without a GPU.  Built by tests/test_generator_host.py.
#include "../../paper_2407_03323_amd/csrc/mj_gen.hip"

namespace mj {
// K_k(D) for k = 0..kmax at a real offset D (voxel steps), voxel edges (1, hy, hz), c dt = r
// (units of the x edge), nq-point rule
extern "C" void host_kernels(double Dx, double Dy, double Dz, double r, double hy, double hz, int nq, int kmax,
                             double *out)
{
    GenArg ga{};
    ga.nq = nq;
    legendre_rule(nq, ga.glx, ga.glw);
    legendre_rule(3, ga.g3x, ga.g3w);
    const double Ds[3] = {Dx, Dy, Dz};
    const double hv[3] = {1.0, hy, hz}, ih[3] = {1.0, 1.0 / hy, 1.0 / hz};
    double Dv[3], sg[3];
    fold_offset(Ds, Dv, sg);
    int a_lo, nsh;
    shell_range_real(Dv, hv, r, a_lo, nsh);
    const double D[3] = {Dv[0] * hv[0], Dv[1] * hv[1], Dv[2] * hv[2]};
    double mom[kShellCap * kMoments] = {0};
    for (int sh = 0; sh < nsh; sh++)
        for (int it = 0; it < gen_items(nq); it++)
            if (hy != 1.0 || hz != 1.0)
                gen_item<true>(ga.nq, ga.glx, ga.glw, ga.g3x, ga.g3w, D, a_lo + sh, r, hv, ih, it, mom + sh * kMoments);
            else
                gen_item<false>(ga.nq, ga.glx, ga.glw, ga.g3x, ga.g3w, D, a_lo + sh, r, hv, ih, it, mom + sh * kMoments);
    for (int k = 0; k <= kmax; k++) {
        kernel_from_shells(mom, a_lo, nsh, k, r, out + 6 * k);
        finish_offgrid(D, sg, out + 6 * k);
    }
}
}  // namespace mj
