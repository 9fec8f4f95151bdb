// Host-side check of the library's Chebyshev coefficients of the Fermi-Dirac
// operator (built by tests/test_host_fermi.py against the library's host.cpp;
// no GPU involved).
//
//   host_fermi_check <beta> <mu> <rescale> <tol> <out.bin>
//
// Writes the coefficients a_k (f(H) = sum_k a_k T_k(H / rescale)) as raw
// doubles to out.bin; exit status 3 if the library declines the expansion.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2209_00806_amd/csrc/tbpm_internal.h"

int main(int argc, char **argv) {
    if (argc != 6) {
        std::fprintf(stderr, "usage: %s beta mu rescale tol out.bin\n", argv[0]);
        return 2;
    }
    const std::vector<double> a = tbpm::fermi_cheb_coeffs(std::atof(argv[1]), std::atof(argv[2]),
                                                          std::atof(argv[3]), std::atof(argv[4]));
    if (a.empty()) return 3;
    FILE *f = std::fopen(argv[5], "wb");
    if (!f) return 2;
    const size_t w = std::fwrite(a.data(), sizeof(double), a.size(), f);
    std::fclose(f);
    return w == a.size() ? 0 : 2;
}
