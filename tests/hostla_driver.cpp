// Test driver for the host-side HPD inverse: reads n and the row-major
// complex matrix (n * n pairs of doubles) from argv[1], writes status and the
// inverse to argv[2]; argv[3] = thread count.
#include <cstdio>
#include <vector>

#include "../paper_2509_03622_amd/csrc/hostla.h"

int main(int argc, char **argv) {
    if (argc < 4) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    int n = 0;
    if (std::fread(&n, sizeof(int), 1, f) != 1) return 4;
    std::vector<std::complex<double>> G((size_t)n * n), Gi;
    if (std::fread(G.data(), sizeof(double) * 2, G.size(), f) != G.size()) return 5;
    std::fclose(f);
    const bool ok = nosdd::hpd_inverse_profile(n, G, Gi, std::atoi(argv[3]));
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 6;
    const int st = ok ? 1 : 0;
    std::fwrite(&st, sizeof(int), 1, o);
    if (ok) std::fwrite(Gi.data(), sizeof(double) * 2, Gi.size(), o);
    std::fclose(o);
    return 0;
}
