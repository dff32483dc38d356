// Host build of the solver's logarithm: reads doubles from argv[1], writes
// lnx of each to argv[2] (raw native-endian doubles).
#include "../paper_1906_09530_amd/csrc/lnx.hpp"

#include <cstdio>
#include <vector>

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *in = std::fopen(argv[1], "rb");
    if (!in) return 3;
    std::vector<double> x;
    double v;
    while (std::fread(&v, sizeof v, 1, in) == 1) x.push_back(v);
    std::fclose(in);
    for (double &t : x) t = cplbm::phys::lnx(t);
    FILE *out = std::fopen(argv[2], "wb");
    if (!out) return 4;
    const size_t n = std::fwrite(x.data(), sizeof(double), x.size(), out);
    std::fclose(out);
    return n == x.size() ? 0 : 5;
}
