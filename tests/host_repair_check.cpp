// Host driver for the hybrid mode's host repair (built for the host only by
// test_host_repair.py; no GPU involved).  Reads "N Lx Ly q" and N lines
// "x y" (positions on the grid 2^-q) from stdin, rebuilds every cell's ring
// from scratch with spv::HostRepair and prints, per cell, its ring length and
// members (tags = input indices), or "err <bits>".
#include <cmath>
#include <cstdio>
#include <vector>

#include "../paper_1702_02939_amd/csrc/spv_host_repair.hpp"

int main()
{
    int n = 0, q = 0;
    double Lx = 0, Ly = 0;
    if (std::scanf("%d %lf %lf %d", &n, &Lx, &Ly, &q) != 4) return 2;
    std::vector<double> x(n), y(n);
    for (int i = 0; i < n; i++)
        if (std::scanf("%lf %lf", &x[i], &y[i]) != 2) return 2;
    std::vector<int> tag(n), sys(n, 0);
    for (int i = 0; i < n; i++) tag[i] = i;
    // one system, set up as the library does at creation (bin side = the
    // mean spacing, first search radius 2.5 spacings)
    spv::SysParam P{};
    P.scale = std::ldexp(1.0, q);
    P.Lx = Lx;
    P.Ly = Ly;
    P.hLx = 0.5 * Lx;
    P.hLy = 0.5 * Ly;
    const double spacing = std::sqrt(Lx * Ly / n);
    P.R0 = 2.5 * spacing;
    P.nbx = std::max(1, (int)std::floor(Lx / spacing));
    P.nby = std::max(1, (int)std::floor(Ly / spacing));
    P.bsx = Lx / P.nbx;
    P.bsy = Ly / P.nby;
    P.n = n;
    std::vector<spv::SysParam> sp{P};
    spv::HostRepair hr;
    hr.build(x.data(), y.data(), sys.data(), n, sp, P.nbx * P.nby);
    for (int i = 0; i < n; i++) {
        const unsigned e = hr.repair(i, x.data(), y.data(), tag.data(), sys.data(), sp, 32);
        if (e) {
            std::printf("err %u\n", e);
            continue;
        }
        std::printf("%d", (int)hr.ring.size());
        for (int m : hr.ring) std::printf(" %d", m);
        std::printf("\n");
    }
    return 0;
}
