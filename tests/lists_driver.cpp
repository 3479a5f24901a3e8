// Host driver for the decomposition lists (lb_lists.hpp): reads cases from
// stdin, one per line,
//     nx ny xbc ybc iface tile_w  blo[0..ntiles)  bhi[0..ntiles)
// (tile_w = 0: one tile) and prints per case the line
//     nfin nproj_low nproj_high  fin...  proj...
#include <cstdio>
#include <vector>

#include "../paper_1007_4895_amd/csrc/lb_lists.hpp"

int main() {
    int nx, ny, xbc, ybc, iface, tw;
    while (std::scanf("%d %d %d %d %d %d", &nx, &ny, &xbc, &ybc, &iface, &tw) == 6) {
        const int nt = tw > 0 ? (nx + tw - 1) / tw : 1;
        std::vector<int32_t> lo(nt), hi(nt);
        for (auto &v : lo)
            if (std::scanf("%d", &v) != 1) return 1;
        for (auto &v : hi)
            if (std::scanf("%d", &v) != 1) return 1;
        const lbl::Decomp D{nx, ny, xbc, ybc, iface, nt, tw > 0 ? tw : nx, lo.data(), hi.data()};
        std::vector<int32_t> fin, proj;
        int np[2];
        const int nf = lbl::build_lists(D, fin, proj, np);
        std::printf("%d %d %d", nf, np[0], np[1]);
        for (int v : fin) std::printf(" %d", v);
        for (int v : proj) std::printf(" %d", v);
        std::printf("\n");
    }
    return 0;
}
