// Host check of the cell order of the binning (common.h): for a set of brick
// grids, cell_rank is a bijection onto 0 .. ncells-1, cell_coords inverts it,
// cell_rank32 agrees with it, and consecutive bricks share a face. Prints one
// line per grid and "ok" or "fail" at the end; built and run by
// test_cell_order.py.
#include "../paper_1309_1889_amd/csrc/common.h"

#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace msmx;

int main()
{
    const int dims[][3] = {{1, 1, 1},  {3, 5, 7},  {11, 11, 11}, {17, 17, 17}, {16, 16, 16}, {5, 8, 3},
                           {4, 17, 2}, {2, 31, 5}, {5, 32, 4},   {3, 33, 5},   {2, 40, 7},   {7, 48, 9},
                           {1, 64, 3}, {30, 65, 65}};
    int bad = 0;
    for (const auto &d : dims) {
        SysPlan p{};
        for (int k = 0; k < 3; ++k) {
            p.nb[k] = d[k];
            p.nc[k] = d[k] * kBrick;
        }
        const int64_t nbricks = (int64_t)d[0] * d[1] * d[2], n = nbricks * kBrickCells;
        std::vector<char> seen(n, 0);
        std::vector<int> bx(nbricks), by(nbricks), bz(nbricks);
        int64_t wrong = 0;
        for (int cz = 0; cz < p.nc[2]; ++cz)
            for (int cy = 0; cy < p.nc[1]; ++cy)
                for (int cx = 0; cx < p.nc[0]; ++cx) {
                    const int64_t r = cell_rank(p, cx, cy, cz);
                    if (r < 0 || r >= n || seen[r]) {
                        ++wrong;
                        continue;
                    }
                    seen[r] = 1;
                    if (cell_rank32(p, cx, cy, cz) != r) ++wrong;
                    int c[3];
                    cell_coords(p, r, c);
                    if (c[0] != cx || c[1] != cy || c[2] != cz) ++wrong;
                    bx[r / kBrickCells] = cx / kBrick;
                    by[r / kBrickCells] = cy / kBrick;
                    bz[r / kBrickCells] = cz / kBrick;
                }
        int64_t jumps = 0;
        for (int64_t b = 1; b < nbricks; ++b)
            if (std::abs(bx[b] - bx[b - 1]) + std::abs(by[b] - by[b - 1]) + std::abs(bz[b] - bz[b - 1]) != 1) ++jumps;
        std::printf("bricks %d %d %d: wrong %lld, consecutive bricks not sharing a face %lld\n", d[0], d[1], d[2],
                    (long long)wrong, (long long)jumps);
        if (wrong) ++bad;
    }
    std::printf(bad ? "fail\n" : "ok\n");
    return bad ? 1 : 0;
}
