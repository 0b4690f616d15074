// Host driver for tests/test_tiles.py: the trace kernels' hand-out of screen
// pixels (paper_2605_05635_amd/csrc/rt_ray.h, compiled for the host from the
// same source).
//   tile_driver quotient  rows of int64 (a, b)               -> int64 quotient(a, b)
//   tile_driver tile      rows of int64 (p, nx, ny, tw, th)  -> int64 tile_pixel(...), by
//                         integer division and by quotient() (two values a row)
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rt_ray.h"

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    const bool tile = !std::strcmp(argv[1], "tile");
    if (!tile && std::strcmp(argv[1], "quotient")) return 2;
    const int width = tile ? 5 : 2;
    std::vector<int64_t> row(width);
    std::vector<int64_t> out;
    while (std::fread(row.data(), sizeof(int64_t), width, stdin) == static_cast<size_t>(width)) {
        if (tile) {
            const int32_t nx = static_cast<int32_t>(row[1]), ny = static_cast<int32_t>(row[2]);
            const int32_t tw = static_cast<int32_t>(row[3]), th = static_cast<int32_t>(row[4]);
            out.push_back(rt::ray::tile_pixel(row[0], nx, ny, tw, th));
            out.push_back(rt::ray::tile_pixel(row[0], nx, ny, tw, th, rt::ray::FpQuotient{}));
        } else
            out.push_back(rt::ray::quotient(static_cast<int32_t>(row[0]), static_cast<int32_t>(row[1])));
    }
    std::fwrite(out.data(), sizeof(int64_t), out.size(), stdout);
    return 0;
}
