// Prints the workgroup -> tile maps of the phase kernels, computed by the
// kernels' own index code (apsp_tilemap.h, compiled here for the host), for
// the CPU tests to compare with their independent derivations.  One line
// per (map, q, r, parameters): "<map> q r a b : I,J I,J ...", tiles in
// workgroup order.  Maps: panels, all, next, rest (a, b = band lo, hi),
// psnap, pnextr, pnext2, prest2 (a, b = band), pfix (a = final), sall,
// srest, snext.
#include <cstdio>

#include "../paper_1902_04446_amd/csrc/apsp_tilemap.h"

using namespace apsp;

namespace {

template <class F>
void line(const char *map, int q, int r, int a, int b, int count, F f) {
    std::printf("%s %d %d %d %d :", map, q, r, a, b);
    for (int t = 0; t < count; ++t) {
        int I = -1, J = -1;
        f(t, I, J);
        std::printf(" %d,%d", I, J);
    }
    std::printf("\n");
}

int nxt_of(int q, int r) {
    const int nx = q - (r + 2);
    return nx < 0 ? 0 : (nx > 2 ? 2 : nx);
}

}  // namespace

int main() {
    const int qs[] = {1, 2, 3, 4, 5, 6, 7, 9, 10, 13, 17, 33};
    for (int q : qs) {
        for (int r = 0; r < q; ++r) {
            line("panels", q, r, 0, 0, (int)tilemap::tile_count(q, r, kPanels, 0, 0),
                 [&](int t, int &I, int &J) { tilemap::tile_of<kPanels>(t, r, q, 0, 0, I, J); });
            line("all", q, r, 0, 0, (int)tilemap::tile_count(q, r, kAll, 0, 0),
                 [&](int t, int &I, int &J) { tilemap::tile_of<kAll>(t, r, q, 0, 0, I, J); });
            line("next", q, r, 0, 0, (int)tilemap::tile_count(q, r, kNext, 0, 0),
                 [&](int t, int &I, int &J) { tilemap::tile_of<kNext>(t, r, q, 0, 0, I, J); });
            for (int bands = 1; bands <= 3; ++bands)
                for (int g = 0; g < bands; ++g) {
                    const int lo = q * g / bands, hi = q * (g + 1) / bands;
                    line("rest", q, r, lo, hi, (int)tilemap::tile_count(q, r, kRest, lo, hi),
                         [&](int t, int &I, int &J) {
                             tilemap::tile_of<kRest>(t, r, q, lo, hi, I, J);
                         });
                }
            // round pairs (r, r+1)
            const int nx = nxt_of(q, r);
            line("psnap", q, r, 0, 0, 2 * (q - 1), [&](int t, int &I, int &J) {
                tilemap::pair_tile_of<tilemap::kPanelsSnap>(t, r, q, nx, 0, 0, 0, I, J);
            });
            if (r + 1 < q) {
                line("pnextr", q, r, 0, 0, 2 * q - 3, [&](int t, int &I, int &J) {
                    tilemap::pair_tile_of<tilemap::kNextR>(t, r, q, nx, 0, 0, 0, I, J);
                });
                const int m = q - 2;
                line("pnext2", q, r, 0, 0, nx * m + nx * (m - nx), [&](int t, int &I, int &J) {
                    tilemap::pair_tile_of<tilemap::kNext2>(t, r, q, nx, 0, 0, 0, I, J);
                });
                for (int bands = 1; bands <= 2; ++bands)
                    for (int g = 0; g < bands; ++g) {
                        const int lo = q * g / bands, hi = q * (g + 1) / bands;
                        const int e1 = r + 2 + nx;
                        const int x0 = r > lo ? r : lo, x1 = e1 < hi ? e1 : hi;
                        const int rows = hi - lo - (x1 > x0 ? x1 - x0 : 0);
                        const int count = rows > 0 ? rows * (q - (e1 - r)) : 0;
                        line("prest2", q, r, lo, hi, count, [&](int t, int &I, int &J) {
                            tilemap::pair_tile_of<tilemap::kRest2>(t, r, q, nx, lo, hi, 0, I, J);
                        });
                    }
                line("pfix", q, r, 0, 0, 2 * nx, [&](int t, int &I, int &J) {
                    tilemap::pair_tile_of<tilemap::kFix>(t, r, q, nx, 0, 0, 0, I, J);
                });
                line("pfix", q, r, 1, 0, (q - 1 - nx) + (q - 2 - nx), [&](int t, int &I, int &J) {
                    tilemap::pair_tile_of<tilemap::kFix>(t, r, q, nx, 0, 0, 1, I, J);
                });
            }
            // symmetric solver (upper tiles)
            line("sall", q, r, 0, 0, (q - 1) * q / 2, [&](int t, int &I, int &J) {
                tilemap::sym_tile_of<tilemap::kSymAll>(t, r, q, I, J);
            });
            if (r + 1 < q) {
                line("srest", q, r, 0, 0, (q - 2) * (q - 1) / 2, [&](int t, int &I, int &J) {
                    tilemap::sym_tile_of<tilemap::kSymRest>(t, r, q, I, J);
                });
                line("snext", q, r, 0, 0, q - 1, [&](int t, int &I, int &J) {
                    tilemap::sym_tile_of<tilemap::kSymNext>(t, r, q, I, J);
                });
            }
        }
    }
    return 0;
}
