// Probing colourings for trace estimation of Pi_p A^-1 (paper Background,
// Probing): a distance-1 colouring of the symmetric part of Pi_p A^k, i.e.
// sites x != y conflict when y is within distance k of x + p z^ or of
// x - p z^ (the graph distance of the Wilson operator is the periodic taxicab
// distance).  Optimality does not matter; the colouring is greedy.
#include "fs_probe.h"

#include <algorithm>
#include <cstdlib>
#include <stdexcept>

namespace fs {

std::vector<int32_t> probing_colours(const int dims[4], int p, int k, int* n_colours) {
    const int Lx = dims[0], Ly = dims[1], Lz = dims[2], Lt = dims[3];
    const long long V = (long long)Lx * Ly * Lz * Lt;
    // offsets of the taxicab ball of radius k (duplicates after wrapping are harmless)
    std::vector<int> off;
    for (int dt = -k; dt <= k; ++dt)
        for (int dz = -k + std::abs(dt); dz <= k - std::abs(dt); ++dz)
            for (int dy = -k + std::abs(dt) + std::abs(dz); dy <= k - std::abs(dt) - std::abs(dz); ++dy) {
                const int r = k - std::abs(dt) - std::abs(dz) - std::abs(dy);
                for (int dx = -r; dx <= r; ++dx) {
                    off.push_back(dx);
                    off.push_back(dy);
                    off.push_back(dz);
                    off.push_back(dt);
                }
            }
    const size_t nb = off.size() / 4;
    // wrapped, stride-scaled coordinate tables: T_mu[v + R] = stride_mu * (v mod L_mu), |v| <= R + L_mu
    const int R = k + p;
    auto table = [R](int L, long long stride) {
        std::vector<long long> t(2 * R + L + 1);
        for (int i = 0; i < (int)t.size(); ++i) t[i] = stride * ((((i - R) % L) + L) % L);
        return t;
    };
    const std::vector<long long> TX = table(Lx, 1), TY = table(Ly, Lx), TZ = table(Lz, (long long)Lx * Ly),
                                 TT = table(Lt, (long long)Lx * Ly * Lz);
    std::vector<int32_t> col(V, -1);
    std::vector<long long> stamp;  // stamp[c] == s: colour c is taken for site s
    int used = 0;
    for (long long s = 0; s < V; ++s) {
        const int x = (int)(s % Lx), y = (int)((s / Lx) % Ly), z = (int)((s / ((long long)Lx * Ly)) % Lz),
                  t = (int)(s / ((long long)Lx * Ly * Lz));
        for (int side = -1; side <= 1; side += 2) {
            const long long* tx = TX.data() + R + x;
            const long long* ty = TY.data() + R + y;
            const long long* tz = TZ.data() + R + z + side * p;
            const long long* tt = TT.data() + R + t;
            for (size_t o = 0; o < nb; ++o) {
                const int* d = &off[4 * o];
                const long long q = tx[d[0]] + ty[d[1]] + tz[d[2]] + tt[d[3]];
                if (q >= s) continue;  // only earlier sites are coloured (q == s is the site itself)
                const int c = col[q];
                if (c >= (int)stamp.size()) stamp.resize(c + 1, -1);
                stamp[c] = s;
            }
        }
        int c = 0;
        while (c < (int)stamp.size() && stamp[c] == s) ++c;
        col[s] = c;
        used = std::max(used, c + 1);
    }
    *n_colours = used;
    return col;
}

}  // namespace fs
