// Canonical Q_p node numbering of general hexahedral meshes (host code).

#include "mfe_mesh.hpp"

#include <algorithm>
#include <array>
#include <cstdio>

namespace mfe {

namespace {

inline int corner(int bx, int by, int bz) { return bx + 2 * by + 4 * bz; }

struct FaceWalk {
    std::array<int32_t, 4> key;   // ascending vertex ids
    std::array<int32_t, 4> path;  // origin, lower neighbour, higher neighbour, opposite
    int o1, o2;                   // origin's corner bits along the free axes d1 < d2
    bool first_d1;                // the walk's first axis is d1
};

// The face of cell row[] with reference coordinate d fixed at `side`.
FaceWalk face_walk(const int32_t* row, int d, int side) {
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    int32_t id[2][2];
    for (int b1 = 0; b1 < 2; ++b1)
        for (int b2 = 0; b2 < 2; ++b2) {
            int bits[3];
            bits[d] = side;
            bits[d1] = b1;
            bits[d2] = b2;
            id[b1][b2] = row[corner(bits[0], bits[1], bits[2])];
        }
    FaceWalk f;
    f.o1 = 0;
    f.o2 = 0;
    for (int b1 = 0; b1 < 2; ++b1)
        for (int b2 = 0; b2 < 2; ++b2)
            if (id[b1][b2] < id[f.o1][f.o2]) {
                f.o1 = b1;
                f.o2 = b2;
            }
    const int32_t n1 = id[1 - f.o1][f.o2], n2 = id[f.o1][1 - f.o2];
    f.first_d1 = n1 < n2;
    f.path = {id[f.o1][f.o2], std::min(n1, n2), std::max(n1, n2), id[1 - f.o1][1 - f.o2]};
    f.key = {id[0][0], id[0][1], id[1][0], id[1][1]};
    std::sort(f.key.begin(), f.key.end());
    return f;
}

}  // namespace

std::string number_hex_nodes(int64_t nv, int64_t ne, const int32_t* ev, int p, std::vector<int32_t>& conn,
                             int64_t& n_nodes) {
    char msg[160];
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t* row = ev + 8 * e;
        for (int v = 0; v < 8; ++v) {
            if (row[v] < 0 || row[v] >= nv) {
                std::snprintf(msg, sizeof(msg), "cell %lld: vertex id %d out of range", (long long)e, row[v]);
                return msg;
            }
            for (int w = 0; w < v; ++w)
                if (row[w] == row[v]) {
                    std::snprintf(msg, sizeof(msg), "cell %lld repeats vertex %d", (long long)e, row[v]);
                    return msg;
                }
        }
    }
    // unique edges, as (lower << 32 | higher)
    std::vector<uint64_t> edges;
    edges.reserve((size_t)ne * 12);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t* row = ev + 8 * e;
        for (int d = 0; d < 3; ++d)
            for (int v = 0; v < 8; ++v)
                if (!((v >> d) & 1)) {
                    const uint32_t a = (uint32_t)row[v], b = (uint32_t)row[v | (1 << d)];
                    edges.push_back((uint64_t)std::min(a, b) << 32 | std::max(a, b));
                }
    }
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    // unique faces: every cell's six, sorted by key; a key may appear twice,
    // with the same path
    struct Entry {
        std::array<int32_t, 4> key, path;
    };
    std::vector<Entry> all;
    all.reserve((size_t)ne * 6);
    for (int64_t e = 0; e < ne; ++e)
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) {
                const FaceWalk f = face_walk(ev + 8 * e, d, side);
                all.push_back({f.key, f.path});
            }
    std::sort(all.begin(), all.end(), [](const Entry& a, const Entry& b) { return a.key < b.key; });
    std::vector<std::array<int32_t, 4>> faces;
    for (size_t i = 0; i < all.size();) {
        size_t j = i + 1;
        while (j < all.size() && all[j].key == all[i].key) {
            if (all[j].path != all[i].path) {
                std::snprintf(msg, sizeof(msg), "two cells disagree on the edges of face (%d %d %d %d)",
                              all[i].key[0], all[i].key[1], all[i].key[2], all[i].key[3]);
                return msg;
            }
            ++j;
        }
        if (j - i > 2) {
            std::snprintf(msg, sizeof(msg), "face (%d %d %d %d) belongs to more than two cells", all[i].key[0],
                          all[i].key[1], all[i].key[2], all[i].key[3]);
            return msg;
        }
        faces.push_back(all[i].key);
        i = j;
    }
    const int64_t m = p - 1, n = p + 1, n3 = n * n * n;
    const int64_t base_e = nv;
    const int64_t base_f = base_e + (int64_t)edges.size() * m;
    const int64_t base_i = base_f + (int64_t)faces.size() * m * m;
    n_nodes = base_i + ne * m * m * m;
    if (3 * n_nodes >= ((int64_t)1 << 31)) return "mesh too large for 32-bit dof indices";
    conn.assign((size_t)(ne * n3), 0);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t* row = ev + 8 * e;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int c[3] = {i, j, k};
                    bool end[3];
                    int ends = 0;
                    for (int d = 0; d < 3; ++d) {
                        end[d] = c[d] == 0 || c[d] == p;
                        ends += end[d];
                    }
                    int64_t node;
                    if (ends == 3) {
                        node = row[corner(i / p, j / p, k / p)];
                    } else if (ends == 2) {
                        const int d = !end[0] ? 0 : (!end[1] ? 1 : 2);
                        int lo[3], hi[3];
                        for (int x = 0; x < 3; ++x) lo[x] = hi[x] = (x == d) ? 0 : c[x] / p;
                        hi[d] = 1;
                        const uint32_t ga = (uint32_t)row[corner(lo[0], lo[1], lo[2])];
                        const uint32_t gb = (uint32_t)row[corner(hi[0], hi[1], hi[2])];
                        const int s = ga < gb ? c[d] : p - c[d];
                        const uint64_t key = (uint64_t)std::min(ga, gb) << 32 | std::max(ga, gb);
                        const int64_t r = std::lower_bound(edges.begin(), edges.end(), key) - edges.begin();
                        node = base_e + r * m + (s - 1);
                    } else if (ends == 1) {
                        const int d = end[0] ? 0 : (end[1] ? 1 : 2);
                        const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
                        const FaceWalk f = face_walk(row, d, c[d] / p);
                        const int s1 = f.o1 ? p - c[d1] : c[d1];
                        const int s2 = f.o2 ? p - c[d2] : c[d2];
                        const int s = f.first_d1 ? s1 : s2, t = f.first_d1 ? s2 : s1;
                        const int64_t r = std::lower_bound(faces.begin(), faces.end(), f.key) - faces.begin();
                        node = base_f + r * m * m + (s - 1) + m * (t - 1);
                    } else {
                        node = base_i + e * m * m * m + (i - 1) + m * ((j - 1) + m * (k - 1));
                    }
                    conn[(size_t)(e * n3 + i + n * (j + n * k))] = (int32_t)node;
                }
    }
    return "";
}

namespace {
// the low 21 bits of v spread to every third bit
uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}
}  // namespace

void morton_order(int64_t nv, const double* xyz, int64_t ne, const int32_t* ev, std::vector<int32_t>& perm) {
    double lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
    for (int64_t v = 1; v < nv; ++v)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], xyz[3 * v + d]);
            hi[d] = std::max(hi[d], xyz[3 * v + d]);
        }
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)ne);
    for (int64_t e = 0; e < ne; ++e) {
        uint64_t code = 0;
        for (int d = 0; d < 3; ++d) {
            double x = 0.0;
            for (int v = 0; v < 8; ++v) x += xyz[3 * (int64_t)ev[8 * e + v] + d];
            const double span = hi[d] - lo[d];
            const double t = span > 0.0 ? (x / 8.0 - lo[d]) / span : 0.0;
            const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097151.0));
            code |= spread3(q) << d;
        }
        key[e] = {code, (int32_t)e};
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint64_t, int32_t>& a, const std::pair<uint64_t, int32_t>& b) {
                         return a.first < b.first;
                     });
    perm.resize((size_t)ne);
    for (int64_t e = 0; e < ne; ++e) perm[e] = key[e].second;
}

}  // namespace mfe
