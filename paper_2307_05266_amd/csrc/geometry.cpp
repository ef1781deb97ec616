// Host-side geometry preprocessing: periodic components, their windings,
// removal of components that cannot carry flow, surface voxel count.
//
// Components are found with a weighted union-find over the fluid adjacency
// (Sec. 2.2 of the paper requires a connected flow domain and fixes the
// pressure up to one constant per component).  Every node stores its
// displacement to its parent in the unwrapped (infinite periodic) lattice.
// Joining two voxels that already share a root closes a cycle; the mismatch
// of their displacements is N times that cycle's winding vector.  A
// component carries flow under the force f exactly when some cycle has a
// winding w with f.w != 0: otherwise a pressure f.(unwrapped position)
// balances the force and the velocity vanishes, so the component is turned
// into solid without changing the solution elsewhere.
#include "geometry.h"

#include <cstring>

namespace stokes {

namespace {

struct UnionFind {
    std::vector<int32_t> parent;
    std::vector<int32_t> size;
    std::vector<int32_t> off;      // 3 per node: displacement to the parent
    std::vector<uint8_t> conducts; // valid at roots

    explicit UnionFind(int64_t n) : parent(n), size(n, 1), off(3 * n, 0), conducts(n, 0) {
        for (int64_t i = 0; i < n; ++i) parent[i] = (int32_t)i;
    }

    // Root of x and the displacement pos(x) - pos(root); compresses the path.
    int32_t find(int32_t x, int32_t o[3]) {
        int32_t r = x;
        int32_t acc[3] = {0, 0, 0};
        while (parent[r] != r) {
            for (int e = 0; e < 3; ++e) acc[e] += off[3 * r + e];
            r = parent[r];
        }
        // second pass: point every node on the path at the root
        int32_t rem[3] = {acc[0], acc[1], acc[2]};
        int32_t y = x;
        while (parent[y] != y) {
            int32_t next = parent[y];
            int32_t my[3] = {off[3 * y], off[3 * y + 1], off[3 * y + 2]};
            parent[y] = r;
            for (int e = 0; e < 3; ++e) off[3 * y + e] = rem[e];
            for (int e = 0; e < 3; ++e) rem[e] -= my[e];
            y = next;
        }
        o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2];
        return r;
    }
};

inline int64_t at(int N, int i, int j, int k) { return (int64_t)i + (int64_t)N * ((int64_t)j + (int64_t)N * k); }

}  // namespace

void preprocess(const uint8_t* mask, int N, const double force[3], bool keep_all, Geometry& g) {
    const int64_t n3 = (int64_t)N * N * N;
    g.N = N;
    g.n3 = n3;
    UnionFind uf(n3);

    // edges to the +x, +y, +z neighbour of every fluid voxel
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const int64_t a = at(N, i, j, k);
                if (!mask[a]) continue;
                const int64_t nb[3] = {at(N, (i + 1) % N, j, k), at(N, i, (j + 1) % N, k),
                                       at(N, i, j, (k + 1) % N)};
                for (int d = 0; d < 3; ++d) {
                    const int64_t b = nb[d];
                    if (!mask[b]) continue;
                    int32_t oa[3], ob[3];
                    int32_t ra = uf.find((int32_t)a, oa);
                    int32_t rb = uf.find((int32_t)b, ob);
                    // unwrapped: pos(b) = pos(a) + e_d
                    int32_t delta[3] = {oa[0] - ob[0], oa[1] - ob[1], oa[2] - ob[2]};
                    delta[d] += 1;  // = pos(rb) - pos(ra) if b is placed next to a
                    if (ra == rb) {
                        double fw = 0.0;
                        for (int e = 0; e < 3; ++e) fw += force[e] * (double)(delta[e] / N);
                        if (fw != 0.0) uf.conducts[ra] = 1;
                        continue;
                    }
                    if (uf.size[ra] < uf.size[rb]) {
                        uf.parent[ra] = rb;
                        for (int e = 0; e < 3; ++e) uf.off[3 * ra + e] = -delta[e];
                        uf.size[rb] += uf.size[ra];
                        uf.conducts[rb] |= uf.conducts[ra];
                    } else {
                        uf.parent[rb] = ra;
                        for (int e = 0; e < 3; ++e) uf.off[3 * rb + e] = delta[e];
                        uf.size[ra] += uf.size[rb];
                        uf.conducts[ra] |= uf.conducts[rb];
                    }
                }
            }

    // number the components by their lowest voxel index
    std::vector<int32_t> id_of_root(n3, -1);
    std::vector<uint8_t> keep;
    int ncomp = 0;
    g.fluid.assign(n3, 0);
    g.nfluid_in = 0;
    for (int64_t x = 0; x < n3; ++x) {
        if (!mask[x]) continue;
        ++g.nfluid_in;
        int32_t o[3];
        int32_t r = uf.find((int32_t)x, o);
        if (id_of_root[r] < 0) {
            id_of_root[r] = ncomp++;
            keep.push_back(keep_all ? 1 : uf.conducts[r]);
        }
    }
    g.ncomp_all = ncomp;
    std::vector<int32_t> kept_id(ncomp, -1);
    int nk = 0;
    for (int c = 0; c < ncomp; ++c)
        if (keep[c]) kept_id[c] = nk++;
    g.ncomp_kept = nk;
    g.comp_size.assign(nk, 0);
    const bool with_labels = nk <= 65535;
    if (with_labels) g.label.assign(n3, 0xFFFFu);
    else g.label.clear();
    g.nfluid = 0;
    for (int64_t x = 0; x < n3; ++x) {
        if (!mask[x]) continue;
        int32_t o[3];
        int c = kept_id[id_of_root[uf.find((int32_t)x, o)]];
        if (c < 0) continue;
        g.fluid[x] = 1;
        ++g.nfluid;
        ++g.comp_size[c];
        if (with_labels) g.label[x] = (uint16_t)c;
    }

    // solid voxels with a fluid face neighbour, on the mask as given
    int64_t ns = 0;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                if (mask[at(N, i, j, k)]) continue;
                const int ip = (i + 1) % N, im = (i + N - 1) % N, jp = (j + 1) % N, jm = (j + N - 1) % N,
                          kp = (k + 1) % N, km = (k + N - 1) % N;
                if (mask[at(N, ip, j, k)] || mask[at(N, im, j, k)] || mask[at(N, i, jp, k)] ||
                    mask[at(N, i, jm, k)] || mask[at(N, i, j, kp)] || mask[at(N, i, j, km)])
                    ++ns;
            }
    g.nsurf = ns;
}

}  // namespace stokes
