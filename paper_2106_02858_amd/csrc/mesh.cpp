// Mesh validation, face connectivity and affine geometry (Section 5.2.2:
// conforming simplicial mesh, interior / PEC / impedance face sets, outward
// normals; the insphere diameter rho_K of the CFL rule of Section 5.3).
//
// Faces are matched through a hash of their sorted global vertex triple; the
// relative orientation of the two copies of an interior face is stored as
// one of the six triangle vertex permutations.  Normals and face areas come
// from the gradients of the barycentric coordinates: n_f = -grad(lambda_f) /
// |grad(lambda_f)|, area_f = 3 |K| |grad(lambda_f)|.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <unordered_map>

#include "internal.h"

namespace cmcg {

namespace {

struct TriKey {
    int64_t a, b, c;
    bool operator==(const TriKey& o) const { return a == o.a && b == o.b && c == o.c; }
};
struct TriHash {
    size_t operator()(const TriKey& k) const {
        uint64_t h = (uint64_t)k.a * 0x9E3779B97F4A7C15ull;
        h ^= (uint64_t)k.b + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
        h ^= (uint64_t)k.c + 0x85EBCA77C2B2AE63ull + (h << 6) + (h >> 2);
        return (size_t)h;
    }
};

void face_vertices(int f, int w[3]) {
    int t = 0;
    for (int v = 0; v < 4; ++v)
        if (v != f) w[t++] = v;
}

}  // namespace

// Spreads the low 21 bits of x to every third bit (Morton interleave).
static uint64_t spread3(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

void locality_order(int64_t nv, const double* xyz, int64_t K, const int64_t* tet, int64_t* order) {
    if (!xyz || !tet || !order) fail(CMCG_ERR_ARG, "locality_order: NULL argument");
    if (nv < 1 || K < 1) fail(CMCG_ERR_ARG, "locality_order: need nv >= 1 and K >= 1");
    for (int64_t i = 0; i < 4 * K; ++i)
        if (tet[i] < 0 || tet[i] >= nv) fail(CMCG_ERR_ARG, "locality_order: vertex index out of range");
    double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    std::vector<double> c(3 * K);
    for (int64_t e = 0; e < K; ++e)
        for (int d = 0; d < 3; ++d) {
            double s = 0;
            for (int v = 0; v < 4; ++v) s += xyz[3 * tet[4 * e + v] + d];
            c[3 * e + d] = 0.25 * s;
            if (!std::isfinite(c[3 * e + d])) fail(CMCG_ERR_ARG, "locality_order: non-finite coordinate");
            lo[d] = std::fmin(lo[d], c[3 * e + d]);
            hi[d] = std::fmax(hi[d], c[3 * e + d]);
        }
    // one scale for all axes keeps the curve's cells cubic
    const double span = std::fmax(std::fmax(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    const double sc = span > 0 ? double((1 << 21) - 1) / span : 0.0;
    std::vector<uint64_t> key(K);
    for (int64_t e = 0; e < K; ++e) {
        uint64_t k = 0;
        for (int d = 0; d < 3; ++d) k |= spread3((uint64_t)((c[3 * e + d] - lo[d]) * sc)) << d;
        key[e] = k;
    }
    std::iota(order, order + K, int64_t(0));
    std::stable_sort(order, order + K, [&](int64_t a, int64_t b) { return key[a] < key[b]; });
}

std::shared_ptr<MeshData> build_mesh(int64_t nv, const double* xyz, int64_t K, const int64_t* tet,
                                     const int8_t* face_tag) {
    if (!xyz || !tet) fail(CMCG_ERR_ARG, "mesh: NULL coordinates or connectivity");
    if (nv < 4 || K < 1) fail(CMCG_ERR_ARG, "mesh: need nv >= 4 and K >= 1");
    if (K >= (int64_t(1) << 26)) fail(CMCG_ERR_ARG, "mesh: K must be below 2^26");
    auto m = std::make_shared<MeshData>();
    m->nv = nv;
    m->K = K;
    m->xyz.assign(xyz, xyz + 3 * nv);
    m->tet.assign(tet, tet + 4 * K);
    for (int64_t i = 0; i < 4 * K; ++i)
        if (tet[i] < 0 || tet[i] >= nv) fail(CMCG_ERR_ARG, "mesh: vertex index out of range");
    m->tag.assign(4 * K, 0);
    m->nbr.assign(4 * K, -1);
    m->nbr_face.assign(4 * K, -1);
    m->perm.assign(4 * K, 0);
    m->G.resize(9 * K);
    m->vol.resize(K);
    m->normal.resize(12 * K);
    m->area.resize(4 * K);
    m->rho.resize(K);
    // geometry
    for (int64_t e = 0; e < K; ++e) {
        const double* v0 = &xyz[3 * tet[4 * e]];
        double J[3][3];  // columns v_a - v_0
        for (int a = 0; a < 3; ++a) {
            const double* va = &xyz[3 * tet[4 * e + a + 1]];
            for (int d = 0; d < 3; ++d) J[d][a] = va[d] - v0[d];
        }
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        double scale = 0;
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) scale = std::fmax(scale, std::fabs(J[d][a]));
        if (!(std::fabs(det) > 1e-14 * scale * scale * scale))
            fail(CMCG_ERR_MESH, "mesh: degenerate tetrahedron " + std::to_string(e));
        // inverse: rows are grad xi_a
        double inv[3][3];
        inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 3; ++k) m->G[9 * e + 3 * a + k] = inv[a][k];
        double vol = std::fabs(det) / 6.0;
        m->vol[e] = vol;
        double asum = 0;
        for (int f = 0; f < 4; ++f) {
            double g[3];
            for (int k = 0; k < 3; ++k)
                g[k] = (f == 0) ? -(inv[0][k] + inv[1][k] + inv[2][k]) : inv[f - 1][k];
            double gn = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            for (int k = 0; k < 3; ++k) m->normal[12 * e + 3 * f + k] = -g[k] / gn;
            m->area[4 * e + f] = 3.0 * vol * gn;
            asum += m->area[4 * e + f];
        }
        m->rho[e] = 6.0 * vol / asum;
    }
    // connectivity
    std::unordered_map<TriKey, int64_t, TriHash> open;
    open.reserve(2 * K + 16);
    for (int64_t e = 0; e < K; ++e) {
        for (int f = 0; f < 4; ++f) {
            int w[3];
            face_vertices(f, w);
            int64_t g[3] = {tet[4 * e + w[0]], tet[4 * e + w[1]], tet[4 * e + w[2]]};
            if (g[0] == g[1] || g[1] == g[2] || g[0] == g[2])
                fail(CMCG_ERR_MESH, "mesh: repeated vertex in tetrahedron " + std::to_string(e));
            int64_t s[3] = {g[0], g[1], g[2]};
            if (s[0] > s[1]) std::swap(s[0], s[1]);
            if (s[1] > s[2]) std::swap(s[1], s[2]);
            if (s[0] > s[1]) std::swap(s[0], s[1]);
            TriKey key{s[0], s[1], s[2]};
            auto it = open.find(key);
            if (it == open.end()) {
                open.emplace(key, 4 * e + f);
                continue;
            }
            int64_t other = it->second;
            if (other < 0) fail(CMCG_ERR_MESH, "mesh: face shared by more than two tetrahedra");
            int64_t e2 = other / 4;
            int f2 = (int)(other % 4);
            it->second = -1;
            m->nbr[4 * e + f] = e2;
            m->nbr_face[4 * e + f] = (int8_t)f2;
            m->nbr[4 * e2 + f2] = e;
            m->nbr_face[4 * e2 + f2] = (int8_t)f;
            int w2[3];
            face_vertices(f2, w2);
            int64_t h[3] = {tet[4 * e2 + w2[0]], tet[4 * e2 + w2[1]], tet[4 * e2 + w2[2]]};
            // permutation seen from e: neighbour vertex j == my vertex perm3[p][j]
            for (int side = 0; side < 2; ++side) {
                const int64_t* A = side == 0 ? g : h;
                const int64_t* Bv = side == 0 ? h : g;
                int found = -1;
                for (int p = 0; p < 6 && found < 0; ++p)
                    if (Bv[0] == A[perm3[p][0]] && Bv[1] == A[perm3[p][1]] && Bv[2] == A[perm3[p][2]]) found = p;
                if (found < 0) fail(CMCG_ERR_MESH, "mesh: inconsistent face vertices");
                if (side == 0)
                    m->perm[4 * e + f] = (int8_t)found;
                else
                    m->perm[4 * e2 + f2] = (int8_t)found;
            }
        }
    }
    for (int64_t e = 0; e < K; ++e)
        for (int f = 0; f < 4; ++f) {
            int64_t i = 4 * e + f;
            if (m->nbr[i] >= 0) continue;
            ++m->n_boundary;
            int t = face_tag ? face_tag[i] : CMCG_TAG_IMPEDANCE;
            if (t != CMCG_TAG_PEC && t != CMCG_TAG_IMPEDANCE)
                fail(CMCG_ERR_MESH, "mesh: boundary face without PEC / impedance tag (element " +
                                        std::to_string(e) + ", face " + std::to_string(f) + ")");
            m->tag[i] = (int8_t)t;
        }
    return m;
}

// Triangle meshes of the 2-D transverse-magnetic setting (Section 5.2.1): edges
// matched through their sorted vertex pair; normals are the edge directions
// turned a quarter turn away from the opposite vertex; rho_K = 4 |K| /
// perimeter, the diameter of the inscribed circle.
std::shared_ptr<MeshData> build_mesh2d(int64_t nv, const double* xy, int64_t K, const int64_t* tri,
                                       const int8_t* edge_tag) {
    if (!xy || !tri) fail(CMCG_ERR_ARG, "mesh2d: NULL coordinates or connectivity");
    if (nv < 3 || K < 1) fail(CMCG_ERR_ARG, "mesh2d: need nv >= 3 and K >= 1");
    if (K >= (int64_t(1) << 26)) fail(CMCG_ERR_ARG, "mesh2d: K must be below 2^26");
    for (int64_t i = 0; i < 3 * K; ++i)
        if (tri[i] < 0 || tri[i] >= nv) fail(CMCG_ERR_ARG, "mesh2d: vertex index out of range");
    auto m = std::make_shared<MeshData>();
    m->dim = 2;
    m->nv = nv;
    m->K = K;
    m->xyz.assign(xy, xy + 2 * nv);
    m->tet.assign(tri, tri + 3 * K);
    m->tag.assign(3 * K, 0);
    m->nbr.assign(3 * K, -1);
    m->nbr_face.assign(3 * K, -1);
    m->perm.assign(3 * K, 0);
    m->G.resize(4 * K);
    m->vol.resize(K);
    m->normal.resize(6 * K);
    m->area.resize(3 * K);
    m->rho.resize(K);
    for (int64_t e = 0; e < K; ++e) {
        const double* v[3] = {&xy[2 * tri[3 * e]], &xy[2 * tri[3 * e + 1]], &xy[2 * tri[3 * e + 2]]};
        const double J00 = v[1][0] - v[0][0], J01 = v[2][0] - v[0][0];
        const double J10 = v[1][1] - v[0][1], J11 = v[2][1] - v[0][1];
        const double det = J00 * J11 - J01 * J10;
        const double scale = std::fmax(std::fmax(std::fabs(J00), std::fabs(J01)), std::fmax(std::fabs(J10), std::fabs(J11)));
        if (!(std::fabs(det) > 1e-14 * scale * scale))
            fail(CMCG_ERR_MESH, "mesh2d: degenerate triangle " + std::to_string(e));
        // rows of the inverse Jacobian: grad xi_1, grad xi_2
        m->G[4 * e + 0] = J11 / det;
        m->G[4 * e + 1] = -J01 / det;
        m->G[4 * e + 2] = -J10 / det;
        m->G[4 * e + 3] = J00 / det;
        m->vol[e] = 0.5 * std::fabs(det);
        double per = 0;
        for (int f = 0; f < 3; ++f) {
            const int a = f == 0 ? 1 : 0, b = f == 2 ? 1 : 2;
            const double tx = v[b][0] - v[a][0], ty = v[b][1] - v[a][1];
            const double L = std::sqrt(tx * tx + ty * ty);
            double nx = ty / L, ny = -tx / L;
            if (nx * (v[f][0] - v[a][0]) + ny * (v[f][1] - v[a][1]) > 0) {
                nx = -nx;
                ny = -ny;
            }
            m->normal[6 * e + 2 * f] = nx;
            m->normal[6 * e + 2 * f + 1] = ny;
            m->area[3 * e + f] = L;
            per += L;
        }
        m->rho[e] = 4.0 * m->vol[e] / per;
    }
    std::unordered_map<TriKey, int64_t, TriHash> open;
    open.reserve(2 * K + 16);
    for (int64_t e = 0; e < K; ++e)
        for (int f = 0; f < 3; ++f) {
            const int a = f == 0 ? 1 : 0, b = f == 2 ? 1 : 2;
            const int64_t ga = tri[3 * e + a], gb = tri[3 * e + b];
            if (ga == gb || tri[3 * e + f] == ga || tri[3 * e + f] == gb)
                fail(CMCG_ERR_MESH, "mesh2d: repeated vertex in triangle " + std::to_string(e));
            TriKey key{std::min(ga, gb), std::max(ga, gb), -1};
            auto it = open.find(key);
            if (it == open.end()) {
                open.emplace(key, 3 * e + f);
                continue;
            }
            const int64_t other = it->second;
            if (other < 0) fail(CMCG_ERR_MESH, "mesh2d: edge shared by more than two triangles");
            const int64_t e2 = other / 3;
            const int f2 = (int)(other % 3);
            it->second = -1;
            const int a2 = f2 == 0 ? 1 : 0;
            const int rev = tri[3 * e2 + a2] != ga ? 1 : 0;  // the neighbour starts the edge at my other end
            m->nbr[3 * e + f] = e2;
            m->nbr_face[3 * e + f] = (int8_t)f2;
            m->perm[3 * e + f] = (int8_t)rev;
            m->nbr[3 * e2 + f2] = e;
            m->nbr_face[3 * e2 + f2] = (int8_t)f;
            m->perm[3 * e2 + f2] = (int8_t)rev;
        }
    for (int64_t i = 0; i < 3 * K; ++i) {
        if (m->nbr[i] >= 0) continue;
        ++m->n_boundary;
        const int t = edge_tag ? edge_tag[i] : CMCG_TAG_IMPEDANCE;
        if (t != CMCG_TAG_PEC && t != CMCG_TAG_IMPEDANCE)
            fail(CMCG_ERR_MESH, "mesh2d: boundary edge without PEC / impedance tag (element " +
                                    std::to_string(i / 3) + ", edge " + std::to_string(i % 3) + ")");
        m->tag[i] = (int8_t)t;
    }
    return m;
}

}  // namespace cmcg
