// Internal declarations of the CMCG Maxwell library (host side + kernel
// launch interfaces).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/cmcg.h"

namespace cmcg {

// ------------------------------------------------------------------ errors
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void set_last_error(const std::string& msg);

#define CMCG_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::cmcg::fail(CMCG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ----------------------------------------------------------- reference element
inline int np_of(int q) { return (q + 1) * (q + 2) * (q + 3) / 6; }
inline int nfp_of(int q) { return (q + 1) * (q + 2) / 2; }
constexpr int kMaxQ = 3;

struct RefElem {
    int q, Np, Nfp;
    std::vector<double> xi;      // [Np][3] node coordinates
    std::vector<double> M;       // [Np][Np] mass, unit-volume element
    std::vector<double> D;       // [3][Np][Np] d/dxi_a at nodes
    std::vector<double> LIFT;    // [Np][4 Nfp] M^-1 E_f, unit-area faces
    std::vector<int> fnode;      // [4][Nfp] element node of face node k
    std::vector<int> fperm;      // [6][Nfp] face node matching under vertex permutation
};
const RefElem& ref_elem(int q);
// vertex permutations of a triangle, index 0..5: neighbour face local vertex
// j carries my face local vertex perm3[p][j]
extern const int perm3[6][3];

// Reference P_q triangle of the 2-D transverse-magnetic space (Section 5.2.1,
// two-dimensional setting): nodes (i, j)/q with j slowest, edge f opposite
// vertex f, edge nodes listed from the edge's lower-numbered vertex.
inline int np2_of(int q) { return (q + 1) * (q + 2) / 2; }
inline int nfp2_of(int q) { return q + 1; }
struct RefElem2D {
    int q, Np, Nfp;
    std::vector<double> xi;      // [Np][2]
    std::vector<double> M;       // [Np][Np] mass, unit-area element
    std::vector<double> D;       // [2][Np][Np] d/dxi_a at nodes
    std::vector<double> LIFT;    // [Np][3 Nfp] M^-1 E_f, unit-length edges
    std::vector<int> fnode;      // [3][Nfp] element node of edge node k
};
const RefElem2D& ref_elem2d(int q);

// ----------------------------------------------------------------- mesh
// dim 3: tetrahedra, 4 faces; dim 2: triangles, 3 edges (the per-face arrays
// then hold 3 entries per element, xyz 2 per vertex, G 4 per element, normal
// 2 per face, area = edge length, vol = triangle area, rho = inscribed-circle
// diameter, perm = 1 when the neighbour runs the edge the other way).
struct MeshData {
    int dim = 3;
    int64_t nv = 0, K = 0;
    std::vector<double> xyz;     // [nv][3]
    std::vector<int64_t> tet;    // [K][4]
    std::vector<int8_t> tag;     // [K][4]  0 interior, 1 PEC, 2 impedance
    std::vector<int64_t> nbr;    // [K][4]  -1 on the boundary
    std::vector<int8_t> nbr_face;// [K][4]
    std::vector<int8_t> perm;    // [K][4]  vertex permutation code 0..5
    std::vector<double> G;       // [K][3][3] d xi_a / d x_k
    std::vector<double> vol;     // [K]
    std::vector<double> normal;  // [K][4][3] outward unit normals
    std::vector<double> area;    // [K][4]
    std::vector<double> rho;     // [K] insphere diameter
    int64_t n_boundary = 0;
};

// Number of per-element geometry values uploaded for the stage kernel.
// Layout per element: G[9] | per face f: n[3], cE1, cE2, cH1, cH2 (28) |
// 1/eps, 1/mu, sigma/eps  -> 40 values.
constexpr int kGeo = 40;
// 2-D: G[4] | per edge f: n[2], cE1, cE2, cH1, cH2 (18) | 1/eps, 1/mu, sigma/eps,
// padded to 28 values so that every element's record starts on a 16-byte
// boundary (the stage kernel stages it with 16-byte loads).
constexpr int kGeo2 = 28;

}  // namespace cmcg

struct cmcg_mesh {
    std::shared_ptr<cmcg::MeshData> d;
};
