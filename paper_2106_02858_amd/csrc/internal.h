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

// ----------------------------------------------------------------- mesh
struct MeshData {
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

}  // namespace cmcg

struct cmcg_mesh {
    std::shared_ptr<cmcg::MeshData> d;
};
