// Reference P_q tetrahedron for the nodal DG space (Section 5.2.2, nodal basis
// of P_q(T_h) lifted from triangles to tetrahedra), and the P_q triangle of
// the 2-D transverse-magnetic space (Section 5.2.1).
//
// Construction (long double): nodal basis from a Cartesian monomial
// Vandermonde at the equispaced nodes; differentiation matrices from the
// monomial derivatives; mass and face-mass matrices by Gauss-Legendre
// quadrature in collapsed (Duffy) coordinates, exact for the polynomial
// degrees involved; LIFT = M^-1 [E_0 | E_1 | E_2 | E_3] on face-node columns.
// Normalisation: unit-volume element, unit-area faces (affine scalings are
// applied per element).
#include <cmath>
#include <mutex>

#include "internal.h"

namespace cmcg {

const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

namespace {

using LD = long double;

// Gauss-Legendre nodes / weights on [0, 1] by Newton iteration.
void gauss01(int n, std::vector<LD>& x, std::vector<LD>& w) {
    x.assign(n, 0);
    w.assign(n, 0);
    const LD pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        LD z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
        LD pp = 0;
        for (int it = 0; it < 100; ++it) {
            LD p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                LD p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1; }
            pp = n * (z * p1 - p0) / (z * z - 1);
            LD dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-19L) break;
        }
        x[i] = 0.5L * (1 - z);
        w[i] = 1.0L / ((1 - z * z) * pp * pp);  // = 0.5 * 2/((1-z^2)p'^2)
    }
}

std::vector<LD> invert(std::vector<LD> A, int n) {
    std::vector<LD> B(n * n, 0);
    for (int i = 0; i < n; ++i) B[i * n + i] = 1;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0) fail(CMCG_ERR_ARG, "singular reference matrix");
        for (int k = 0; k < n; ++k) {
            std::swap(A[c * n + k], A[p * n + k]);
            std::swap(B[c * n + k], B[p * n + k]);
        }
        LD piv = A[c * n + c];
        for (int k = 0; k < n; ++k) {
            A[c * n + k] /= piv;
            B[c * n + k] /= piv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            LD f = A[r * n + c];
            if (f == 0) continue;
            for (int k = 0; k < n; ++k) {
                A[r * n + k] -= f * A[c * n + k];
                B[r * n + k] -= f * B[c * n + k];
            }
        }
    }
    return B;
}

struct Basis {
    int q, Np;
    std::vector<int> ex;     // [Np][3] monomial exponents
    std::vector<LD> Vinv;    // [Np][Np] coefficients: phi_n = sum_m Vinv[m][n] mono_m
    LD mono(int m, const LD* x) const {
        return std::pow(x[0], ex[3 * m]) * std::pow(x[1], ex[3 * m + 1]) * std::pow(x[2], ex[3 * m + 2]);
    }
    void phi(const LD* x, LD* out) const {
        std::vector<LD> mv(Np);
        for (int m = 0; m < Np; ++m) mv[m] = mono(m, x);
        for (int n = 0; n < Np; ++n) {
            LD s = 0;
            for (int m = 0; m < Np; ++m) s += Vinv[m * Np + n] * mv[m];
            out[n] = s;
        }
    }
};

RefElem build(int q) {
    RefElem r;
    r.q = q;
    r.Np = np_of(q);
    r.Nfp = nfp_of(q);
    const int Np = r.Np, Nfp = r.Nfp;
    // nodes: k slowest, j, i fastest
    std::vector<int> lab;
    for (int k = 0; k <= q; ++k)
        for (int j = 0; j <= q - k; ++j)
            for (int i = 0; i <= q - j - k; ++i) {
                lab.push_back(i);
                lab.push_back(j);
                lab.push_back(k);
            }
    std::vector<LD> xi(3 * Np);
    r.xi.resize(3 * Np);
    for (int n = 0; n < 3 * Np; ++n) {
        xi[n] = (LD)lab[n] / q;
        r.xi[n] = (double)xi[n];
    }
    Basis B;
    B.q = q;
    B.Np = Np;
    for (int a = 0; a <= q; ++a)
        for (int b = 0; b <= q - a; ++b)
            for (int c = 0; c <= q - a - b; ++c) {
                B.ex.push_back(a);
                B.ex.push_back(b);
                B.ex.push_back(c);
            }
    std::vector<LD> V(Np * Np);
    for (int n = 0; n < Np; ++n)
        for (int m = 0; m < Np; ++m) V[n * Np + m] = B.mono(m, &xi[3 * n]);
    B.Vinv = invert(V, Np);
    // differentiation matrices
    r.D.assign(3 * Np * Np, 0);
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < Np; ++i)
            for (int j = 0; j < Np; ++j) {
                LD s = 0;
                for (int m = 0; m < Np; ++m) {
                    int e = B.ex[3 * m + a];
                    if (e == 0) continue;
                    LD x[3] = {xi[3 * i], xi[3 * i + 1], xi[3 * i + 2]};
                    LD d = e * std::pow(x[a], e - 1);
                    for (int b = 0; b < 3; ++b)
                        if (b != a) d *= std::pow(x[b], B.ex[3 * m + b]);
                    s += B.Vinv[m * Np + j] * d;
                }
                r.D[(a * Np + i) * Np + j] = (double)s;
            }
    // volume mass: 6 * int over the unit simplex (volume 1/6)
    std::vector<LD> gx, gw;
    gauss01(q + 3, gx, gw);
    std::vector<LD> M(Np * Np, 0), ph(Np);
    for (size_t a = 0; a < gx.size(); ++a)
        for (size_t b = 0; b < gx.size(); ++b)
            for (size_t c = 0; c < gx.size(); ++c) {
                LD u = gx[a], v = gx[b], s = gx[c];
                LD x[3] = {u, v * (1 - u), s * (1 - u) * (1 - v)};
                LD w = gw[a] * gw[b] * gw[c] * (1 - u) * (1 - u) * (1 - v) * 6;
                B.phi(x, ph.data());
                for (int i = 0; i < Np; ++i)
                    for (int j = 0; j < Np; ++j) M[i * Np + j] += w * ph[i] * ph[j];
            }
    r.M.resize(Np * Np);
    for (int i = 0; i < Np * Np; ++i) r.M[i] = (double)M[i];
    // faces: face f opposite vertex f; face vertices in increasing local order
    const LD V4[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    r.fnode.assign(4 * Nfp, -1);
    std::vector<LD> Minv = invert(M, Np);
    r.LIFT.assign(Np * 4 * Nfp, 0);
    for (int f = 0; f < 4; ++f) {
        int w3[3], t = 0;
        for (int v = 0; v < 4; ++v)
            if (v != f) w3[t++] = v;
        // barycentric labels of nodes
        int cnt = 0;
        for (int n = 0; n < Np; ++n) {
            int bl[4] = {q - lab[3 * n] - lab[3 * n + 1] - lab[3 * n + 2], lab[3 * n], lab[3 * n + 1],
                         lab[3 * n + 2]};
            if (bl[f] != 0) continue;
            // canonical face order: c2 slowest, c1 fastest (c_i = label of face vertex i)
            int c1 = bl[w3[1]], c2 = bl[w3[2]];
            int idx = 0;
            for (int tt = 0; tt < c2; ++tt) idx += q + 1 - tt;
            idx += c1;
            if (idx != cnt) fail(CMCG_ERR_ARG, "face node order is not canonical");
            r.fnode[f * Nfp + cnt] = n;
            ++cnt;
        }
        // face mass on unit area: 2 * int over the unit triangle
        std::vector<LD> E(Np * Np, 0);
        for (size_t a = 0; a < gx.size(); ++a)
            for (size_t b = 0; b < gx.size(); ++b) {
                LD s = gx[a], tt = gx[b] * (1 - gx[a]);
                LD w = gw[a] * gw[b] * (1 - gx[a]) * 2;
                LD x[3];
                for (int d = 0; d < 3; ++d)
                    x[d] = V4[w3[0]][d] + s * (V4[w3[1]][d] - V4[w3[0]][d]) + tt * (V4[w3[2]][d] - V4[w3[0]][d]);
                B.phi(x, ph.data());
                for (int i = 0; i < Np; ++i)
                    for (int j = 0; j < Np; ++j) E[i * Np + j] += w * ph[i] * ph[j];
            }
        for (int i = 0; i < Np; ++i)
            for (int k = 0; k < Nfp; ++k) {
                LD s = 0;
                int col = r.fnode[f * Nfp + k];
                for (int j = 0; j < Np; ++j) s += Minv[i * Np + j] * E[j * Np + col];
                r.LIFT[i * 4 * Nfp + f * Nfp + k] = (double)s;
            }
    }
    // matching of canonical face nodes under the 6 vertex permutations:
    // neighbour label d_j = c_{perm3[p][j]}
    r.fperm.assign(6 * Nfp, -1);
    for (int p = 0; p < 6; ++p) {
        int k = 0;
        for (int c2 = 0; c2 <= q; ++c2)
            for (int c1 = 0; c1 <= q - c2; ++c1, ++k) {
                int c[3] = {q - c1 - c2, c1, c2};
                int d1 = c[perm3[p][1]], d2 = c[perm3[p][2]];
                int idx = 0;
                for (int tt = 0; tt < d2; ++tt) idx += q + 1 - tt;
                idx += d1;
                r.fperm[p * Nfp + k] = idx;
            }
    }
    return r;
}

// Reference triangle: the same construction in two variables.  Edge f is
// opposite vertex f; its nodes run from its lower-numbered vertex.
RefElem2D build2d(int q) {
    RefElem2D r;
    r.q = q;
    r.Np = np2_of(q);
    r.Nfp = nfp2_of(q);
    const int Np = r.Np, Nfp = r.Nfp;
    std::vector<int> lab;  // (i, j), j slowest
    for (int j = 0; j <= q; ++j)
        for (int i = 0; i <= q - j; ++i) {
            lab.push_back(i);
            lab.push_back(j);
        }
    std::vector<LD> xi(2 * Np);
    r.xi.resize(2 * Np);
    for (int n = 0; n < 2 * Np; ++n) {
        xi[n] = (LD)lab[n] / q;
        r.xi[n] = (double)xi[n];
    }
    std::vector<int> ex;  // monomials x^a y^b, a + b <= q
    for (int a = 0; a <= q; ++a)
        for (int b = 0; b <= q - a; ++b) {
            ex.push_back(a);
            ex.push_back(b);
        }
    auto mono = [&](int m, LD x, LD y) { return std::pow(x, ex[2 * m]) * std::pow(y, ex[2 * m + 1]); };
    std::vector<LD> V(Np * Np);
    for (int n = 0; n < Np; ++n)
        for (int m = 0; m < Np; ++m) V[n * Np + m] = mono(m, xi[2 * n], xi[2 * n + 1]);
    const std::vector<LD> Vinv = invert(V, Np);
    auto phi = [&](LD x, LD y, LD* out) {
        for (int nn = 0; nn < Np; ++nn) {
            LD t = 0;
            for (int m = 0; m < Np; ++m) t += Vinv[m * Np + nn] * mono(m, x, y);
            out[nn] = t;
        }
    };
    r.D.assign(2 * Np * Np, 0);
    for (int a = 0; a < 2; ++a)
        for (int i = 0; i < Np; ++i)
            for (int j = 0; j < Np; ++j) {
                LD t = 0;
                for (int m = 0; m < Np; ++m) {
                    const int e = ex[2 * m + a];
                    if (e == 0) continue;
                    const LD x = xi[2 * i], y = xi[2 * i + 1];
                    const LD d = a == 0 ? e * std::pow(x, e - 1) * std::pow(y, ex[2 * m + 1])
                                        : e * std::pow(y, e - 1) * std::pow(x, ex[2 * m]);
                    t += Vinv[m * Np + j] * d;
                }
                r.D[(a * Np + i) * Np + j] = (double)t;
            }
    // mass: 2 * int over the unit triangle (area 1/2), collapsed coordinates
    std::vector<LD> gx, gw;
    gauss01(q + 3, gx, gw);
    std::vector<LD> M(Np * Np, 0), ph(Np);
    for (size_t a = 0; a < gx.size(); ++a)
        for (size_t b = 0; b < gx.size(); ++b) {
            const LD u = gx[a], v = gx[b] * (1 - gx[a]);
            const LD w = gw[a] * gw[b] * (1 - gx[a]) * 2;
            phi(u, v, ph.data());
            for (int i = 0; i < Np; ++i)
                for (int j = 0; j < Np; ++j) M[i * Np + j] += w * ph[i] * ph[j];
        }
    r.M.resize(Np * Np);
    for (int i = 0; i < Np * Np; ++i) r.M[i] = (double)M[i];
    const std::vector<LD> Minv = invert(M, Np);
    const LD V3[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    r.fnode.assign(3 * Nfp, -1);
    r.LIFT.assign(Np * 3 * Nfp, 0);
    for (int f = 0; f < 3; ++f) {
        const int va = f == 0 ? 1 : 0, vb = f == 2 ? 1 : 2;
        // edge nodes ordered by their distance from va
        int cnt = 0;
        for (int k = 0; k <= q; ++k)
            for (int n = 0; n < Np; ++n) {
                const int bl[3] = {q - lab[2 * n] - lab[2 * n + 1], lab[2 * n], lab[2 * n + 1]};
                if (bl[f] == 0 && bl[vb] == k) r.fnode[f * Nfp + cnt++] = n;
            }
        if (cnt != Nfp) fail(CMCG_ERR_ARG, "edge node count");
        // edge mass per unit length
        std::vector<LD> E(Np * Np, 0);
        for (size_t a = 0; a < gx.size(); ++a) {
            const LD t = gx[a];
            phi(V3[va][0] + t * (V3[vb][0] - V3[va][0]), V3[va][1] + t * (V3[vb][1] - V3[va][1]), ph.data());
            for (int i = 0; i < Np; ++i)
                for (int j = 0; j < Np; ++j) E[i * Np + j] += gw[a] * ph[i] * ph[j];
        }
        for (int i = 0; i < Np; ++i)
            for (int k = 0; k < Nfp; ++k) {
                LD t = 0;
                const int col = r.fnode[f * Nfp + k];
                for (int j = 0; j < Np; ++j) t += Minv[i * Np + j] * E[j * Np + col];
                r.LIFT[i * 3 * Nfp + f * Nfp + k] = (double)t;
            }
    }
    return r;
}

}  // namespace

const RefElem2D& ref_elem2d(int q) {
    static RefElem2D cache[kMaxQ + 1];
    static std::once_flag once[kMaxQ + 1];
    if (q < 1 || q > kMaxQ) fail(CMCG_ERR_ARG, "q must be 1, 2 or 3");
    std::call_once(once[q], [q] { cache[q] = build2d(q); });
    return cache[q];
}

const RefElem& ref_elem(int q) {
    static RefElem cache[kMaxQ + 1];
    static std::once_flag once[kMaxQ + 1];
    if (q < 1 || q > kMaxQ) fail(CMCG_ERR_ARG, "q must be 1, 2 or 3");
    std::call_once(once[q], [q] { cache[q] = build(q); });
    return cache[q];
}

}  // namespace cmcg
