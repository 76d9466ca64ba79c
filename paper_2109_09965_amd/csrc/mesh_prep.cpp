// Host preprocessing of a face-based hybrid mesh: face Gauss points, cell
// geometry, compact-reconstruction operators, multicolour classes and the
// library cell order.  Runs once per mesh on the host (FP64, long double for
// the small dense factorisations).
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "cgks_internal.h"

namespace cgks {
namespace {

struct V3 {
    double x[3] = {0, 0, 0};
};

inline void sub(const double *a, const double *b, double *c, int d) {
    for (int k = 0; k < d; ++k) c[k] = a[k] - b[k];
}
inline void cross(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
inline double norm(const double *a, int d) {
    double s = 0;
    for (int k = 0; k < d; ++k) s += a[k] * a[k];
    return std::sqrt(s);
}

// Vertex k of face f in the frame of the cell on `side` (neighbour frame =
// owner frame minus the periodic shift).
void face_pt(const HostMesh &m, int64_t f, int k, int side, double *x) {
    const int64_t v = m.fvert[m.fptr[f] + k];
    for (int a = 0; a < m.dim; ++a) {
        x[a] = m.xyz[v * m.dim + a];
        if (side) x[a] -= m.shift[f * m.dim + a];
    }
}

// Point and unnormalised normal of the bilinear map of a quad at (s, t).
void quad_map(const double P[4][3], double s, double t, double *x, double *N) {
    double xs[3], xt[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = P[0][a] + s * (P[1][a] - P[0][a]) + t * (P[3][a] - P[0][a]) +
               s * t * (P[0][a] - P[1][a] + P[2][a] - P[3][a]);
        xs[a] = (P[1][a] - P[0][a]) + t * (P[0][a] - P[1][a] + P[2][a] - P[3][a]);
        xt[a] = (P[3][a] - P[0][a]) + s * (P[0][a] - P[1][a] + P[2][a] - P[3][a]);
    }
    cross(xs, xt, N);
}

// Face quadrature used by the scheme (Sec. 2.1): 2-point Gauss-Legendre on
// edges, the 3-point interior rule on triangles, 2x2 Gauss-Legendre on the
// bilinear quad with the Jacobian and normal of each point.
cgks_status face_quadrature(HostMesh &m) {
    const int d = m.dim;
    const double r3 = 1.0 / std::sqrt(3.0);
    const double gl2[2] = {0.5 * (1.0 - r3), 0.5 * (1.0 + r3)};
    m.ngp.assign(m.n_face, 0);
    m.gp_off.assign(m.n_face + 1, 0);
    for (int64_t f = 0; f < m.n_face; ++f) {
        const int nfv = int(m.fptr[f + 1] - m.fptr[f]);
        int n = 0;
        if (d == 2 && nfv == 2) n = 2;
        else if (d == 3 && nfv == 3) n = 3;
        else if (d == 3 && nfv == 4) n = 4;
        else return CGKS_EMESH;
        m.ngp[f] = n;
        m.gp_off[f + 1] = m.gp_off[f] + n;
    }
    m.n_gp = m.gp_off[m.n_face];
    m.gx.assign(m.n_gp * d, 0.0);
    m.gn.assign(m.n_gp * d, 0.0);
    m.gw.assign(m.n_gp, 0.0);
    m.avec.assign(m.n_face * d, 0.0);
    m.S.assign(m.n_face, 0.0);
    for (int64_t f = 0; f < m.n_face; ++f) {
        double P[4][3] = {};
        const int nfv = int(m.fptr[f + 1] - m.fptr[f]);
        for (int k = 0; k < nfv; ++k) face_pt(m, f, k, 0, P[k]);
        const int64_t g0 = m.gp_off[f];
        if (d == 2) {
            const double e[2] = {P[1][0] - P[0][0], P[1][1] - P[0][1]};
            const double len = std::hypot(e[0], e[1]);
            if (!(len > 0)) return CGKS_EMESH;
            for (int g = 0; g < 2; ++g) {
                m.gx[(g0 + g) * 2 + 0] = P[0][0] + gl2[g] * e[0];
                m.gx[(g0 + g) * 2 + 1] = P[0][1] + gl2[g] * e[1];
                m.gn[(g0 + g) * 2 + 0] = e[1] / len;
                m.gn[(g0 + g) * 2 + 1] = -e[0] / len;
                m.gw[g0 + g] = 0.5 * len;
            }
        } else if (nfv == 3) {
            double e1[3], e2[3], N[3];
            sub(P[1], P[0], e1, 3);
            sub(P[2], P[0], e2, 3);
            cross(e1, e2, N);
            const double twoA = norm(N, 3);
            if (!(twoA > 0)) return CGKS_EMESH;
            for (int g = 0; g < 3; ++g) {
                // barycentric weight 2/3 on vertex g, 1/6 on the other two
                for (int a = 0; a < 3; ++a) {
                    const double s = P[0][a] + P[1][a] + P[2][a];
                    m.gx[(g0 + g) * 3 + a] = (s + 3.0 * P[g][a]) / 6.0;
                    m.gn[(g0 + g) * 3 + a] = N[a] / twoA;
                }
                m.gw[g0 + g] = twoA / 6.0;
            }
        } else {
            int g = 0;
            for (int jt = 0; jt < 2; ++jt)
                for (int js = 0; js < 2; ++js, ++g) {
                    double x[3], N[3];
                    quad_map(P, gl2[js], gl2[jt], x, N);
                    const double J = norm(N, 3);
                    if (!(J > 0)) return CGKS_EMESH;
                    for (int a = 0; a < 3; ++a) {
                        m.gx[(g0 + g) * 3 + a] = x[a];
                        m.gn[(g0 + g) * 3 + a] = N[a] / J;
                    }
                    m.gw[g0 + g] = 0.25 * J;
                }
        }
        double s2 = 0;
        for (int a = 0; a < d; ++a) {
            double acc = 0;
            for (int g = 0; g < m.ngp[f]; ++g) acc += m.gw[g0 + g] * m.gn[(g0 + g) * d + a];
            m.avec[f * d + a] = acc;
            s2 += acc * acc;
        }
        m.S[f] = std::sqrt(s2);
    }
    return CGKS_OK;
}

// Moments of a polyhedral / polygonal cell by the divergence theorem:
//   |V| = 1/d  oint y.n,  int y_a = oint y_a^2/2 n_a,
//   int y_a^2 = oint y_a^3/3 n_a,  int y_a y_b = oint y_a^2 y_b / 2 n_a,
// with y relative to a vertex of the cell.  The face integrals of these
// cubics are exact with Simpson's rule on edges, a collapsed 3x3
// Gauss-Legendre rule on triangles and 4x4 Gauss-Legendre on bilinear quads.
struct Moments {
    double V = 0, M1[3] = {0, 0, 0}, M2[3][3] = {{0}};
    void add(int d, const double *y, const double *nw) {
        for (int a = 0; a < d; ++a) {
            V += y[a] * nw[a] / d;
            M1[a] += 0.5 * y[a] * y[a] * nw[a];
            for (int b = 0; b < d; ++b)
                M2[a][b] += (a == b ? y[a] * y[a] * y[a] / 3.0 : 0.5 * y[a] * y[a] * y[b]) * nw[a];
        }
    }
};

cgks_status cell_geometry(HostMesh &m) {
    const int d = m.dim;
    const double q3x[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
    const double q3w[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    const double a4 = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(1.2));
    const double b4 = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(1.2));
    const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
    const double q4x[4] = {0.5 * (1 - b4), 0.5 * (1 - a4), 0.5 * (1 + a4), 0.5 * (1 + b4)};
    const double q4w[4] = {0.5 * wb, 0.5 * wa, 0.5 * wa, 0.5 * wb};
    m.vol.assign(m.n_cell, 0.0);
    m.ctr.assign(m.n_cell * d, 0.0);
    m.sec.assign(m.n_cell * m.nq, 0.0);
    m.h.assign(m.n_cell, 0.0);
    std::atomic<bool> bad{false};
    parallel_for(m.n_cell, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            double ref[3] = {0, 0, 0};
            {
                const int64_t f = m.cf_face[m.cf_ptr[i]];
                face_pt(m, f, 0, m.cf_side[m.cf_ptr[i]], ref);
            }
            Moments mo;
            double sumS = 0;
            for (int64_t q = m.cf_ptr[i]; q < m.cf_ptr[i + 1]; ++q) {
                const int64_t f = m.cf_face[q];
                const int side = m.cf_side[q];
                const double sg = side ? -1.0 : 1.0;
                const int nfv = int(m.fptr[f + 1] - m.fptr[f]);
                double P[4][3] = {};
                for (int k = 0; k < nfv; ++k) {
                    face_pt(m, f, k, side, P[k]);
                    for (int a = 0; a < d; ++a) P[k][a] -= ref[a];
                }
                sumS += m.S[f];
                if (d == 2) {
                    const double n[2] = {sg * (P[1][1] - P[0][1]), -sg * (P[1][0] - P[0][0])};  // |n| = length
                    const double sw[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
                    for (int k = 0; k < 3; ++k) {
                        const double t = 0.5 * k;
                        const double y[2] = {P[0][0] + t * (P[1][0] - P[0][0]), P[0][1] + t * (P[1][1] - P[0][1])};
                        const double nw[2] = {n[0] * sw[k], n[1] * sw[k]};
                        mo.add(2, y, nw);
                    }
                } else if (nfv == 3) {
                    double e1[3], e2[3], N[3];
                    sub(P[1], P[0], e1, 3);
                    sub(P[2], P[0], e2, 3);
                    cross(e1, e2, N);  // |N| = 2A
                    for (int js = 0; js < 3; ++js)
                        for (int jt = 0; jt < 3; ++jt) {
                            const double s = q3x[js], t = q3x[jt];
                            const double a = s, b = t * (1.0 - s);
                            const double w = q3w[js] * q3w[jt] * (1.0 - s);
                            double y[3], nw[3];
                            for (int c = 0; c < 3; ++c) {
                                y[c] = P[0][c] + a * e1[c] + b * e2[c];
                                nw[c] = sg * N[c] * w;
                            }
                            mo.add(3, y, nw);
                        }
                } else {
                    for (int js = 0; js < 4; ++js)
                        for (int jt = 0; jt < 4; ++jt) {
                            double y[3], N[3], nw[3];
                            quad_map(P, q4x[js], q4x[jt], y, N);
                            for (int c = 0; c < 3; ++c) nw[c] = sg * N[c] * q4w[js] * q4w[jt];
                            mo.add(3, y, nw);
                        }
                }
            }
            if (!(mo.V > 0)) {
                bad = true;
                continue;
            }
            m.vol[i] = mo.V;
            double yc[3];
            for (int a = 0; a < d; ++a) {
                yc[a] = mo.M1[a] / mo.V;
                m.ctr[i * d + a] = ref[a] + yc[a];
            }
            int q = 0;
            for (int a = 0; a < d; ++a)
                for (int b = a; b < d; ++b) m.sec[i * m.nq + q++] = mo.M2[a][b] / mo.V - yc[a] * yc[b];
            m.h[i] = 2.0 * d * mo.V / sumS;
        }
    });
    return bad ? CGKS_EMESH : CGKS_OK;
}

// index of (a, b), a <= b, in the packed second-moment arrays
inline int qidx(int d, int a, int b) {
    if (a > b) std::swap(a, b);
    if (d == 2) return a + b;
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}
// quadratic basis order: 2-D (00, 01, 11); 3-D (00, 11, 22, 01, 02, 12)
const int kQa[2][6] = {{0, 0, 1, 0, 0, 0}, {0, 1, 2, 0, 0, 1}};
const int kQb[2][6] = {{0, 1, 1, 0, 0, 0}, {0, 1, 2, 1, 2, 2}};

// Basis averages <phi_k> over a cell with centroid c and central second
// moments s (packed), in the scaled frame of cell i (centre xc, size h).
void basis_avg(int d, const double *c, const double *s, const double *xc, double h, double *avg) {
    double dx[3];
    for (int a = 0; a < d; ++a) {
        dx[a] = c[a] - xc[a];
        avg[a] = dx[a] / h;
    }
    for (int q = 0; q < nquad_of(d); ++q) {
        const int a = kQa[d - 2][q], b = kQb[d - 2][q];
        avg[d + q] = (s[qidx(d, a, b)] + dx[a] * dx[b]) / (h * h);
    }
}

// Ghost basis averages of boundary face f for its owner: the owner mirrored
// in the plane through the face centroid normal to the face.
void ghost_avg(const HostMesh &m, int64_t f, double *avg) {
    const int d = m.dim;
    const int64_t i = m.owner[f];
    double n[3] = {0, 0, 0}, xf[3] = {0, 0, 0}, sw = 0;
    for (int a = 0; a < d; ++a) n[a] = m.avec[f * d + a] / m.S[f];
    for (int64_t g = m.gp_off[f]; g < m.gp_off[f + 1]; ++g) {
        sw += m.gw[g];
        for (int a = 0; a < d; ++a) xf[a] += m.gw[g] * m.gx[g * d + a];
    }
    double dist = 0;
    for (int a = 0; a < d; ++a) dist += (xf[a] / sw - m.ctr[i * d + a]) * n[a];
    double cg[3], S[3][3], RS[3][3], sg[6];
    for (int a = 0; a < d; ++a) cg[a] = m.ctr[i * d + a] + 2.0 * dist * n[a];
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) S[a][b] = m.sec[i * m.nq + qidx(d, a, b)];
    // R S R with R = I - 2 n n^T
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
            double acc = 0;
            for (int k = 0; k < d; ++k) acc += ((a == k) - 2.0 * n[a] * n[k]) * S[k][b];
            RS[a][b] = acc;
        }
    for (int a = 0; a < d; ++a)
        for (int b = a; b < d; ++b) {
            double acc = 0;
            for (int k = 0; k < d; ++k) acc += RS[a][k] * ((k == b) - 2.0 * n[k] * n[b]);
            sg[qidx(d, a, b)] = acc;
        }
    basis_avg(d, cg, sg, m.ctr.data() + i * d, m.h[i], avg);
}

// Householder QR of A [nr][nc] in long double; returns R's diagonal ratio and
// leaves R in the upper triangle.
long double qr_ratio(int nr, int nc, std::vector<long double> &A) {
    for (int k = 0; k < nc; ++k) {
        long double nrm = 0;
        for (int r = k; r < nr; ++r) nrm += A[r * nc + k] * A[r * nc + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0) continue;
        const long double alpha = A[k * nc + k] > 0 ? -nrm : nrm;
        std::vector<long double> v(nr, 0);
        for (int r = k; r < nr; ++r) v[r] = A[r * nc + k];
        v[k] -= alpha;
        long double vv = 0;
        for (int r = k; r < nr; ++r) vv += v[r] * v[r];
        if (vv == 0) continue;
        for (int j = k; j < nc; ++j) {
            long double s = 0;
            for (int r = k; r < nr; ++r) s += v[r] * A[r * nc + j];
            s = 2 * s / vv;
            for (int r = k; r < nr; ++r) A[r * nc + j] -= s * v[r];
        }
    }
    long double mn = INFINITY, mx = 0;
    for (int k = 0; k < nc; ++k) {
        const long double r = std::fabs(A[k * nc + k]);
        mn = std::min(mn, r);
        mx = std::max(mx, r);
    }
    return mx > 0 ? mn / mx : 0;
}

// (R^T R)^-1 = R^-1 R^-T from the upper triangle of A [..][nc], into out
// (an nk x nk block at offset 0)
void inverse_normal(int nc, const std::vector<long double> &A, int nk, double *out) {
    std::vector<long double> X(nc * nc, 0);  // X = R^-1 (upper)
    for (int j = 0; j < nc; ++j) {
        X[j * nc + j] = 1.0L / A[j * nc + j];
        for (int i = j - 1; i >= 0; --i) {
            long double s = 0;
            for (int k = i + 1; k <= j; ++k) s += A[i * nc + k] * X[k * nc + j];
            X[i * nc + j] = -s / A[i * nc + i];
        }
    }
    for (int i = 0; i < nk * nk; ++i) out[i] = 0.0;
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) {
            long double s = 0;
            for (int k = std::max(i, j); k < nc; ++k) s += X[i * nc + k] * X[j * nc + k];
            out[i * nk + j] = double(s);
        }
}

// Least-squares rows of cell i (slot order = increasing face index):
// per face neighbour (or ghost) one average row and d gradient rows, then
// d own-gradient rows.  Mirrors the device-side row generation.
void recon_rows(const HostMesh &m, int64_t i, std::vector<long double> &A, int &nr) {
    const int d = m.dim, nk = m.nk;
    const double *xc = m.ctr.data() + i * d;
    const double h = m.h[i];
    double own[9];
    basis_avg(d, xc, m.sec.data() + i * m.nq, xc, h, own);
    nr = 0;
    A.clear();
    auto push_block = [&](const double *avg) {
        A.resize((nr + 1 + d) * nk);
        for (int k = 0; k < nk; ++k) A[nr * nk + k] = avg[k] - own[k];
        ++nr;
        for (int a = 0; a < d; ++a, ++nr) {
            for (int k = 0; k < nk; ++k) A[nr * nk + k] = 0;
            A[nr * nk + a] = 1.0;
            for (int q = 0; q < nquad_of(d); ++q) {
                const int p = kQa[d - 2][q], r = kQb[d - 2][q];
                A[nr * nk + d + q] = (p == a ? avg[r] : 0.0) + (r == a ? avg[p] : 0.0);
            }
        }
    };
    for (int64_t q = m.cf_ptr[i]; q < m.cf_ptr[i + 1]; ++q) {
        const int64_t f = m.cf_face[q];
        double avg[9];
        if (m.neigh[f] >= 0) {
            const int side = m.cf_side[q];
            const int64_t nb = side ? m.owner[f] : m.neigh[f];
            double c[3];
            for (int a = 0; a < d; ++a)
                c[a] = m.ctr[nb * d + a] + (side ? -m.shift[f * d + a] : m.shift[f * d + a]);
            basis_avg(d, c, m.sec.data() + nb * m.nq, xc, h, avg);
        } else {
            for (int k = 0; k < nk; ++k) avg[k] = m.gavg[f * nk + k];
        }
        push_block(avg);
    }
    A.resize((nr + d) * nk);
    for (int a = 0; a < d; ++a, ++nr) {
        for (int k = 0; k < nk; ++k) A[nr * nk + k] = 0;
        A[nr * nk + a] = 1.0;
    }
}

// The reconstruction operators (M^T M)^-1 of every cell.  With the ghost
// rows of boundary faces every stencil of a valid mesh fixes the whole
// quadratic (each face brings d + 1 rows); one that does not is rejected.
cgks_status recon_setup(HostMesh &m) {
    const int nk = m.nk;
    m.gavg.assign(m.n_face * nk, 0.0);
    for (int64_t f = 0; f < m.n_face; ++f)
        if (m.neigh[f] < 0) ghost_avg(m, f, m.gavg.data() + f * nk);
    m.minv.assign(m.n_cell * nk * nk, 0.0);
    std::atomic<bool> bad{false};
    parallel_for(m.n_cell, [&](int64_t i0, int64_t i1) {
        std::vector<long double> A;
        for (int64_t i = i0; i < i1; ++i) {
            int nr = 0;
            recon_rows(m, i, A, nr);
            std::vector<long double> Q(A);
            if (nr >= nk && qr_ratio(nr, nk, Q) > kRankTol) inverse_normal(nk, Q, nk, m.minv.data() + i * nk * nk);
            else bad = true;
        }
    });
    return bad ? CGKS_EMESH : CGKS_OK;
}

// Morton (Z-order) key: the bits of 21-bit (3-D) or 32-bit (2-D) grid
// coordinates interleaved
static uint64_t spread3(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}
static uint64_t spread2(uint64_t x) {
    x &= 0xffffffffull;
    x = (x | x << 16) & 0x0000ffff0000ffffull;
    x = (x | x << 8) & 0x00ff00ff00ff00ffull;
    x = (x | x << 4) & 0x0f0f0f0f0f0f0f0full;
    x = (x | x << 2) & 0x3333333333333333ull;
    x = (x | x << 1) & 0x5555555555555555ull;
    return x;
}

// Cells along a Morton curve of their centroids (the bounding box mapped
// onto the grid; ties by caller id): consecutive cells are close in space.
static std::vector<int64_t> morton_order(const HostMesh &m) {
    const int d = m.dim;
    const int64_t n = m.n_cell;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) lo[a] = hi[a] = m.ctr[a];
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a) {
            lo[a] = std::min(lo[a], m.ctr[i * d + a]);
            hi[a] = std::max(hi[a], m.ctr[i * d + a]);
        }
    const double cells = d == 3 ? double(1 << 21) : 4294967296.0;
    std::vector<uint64_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t k = 0;
        for (int a = 0; a < d; ++a) {
            const double w = hi[a] > lo[a] ? (m.ctr[i * d + a] - lo[a]) / (hi[a] - lo[a]) : 0.0;
            const uint64_t g = uint64_t(std::min(cells - 1.0, std::max(0.0, std::floor(w * cells))));
            k |= (d == 3 ? spread3(g) : spread2(g)) << a;
        }
        key[i] = k;
    }
    std::vector<int64_t> order(n);
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return key[x] < key[y]; });
    return order;
}

// Multicolour classes of the relaxation sweeps (Algorithm 1 in a
// deterministic parallel order).  Largest-degree-first greedy colouring
// (Welsh-Powell): cells in order of decreasing count of faces with a
// neighbour cell, ties by caller id, each given the smallest colour absent
// from its coloured neighbours.  Class ids are then assigned by size: a step's
// passes visit colour 0 three times, colour C-1 twice and the others four
// times, so the largest class takes C-1, the next largest 0 and the rest
// 1..C-2 by decreasing size (stable on the greedy id).
void order_cells(HostMesh &m);

// Multicolour classes and the library cell order.  colour (may be NULL):
// the caller's classes, checked to be independent sets.
cgks_status colour_and_order(HostMesh &m, const int32_t *caller_colour) {
    const int64_t n = m.n_cell;
    auto neighbour = [&](int64_t q) { return m.cf_side[q] ? m.owner[m.cf_face[q]] : m.neigh[m.cf_face[q]]; };
    if (caller_colour) {
        int ncol = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (caller_colour[i] < 0 || caller_colour[i] >= kMaxColoursMesh) return CGKS_EMESH;
            ncol = std::max(ncol, caller_colour[i] + 1);
        }
        for (int64_t f = 0; f < m.n_face; ++f)
            if (m.neigh[f] >= 0 && caller_colour[m.owner[f]] == caller_colour[m.neigh[f]]) return CGKS_EMESH;
        m.colour.assign(caller_colour, caller_colour + n);
        m.n_colour = ncol;
        order_cells(m);
        return CGKS_OK;
    }
    std::vector<int> deg(n, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = m.cf_ptr[i]; q < m.cf_ptr[i + 1]; ++q) deg[i] += neighbour(q) >= 0;
    std::vector<int64_t> visit(n);
    for (int64_t i = 0; i < n; ++i) visit[i] = i;
    std::stable_sort(visit.begin(), visit.end(), [&](int64_t x, int64_t y) { return deg[x] > deg[y]; });
    m.colour.assign(n, -1);
    int ncol = 0;
    std::vector<char> used;
    for (int64_t i : visit) {
        used.assign(ncol + 1, 0);
        for (int64_t q = m.cf_ptr[i]; q < m.cf_ptr[i + 1]; ++q) {
            const int64_t nb = neighbour(q);
            if (nb >= 0 && m.colour[nb] >= 0) used[m.colour[nb]] = 1;
        }
        int c = 0;
        while (used[c]) ++c;
        m.colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    std::vector<int64_t> size(ncol, 0);
    for (int64_t i = 0; i < n; ++i) size[m.colour[i]]++;
    std::vector<int> by_size(ncol);
    for (int c = 0; c < ncol; ++c) by_size[c] = c;
    std::stable_sort(by_size.begin(), by_size.end(), [&](int x, int y) { return size[x] > size[y]; });
    std::vector<int> relabel(ncol);
    for (int k = 0; k < ncol; ++k) relabel[by_size[k]] = k == 0 ? ncol - 1 : k - 1;
    for (int64_t i = 0; i < n; ++i) m.colour[i] = relabel[m.colour[i]];
    m.n_colour = ncol;
    order_cells(m);
    return CGKS_OK;
}

// library order from the colour classes: tiles of m.tile consecutive cells
// of the Morton curve, colour-major inside each tile; faces follow
void order_cells(HostMesh &m) {
    const int ncol = m.n_colour;
    m.colour_count.assign(ncol, 0);
    for (int64_t i = 0; i < m.n_cell; ++i) m.colour_count[m.colour[i]]++;
    // library order: tiles of m.tile consecutive cells of the Morton curve,
    // colour-major inside each tile (curve order within a colour)
    const std::vector<int64_t> curve = morton_order(m);
    m.lib2caller.assign(m.n_cell, 0);
    m.caller2lib.assign(m.n_cell, 0);
    std::vector<std::vector<std::pair<int64_t, int64_t>>> runs(ncol);
    int64_t l = 0;
    for (int64_t t0 = 0; t0 < m.n_cell; t0 += m.tile) {
        const int64_t t1 = std::min(m.n_cell, t0 + m.tile);
        for (int c = 0; c < ncol; ++c) {
            const int64_t first = l;
            for (int64_t r = t0; r < t1; ++r) {
                const int64_t i = curve[r];
                if (m.colour[i] == c) {
                    m.lib2caller[l] = i;
                    m.caller2lib[i] = l++;
                }
            }
            if (l > first) runs[c].push_back({first, l - first});
        }
    }
    m.run_ptr.assign(ncol + 1, 0);
    m.run_start.clear();
    m.run_count.clear();
    for (int c = 0; c < ncol; ++c) {
        for (const auto &r : runs[c]) {
            m.run_start.push_back(r.first);
            m.run_count.push_back(r.second);
        }
        m.run_ptr[c + 1] = int64_t(m.run_start.size());
    }
    // faces follow their cells; boundary faces after the interior ones, so
    // that a face kernel's waves do not mix the two paths
    std::vector<int64_t> fkey(m.n_face);
    for (int64_t f = 0; f < m.n_face; ++f) {
        const int64_t a = m.caller2lib[m.owner[f]];
        fkey[f] = m.neigh[f] >= 0 ? std::min(a, m.caller2lib[m.neigh[f]]) : m.n_cell + a;
    }
    m.libf2caller.resize(m.n_face);
    for (int64_t f = 0; f < m.n_face; ++f) m.libf2caller[f] = f;
    std::stable_sort(m.libf2caller.begin(), m.libf2caller.end(),
                     [&](int64_t x, int64_t y) { return fkey[x] < fkey[y]; });
    m.caller2libf.assign(m.n_face, 0);
    for (int64_t lf = 0; lf < m.n_face; ++lf) m.caller2libf[m.libf2caller[lf]] = lf;
}


// Canonical face form: the owner is the smaller cell id (a swap reverses
// the vertex cycle and the periodic shift), a 3-D face's vertex cycle
// starts at its smallest id, and faces are sorted by owner, neighbour
// (boundary faces last) and vertex list.  Results then depend on the mesh
// alone, not on how its faces were listed.
void canonical_faces(HostMesh &m) {
    const int d = m.dim;
    const int64_t nf = m.n_face;
    std::vector<std::vector<int64_t>> fv(nf);
    for (int64_t f = 0; f < nf; ++f) {
        fv[f].assign(m.fvert.begin() + m.fptr[f], m.fvert.begin() + m.fptr[f + 1]);
        if (m.neigh[f] >= 0 && m.owner[f] > m.neigh[f]) {
            std::swap(m.owner[f], m.neigh[f]);
            std::reverse(fv[f].begin(), fv[f].end());
            for (int a = 0; a < d; ++a) m.shift[f * d + a] = -m.shift[f * d + a];
        }
        if (d == 3) {
            auto it = std::min_element(fv[f].begin(), fv[f].end());
            std::rotate(fv[f].begin(), it, fv[f].end());
        }
    }
    std::vector<int64_t> ord(nf);
    for (int64_t f = 0; f < nf; ++f) ord[f] = f;
    const int64_t big = m.n_cell;
    std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
        if (m.owner[x] != m.owner[y]) return m.owner[x] < m.owner[y];
        const int64_t nx = m.neigh[x] < 0 ? big : m.neigh[x], ny = m.neigh[y] < 0 ? big : m.neigh[y];
        if (nx != ny) return nx < ny;
        return fv[x] < fv[y];
    });
    std::vector<int64_t> ptr(nf + 1, 0), vert, own(nf), nb(nf);
    std::vector<int32_t> bc(nf);
    std::vector<double> sh(nf * d);
    for (int64_t k = 0; k < nf; ++k) {
        const int64_t f = ord[k];
        vert.insert(vert.end(), fv[f].begin(), fv[f].end());
        ptr[k + 1] = int64_t(vert.size());
        own[k] = m.owner[f];
        nb[k] = m.neigh[f];
        bc[k] = m.bc[f];
        for (int a = 0; a < d; ++a) sh[k * d + a] = m.shift[f * d + a];
    }
    m.fptr.swap(ptr);
    m.fvert.swap(vert);
    m.owner.swap(own);
    m.neigh.swap(nb);
    m.bc.swap(bc);
    m.shift.swap(sh);
}

}  // namespace

cgks_status build_host_mesh(const cgks_face_mesh_desc *ds, HostMesh &m) {
    if (!ds || (ds->dim != 2 && ds->dim != 3) || ds->n_cell <= 0 || ds->n_face <= 0 || ds->n_vert <= 0 ||
        !ds->xyz || !ds->face_vert_ptr || !ds->face_vert || !ds->face_owner || !ds->face_neigh || !ds->face_bc)
        return CGKS_EINVAL;
    if (ds->order_tile < 0) return CGKS_EINVAL;
    const int d = ds->dim;
    m.dim = d;
    m.tile = ds->order_tile > 0 ? ds->order_tile : CGKS_ORDER_TILE_DEFAULT;
    m.nv = d + 2;
    m.nk = ncoef_of(d);
    m.nq = nquad_of(d);
    m.n_cell = ds->n_cell;
    m.n_face = ds->n_face;
    m.xyz.assign(ds->xyz, ds->xyz + ds->n_vert * d);
    m.fptr.assign(ds->face_vert_ptr, ds->face_vert_ptr + ds->n_face + 1);
    if (m.fptr[0] != 0) return CGKS_EINVAL;
    for (int64_t f = 0; f < m.n_face; ++f)
        if (m.fptr[f + 1] < m.fptr[f]) return CGKS_EINVAL;
    m.fvert.assign(ds->face_vert, ds->face_vert + m.fptr[m.n_face]);
    m.owner.assign(ds->face_owner, ds->face_owner + m.n_face);
    m.neigh.assign(ds->face_neigh, ds->face_neigh + m.n_face);
    m.bc.assign(ds->face_bc, ds->face_bc + m.n_face);
    m.shift.assign(m.n_face * d, 0.0);
    if (ds->face_shift) m.shift.assign(ds->face_shift, ds->face_shift + m.n_face * d);
    for (int64_t v : m.fvert)
        if (v < 0 || v >= ds->n_vert) return CGKS_EMESH;
    m.n_bface = 0;
    for (int64_t f = 0; f < m.n_face; ++f) {
        if (m.owner[f] < 0 || m.owner[f] >= m.n_cell || m.neigh[f] >= m.n_cell || m.neigh[f] == m.owner[f])
            return CGKS_EMESH;
        if (m.neigh[f] < 0) {
            ++m.n_bface;
            if (m.bc[f] != CGKS_BC_SLIP_WALL && m.bc[f] != CGKS_BC_NOSLIP_ISOTHERMAL &&
                m.bc[f] != CGKS_BC_NOSLIP_ADIABATIC && m.bc[f] != CGKS_BC_FARFIELD)
                return CGKS_EMESH;
        }
    }
    canonical_faces(m);
    // faces of each cell in increasing face index
    m.cf_ptr.assign(m.n_cell + 1, 0);
    for (int64_t f = 0; f < m.n_face; ++f) {
        m.cf_ptr[m.owner[f] + 1]++;
        if (m.neigh[f] >= 0) m.cf_ptr[m.neigh[f] + 1]++;
    }
    for (int64_t i = 0; i < m.n_cell; ++i) {
        if (m.cf_ptr[i + 1] < d + 1 || m.cf_ptr[i + 1] > (d == 2 ? 4 : kMaxSlots)) return CGKS_EMESH;
        m.cf_ptr[i + 1] += m.cf_ptr[i];
    }
    m.cf_face.assign(m.cf_ptr[m.n_cell], 0);
    m.cf_side.assign(m.cf_ptr[m.n_cell], 0);
    {
        std::vector<int64_t> fill(m.cf_ptr.begin(), m.cf_ptr.end() - 1);
        for (int64_t f = 0; f < m.n_face; ++f) {
            const int64_t o = m.owner[f];
            m.cf_face[fill[o]] = f;
            m.cf_side[fill[o]++] = 0;
            if (m.neigh[f] >= 0) {
                const int64_t r = m.neigh[f];
                m.cf_face[fill[r]] = f;
                m.cf_side[fill[r]++] = 1;
            }
        }
    }
    cgks_status st = face_quadrature(m);
    if (st != CGKS_OK) return st;
    st = cell_geometry(m);
    if (st != CGKS_OK) return st;
    st = colour_and_order(m, ds->colour);
    if (st != CGKS_OK) return st;
    return recon_setup(m);
}

// ---------------------------------------------------------------------
// Faces from cells.
// ---------------------------------------------------------------------
namespace {

// local faces of the standard cell types (vertex positions in the cell's
// list; -1 ends a face)
struct TypeFaces {
    int dim, nvert, nface;
    int face[6][4];
};
const TypeFaces *type_faces(int t) {
    static const TypeFaces tri{2, 3, 3, {{0, 1, -1}, {1, 2, -1}, {2, 0, -1}}};
    static const TypeFaces quad{2, 4, 4, {{0, 1, -1}, {1, 2, -1}, {2, 3, -1}, {3, 0, -1}}};
    static const TypeFaces tet{3, 4, 4, {{0, 1, 2, -1}, {0, 1, 3, -1}, {1, 2, 3, -1}, {0, 2, 3, -1}}};
    static const TypeFaces pyr{3, 5, 5, {{0, 1, 2, 3}, {0, 1, 4, -1}, {1, 2, 4, -1}, {2, 3, 4, -1}, {3, 0, 4, -1}}};
    static const TypeFaces prism{3, 6, 5, {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}}};
    static const TypeFaces hex{3, 8, 6,
                               {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}}};
    switch (t) {
        case CGKS_CELL_TRI: return &tri;
        case CGKS_CELL_QUAD: return &quad;
        case CGKS_CELL_TET: return &tet;
        case CGKS_CELL_PYR: return &pyr;
        case CGKS_CELL_PRISM: return &prism;
        case CGKS_CELL_HEX: return &hex;
        default: return nullptr;
    }
}

struct CellFace {
    std::array<int64_t, 4> key;   // sorted vertex ids, padded with -1
    int64_t cell;
    int64_t v[4];
    int nv;
};

std::array<int64_t, 4> face_key(const int64_t *v, int nv) {
    std::array<int64_t, 4> k{-1, -1, -1, -1};
    for (int a = 0; a < nv; ++a) k[a] = v[a];
    std::sort(k.begin(), k.begin() + nv);
    return k;
}

}  // namespace

cgks_status build_host_mesh_cells(const cgks_mesh_desc *ds, HostMesh &m) {
    if (!ds || (ds->dim != 2 && ds->dim != 3) || ds->n_cell <= 0 || ds->n_vert <= 0 || !ds->xyz || !ds->cell_type ||
        !ds->cell_vert_ptr || !ds->cell_vert || ds->n_bface < 0 || ds->order_tile < 0)
        return CGKS_EINVAL;
    if (ds->n_bface > 0 && (!ds->bface_vert_ptr || !ds->bface_vert || !ds->bface_tag)) return CGKS_EINVAL;
    const int d = ds->dim;
    const int64_t nc = ds->n_cell, nvx = ds->n_vert, nb = ds->n_bface;
    const int64_t *cp = ds->cell_vert_ptr, *cv = ds->cell_vert;
    if (cp[0] != 0) return CGKS_EINVAL;
    auto vert_ok = [&](int64_t v) { return v >= 0 && v < nvx; };
    // 1. every cell's faces, and the cell's vertex centroid
    std::vector<CellFace> faces;
    faces.reserve(size_t(nc) * (d == 2 ? 3 : 5));
    std::vector<double> vctr(nc * d, 0.0);
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t b = cp[i], e = cp[i + 1];
        if (e <= b) return CGKS_EINVAL;
        const int t = ds->cell_type[i];
        std::vector<std::vector<int64_t>> fl;
        if (t == CGKS_CELL_POLY) {
            int64_t k = b;
            const int64_t n_f = cv[k++];
            if (n_f < d + 1 || n_f > (d == 2 ? 4 : kMaxSlots)) return CGKS_EMESH;
            for (int64_t q = 0; q < n_f; ++q) {
                if (k >= e) return CGKS_EINVAL;
                const int64_t nfv = cv[k++];
                if ((d == 2 && nfv != 2) || (d == 3 && nfv != 3 && nfv != 4) || k + nfv > e) return CGKS_EMESH;
                fl.emplace_back(cv + k, cv + k + nfv);
                k += nfv;
            }
            if (k != e) return CGKS_EINVAL;
        } else {
            const TypeFaces *tf = type_faces(t);
            if (!tf || tf->dim != d || e - b != tf->nvert) return CGKS_EINVAL;
            for (int q = 0; q < tf->nface; ++q) {
                std::vector<int64_t> f;
                for (int a = 0; a < 4 && tf->face[q][a] >= 0; ++a) f.push_back(cv[b + tf->face[q][a]]);
                fl.push_back(f);
            }
        }
        // vertex centroid over the cell's distinct vertices
        std::vector<int64_t> vs;
        for (auto &f : fl)
            for (int64_t v : f) {
                if (!vert_ok(v)) return CGKS_EMESH;
                vs.push_back(v);
            }
        std::sort(vs.begin(), vs.end());
        vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
        for (int64_t v : vs)
            for (int a = 0; a < d; ++a) vctr[i * d + a] += ds->xyz[v * d + a] / double(vs.size());
        for (auto &f : fl) {
            CellFace c{};
            c.nv = int(f.size());
            for (int a = 0; a < c.nv; ++a) c.v[a] = f[a];
            c.key = face_key(c.v, c.nv);
            for (int a = 1; a < c.nv; ++a)
                if (c.key[a] == c.key[a - 1]) return CGKS_EMESH;   // repeated vertex in a face
            c.cell = i;
            faces.push_back(c);
        }
    }
    // 2. shared faces: equal vertex sets
    std::vector<int64_t> ord(faces.size());
    for (size_t k = 0; k < faces.size(); ++k) ord[k] = int64_t(k);
    std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
        if (faces[x].key != faces[y].key) return faces[x].key < faces[y].key;
        return faces[x].cell < faces[y].cell;
    });
    // 3. the boundary list, by vertex set
    std::vector<std::array<int64_t, 4>> bkey(nb);
    for (int64_t q = 0; q < nb; ++q) {
        const int64_t b = ds->bface_vert_ptr[q], e = ds->bface_vert_ptr[q + 1];
        const int64_t nfv = e - b;
        if ((d == 2 && nfv != 2) || (d == 3 && nfv != 3 && nfv != 4)) return CGKS_EMESH;
        for (int64_t k = b; k < e; ++k)
            if (!vert_ok(ds->bface_vert[k])) return CGKS_EMESH;
        bkey[q] = face_key(ds->bface_vert + b, int(nfv));
        const int32_t tag = ds->bface_tag[q];
        if (tag != CGKS_BC_SLIP_WALL && tag != CGKS_BC_NOSLIP_ISOTHERMAL && tag != CGKS_BC_NOSLIP_ADIABATIC &&
            tag != CGKS_BC_FARFIELD && tag != CGKS_BC_PERIODIC)
            return CGKS_EMESH;
        if (tag == CGKS_BC_PERIODIC) {
            if (!ds->bface_pair) return CGKS_EINVAL;
            const int64_t p = ds->bface_pair[q];
            if (p < 0 || p >= nb || p == q || ds->bface_tag[p] != CGKS_BC_PERIODIC || ds->bface_pair[p] != q)
                return CGKS_EMESH;
        }
    }
    std::vector<int64_t> bord(nb);
    for (int64_t q = 0; q < nb; ++q) bord[q] = q;
    std::sort(bord.begin(), bord.end(), [&](int64_t x, int64_t y) { return bkey[x] < bkey[y]; });
    for (int64_t q = 1; q < nb; ++q)
        if (bkey[bord[q]] == bkey[bord[q - 1]]) return CGKS_EMESH;   // a boundary face listed twice
    std::vector<int64_t> bface_of(nb, -1);     // boundary face -> cell face
    // output arrays of the face-based form
    std::vector<int64_t> fptr{0}, fvert, own, nbr;
    std::vector<int32_t> fbc;
    std::vector<double> shift;
    // vertex average of a face, summed in increasing vertex id
    auto face_centre = [&](const CellFace &c, double *x) {
        for (int a = 0; a < d; ++a) {
            double s = ds->xyz[c.key[0] * d + a];
            for (int k = 1; k < c.nv; ++k) s += ds->xyz[c.key[k] * d + a];
            x[a] = s / c.nv;
        }
    };
    // the face's vertex cycle oriented outward from cell `owner`
    auto emit = [&](const CellFace &c, int64_t owner, int64_t neigh, int32_t tag, const double *sh) {
        const double *P[4];
        for (int k = 0; k < c.nv; ++k) P[k] = ds->xyz + c.v[k] * d;
        double nrm[3] = {0, 0, 0}, fc[3];
        face_centre(c, fc);
        if (d == 2) {
            nrm[0] = P[1][1] - P[0][1];
            nrm[1] = -(P[1][0] - P[0][0]);
        } else {
            double a[3], b[3];
            for (int k = 0; k < 3; ++k) {
                a[k] = c.nv == 4 ? P[2][k] - P[0][k] : P[1][k] - P[0][k];
                b[k] = c.nv == 4 ? P[3][k] - P[1][k] : P[2][k] - P[0][k];
            }
            cross(a, b, nrm);
        }
        double dot = 0;
        for (int k = 0; k < d; ++k) dot += nrm[k] * (fc[k] - vctr[owner * d + k]);
        for (int k = 0; k < c.nv; ++k) fvert.push_back(dot < 0 ? c.v[c.nv - 1 - k] : c.v[k]);
        fptr.push_back(int64_t(fvert.size()));
        own.push_back(owner);
        nbr.push_back(neigh);
        fbc.push_back(tag);
        for (int k = 0; k < d; ++k) shift.push_back(sh ? sh[k] : 0.0);
    };
    for (size_t k = 0; k < ord.size();) {
        size_t r = k + 1;
        while (r < ord.size() && faces[ord[r]].key == faces[ord[k]].key) ++r;
        if (r - k > 2) return CGKS_EMESH;                        // shared by more than two cells
        const CellFace &a = faces[ord[k]];
        if (r - k == 2) {
            const CellFace &b = faces[ord[k + 1]];
            if (a.cell == b.cell) return CGKS_EMESH;
            emit(a, a.cell, b.cell, CGKS_BC_INTERIOR, nullptr);   // a.cell < b.cell (sorted)
        } else {
            // a boundary face: find it in the list
            auto it = std::lower_bound(bord.begin(), bord.end(), a.key,
                                       [&](int64_t q, const std::array<int64_t, 4> &key) { return bkey[q] < key; });
            if (it == bord.end() || bkey[*it] != a.key) return CGKS_EMESH;
            bface_of[*it] = int64_t(ord[k]);
            if (ds->bface_tag[*it] != CGKS_BC_PERIODIC) emit(a, a.cell, -1, ds->bface_tag[*it], nullptr);
        }
        k = r;
    }
    for (int64_t q = 0; q < nb; ++q)
        if (bface_of[q] < 0) return CGKS_EMESH;                  // listed but matching no cell face
    // periodic pairs: one interior face, owner the smaller cell
    for (int64_t q = 0; q < nb; ++q) {
        if (ds->bface_tag[q] != CGKS_BC_PERIODIC || ds->bface_pair[q] < q) continue;
        const CellFace &a = faces[bface_of[q]], &b = faces[bface_of[ds->bface_pair[q]]];
        if (a.cell == b.cell) return CGKS_EMESH;
        const CellFace &o = a.cell < b.cell ? a : b, &n = a.cell < b.cell ? b : a;
        double co[3], cn[3], sh[3];
        face_centre(o, co);
        face_centre(n, cn);
        // the period: the offset of the two face centroids; components at
        // round-off level of the coordinates are zero
        for (int k = 0; k < d; ++k) {
            sh[k] = co[k] - cn[k];
            if (std::fabs(sh[k]) < 1e-12 * std::max({1.0, std::fabs(co[k]), std::fabs(cn[k])})) sh[k] = 0.0;
        }
        emit(o, o.cell, n.cell, CGKS_BC_INTERIOR, sh);
    }
    cgks_face_mesh_desc fd{};
    fd.dim = d;
    fd.n_vert = nvx;
    fd.xyz = ds->xyz;
    fd.n_cell = nc;
    fd.n_face = int64_t(own.size());
    fd.face_vert_ptr = fptr.data();
    fd.face_vert = fvert.data();
    fd.face_owner = own.data();
    fd.face_neigh = nbr.data();
    fd.face_bc = fbc.data();
    fd.face_shift = shift.data();
    fd.colour = ds->colour;
    fd.order_tile = ds->order_tile;
    return build_host_mesh(&fd, m);
}

}  // namespace cgks
