// Basis and quadrature tables for the device kernels.
//
// Basis: orthonormal Dubiner polynomials on the unit triangle / tetrahedron
// (the paper's Eq. 2 needs an orthonormal modal basis; the family is this
// project's reading), evaluated in collapsed coordinates with normalised
// Jacobi polynomials; gradients by the chain rule through the collapsed map.
// Quadrature: Gauss-Jacobi nodes by Newton's method with deflation on the
// Jacobi polynomial, weights by the Christoffel formula
//   w_k = 2^(a+b+1) G(n+a+1) G(n+b+1) / (G(n+a+b+1) n!) / ((1-x_k^2) P_n'(x_k)^2).
#include <cmath>

#include "internal.hpp"

namespace dgc {

namespace {

const double kPi = 3.14159265358979323846;

// P_n^(a,b)(x) and its derivative
void jacobi_pd(int n, double a, double b, double x, double *P, double *dP) {
    // value by the three-term recurrence
    auto val = [](int nn, double al, double be, double xx) {
        double p0 = 1.0;
        if (nn == 0) return p0;
        double p1 = 0.5 * ((al + be + 2.0) * xx + (al - be));
        for (int k = 1; k < nn; ++k) {
            double c = 2.0 * k + al + be;
            double num = (c + 1.0) * ((c + 2.0) * c * xx + al * al - be * be) * p1 - 2.0 * (k + al) * (k + be) * (c + 2.0) * p0;
            double den = 2.0 * (k + 1) * (k + al + be + 1.0) * c;
            p0 = p1;
            p1 = num / den;
        }
        return p1;
    };
    *P = val(n, a, b, x);
    *dP = n == 0 ? 0.0 : 0.5 * (n + a + b + 1.0) * val(n - 1, a + 1.0, b + 1.0, x);
}

double jacobi_h(int n, double a, double b) {  // squared norm
    return std::pow(2.0, a + b + 1.0) / (2.0 * n + a + b + 1.0) * std::tgamma(n + a + 1.0) * std::tgamma(n + b + 1.0) /
           (std::tgamma(n + a + b + 1.0) * std::tgamma(n + 1.0));
}

// normalised Jacobi value and derivative
void pnorm(int n, double a, double b, double x, double *v, double *d) {
    double P, dP;
    jacobi_pd(n, a, b, x, &P, &dP);
    double s = 1.0 / std::sqrt(jacobi_h(n, a, b));
    *v = P * s;
    *d = dP * s;
}

void gauss_jacobi(int n, double a, double b, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        // Chebyshev-like initial guess, averaged with the previous root
        double r = -std::cos((2.0 * k + 1.0) * kPi / (2.0 * n));
        if (k > 0) r = 0.5 * (r + x[k - 1]);
        for (int it = 0; it < 200; ++it) {
            double P, dP;
            jacobi_pd(n, a, b, r, &P, &dP);
            double s = 0.0;
            for (int i = 0; i < k; ++i) s += 1.0 / (r - x[i]);
            double delta = P / (dP - s * P);
            r -= delta;
            if (std::fabs(delta) < 1e-16) break;
        }
        x[k] = r;
    }
    double c = std::pow(2.0, a + b + 1.0) * std::tgamma(n + a + 1.0) * std::tgamma(n + b + 1.0) /
               (std::tgamma(n + a + b + 1.0) * std::tgamma(n + 1.0));
    for (int k = 0; k < n; ++k) {
        double P, dP;
        jacobi_pd(n, a, b, x[k], &P, &dP);
        w[k] = c / ((1.0 - x[k] * x[k]) * dP * dP);
    }
}

int nmodes(int dim, int p) { return dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6; }

// value and reference gradient of every mode at a point of the unit element
void dubiner(int dim, int p, const double *xi, double *phi, double *grad /* [dim][Np] or null */) {
    const int np = nmodes(dim, p);
    int m = 0;
    if (dim == 2) {
        double r = 2.0 * xi[0] - 1.0, s = 2.0 * xi[1] - 1.0;
        double one_s = 1.0 - s;
        double a = std::fabs(one_s) > 1e-15 ? 2.0 * (1.0 + r) / one_s - 1.0 : -1.0;
        double b = s;
        const double C = 2.0 * std::sqrt(2.0);
        for (int d = 0; d <= p; ++d) {
            for (int j = 0; j <= d; ++j) {
                int i = d - j;
                double fa, dfa, gb, dgb;
                pnorm(i, 0.0, 0.0, a, &fa, &dfa);
                pnorm(j, 2.0 * i + 1.0, 0.0, b, &gb, &dgb);
                double w = std::pow(1.0 - b, i);
                double g = gb * w;
                double dg = dgb * w - (i > 0 ? i * gb * std::pow(1.0 - b, i - 1) : 0.0);
                phi[m] = C * fa * g;
                if (grad) {
                    double dr = C * dfa * g * 2.0 / (1.0 - b);
                    double ds = C * (dfa * g * (1.0 + a) / (1.0 - b) + fa * dg);
                    grad[0 * np + m] = 2.0 * dr;
                    grad[1 * np + m] = 2.0 * ds;
                }
                ++m;
            }
        }
        return;
    }
    double r = 2.0 * xi[0] - 1.0, s = 2.0 * xi[1] - 1.0, t = 2.0 * xi[2] - 1.0;
    double st = s + t;
    double a = std::fabs(st) > 1e-15 ? -2.0 * (1.0 + r) / st - 1.0 : -1.0;
    double b = std::fabs(1.0 - t) > 1e-15 ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
    double c = t;
    const double C = 8.0;  // sqrt(8) (unit element) x 2 sqrt(2) (biunit normalisation)
    double da_dr = -2.0 / st, da_ds = 2.0 * (1.0 + r) / (st * st), da_dt = da_ds;
    double db_ds = 2.0 / (1.0 - t), db_dt = 2.0 * (1.0 + s) / ((1.0 - t) * (1.0 - t));
    for (int d = 0; d <= p; ++d) {
        for (int k = 0; k <= d; ++k) {
            for (int j = 0; j <= d - k; ++j) {
                int i = d - j - k;
                double fa, dfa, gb, dgb, hc, dhc;
                pnorm(i, 0.0, 0.0, a, &fa, &dfa);
                pnorm(j, 2.0 * i + 1.0, 0.0, b, &gb, &dgb);
                pnorm(k, 2.0 * i + 2.0 * j + 2.0, 0.0, c, &hc, &dhc);
                double wb = std::pow(1.0 - b, i), wc = std::pow(1.0 - c, i + j);
                double g = gb * wb, h = hc * wc;
                double dg = dgb * wb - (i > 0 ? i * gb * std::pow(1.0 - b, i - 1) : 0.0);
                double dh = dhc * wc - (i + j > 0 ? (i + j) * hc * std::pow(1.0 - c, i + j - 1) : 0.0);
                phi[m] = C * fa * g * h;
                if (grad) {
                    double dr = C * dfa * g * h * da_dr;
                    double ds = C * (dfa * g * h * da_ds + fa * dg * h * db_ds);
                    double dt = C * (dfa * g * h * da_dt + fa * dg * h * db_dt + fa * g * dh);
                    grad[0 * np + m] = 2.0 * dr;
                    grad[1 * np + m] = 2.0 * ds;
                    grad[2 * np + m] = 2.0 * dt;
                }
                ++m;
            }
        }
    }
}

// tensor Legendre basis of the unit square: phi_(a,b) = L_a(x) L_b(y) with
// L_n(x) = sqrt(2) Phat_n(2x - 1) (Phat_n normalised on [-1, 1]), mode
// j = b (p + 1) + a; gradients by the product rule
void legendre_tensor(int p, const double *xi, double *phi, double *grad /* [2][Np] or null */) {
    const int n = p + 1, np = n * n;
    std::vector<double> lx(n), dlx(n), ly(n), dly(n);
    for (int a = 0; a < n; ++a) {
        pnorm(a, 0.0, 0.0, 2.0 * xi[0] - 1.0, &lx[a], &dlx[a]);
        pnorm(a, 0.0, 0.0, 2.0 * xi[1] - 1.0, &ly[a], &dly[a]);
    }
    const double r2 = std::sqrt(2.0);
    for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a) {
            const int m = b * n + a;
            phi[m] = 2.0 * lx[a] * ly[b];
            if (grad) {
                grad[0 * np + m] = r2 * 2.0 * dlx[a] * r2 * ly[b];
                grad[1 * np + m] = r2 * lx[a] * r2 * 2.0 * dly[b];
            }
        }
}

const double kRefTri[3][2] = {{0, 0}, {1, 0}, {0, 1}};
const double kRefQuad[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
const int kQuadEdge[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
const double kRefTet[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
const int kTriEdge[3][2] = {{0, 1}, {1, 2}, {2, 0}};
const int kTetFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
const int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

}  // namespace

// Mixed meshes: the triangle's and the quadrilateral's tables side by side,
// the triangle's padded with zeros to the quadrilateral's (p+1)^2 modes.
dgc_status build_mixed_tables(int p, dgc_table_info *info, std::vector<double> *out) {
    if (p < 0 || p > 3) return fail(DGC_E_UNSUPPORTED, "order p=" + std::to_string(p) + " is not supported for mixed meshes");
    dgc_table_info tt, tq;
    std::vector<double> vt, vq;
    dgc_status s = build_tables(DGC_TRI, p, &tt, out ? &vt : nullptr);
    if (s == DGC_OK) s = build_tables(DGC_QUAD, p, &tq, out ? &vq : nullptr);
    if (s != DGC_OK) return s;
    dgc_table_info ti = tq;
    ti.elem_type = DGC_MIXED;
    ti.n_codes = tt.n_codes + tq.n_codes;
    const int np = tq.n_p, ntp = tt.n_p, qf = tq.n_qf, qv = tq.n_qv;
    ti.off_trace = 0;
    ti.off_proj = (int64_t)ti.n_codes * qf * np;
    ti.off_vb = ti.off_proj + (int64_t)ti.n_codes * qf * np;
    ti.off_vd = ti.off_vb + 2 * (int64_t)qv * np;
    ti.off_prolong = ti.off_vd + 2 * 2 * (int64_t)qv * np;
    ti.total = ti.off_prolong;
    if (info) *info = ti;
    if (!out) return DGC_OK;
    out->assign(ti.total, 0.0);
    double *T = out->data();
    // rows of n_src values (tri) or np values (quad) copied into rows of np
    auto rows = [&](int64_t dst, const double *src, int64_t n_rows, int n_src) {
        for (int64_t r = 0; r < n_rows; ++r)
            for (int j = 0; j < n_src; ++j) T[dst + r * np + j] = src[r * n_src + j];
    };
    rows(ti.off_trace, vt.data() + tt.off_trace, (int64_t)tt.n_codes * qf, ntp);
    rows(ti.off_trace + (int64_t)tt.n_codes * qf * np, vq.data() + tq.off_trace, (int64_t)tq.n_codes * qf, np);
    rows(ti.off_proj, vt.data() + tt.off_proj, (int64_t)tt.n_codes * qf, ntp);
    rows(ti.off_proj + (int64_t)tt.n_codes * qf * np, vq.data() + tq.off_proj, (int64_t)tq.n_codes * qf, np);
    rows(ti.off_vb, vt.data() + tt.off_vb, qv, ntp);
    rows(ti.off_vb + (int64_t)qv * np, vq.data() + tq.off_vb, qv, np);
    rows(ti.off_vd, vt.data() + tt.off_vd, 2 * (int64_t)qv, ntp);
    rows(ti.off_vd + 2 * (int64_t)qv * np, vq.data() + tq.off_vd, 2 * (int64_t)qv, np);
    return DGC_OK;
}

dgc_status build_tables(int32_t elem_type, int p, dgc_table_info *info, std::vector<double> *out) {
    if (elem_type == DGC_MIXED) return build_mixed_tables(p, info, out);
    if (elem_type != DGC_TRI && elem_type != DGC_QUAD && elem_type != DGC_TET)
        return fail(DGC_E_ARG, "unknown element type");
    const bool quad = elem_type == DGC_QUAD;
    const int dim = elem_type == DGC_TET ? 3 : 2;
    if (p < 0 || (elem_type == DGC_TRI && p > 5) || (quad && p > 3) || (dim == 3 && p > 2))
        return fail(DGC_E_UNSUPPORTED, "order p=" + std::to_string(p) + " is not supported for this element");
    dgc_table_info ti{};
    ti.elem_type = elem_type;
    ti.p = p;
    ti.dim = dim;
    ti.n_p = quad ? (p + 1) * (p + 1) : nmodes(dim, p);
    const int n = p + 1;
    ti.n_qv = dim == 2 ? n * n : n * n * n;
    ti.n_qf = dim == 2 ? p + 1 : (p <= 1 ? 3 : n * n);
    ti.n_orient = dim == 2 ? 4 : 6;
    const int nfaces = dim == 2 && !quad ? 3 : 4;
    ti.n_codes = nfaces * ti.n_orient;
    const int np = ti.n_p, qf = ti.n_qf, qv = ti.n_qv;
    ti.off_trace = 0;
    ti.off_proj = ti.off_trace + (int64_t)ti.n_codes * qf * np;
    ti.off_vb = ti.off_proj + (int64_t)ti.n_codes * qf * np;
    ti.off_vd = ti.off_vb + (int64_t)qv * np;
    ti.off_prolong = ti.off_vd + (int64_t)dim * qv * np;
    ti.total = ti.off_prolong + (elem_type == DGC_TRI ? 4 * (int64_t)np * np : 0);
    if (info) *info = ti;
    if (!out) return DGC_OK;
    out->assign(ti.total, 0.0);
    double *T = out->data();

    // face rule.  Edges: Gauss-Legendre on [0, 1].  Tetrahedron faces, as
    // barycentric weights fb[q][u] of the face's vertices in the left
    // element's order: the symmetric 3-point rule (2/3, 1/6, 1/6) up to
    // p = 1, else the collapsed Gauss-Jacobi product with n points per
    // direction (exact for degree 2n - 1), weights summing to 1.
    std::vector<double> fs, fw, fb;
    if (dim == 2) {
        gauss_jacobi(qf, 0.0, 0.0, fs, fw);
        for (int q = 0; q < qf; ++q) {
            fs[q] = 0.5 * (fs[q] + 1.0);
            fw[q] *= 0.5;
        }
    } else if (p <= 1) {
        fw.assign(3, 1.0 / 3.0);
        fb.assign(9, 1.0 / 6.0);
        for (int q = 0; q < 3; ++q) fb[q * 3 + q] = 2.0 / 3.0;
    } else {
        std::vector<double> xa, wa, xb, wb;
        gauss_jacobi(n, 0.0, 0.0, xa, wa);
        gauss_jacobi(n, 1.0, 0.0, xb, wb);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                double r = 0.5 * (1.0 + xa[i]) * (1.0 - xb[k]) - 1.0, s = xb[k];
                double x = 0.5 * (1.0 + r), y = 0.5 * (1.0 + s);
                fb.push_back(1.0 - x - y);
                fb.push_back(x);
                fb.push_back(y);
                fw.push_back(wa[i] * wb[k] / 4.0);
            }
    }
    std::vector<double> phi(np), grad(dim * np);
    auto basis = [&](const double *xi, double *ph, double *gr) {
        if (quad)
            legendre_tensor(p, xi, ph, gr);
        else
            dubiner(dim, p, xi, ph, gr);
    };
    for (int f = 0; f < nfaces; ++f) {
        for (int o = 0; o < ti.n_orient; ++o) {
            const int code = f * ti.n_orient + o;
            for (int q = 0; q < qf; ++q) {
                double xi[3] = {0, 0, 0};
                if (dim == 2) {
                    double t;
                    switch (o) {
                        case 0: t = fs[q]; break;
                        case 1: t = 1.0 - fs[q]; break;
                        case 2: t = 0.5 - 0.5 * fs[q]; break;
                        default: t = 1.0 - 0.5 * fs[q]; break;
                    }
                    const double *A = quad ? kRefQuad[kQuadEdge[f][0]] : kRefTri[kTriEdge[f][0]];
                    const double *B = quad ? kRefQuad[kQuadEdge[f][1]] : kRefTri[kTriEdge[f][1]];
                    xi[0] = A[0] + t * (B[0] - A[0]);
                    xi[1] = A[1] + t * (B[1] - A[1]);
                } else {
                    // the left element's face vertex u is this side's face vertex kPerm3[o][u]
                    for (int u = 0; u < 3; ++u) {
                        const double *V = kRefTet[kTetFace[f][kPerm3[o][u]]];
                        for (int e = 0; e < 3; ++e) xi[e] += fb[q * 3 + u] * V[e];
                    }
                }
                basis(xi, phi.data(), nullptr);
                for (int j = 0; j < np; ++j) {
                    T[ti.off_trace + ((int64_t)code * qf + q) * np + j] = phi[j];
                    T[ti.off_proj + ((int64_t)code * qf + q) * np + j] = fw[q] * phi[j];
                }
            }
        }
    }

    // volume rule: collapsed Gauss-Jacobi product
    std::vector<double> xa, wa, xb, wb, xc, wc;
    gauss_jacobi(n, 0.0, 0.0, xa, wa);
    gauss_jacobi(n, 1.0, 0.0, xb, wb);
    if (dim == 3) gauss_jacobi(n, 2.0, 0.0, xc, wc);
    int q = 0;
    auto put = [&](const double *xi, double w) {
        basis(xi, phi.data(), grad.data());
        for (int j = 0; j < np; ++j) {
            T[ti.off_vb + (int64_t)q * np + j] = phi[j];
            for (int d = 0; d < dim; ++d) T[ti.off_vd + ((int64_t)d * qv + q) * np + j] = w * grad[d * np + j];
        }
        ++q;
    };
    if (quad) {
        // tensor Gauss-Legendre, first coordinate fastest
        for (int iy = 0; iy < n; ++iy)
            for (int ix = 0; ix < n; ++ix) {
                double xi[2] = {0.5 * (1.0 + xa[ix]), 0.5 * (1.0 + xa[iy])};
                put(xi, wa[ix] * wa[iy] / 4.0);
            }
    } else if (dim == 2) {
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                double r = 0.5 * (1.0 + xa[i]) * (1.0 - xb[k]) - 1.0, s = xb[k];
                double xi[2] = {0.5 * (1.0 + r), 0.5 * (1.0 + s)};
                put(xi, wa[i] * wb[k] / 8.0);
            }
    } else {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    double r = 0.25 * (1.0 + xa[i]) * (1.0 - xb[j]) * (1.0 - xc[k]) - 1.0;
                    double s = 0.5 * (1.0 + xb[j]) * (1.0 - xc[k]) - 1.0;
                    double t = xc[k];
                    double xi[3] = {0.5 * (1.0 + r), 0.5 * (1.0 + s), 0.5 * (1.0 + t)};
                    put(xi, wa[i] * wb[j] * wc[k] / 64.0);
                }
    }

    // prolongation onto the four children of the midpoint split:
    // P_k[j][l] = 1/2 sum_q w_q phi_j(xi_q) phi_l(child_k(xi_q)), the factor
    // 1/2 = sqrt(det J_child / det J_parent) of the physical basis; the
    // product has degree 2p, within the volume rule's exactness 2p+1
    if (elem_type == DGC_TRI) {
        // child vertices in the parent's reference coordinates, each child's own order
        const double C[4][3][2] = {{{0, 0}, {0.5, 0}, {0, 0.5}},
                                   {{0.5, 0}, {1, 0}, {0.5, 0.5}},
                                   {{0, 0.5}, {0.5, 0.5}, {0, 1}},
                                   {{0.5, 0.5}, {0, 0.5}, {0.5, 0}}};
        std::vector<double> phic(np), phip(np);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                double r = 0.5 * (1.0 + xa[i]) * (1.0 - xb[k]) - 1.0, s = xb[k];
                double xi[2] = {0.5 * (1.0 + r), 0.5 * (1.0 + s)};
                const double w = wa[i] * wb[k] / 8.0;
                dubiner(dim, p, xi, phic.data(), nullptr);
                for (int c = 0; c < 4; ++c) {
                    double xp[2];
                    for (int d = 0; d < 2; ++d)
                        xp[d] = C[c][0][d] + xi[0] * (C[c][1][d] - C[c][0][d]) + xi[1] * (C[c][2][d] - C[c][0][d]);
                    dubiner(dim, p, xp, phip.data(), nullptr);
                    double *Pk = T + ti.off_prolong + (int64_t)c * np * np;
                    for (int j = 0; j < np; ++j)
                        for (int l = 0; l < np; ++l) Pk[j * np + l] += 0.5 * w * phic[j] * phip[l];
                }
            }
    }
    return DGC_OK;
}

}  // namespace dgc
