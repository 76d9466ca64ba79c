/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow FP64 CPU implementation of one two-level p-multigrid cycle
 * of the compact gas-kinetic scheme (CGKS), written from the paper
 * "A p-multigrid compact gas-kinetic scheme for steady-state acceleration"
 * (Ji, Shyy, Xu).  Only the test suite, the smoke check and the benchmark's
 * CPU baseline load it; the HIP library never links or calls it, and the two
 * share no code.  Loops are written in the order the paper states the steps;
 * nothing is blocked, fused or reordered.
 *
 * Where the paper defers a detail to other work the reading taken here is
 * named in the comment of the function that implements it.
 *
 * Parity unpinned (no check independent of this file beyond agreement with
 * the HIP path and behavioural tests): the weights of the reconstruction's
 * least-squares rows (recon_cell; its exactness on quadratic data, with
 * and without the mirror ghost rows of walls, is pinned), the high-order
 * time-step rule (cell_dt, om_dt), the viscous term of the implicit
 * operator's spectral radius (side_radius: its inviscid part |U.n| + c and
 * the larger-of-two-sides rule are pinned through the Lax-Friedrichs mass
 * flux at rest) and the low level's local time step (cell_dt with
 * cfl_low).  The relaxation update of om_lowlevel is pinned through the
 * backward-Euler equation its converged sweeps solve, ghost_cell through
 * mirror-symmetric quadratics and farfield_state through the Riemann
 * invariants, entropy and tangential velocity it must carry.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fPIC -shared.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NVMAX 5
#define DMAX 3
#define NCMAX 9    /* quadratic basis size in 3-D */
#define MAXGP 4

enum { BC_INTERIOR = 0, BC_SLIP = 1, BC_ISOTHERMAL = 2, BC_ADIABATIC = 3, BC_FARFIELD = 4 };

typedef struct {
    double gamma, mu, Pr, T_wall;
    double W_inf[NVMAX];
    double cfl_high, cfl_low;
    int n_implicit, n_sweeps;
    int time_scheme;   /* 0 = two-stage fourth order (S2O4), 1 = one-step second order (S1O2) */
    int explicit_only; /* 1: high-order step only, no low-order level */
    double dt_fixed;   /* > 0: use this global time step instead of the CFL rule */
    int low_flux;      /* first-order flux of the low-order level: 0 KFVS, 1 Lax-Friedrichs */
    int flux_kind;     /* high-order flux: 0 smooth solution, 1 full time-dependent solution */
    double weno_eps;   /* > 0: nonlinear reconstruction weights with this epsilon; 0: linear weights */
} om_params;

typedef struct {
    int dim, nv, ncoef;
    long n_cell, n_face, n_vert;
    const double *xyz;
    long *fptr, *fvert, *owner, *neigh;
    int *bc;
    double *shift;
    /* face quadrature */
    int *ngp;
    double *gx, *gn, *gw; /* [f*MAXGP+g][d], [..][d], [..] : point, unit normal, weight*Jacobian */
    double *avec, *S;     /* area vector [f][d], its magnitude */
    /* cells */
    double *vol, *ctr, *sec, *h; /* sec: central second moments (1/|V|) int (x-c)_a (x-c)_b, [i][6] */
    long *cf_ptr, *cf_face;
    int *cf_sign;
    int *colour;
    int n_colour;
} om_mesh;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */
static void vcopy(double *a, const double *b, int n) { memcpy(a, b, sizeof(double) * n); }

/* coordinate of vertex k of face f as seen from the cell on side `side`
   (0 owner, 1 neighbour): the neighbour's frame is the owner's minus shift */
static void face_vertex(const om_mesh *m, long f, int k, int side, double *x) {
    long v = m->fvert[m->fptr[f] + k];
    for (int a = 0; a < m->dim; a++) {
        x[a] = m->xyz[v * m->dim + a];
        if (side) x[a] -= m->shift[f * m->dim + a];
    }
}

static void local_frame(int dim, const double *n, double e[3][3]);
static void state_to_local(int dim, double e[3][3], const double *W, double *Wl);
static void vec_to_global(int dim, double e[3][3], const double *Fl, double *F);
static void farfield_state(int dim, double gamma, const double *Wl, const double *Winf_l, double *Wb);

static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------ */
/* Geometry: face Gauss points (Sec. 2.1).  The paper uses 3 points on a */
/* triangular face and 4 on a quadrilateral one with an iso-parametric   */
/* (bilinear) map and a normal at every Gauss point.  Reading: the       */
/* 3-point degree-2 triangle rule at barycentric (2/3,1/6,1/6), the 2x2  */
/* Gauss-Legendre rule on the bilinear quad, and 2-point Gauss-Legendre  */
/* on 2-D edges.                                                         */
/* ------------------------------------------------------------------ */
static void bilinear(const double P[4][3], double s, double t, double *x, double *xs, double *xt) {
    for (int a = 0; a < 3; a++) {
        x[a] = (1 - s) * (1 - t) * P[0][a] + s * (1 - t) * P[1][a] + s * t * P[2][a] + (1 - s) * t * P[3][a];
        xs[a] = (1 - t) * (P[1][a] - P[0][a]) + t * (P[2][a] - P[3][a]);
        xt[a] = (1 - s) * (P[3][a] - P[0][a]) + s * (P[2][a] - P[1][a]);
    }
}

static void face_quadrature(om_mesh *m) {
    int d = m->dim;
    const double g2[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    for (long f = 0; f < m->n_face; f++) {
        int nfv = (int)(m->fptr[f + 1] - m->fptr[f]);
        double P[4][3] = {{0}};
        for (int k = 0; k < nfv; k++) face_vertex(m, f, k, 0, P[k]);
        double *gx = m->gx + f * MAXGP * d, *gn = m->gn + f * MAXGP * d, *gw = m->gw + f * MAXGP;
        if (d == 2) {
            double tx = P[1][0] - P[0][0], ty = P[1][1] - P[0][1];
            double L = sqrt(tx * tx + ty * ty);
            m->ngp[f] = 2;
            for (int g = 0; g < 2; g++) {
                gx[g * 2 + 0] = P[0][0] + g2[g] * tx;
                gx[g * 2 + 1] = P[0][1] + g2[g] * ty;
                gn[g * 2 + 0] = ty / L;
                gn[g * 2 + 1] = -tx / L;
                gw[g] = 0.5 * L;
            }
        } else if (nfv == 3) {
            double e1[3], e2[3], c[3];
            for (int a = 0; a < 3; a++) { e1[a] = P[1][a] - P[0][a]; e2[a] = P[2][a] - P[0][a]; }
            cross3(e1, e2, c);
            double A2 = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            m->ngp[f] = 3;
            for (int g = 0; g < 3; g++) {
                double b[3] = {1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
                b[g] = 2.0 / 3.0;
                for (int a = 0; a < 3; a++) {
                    gx[g * 3 + a] = b[0] * P[0][a] + b[1] * P[1][a] + b[2] * P[2][a];
                    gn[g * 3 + a] = c[a] / A2;
                }
                gw[g] = 0.5 * A2 / 3.0;
            }
        } else {
            m->ngp[f] = 4;
            int g = 0;
            for (int it = 0; it < 2; it++)
                for (int is = 0; is < 2; is++, g++) {
                    double x[3], xs[3], xt[3], c[3];
                    bilinear(P, g2[is], g2[it], x, xs, xt);
                    cross3(xs, xt, c);
                    double J = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
                    for (int a = 0; a < 3; a++) { gx[g * 3 + a] = x[a]; gn[g * 3 + a] = c[a] / J; }
                    gw[g] = 0.25 * J;
                }
        }
        /* area vector = sum of weight * normal (exact for the linear element) */
        double s2 = 0;
        for (int a = 0; a < d; a++) {
            double acc = 0;
            for (int g = 0; g < m->ngp[f]; g++) acc += gw[g] * gn[g * d + a];
            m->avec[f * d + a] = acc;
            s2 += acc * acc;
        }
        m->S[f] = sqrt(s2);
    }
}

/* ------------------------------------------------------------------ */
/* Cell volume, centroid and central second moments by the divergence   */
/* theorem over the cell's faces, with face rules exact for the cubic   */
/* integrands (edges: 2-point Gauss; triangles: 6-point degree-4 rule;  */
/* bilinear quads: 3x3 Gauss on the parameter square).                 */
/* ------------------------------------------------------------------ */
static void accumulate_moments(int d, const double *y, const double *nw, double *V, double *M1, double *M2) {
    /* nw = normal * weight (outward); y = point relative to the reference */
    for (int a = 0; a < d; a++) {
        *V += y[a] * nw[a] / d;
        M1[a] += 0.5 * y[a] * y[a] * nw[a];
    }
    for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++) {
            if (a == b) M2[a * 3 + b] += y[a] * y[a] * y[a] / 3.0 * nw[a];
            else M2[a * 3 + b] += 0.5 * y[a] * y[a] * y[b] * nw[a];
        }
}

static void cell_geometry(om_mesh *m) {
    int d = m->dim;
    static const double t6p[2][3] = {{0.445948490915965, 0.445948490915965, 0.108103018168070},
                                     {0.091576213509771, 0.091576213509771, 0.816847572980459}};
    static const double t6w[2] = {0.223381589678011, 0.109951743655322};
    const double g3[3] = {0.5 - 0.5 * sqrt(0.6), 0.5, 0.5 + 0.5 * sqrt(0.6)};
    const double w3[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    const double g2[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    for (long i = 0; i < m->n_cell; i++) {
        /* reference point: mean of the vertices of the cell's faces */
        double ref[3] = {0, 0, 0};
        int nref = 0;
        for (long q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; q++) {
            long f = m->cf_face[q];
            int side = m->cf_sign[q] > 0 ? 0 : 1;
            int nfv = (int)(m->fptr[f + 1] - m->fptr[f]);
            for (int k = 0; k < nfv; k++) {
                double x[3];
                face_vertex(m, f, k, side, x);
                for (int a = 0; a < d; a++) ref[a] += x[a];
                nref++;
            }
        }
        for (int a = 0; a < d; a++) ref[a] /= nref;
        double V = 0, M1[3] = {0, 0, 0}, M2[9] = {0};
        double sumS = 0;
        for (long q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; q++) {
            long f = m->cf_face[q];
            int sg = m->cf_sign[q];
            int side = sg > 0 ? 0 : 1;
            int nfv = (int)(m->fptr[f + 1] - m->fptr[f]);
            double P[4][3] = {{0}};
            for (int k = 0; k < nfv; k++) {
                face_vertex(m, f, k, side, P[k]);
                for (int a = 0; a < d; a++) P[k][a] -= ref[a];
            }
            sumS += m->S[f];
            if (d == 2) {
                double tx = P[1][0] - P[0][0], ty = P[1][1] - P[0][1];
                double L = sqrt(tx * tx + ty * ty);
                double n[2] = {sg * ty / L, -sg * tx / L};
                for (int g = 0; g < 2; g++) {
                    double y[2] = {P[0][0] + g2[g] * tx, P[0][1] + g2[g] * ty};
                    double nw[2] = {n[0] * 0.5 * L, n[1] * 0.5 * L};
                    accumulate_moments(2, y, nw, &V, M1, M2);
                }
            } else if (nfv == 3) {
                double e1[3], e2[3], c[3];
                for (int a = 0; a < 3; a++) { e1[a] = P[1][a] - P[0][a]; e2[a] = P[2][a] - P[0][a]; }
                cross3(e1, e2, c); /* |c| = 2 * area */
                for (int grp = 0; grp < 2; grp++)
                    for (int r = 0; r < 3; r++) {
                        double b[3];
                        for (int k = 0; k < 3; k++) b[k] = t6p[grp][(k + r) % 3];
                        double y[3], nw[3];
                        for (int a = 0; a < 3; a++) {
                            y[a] = b[0] * P[0][a] + b[1] * P[1][a] + b[2] * P[2][a];
                            nw[a] = sg * c[a] * 0.5 * t6w[grp];
                        }
                        accumulate_moments(3, y, nw, &V, M1, M2);
                    }
            } else {
                for (int it = 0; it < 3; it++)
                    for (int is = 0; is < 3; is++) {
                        double y[3], xs[3], xt[3], c[3], nw[3];
                        bilinear(P, g3[is], g3[it], y, xs, xt);
                        cross3(xs, xt, c);
                        for (int a = 0; a < 3; a++) nw[a] = sg * c[a] * w3[is] * w3[it];
                        accumulate_moments(3, y, nw, &V, M1, M2);
                    }
            }
        }
        m->vol[i] = V;
        double yc[3];
        for (int a = 0; a < d; a++) {
            yc[a] = M1[a] / V;
            m->ctr[i * d + a] = ref[a] + yc[a];
        }
        int q = 0;
        for (int a = 0; a < d; a++)
            for (int b = a; b < d; b++) m->sec[i * 6 + q++] = M2[a * 3 + b] / V - yc[a] * yc[b];
        m->h[i] = 2.0 * d * V / sumS;
    }
}

/* Multicolour ordering of the smoother (a reading: the paper sweeps by
   element index).  Welsh-Powell greedy colouring: cells are visited by
   decreasing number of faces shared with another cell (ties: increasing cell
   id) and each takes the smallest colour no already coloured face neighbour
   has.  The classes are then renumbered for the sweep, which visits the first
   colour three times per implicit step, the last twice and the others four
   times: the largest class becomes the last colour, the second largest the
   first, the remaining ones the colours between in decreasing size (equal
   sizes: smaller greedy colour first). */
static void colour_cells(om_mesh *m) {
    long n = m->n_cell;
    int *deg = (int *)calloc(n, sizeof(int));
    int maxdeg = 0;
    for (long i = 0; i < n; i++) {
        m->colour[i] = -1;
        for (long q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; q++) {
            long f = m->cf_face[q];
            long o = m->cf_sign[q] > 0 ? m->neigh[f] : m->owner[f];
            if (o >= 0) deg[i]++;
        }
        if (deg[i] > maxdeg) maxdeg = deg[i];
    }
    int ncol = 0;
    for (int dg = maxdeg; dg >= 0; dg--)
        for (long i = 0; i < n; i++) {
            if (deg[i] != dg) continue;
            int used[64] = {0};
            for (long q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; q++) {
                long f = m->cf_face[q];
                long o = m->cf_sign[q] > 0 ? m->neigh[f] : m->owner[f];
                if (o >= 0 && m->colour[o] >= 0) used[m->colour[o]] = 1;
            }
            int c = 0;
            while (used[c]) c++;
            m->colour[i] = c;
            if (c + 1 > ncol) ncol = c + 1;
        }
    free(deg);
    /* classes by decreasing size, then the new colour of each */
    long size[64] = {0};
    int rank[64], newc[64];
    for (long i = 0; i < n; i++) size[m->colour[i]]++;
    for (int c = 0; c < ncol; c++) rank[c] = c;
    for (int a = 1; a < ncol; a++)        /* insertion sort: stable, so ties keep the greedy order */
        for (int b = a; b > 0 && size[rank[b]] > size[rank[b - 1]]; b--) {
            int t = rank[b]; rank[b] = rank[b - 1]; rank[b - 1] = t;
        }
    for (int k = 0; k < ncol; k++) {
        if (k == 0) newc[rank[k]] = ncol - 1;
        else if (k == 1) newc[rank[k]] = 0;
        else newc[rank[k]] = k - 1;
    }
    for (long i = 0; i < n; i++) m->colour[i] = newc[m->colour[i]];
    m->n_colour = ncol;
}

/* ------------------------------------------------------------------ */
/* mesh construction                                                     */
/* ------------------------------------------------------------------ */
om_mesh *om_mesh_create(int dim, long n_vert, const double *xyz, long n_cell, long n_face, const long *fptr,
                        const long *fvert, const long *owner, const long *neigh, const int *bc,
                        const double *shift) {
    om_mesh *m = (om_mesh *)calloc(1, sizeof(om_mesh));
    m->dim = dim;
    m->nv = dim + 2;
    m->ncoef = dim == 2 ? 5 : 9;
    m->n_cell = n_cell;
    m->n_face = n_face;
    m->n_vert = n_vert;
    double *x = (double *)malloc(sizeof(double) * n_vert * dim);
    vcopy(x, xyz, (int)(n_vert * dim));
    m->xyz = x;
    m->fptr = (long *)malloc(sizeof(long) * (n_face + 1));
    memcpy(m->fptr, fptr, sizeof(long) * (n_face + 1));
    m->fvert = (long *)malloc(sizeof(long) * fptr[n_face]);
    memcpy(m->fvert, fvert, sizeof(long) * fptr[n_face]);
    m->owner = (long *)malloc(sizeof(long) * n_face);
    memcpy(m->owner, owner, sizeof(long) * n_face);
    m->neigh = (long *)malloc(sizeof(long) * n_face);
    memcpy(m->neigh, neigh, sizeof(long) * n_face);
    m->bc = (int *)malloc(sizeof(int) * n_face);
    memcpy(m->bc, bc, sizeof(int) * n_face);
    m->shift = (double *)calloc(n_face * dim, sizeof(double));
    if (shift) memcpy(m->shift, shift, sizeof(double) * n_face * dim);
    m->ngp = (int *)calloc(n_face, sizeof(int));
    m->gx = (double *)calloc(n_face * MAXGP * dim, sizeof(double));
    m->gn = (double *)calloc(n_face * MAXGP * dim, sizeof(double));
    m->gw = (double *)calloc(n_face * MAXGP, sizeof(double));
    m->avec = (double *)calloc(n_face * dim, sizeof(double));
    m->S = (double *)calloc(n_face, sizeof(double));
    m->vol = (double *)calloc(n_cell, sizeof(double));
    m->ctr = (double *)calloc(n_cell * dim, sizeof(double));
    m->sec = (double *)calloc(n_cell * 6, sizeof(double));
    m->h = (double *)calloc(n_cell, sizeof(double));
    m->colour = (int *)calloc(n_cell, sizeof(int));
    /* cell -> face lists, faces in increasing face index */
    m->cf_ptr = (long *)calloc(n_cell + 1, sizeof(long));
    for (long f = 0; f < n_face; f++) {
        m->cf_ptr[owner[f] + 1]++;
        if (neigh[f] >= 0) m->cf_ptr[neigh[f] + 1]++;
    }
    for (long i = 0; i < n_cell; i++) m->cf_ptr[i + 1] += m->cf_ptr[i];
    m->cf_face = (long *)malloc(sizeof(long) * m->cf_ptr[n_cell]);
    m->cf_sign = (int *)malloc(sizeof(int) * m->cf_ptr[n_cell]);
    long *fill = (long *)calloc(n_cell, sizeof(long));
    for (long f = 0; f < n_face; f++) {
        long o = owner[f];
        m->cf_face[m->cf_ptr[o] + fill[o]] = f;
        m->cf_sign[m->cf_ptr[o] + fill[o]++] = 1;
        if (neigh[f] >= 0) {
            long r = neigh[f];
            m->cf_face[m->cf_ptr[r] + fill[r]] = f;
            m->cf_sign[m->cf_ptr[r] + fill[r]++] = -1;
        }
    }
    free(fill);
    face_quadrature(m);
    cell_geometry(m);
    colour_cells(m);
    return m;
}

void om_mesh_destroy(om_mesh *m) {
    if (!m) return;
    free((void *)m->xyz); free(m->fptr); free(m->fvert); free(m->owner); free(m->neigh); free(m->bc);
    free(m->shift); free(m->ngp); free(m->gx); free(m->gn); free(m->gw); free(m->avec); free(m->S);
    free(m->vol); free(m->ctr); free(m->sec); free(m->h); free(m->colour); free(m->cf_ptr);
    free(m->cf_face); free(m->cf_sign);
    free(m);
}

/* geometry export for the tests */
int om_mesh_n_colour(const om_mesh *m) { return m->n_colour; }

/* replace the colouring by a caller's (class ids 0..63; the classes must be
   independent sets, which the relaxation's order relies on).  Returns -1
   if two face neighbours share a colour or an id is out of range. */
int om_mesh_set_colour(om_mesh *m, const int *colour) {
    int ncol = 0;
    for (long i = 0; i < m->n_cell; i++) {
        if (colour[i] < 0 || colour[i] >= 64) return -1;
        if (colour[i] + 1 > ncol) ncol = colour[i] + 1;
    }
    for (long f = 0; f < m->n_face; f++)
        if (m->neigh[f] >= 0 && colour[m->owner[f]] == colour[m->neigh[f]]) return -1;
    for (long i = 0; i < m->n_cell; i++) m->colour[i] = colour[i];
    m->n_colour = ncol;
    return 0;
}
void om_mesh_cells(const om_mesh *m, double *vol, double *ctr, double *sec, double *h, int *colour) {
    for (long i = 0; i < m->n_cell; i++) {
        vol[i] = m->vol[i];
        h[i] = m->h[i];
        colour[i] = m->colour[i];
        for (int a = 0; a < m->dim; a++) ctr[i * m->dim + a] = m->ctr[i * m->dim + a];
        for (int q = 0; q < 6; q++) sec[i * 6 + q] = m->sec[i * 6 + q];
    }
}
void om_mesh_faces(const om_mesh *m, int *ngp, double *gx, double *gn, double *gw, double *avec, double *S) {
    int d = m->dim;
    for (long f = 0; f < m->n_face; f++) {
        ngp[f] = m->ngp[f];
        S[f] = m->S[f];
        for (int a = 0; a < d; a++) avec[f * d + a] = m->avec[f * d + a];
        for (int g = 0; g < MAXGP; g++) {
            gw[f * MAXGP + g] = m->gw[f * MAXGP + g];
            for (int a = 0; a < d; a++) {
                gx[(f * MAXGP + g) * d + a] = m->gx[(f * MAXGP + g) * d + a];
                gn[(f * MAXGP + g) * d + a] = m->gn[(f * MAXGP + g) * d + a];
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Compact reconstruction (Sec. 2.2 defers it; linear weights are used  */
/* for smooth flow, Sec. 4).  Reading: one quadratic per cell,           */
/*   P_i(x) = W_i + sum_k c_k (phi_k(x) - <phi_k>_i),                    */
/* phi_k the monomials of degree 1..2 in xi = (x - x_i)/h_i, which keeps */
/* the cell average exactly; the c_k solve, in the least-squares sense,  */
/*   <P_i>_m = W_m and h_i <grad P_i>_m = h_i gradW_m  for every face     */
/*   neighbour m, and h_i <grad P_i>_i = h_i gradW_i,                     */
/* unweighted rows, by Householder QR.  A boundary face brings the rows  */
/* of its ghost cell (ghost_cell below) when boundary data are given.    */
/* ------------------------------------------------------------------ */
/* a stencil whose rows do not fix every quadratic coefficient (an R
   diagonal below RANK_TOL of the largest) falls back to the linear
   reconstruction from the same rows */
#define RANK_TOL 1e-8
static const int QA[2][6] = {{0, 0, 1, 0, 0, 0}, {0, 1, 2, 0, 0, 1}};
static const int QB[2][6] = {{0, 1, 1, 0, 0, 0}, {0, 1, 2, 1, 2, 2}};

/* index of sec[] for the pair (a, b), a <= b */
static int sec_index(int d, int a, int b) {
    if (a > b) { int t = a; a = b; b = t; }
    if (d == 2) return a == 0 ? b : 2;
    static const int idx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    return idx[a][b];
}

/* centroid of face-neighbour m of cell i through face f, in i's frame */
static void neighbour_centroid(const om_mesh *m, long i, long f, long nb, double *c) {
    int d = m->dim;
    for (int a = 0; a < d; a++) {
        c[a] = m->ctr[nb * d + a];
        if (m->owner[f] == i) c[a] += m->shift[f * d + a];
        else c[a] -= m->shift[f * d + a];
    }
}

/* <phi_k> over a cell with centroid c and central second moments sec,
   in the basis of cell i (centre xi_c, scale h) */
static void basis_average(const om_mesh *m, const double *c, const double *sec, const double *xc, double h,
                          double *avg) {
    int d = m->dim, nq = d == 2 ? 3 : 6;
    double y[3];
    for (int a = 0; a < d; a++) { y[a] = (c[a] - xc[a]) / h; avg[a] = y[a]; }
    for (int q = 0; q < nq; q++) {
        int a = QA[d - 2][q], b = QB[d - 2][q];
        avg[d + q] = (sec[sec_index(d, a, b)] + (c[a] - xc[a]) * (c[b] - xc[b])) / (h * h);
    }
}

/* least squares by Householder QR: A[nr][nc] (row major), B[nr][nrhs];
   the solution overwrites the first nc rows of B.  Returns
   min |R_kk| / max |R_kk| (0 when a column is dependent). */
static double lsq_qr(int nr, int nc, double *A, int nrhs, double *B) {
    for (int k = 0; k < nc; k++) {
        double nrm = 0;
        for (int r = k; r < nr; r++) nrm += A[r * nc + k] * A[r * nc + k];
        nrm = sqrt(nrm);
        double alpha = A[k * nc + k] > 0 ? -nrm : nrm;
        double v[64];
        for (int r = k; r < nr; r++) v[r] = A[r * nc + k];
        v[k] -= alpha;
        double vv = 0;
        for (int r = k; r < nr; r++) vv += v[r] * v[r];
        if (vv == 0) continue;
        for (int j = k; j < nc; j++) {
            double s = 0;
            for (int r = k; r < nr; r++) s += v[r] * A[r * nc + j];
            s = 2 * s / vv;
            for (int r = k; r < nr; r++) A[r * nc + j] -= s * v[r];
        }
        for (int j = 0; j < nrhs; j++) {
            double s = 0;
            for (int r = k; r < nr; r++) s += v[r] * B[r * nrhs + j];
            s = 2 * s / vv;
            for (int r = k; r < nr; r++) B[r * nrhs + j] -= s * v[r];
        }
    }
    double rmin = INFINITY, rmax = 0;
    for (int k = 0; k < nc; k++) {
        double r = fabs(A[k * nc + k]);
        if (r < rmin) rmin = r;
        if (r > rmax) rmax = r;
    }
    if (!(rmin > RANK_TOL * rmax)) return 0.0;
    for (int j = 0; j < nrhs; j++)
        for (int k = nc - 1; k >= 0; k--) {
            double s = B[k * nrhs + j];
            for (int q = k + 1; q < nc; q++) s -= A[k * nc + q] * B[q * nrhs + j];
            B[k * nrhs + j] = s / A[k * nc + k];
        }
    return rmin / rmax;
}

/* Ghost cell of boundary face f seen from cell i: the mirror image of i
   in the plane through the face centroid with the face normal, carrying
   the boundary data
     far field:        average = characteristic boundary state of W_i,
                       gradient = 0;
     slip wall:        W_g(x) = M W_i(R x), M reflecting the momentum;
     no-slip wall:     W_g(x) = M W_i(R x), M reversing the momentum;
   R = I - 2 n n^T.  Returns 0, or -3 for an unsupported tag. */
static int ghost_cell(const om_mesh *m, const om_params *P, long i, long f, const double *W, const double *dW,
                      double *cg, double *secg, double *Wg, double *dWg) {
    int d = m->dim, nv = m->nv;
    long N = m->n_cell;
    double n[3] = {0, 0, 0}, xf[3] = {0, 0, 0}, sw = 0;
    for (int a = 0; a < d; a++) n[a] = m->avec[f * d + a] / m->S[f];
    for (int g = 0; g < m->ngp[f]; g++) {
        double w = m->gw[f * MAXGP + g];
        sw += w;
        for (int a = 0; a < d; a++) xf[a] += w * m->gx[(f * MAXGP + g) * d + a];
    }
    for (int a = 0; a < d; a++) xf[a] /= sw;
    const double *ci = m->ctr + i * d;
    double dist = 0;
    for (int a = 0; a < d; a++) dist += (xf[a] - ci[a]) * n[a];
    for (int a = 0; a < d; a++) cg[a] = ci[a] + 2.0 * dist * n[a];
    double R[3][3], S[3][3], T[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            R[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * n[a] * n[b];
            S[a][b] = (a < d && b < d) ? m->sec[i * 6 + sec_index(d, a, b)] : 0.0;
        }
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += R[a][k] * S[k][b];
            T[a][b] = acc;
        }
    for (int a = 0; a < d; a++)
        for (int b = a; b < d; b++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += T[a][k] * R[k][b];
            secg[sec_index(d, a, b)] = acc;
        }
    double Wi[NVMAX];
    for (int v = 0; v < nv; v++) Wi[v] = W[v * N + i];
    int bc = m->bc[f];
    if (bc == BC_FARFIELD) {
        double e[3][3], Wl[NVMAX], Winf_l[NVMAX], Wb[NVMAX];
        local_frame(d, n, e);
        state_to_local(d, e, Wi, Wl);
        state_to_local(d, e, P->W_inf, Winf_l);
        farfield_state(d, P->gamma, Wl, Winf_l, Wb);
        vec_to_global(d, e, Wb, Wg);
        for (int k = 0; k < d * nv; k++) dWg[k] = 0.0;
        return 0;
    }
    if (bc != BC_SLIP && bc != BC_ISOTHERMAL && bc != BC_ADIABATIC) return -3;
    /* M acting on (rho, m, E): identity on scalars, R (slip) or -I (no slip) on m */
    double Mm[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Mm[a][b] = bc == BC_SLIP ? R[a][b] : (a == b ? -1.0 : 0.0);
    Wg[0] = Wi[0];
    Wg[nv - 1] = Wi[nv - 1];
    for (int a = 0; a < d; a++) {
        double acc = 0;
        for (int b = 0; b < d; b++) acc += Mm[a][b] * Wi[1 + b];
        Wg[1 + a] = acc;
    }
    /* gradient of x -> M W_i(R x): G_g[a][v] = sum_b R[a][b] (M G_i[b])_v */
    for (int a = 0; a < d; a++)
        for (int v = 0; v < nv; v++) {
            double acc = 0;
            for (int b = 0; b < d; b++) {
                double mg;
                if (v == 0 || v == nv - 1) mg = dW[(b * nv + v) * N + i];
                else {
                    mg = 0;
                    for (int c = 0; c < d; c++) mg += Mm[v - 1][c] * dW[(b * nv + 1 + c) * N + i];
                }
                acc += R[a][b] * mg;
            }
            dWg[a * nv + v] = acc;
        }
    return 0;
}

/* Nonlinear weights of the compact reconstruction, for flows with
   discontinuities (Sec. 4 uses WENO-type weights there with a small
   positive epsilon; their form is taken from other work).  Reading: the
   candidates are the quadratic P0 of the least-squares fit and, for every
   face neighbour or ghost m of the stencil, the linear polynomial P_m that
   fits m's average and h-scaled averaged gradient alone in the least-squares
   sense; linear weights gamma_0 = 0.95 for P0 and (1 - gamma_0)/M for each
   of the M linear candidates; smoothness indicators in the cell's scaled
   coordinates xi = (x - x_i)/h_i,
     beta = sum_a <(dP/dxi_a)^2>_i + sum_{a<=b} (d2P/dxi_a dxi_b)^2
   (<.>_i the cell average); weights omega_k proportional to
   gamma_k / (eps + beta_k)^2, normalised per variable; and the result
     P = omega_0/gamma_0 (P0 - sum_m gamma_m P_m) + sum_m omega_m P_m,
   which is P0 when the indicators agree (linear data) and tends to P0 as
   eps grows. */
#define WENO_GAMMA0 0.95
static void weno_combine(const om_mesh *m, long i, int nb_count, const double *nb_xi, const double *nb_dW,
                         const double *nb_dU, double eps, double *coef) {
    int d = m->dim, nv = m->nv, nq = d == 2 ? 3 : 6;
    double h = m->h[i];
    /* linear candidates: rows xi_m . c = W_m - W_i and c = h grad W_m */
    double cand[8][DMAX * NVMAX];
    for (int k = 0; k < nb_count; k++) {
        double A[(DMAX + 1) * DMAX], B[(DMAX + 1) * NVMAX];
        for (int a = 0; a < d; a++) A[a] = nb_xi[k * d + a];
        for (int v = 0; v < nv; v++) B[v] = nb_dU[k * nv + v];
        for (int r = 0; r < d; r++) {
            for (int a = 0; a < d; a++) A[(1 + r) * d + a] = r == a ? 1.0 : 0.0;
            for (int v = 0; v < nv; v++) B[(1 + r) * nv + v] = h * nb_dW[(k * d + r) * nv + v];
        }
        lsq_qr(d + 1, d, A, nv, B);
        for (int a = 0; a < d; a++)
            for (int v = 0; v < nv; v++) cand[k][a * nv + v] = B[a * nv + v];
    }
    /* second moments of the cell in xi */
    double Mxx[3][3];
    for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++) Mxx[a][b] = m->sec[i * 6 + sec_index(d, a, b)] / (h * h);
    double g0 = WENO_GAMMA0, gk = (1.0 - WENO_GAMMA0) / nb_count;
    for (int v = 0; v < nv; v++) {
        /* Hessian of P0 in xi */
        double D[3][3] = {{0}};
        for (int q = 0; q < nq; q++) {
            int p = QA[d - 2][q], r = QB[d - 2][q];
            double c = coef[(d + q) * nv + v];
            if (p == r) D[p][p] += 2.0 * c;
            else { D[p][r] += c; D[r][p] += c; }
        }
        double beta0 = 0;
        for (int a = 0; a < d; a++) {
            double ca = coef[a * nv + v];
            double quad = 0;
            for (int b = 0; b < d; b++)
                for (int b2 = 0; b2 < d; b2++) quad += D[a][b] * D[a][b2] * Mxx[b][b2];
            beta0 += ca * ca + quad;
            for (int b = a; b < d; b++) beta0 += D[a][b] * D[a][b];
        }
        double w0 = g0 / ((eps + beta0) * (eps + beta0));
        double wk[8], wsum = w0;
        for (int k = 0; k < nb_count; k++) {
            double beta = 0;
            for (int a = 0; a < d; a++) beta += cand[k][a * nv + v] * cand[k][a * nv + v];
            wk[k] = gk / ((eps + beta) * (eps + beta));
            wsum += wk[k];
        }
        double om0 = w0 / wsum;
        for (int a = 0; a < d; a++) {
            double lin = coef[a * nv + v], mix = 0;
            for (int k = 0; k < nb_count; k++) {
                lin -= gk * cand[k][a * nv + v];
                mix += wk[k] / wsum * cand[k][a * nv + v];
            }
            coef[a * nv + v] = om0 / g0 * lin + mix;
        }
        for (int q = 0; q < nq; q++) coef[(d + q) * nv + v] *= om0 / g0;
    }
}

/* coefficients c[k][v] of cell i; returns 0 (quadratic), 1 (linear
   fallback, only without boundary data), -1 if the stencil fixes no
   quadratic (with boundary data) or not even a linear fit, -3 on an
   unsupported tag.  With boundary data and weno_eps > 0 the nonlinear
   weights above are applied. */
static int recon_cell(const om_mesh *m, const om_params *P, long i, const double *W, const double *dW,
                      double *coef) {
    int d = m->dim, nv = m->nv, nc = m->ncoef;
    long N = m->n_cell;
    double A[64 * NCMAX], B[64 * NVMAX];
    double nb_xi[8 * DMAX], nb_dW[8 * DMAX * NVMAX], nb_dU[8 * NVMAX];
    int nb_count = 0;
    int nr = 0;
    const double *xc = m->ctr + i * d;
    double h = m->h[i];
    double own[NCMAX];
    basis_average(m, xc, m->sec + i * 6, xc, h, own);
    for (long q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; q++) {
        long f = m->cf_face[q];
        long nb = m->cf_sign[q] > 0 ? m->neigh[f] : m->owner[f];
        double c[3], sec[6], Wnb[NVMAX], dWnb[DMAX * NVMAX], avg[NCMAX];
        if (nb >= 0) {
            neighbour_centroid(m, i, f, nb, c);
            for (int k = 0; k < 6; k++) sec[k] = m->sec[nb * 6 + k];
            for (int v = 0; v < nv; v++) {
                Wnb[v] = W[v * N + nb];
                for (int a = 0; a < d; a++) dWnb[a * nv + v] = dW[(a * nv + v) * N + nb];
            }
        } else {
            if (!P) continue;
            int st = ghost_cell(m, P, i, f, W, dW, c, sec, Wnb, dWnb);
            if (st) return st;
        }
        basis_average(m, c, sec, xc, h, avg);
        for (int a = 0; a < d; a++) nb_xi[nb_count * d + a] = avg[a];
        for (int v = 0; v < nv; v++) {
            nb_dU[nb_count * nv + v] = Wnb[v] - W[v * N + i];
            for (int a = 0; a < d; a++) nb_dW[(nb_count * d + a) * nv + v] = dWnb[a * nv + v];
        }
        nb_count++;
        /* average row */
        for (int k = 0; k < nc; k++) A[nr * nc + k] = avg[k] - own[k];
        for (int v = 0; v < nv; v++) B[nr * nv + v] = Wnb[v] - W[v * N + i];
        nr++;
        /* gradient rows: <d phi_k / d xi_a>_m, exact since d phi / d xi is linear */
        for (int a = 0; a < d; a++) {
            for (int k = 0; k < nc; k++) A[nr * nc + k] = 0;
            A[nr * nc + a] = 1.0;
            for (int qq = 0; qq < (d == 2 ? 3 : 6); qq++) {
                int p = QA[d - 2][qq], r = QB[d - 2][qq];
                double val = 0;
                if (p == a) val += avg[r];
                if (r == a) val += avg[p];
                A[nr * nc + d + qq] = val;
            }
            for (int v = 0; v < nv; v++) B[nr * nv + v] = h * dWnb[a * nv + v];
            nr++;
        }
    }
    /* own-gradient rows */
    for (int a = 0; a < d; a++) {
        for (int k = 0; k < nc; k++) A[nr * nc + k] = 0;
        A[nr * nc + a] = 1.0;
        for (int v = 0; v < nv; v++) B[nr * nv + v] = h * dW[(a * nv + v) * N + i];
        nr++;
    }
    /* keep copies for the linear fallback */
    double A1[64 * NCMAX], B1[64 * NVMAX];
    for (int r = 0; r < nr; r++) {
        for (int k = 0; k < d; k++) A1[r * d + k] = A[r * nc + k];
        for (int v = 0; v < nv; v++) B1[r * nv + v] = B[r * nv + v];
    }
    if (nr >= nc && lsq_qr(nr, nc, A, nv, B) > 0) {
        for (int k = 0; k < nc; k++)
            for (int v = 0; v < nv; v++) coef[k * nv + v] = B[k * nv + v];
        if (P && P->weno_eps > 0) weno_combine(m, i, nb_count, nb_xi, nb_dW, nb_dU, P->weno_eps, coef);
        return 0;
    }
    /* with the boundary rows every stencil of a valid mesh fixes the
       quadratic; the linear fit serves the pins without boundary rows */
    if (P) return -1;
    if (lsq_qr(nr, d, A1, nv, B1) <= 0) return -1;
    for (int k = 0; k < nc; k++)
        for (int v = 0; v < nv; v++) coef[k * nv + v] = k < d ? B1[k * nv + v] : 0.0;
    return 1;
}

/* exported: 1 for cells whose stencil falls back to linear, else 0 */
void om_recon_linear_cells(const om_mesh *m, const om_params *P, int *flag) {
    long N = m->n_cell;
    int nv = m->nv, d = m->dim;
    double *W = (double *)calloc(nv * N, sizeof(double));
    double *dW = (double *)calloc(d * nv * N, sizeof(double));
    double coef[NCMAX * NVMAX];
    for (long i = 0; i < N; i++) {
        W[i] = 1.0;
        W[(nv - 1) * N + i] = 2.5;
        if (P)
            for (int v = 0; v < nv; v++) W[v * N + i] = P->W_inf[v];
    }
    for (long i = 0; i < N; i++) flag[i] = recon_cell(m, P, i, W, dW, coef);
    free(W);
    free(dW);
}

/* value and gradient of P_i at point x (given in i's frame) */
static void recon_eval(const om_mesh *m, long i, const double *W, const double *coef, const double *x,
                       double *Wx, double *dWx) {
    int d = m->dim, nv = m->nv, nc = m->ncoef;
    long N = m->n_cell;
    const double *xc = m->ctr + i * d;
    double h = m->h[i];
    double own[NCMAX], y[3], phi[NCMAX], dphi[3][NCMAX];
    basis_average(m, xc, m->sec + i * 6, xc, h, own);
    for (int a = 0; a < d; a++) y[a] = (x[a] - xc[a]) / h;
    for (int a = 0; a < d; a++) phi[a] = y[a];
    for (int q = 0; q < (d == 2 ? 3 : 6); q++) phi[d + q] = y[QA[d - 2][q]] * y[QB[d - 2][q]];
    for (int a = 0; a < d; a++) {
        for (int k = 0; k < nc; k++) dphi[a][k] = 0;
        dphi[a][a] = 1.0;
        for (int q = 0; q < (d == 2 ? 3 : 6); q++) {
            int p = QA[d - 2][q], r = QB[d - 2][q];
            double val = 0;
            if (p == a) val += y[r];
            if (r == a) val += y[p];
            dphi[a][d + q] = val;
        }
    }
    for (int v = 0; v < nv; v++) {
        double s = W[v * N + i];
        for (int k = 0; k < nc; k++) s += coef[k * nv + v] * (phi[k] - own[k]);
        Wx[v] = s;
        for (int a = 0; a < d; a++) {
            double g = 0;
            for (int k = 0; k < nc; k++) g += coef[k * nv + v] * dphi[a][k];
            dWx[a * nv + v] = g / h;
        }
    }
}

/* exported: reconstruct every cell and evaluate P_i at given points */
int om_recon_eval(const om_mesh *m, const om_params *P, const double *W, const double *dW, long n_pts,
                  const long *cell, const double *x, double *Wx, double *dWx) {
    int nv = m->nv, d = m->dim;
    for (long p = 0; p < n_pts; p++) {
        double coef[NCMAX * NVMAX];
        if (recon_cell(m, P, cell[p], W, dW, coef) < 0) return -1;
        recon_eval(m, cell[p], W, coef, x + p * d, Wx + p * nv, dWx + p * d * nv);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Kinetic moments (Sec. 2.2).  Moments are expectations per unit       */
/* density of the Maxwellian g = rho (lam/pi)^{(K+D)/2}                  */
/*   exp(-lam((u-U)^2 + xi^2)),                                          */
/* in the local face frame (u along the normal).  K internal degrees of  */
/* freedom: (5-3 gamma)/(gamma-1) in 3-D (the paper's value);            */
/* reading for 2-D: (4-2 gamma)/(gamma-1), so both have 2/(gamma-1)      */
/* total degrees of freedom.                                              */
/* ------------------------------------------------------------------ */
#define NMOM 10
typedef struct {
    double u[NMOM], v[NMOM], w[NMOM], xi[3]; /* <u^k>, <v^k>, <w^k>, <xi^{2e}> */
} moments;

static void full_moments(double U, double lam, double *mu) {
    mu[0] = 1.0;
    mu[1] = U;
    for (int k = 0; k + 2 < NMOM; k++) mu[k + 2] = U * mu[k + 1] + (k + 1) / (2.0 * lam) * mu[k];
}

/* half-range moments over u > 0 (sgn = +1) or u < 0 (sgn = -1) */
static void half_moments(double U, double lam, int sgn, double *mu) {
    double s = sqrt(lam);
    mu[0] = 0.5 * erfc(-sgn * s * U);
    mu[1] = U * mu[0] + sgn * 0.5 * exp(-lam * U * U) / sqrt(M_PI * lam);
    for (int k = 0; k + 2 < NMOM; k++) mu[k + 2] = U * mu[k + 1] + (k + 1) / (2.0 * lam) * mu[k];
}

static void xi_moments(double lam, double K, double *mx) {
    mx[0] = 1.0;
    mx[1] = K / (2.0 * lam);
    mx[2] = (K * K + 2.0 * K) / (4.0 * lam * lam);
}

static double internal_dof(int dim, double gamma) {
    return dim == 3 ? (5.0 - 3.0 * gamma) / (gamma - 1.0) : (4.0 - 2.0 * gamma) / (gamma - 1.0);
}

/* polynomials in (u, v, w, xi^2) as term lists */
#define PMAX 512
typedef struct {
    int n;
    double c[PMAX];
    unsigned char a[PMAX], b[PMAX], g[PMAX], e[PMAX];
} poly;

static void p_zero(poly *p) { p->n = 0; }
static void p_term(poly *p, double c, int a, int b, int g, int e) {
    p->c[p->n] = c; p->a[p->n] = (unsigned char)a; p->b[p->n] = (unsigned char)b;
    p->g[p->n] = (unsigned char)g; p->e[p->n] = (unsigned char)e; p->n++;
}
/* psi_k for k = 0..nv-1: 1, u, v, [w], (u^2+v^2+[w^2]+xi^2)/2 */
static void p_psi(poly *p, int k, int dim) {
    p_zero(p);
    int nv = dim + 2;
    if (k == 0) p_term(p, 1, 0, 0, 0, 0);
    else if (k == 1) p_term(p, 1, 1, 0, 0, 0);
    else if (k == 2) p_term(p, 1, 0, 1, 0, 0);
    else if (k == 3 && dim == 3) p_term(p, 1, 0, 0, 1, 0);
    if (k == nv - 1) {
        p_term(p, 0.5, 2, 0, 0, 0);
        p_term(p, 0.5, 0, 2, 0, 0);
        if (dim == 3) p_term(p, 0.5, 0, 0, 2, 0);
        p_term(p, 0.5, 0, 0, 0, 1);
    }
}
/* sum_k coef_k psi_k */
static void p_combo(poly *p, const double *coef, int dim) {
    p_zero(p);
    for (int k = 0; k < dim + 2; k++) {
        poly q;
        p_psi(&q, k, dim);
        for (int t = 0; t < q.n; t++) p_term(p, coef[k] * q.c[t], q.a[t], q.b[t], q.g[t], q.e[t]);
    }
}
static void p_mul(const poly *x, const poly *y, poly *z) {
    p_zero(z);
    for (int s = 0; s < x->n; s++)
        for (int t = 0; t < y->n; t++)
            p_term(z, x->c[s] * y->c[t], x->a[s] + y->a[t], x->b[s] + y->b[t], x->g[s] + y->g[t],
                   x->e[s] + y->e[t]);
}
/* multiply by the velocity component j (0 = u, 1 = v, 2 = w) */
static void p_mulvar(const poly *x, int j, poly *z) {
    *z = *x;
    for (int t = 0; t < z->n; t++) {
        if (j == 0) z->a[t]++;
        else if (j == 1) z->b[t]++;
        else z->g[t]++;
    }
}
static void p_add(poly *x, const poly *y) {
    for (int t = 0; t < y->n; t++) p_term(x, y->c[t], y->a[t], y->b[t], y->g[t], y->e[t]);
}
static double p_expect(const poly *p, const moments *M) {
    double s = 0;
    for (int t = 0; t < p->n; t++) s += p->c[t] * M->u[p->a[t]] * M->v[p->b[t]] * M->w[p->g[t]] * M->xi[p->e[t]];
    return s;
}

static void gauss_solve(int n, double *A, double *b) {
    for (int k = 0; k < n; k++) {
        int piv = k;
        for (int r = k + 1; r < n; r++)
            if (fabs(A[r * n + k]) > fabs(A[piv * n + k])) piv = r;
        if (piv != k) {
            for (int j = 0; j < n; j++) { double t = A[k * n + j]; A[k * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < n; r++) {
            double f = A[r * n + k] / A[k * n + k];
            for (int j = k; j < n; j++) A[r * n + j] -= f * A[k * n + j];
            b[r] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; k--) {
        double s = b[k];
        for (int j = k + 1; j < n; j++) s -= A[k * n + j] * b[j];
        b[k] = s / A[k * n + k];
    }
}

/* Micro-slope a = sum_k a_k psi_k from <a psi> = b (b = dW / rho):
   solve the moment system E[psi_p psi_q] a_q = b_p. */
static void micro_slope(const moments *M, int dim, const double *b, double *a) {
    int nv = dim + 2;
    double A[NVMAX * NVMAX];
    for (int p = 0; p < nv; p++)
        for (int q = 0; q < nv; q++) {
            poly x, y, z;
            p_psi(&x, p, dim);
            p_psi(&y, q, dim);
            p_mul(&x, &y, &z);
            A[p * nv + q] = p_expect(&z, M);
        }
    for (int p = 0; p < nv; p++) a[p] = b[p];
    gauss_solve(nv, A, a);
}

typedef struct {
    double rho, U[3], p, lam;
} prim;

static prim to_prim(const double *W, int dim, double gamma) {
    prim q;
    q.rho = W[0];
    double ke = 0;
    for (int a = 0; a < 3; a++) q.U[a] = a < dim ? W[1 + a] / W[0] : 0.0;
    for (int a = 0; a < dim; a++) ke += q.U[a] * q.U[a];
    q.p = (gamma - 1.0) * (W[dim + 1] - 0.5 * q.rho * ke);
    q.lam = q.rho / (2.0 * q.p);
    return q;
}

static void make_moments(const prim *q, double K, moments *M) {
    full_moments(q->U[0], q->lam, M->u);
    full_moments(q->U[1], q->lam, M->v);
    full_moments(q->U[2], q->lam, M->w);
    xi_moments(q->lam, K, M->xi);
}

/* Smooth-flow gas-kinetic flux (the simplified BGK solution for smooth
   flow, Sec. 2.2):  f = g^c [1 - tau (a.u + A) + A t],  with a^(j) the
   micro-slopes of dW^c along the local axis j and A from the compatibility
   condition <A + a.u> = 0.  Local frame, axis 0 = face normal.
   Out: F0 (flux at t = 0), Ft (its time derivative), Wt = <A psi> rho.
   With Pr != 1 the energy flux gets (1/Pr - 1) times the Fourier heat flux
   of the macroscopic state (BGK gives Pr = 1). */
int om_gks_flux(int dim, double gamma, double mu, double Pr, const double *Wc, const double *dWc, double *F0,
                double *Ft, double *Wt) {
    int nv = dim + 2;
    prim q = to_prim(Wc, dim, gamma);
    if (!(q.rho > 0) || !(q.p > 0)) return -1;
    double K = internal_dof(dim, gamma);
    moments M;
    make_moments(&q, K, &M);
    double tau = mu / q.p;
    double a[3][NVMAX], A[NVMAX], b[NVMAX];
    for (int j = 0; j < dim; j++) {
        for (int v = 0; v < nv; v++) b[v] = dWc[j * nv + v] / q.rho;
        micro_slope(&M, dim, b, a[j]);
    }
    /* a.u = sum_j a^(j) u_j */
    poly au, tmp, t2;
    p_zero(&au);
    for (int j = 0; j < dim; j++) {
        p_combo(&tmp, a[j], dim);
        p_mulvar(&tmp, j, &t2);
        p_add(&au, &t2);
    }
    for (int p = 0; p < nv; p++) {
        poly ps, z;
        p_psi(&ps, p, dim);
        p_mul(&ps, &au, &z);
        b[p] = -p_expect(&z, &M);
    }
    micro_slope(&M, dim, b, A);
    poly PA;
    p_combo(&PA, A, dim);
    poly sum = au;
    p_add(&sum, &PA);
    for (int p = 0; p < nv; p++) {
        poly ps, ups, z;
        p_psi(&ps, p, dim);
        p_mulvar(&ps, 0, &ups);
        double e_ups = p_expect(&ups, &M);
        p_mul(&ups, &sum, &z);
        double e_tau = p_expect(&z, &M);
        p_mul(&ups, &PA, &z);
        double e_t = p_expect(&z, &M);
        p_mul(&ps, &PA, &z);
        double e_w = p_expect(&z, &M);
        F0[p] = q.rho * (e_ups - tau * e_tau);
        Ft[p] = q.rho * e_t;
        Wt[p] = q.rho * e_w;
    }
    if (Pr != 1.0 && mu != 0.0) {
        /* q_n = -mu cp dT/dn with R = 1, T = p / rho */
        const double *dn = dWc; /* derivatives along the normal */
        double ke_d = 0, ke = 0;
        for (int a2 = 0; a2 < dim; a2++) {
            ke_d += q.U[a2] * dn[1 + a2];
            ke += q.U[a2] * q.U[a2];
        }
        double pn = (gamma - 1.0) * (dn[nv - 1] - ke_d + 0.5 * ke * dn[0]);
        double Tn = (pn * q.rho - q.p * dn[0]) / (q.rho * q.rho);
        double qn = -mu * gamma / (gamma - 1.0) * Tn;
        F0[nv - 1] += (1.0 / Pr - 1.0) * qn;
    }
    return 0;
}

/* Interface equilibrium state from the left/right Maxwellians by kinetic
   half-space combination (u_n > 0 from the left, u_n < 0 from the right). */
int om_halfspace_state(int dim, double gamma, const double *WL, const double *WR, double *Wc) {
    int nv = dim + 2;
    double K = internal_dof(dim, gamma);
    prim L = to_prim(WL, dim, gamma), R = to_prim(WR, dim, gamma);
    if (!(L.rho > 0) || !(L.p > 0) || !(R.rho > 0) || !(R.p > 0)) return -1;
    moments ML, MR;
    make_moments(&L, K, &ML);
    make_moments(&R, K, &MR);
    half_moments(L.U[0], L.lam, +1, ML.u);
    half_moments(R.U[0], R.lam, -1, MR.u);
    for (int p = 0; p < nv; p++) {
        poly ps;
        p_psi(&ps, p, dim);
        Wc[p] = L.rho * p_expect(&ps, &ML) + R.rho * p_expect(&ps, &MR);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Full time-dependent gas-kinetic solution at a Gauss point (Sec. 2.2, */
/* the 2nd-flux equation), for flows with discontinuities (Sec. 4):     */
/*  f(t) = (1 - e) g^c + [(t + tau) e - tau] (a^c.u) g^c               */
/*       + (t - tau + tau e) A^c g^c                                   */
/*       + e g^l [1 - (tau + t) a^l.u - tau A^l] H(u)                  */
/*       + e g^r [1 - (tau + t) a^r.u - tau A^r] (1 - H(u)),           */
/* e = exp(-t / tau_n), u the normal velocity.  g^l, g^r are the        */
/* Maxwellians of the left and right interface states, a^l, a^r their  */
/* micro-slopes from the left and right gradients, A^l, A^r from their  */
/* own compatibility conditions; g^c is the half-space combination W^c  */
/* with the slopes of 1/2 (grad W^l + grad W^r), as on the smooth path. */
/* tau = mu / p^c.  Reading of the numerical collision time, which the  */
/* paper takes from other work: tau_n = tau + |p^l - p^r|/(p^l + p^r) dt.*/
/* The time marching takes the flux as F0 + t Ft, the linear function   */
/* with the same integrals over [0, dt/2] and [0, dt], and the          */
/* interface state as W0 + t Wt through its values at dt/2 and dt.  For  */
/* equal left and right states and gradients the solution is the smooth */
/* one (Eq. 2nd-smooth-flux) exactly, whatever tau_n.                   */
/* ------------------------------------------------------------------ */
typedef struct {
    double g[NVMAX], a[NVMAX], A[NVMAX]; /* rho <w psi>, rho <w psi a.u>, rho <w psi A> */
} kin_terms;

/* micro-slopes a^(j) (axis j of the local frame) of the Maxwellian with
   moments M and density rho from the gradient dW [dim][nv], and A from the
   compatibility condition <(a.u + A) psi> = 0, both over the whole
   velocity space */
static void slopes_and_A(const moments *M, int dim, double rho, const double *dW, double a[3][NVMAX], double *A) {
    int nv = dim + 2;
    double b[NVMAX];
    for (int j = 0; j < dim; j++) {
        for (int v = 0; v < nv; v++) b[v] = dW[j * nv + v] / rho;
        micro_slope(M, dim, b, a[j]);
    }
    poly au, tmp, t2;
    p_zero(&au);
    for (int j = 0; j < dim; j++) {
        p_combo(&tmp, a[j], dim);
        p_mulvar(&tmp, j, &t2);
        p_add(&au, &t2);
    }
    for (int p = 0; p < nv; p++) {
        poly ps, z;
        p_psi(&ps, p, dim);
        p_mul(&ps, &au, &z);
        b[p] = -p_expect(&z, M);
    }
    micro_slope(M, dim, b, A);
}

/* rho <w psi>, rho <w psi (a.u)>, rho <w psi A> under the moments M, with
   the weight w = 1 (ku = 0) or the normal velocity u (ku = 1) */
static void kinetic_terms(const moments *M, int dim, double rho, double a[3][NVMAX], const double *A, int ku,
                          kin_terms *t) {
    int nv = dim + 2;
    poly au, tmp, t2, PA;
    p_zero(&au);
    for (int j = 0; j < dim; j++) {
        p_combo(&tmp, a[j], dim);
        p_mulvar(&tmp, j, &t2);
        p_add(&au, &t2);
    }
    p_combo(&PA, A, dim);
    for (int p = 0; p < nv; p++) {
        poly ps, w, z;
        p_psi(&ps, p, dim);
        if (ku) p_mulvar(&ps, 0, &w);
        else w = ps;
        t->g[p] = rho * p_expect(&w, M);
        p_mul(&w, &au, &z);
        t->a[p] = rho * p_expect(&z, M);
        p_mul(&w, &PA, &z);
        t->A[p] = rho * p_expect(&z, M);
    }
}

/* the five time functions of the full solution -- 1 - e, (t + tau) e - tau,
   t - tau + tau e, e, (tau + t) e -- at t = T (integral = 0) or integrated
   over [0, T] (integral = 1) */
static void full_time_weights(double T, double tau, double taun, int integral, double w[5]) {
    double E = taun > 0 ? exp(-T / taun) : 0.0;
    if (!integral) {
        w[0] = 1.0 - E;
        w[1] = (T + tau) * E - tau;
        w[2] = T - tau + tau * E;
        w[3] = E;
        w[4] = (tau + T) * E;
        return;
    }
    double omE = 1.0 - E;
    w[0] = T - taun * omE;
    w[1] = taun * taun * omE - taun * T * E + tau * taun * omE - tau * T;
    w[2] = 0.5 * T * T - tau * T + tau * taun * omE;
    w[3] = taun * omE;
    w[4] = tau * taun * omE + taun * taun * omE - taun * T * E;
}

static void full_combine(const double w[5], double tau, int nv, const kin_terms *c, const kin_terms *l,
                         const kin_terms *r, double *out) {
    for (int p = 0; p < nv; p++)
        out[p] = w[0] * c->g[p] + w[1] * c->a[p] + w[2] * c->A[p] +
                 w[3] * (l->g[p] + r->g[p] - tau * (l->A[p] + r->A[p])) - w[4] * (l->a[p] + r->a[p]);
}

/* Local frame (axis 0 = face normal, from left to right).  In: left and
   right states and gradients [dim][nv] (local axes), the time step dt.
   Out: F0, Ft (flux and its time slope of the linear fit), W0, Wt
   (interface state and its time slope).  Returns -1 for a non-physical
   state. */
int om_gks_flux_full(int dim, double gamma, double mu, double Pr, double dt, const double *WL, const double *dWL,
                     const double *WR, const double *dWR, double *F0, double *Ft, double *W0, double *Wt) {
    int nv = dim + 2;
    double K = internal_dof(dim, gamma);
    double Wc[NVMAX], dWc[DMAX * NVMAX];
    if (om_halfspace_state(dim, gamma, WL, WR, Wc)) return -1;
    for (int k = 0; k < dim * nv; k++) dWc[k] = 0.5 * (dWL[k] + dWR[k]);
    prim qc = to_prim(Wc, dim, gamma), ql = to_prim(WL, dim, gamma), qr = to_prim(WR, dim, gamma);
    if (!(qc.rho > 0) || !(qc.p > 0)) return -1;
    moments Mc, Ml, Mr, Hl, Hr;
    make_moments(&qc, K, &Mc);
    make_moments(&ql, K, &Ml);
    make_moments(&qr, K, &Mr);
    Hl = Ml;
    half_moments(ql.U[0], ql.lam, +1, Hl.u);
    Hr = Mr;
    half_moments(qr.U[0], qr.lam, -1, Hr.u);
    double ac[3][NVMAX], al[3][NVMAX], ar[3][NVMAX], Ac[NVMAX], Al[NVMAX], Ar[NVMAX];
    slopes_and_A(&Mc, dim, qc.rho, dWc, ac, Ac);
    slopes_and_A(&Ml, dim, ql.rho, dWL, al, Al);
    slopes_and_A(&Mr, dim, qr.rho, dWR, ar, Ar);
    double tau = mu / qc.p;
    double taun = tau + fabs(ql.p - qr.p) / (ql.p + qr.p) * dt;
    kin_terms fc, fl, fr, wc, wl, wr;
    kinetic_terms(&Mc, dim, qc.rho, ac, Ac, 1, &fc);
    kinetic_terms(&Hl, dim, ql.rho, al, Al, 1, &fl);
    kinetic_terms(&Hr, dim, qr.rho, ar, Ar, 1, &fr);
    kinetic_terms(&Mc, dim, qc.rho, ac, Ac, 0, &wc);
    kinetic_terms(&Hl, dim, ql.rho, al, Al, 0, &wl);
    kinetic_terms(&Hr, dim, qr.rho, ar, Ar, 0, &wr);
    double w[5], I1[NVMAX], I2[NVMAX], V1[NVMAX], V2[NVMAX];
    full_time_weights(dt, tau, taun, 1, w);
    full_combine(w, tau, nv, &fc, &fl, &fr, I1);
    full_time_weights(0.5 * dt, tau, taun, 1, w);
    full_combine(w, tau, nv, &fc, &fl, &fr, I2);
    full_time_weights(dt, tau, taun, 0, w);
    full_combine(w, tau, nv, &wc, &wl, &wr, V1);
    full_time_weights(0.5 * dt, tau, taun, 0, w);
    full_combine(w, tau, nv, &wc, &wl, &wr, V2);
    for (int p = 0; p < nv; p++) {
        F0[p] = (4.0 * I2[p] - I1[p]) / dt;
        Ft[p] = 4.0 * (I1[p] - 2.0 * I2[p]) / (dt * dt);
        W0[p] = 2.0 * V2[p] - V1[p];
        Wt[p] = 2.0 * (V1[p] - V2[p]) / dt;
    }
    if (Pr != 1.0 && mu != 0.0) {
        /* as on the smooth path: q_n = -mu cp dT/dn from W^c, grad W^c */
        const double *dn = dWc;
        double ke_d = 0, ke = 0;
        for (int a2 = 0; a2 < dim; a2++) {
            ke_d += qc.U[a2] * dn[1 + a2];
            ke += qc.U[a2] * qc.U[a2];
        }
        double pn = (gamma - 1.0) * (dn[nv - 1] - ke_d + 0.5 * ke * dn[0]);
        double Tn = (pn * qc.rho - qc.p * dn[0]) / (qc.rho * qc.rho);
        double qn = -mu * gamma / (gamma - 1.0) * Tn;
        F0[nv - 1] += (1.0 / Pr - 1.0) * qn;
    }
    return 0;
}

/* First-order kinetic flux vector splitting flux in the local frame:
   F = rho_L <u psi>_{u>0,L} + rho_R <u psi>_{u<0,R}. */
int om_kfvs(int dim, double gamma, const double *UL, const double *UR, double *F) {
    int nv = dim + 2;
    double K = internal_dof(dim, gamma);
    prim L = to_prim(UL, dim, gamma), R = to_prim(UR, dim, gamma);
    if (!(L.rho > 0) || !(L.p > 0) || !(R.rho > 0) || !(R.p > 0)) return -1;
    moments ML, MR;
    make_moments(&L, K, &ML);
    make_moments(&R, K, &MR);
    half_moments(L.U[0], L.lam, +1, ML.u);
    half_moments(R.U[0], R.lam, -1, MR.u);
    for (int p = 0; p < nv; p++) {
        poly ps, ups;
        p_psi(&ps, p, dim);
        p_mulvar(&ps, 0, &ups);
        F[p] = L.rho * p_expect(&ups, &ML) + R.rho * p_expect(&ups, &MR);
    }
    return 0;
}

/* exported for the moment pins: <u^a v^b w^c xi^(2e)> of a Maxwellian */
double om_moment(int dim, double gamma, const double *W, int a, int b, int c, int e, int half) {
    prim q = to_prim(W, dim, gamma);
    moments M;
    make_moments(&q, internal_dof(dim, gamma), &M);
    if (half) half_moments(q.U[0], q.lam, half, M.u);
    return M.u[a] * M.v[b] * M.w[c] * M.xi[e];
}

/* exported: micro-slope coefficients for the pins */
void om_micro_slope(int dim, double gamma, const double *W, const double *dW, double *a) {
    int nv = dim + 2;
    prim q = to_prim(W, dim, gamma);
    moments M;
    make_moments(&q, internal_dof(dim, gamma), &M);
    double b[NVMAX];
    for (int v = 0; v < nv; v++) b[v] = dW[v] / q.rho;
    micro_slope(&M, dim, b, a);
}

/* ------------------------------------------------------------------ */
/* Local frame and boundary states                                       */
/* ------------------------------------------------------------------ */
static void local_frame(int dim, const double *n, double e[3][3]) {
    memset(e, 0, sizeof(double) * 9);
    if (dim == 2) {
        e[0][0] = n[0]; e[0][1] = n[1];
        e[1][0] = -n[1]; e[1][1] = n[0];
        return;
    }
    int k = 0;
    for (int a = 1; a < 3; a++)
        if (fabs(n[a]) < fabs(n[k])) k = a;
    double ax[3] = {0, 0, 0};
    ax[k] = 1.0;
    double t1[3], t2[3];
    cross3(n, ax, t1);
    double l = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    for (int a = 0; a < 3; a++) t1[a] /= l;
    cross3(n, t1, t2);
    for (int a = 0; a < 3; a++) { e[0][a] = n[a]; e[1][a] = t1[a]; e[2][a] = t2[a]; }
}

static void state_to_local(int dim, double e[3][3], const double *W, double *Wl) {
    int nv = dim + 2;
    Wl[0] = W[0];
    Wl[nv - 1] = W[nv - 1];
    for (int a = 0; a < dim; a++) {
        double s = 0;
        for (int b = 0; b < dim; b++) s += e[a][b] * W[1 + b];
        Wl[1 + a] = s;
    }
}
static void vec_to_global(int dim, double e[3][3], const double *Fl, double *F) {
    int nv = dim + 2;
    F[0] = Fl[0];
    F[nv - 1] = Fl[nv - 1];
    for (int b = 0; b < dim; b++) {
        double s = 0;
        for (int a = 0; a < dim; a++) s += e[a][b] * Fl[1 + a];
        F[1 + b] = s;
    }
}
/* gradient [a][v] (global axes) -> local axes and local momentum components */
static void grad_to_local(int dim, double e[3][3], const double *dW, double *dWl) {
    int nv = dim + 2;
    double tmp[DMAX * NVMAX];
    for (int v = 0; v < nv; v++)
        for (int a = 0; a < dim; a++) {
            double s = 0;
            for (int b = 0; b < dim; b++) s += e[a][b] * dW[b * nv + v];
            tmp[a * nv + v] = s;
        }
    for (int a = 0; a < dim; a++) state_to_local(dim, e, tmp + a * nv, dWl + a * nv);
}

/* non-reflecting far field from the normal Riemann invariants of the
   interior state and the free stream (local frame, axis 0 outward):
   the outgoing invariant U_n + 2c/(gamma-1) comes from the interior, the
   incoming U_n - 2c/(gamma-1) from the free stream; entropy p/rho^gamma and
   the tangential velocity from the side the flow comes from; supersonic
   inflow takes the free stream, supersonic outflow the interior */
static void farfield_state(int dim, double gamma, const double *Wl, const double *Winf_l, double *Wb) {
    int nv = dim + 2;
    prim I = to_prim(Wl, dim, gamma), O = to_prim(Winf_l, dim, gamma);
    double cI = sqrt(gamma * I.p / I.rho), cO = sqrt(gamma * O.p / O.rho);
    if (O.U[0] <= -cO) { vcopy(Wb, Winf_l, nv); return; } /* supersonic inflow */
    if (I.U[0] >= cI) { vcopy(Wb, Wl, nv); return; }      /* supersonic outflow */
    double Rp = I.U[0] + 2.0 * cI / (gamma - 1.0);
    double Rm = O.U[0] - 2.0 * cO / (gamma - 1.0);
    double Un = 0.5 * (Rp + Rm);
    double c = 0.25 * (gamma - 1.0) * (Rp - Rm);
    const prim *up = Un > 0 ? &I : &O;
    double s = up->p / pow(up->rho, gamma);
    double rho = pow(c * c / (gamma * s), 1.0 / (gamma - 1.0));
    double p = rho * c * c / gamma;
    double U[3] = {Un, up->U[1], up->U[2]};
    Wb[0] = rho;
    double ke = 0;
    for (int a = 0; a < dim; a++) { Wb[1 + a] = rho * U[a]; ke += U[a] * U[a]; }
    Wb[nv - 1] = p / (gamma - 1.0) + 0.5 * rho * ke;
}

/* exported for the far-field pins (local frame, axis 0 outward) */
void om_farfield_state(int dim, double gamma, const double *Wl, const double *Winf_l, double *Wb) {
    farfield_state(dim, gamma, Wl, Winf_l, Wb);
}

/* ------------------------------------------------------------------ */
/* High-order pass: reconstruction, interface states, gas-kinetic flux   */
/* at every face Gauss point, and the per-cell sums                      */
/*   F0s_i  = sum_f s sum_g wJ F0.n,  Fts_i similarly,                    */
/*   G0s_i  = sum_f s sum_g wJ W_g n,  Gts_i = sum_f s sum_g wJ W_t n,    */
/* with s = +1 for the owner, -1 for the neighbour.  Each face is        */
/* evaluated once.  Cd accumulates the wall momentum flux.               */
/* ------------------------------------------------------------------ */
typedef struct {
    double *F0s, *Fts, *G0s, *Gts; /* [nv][N], [nv][N], [d][nv][N], [d][nv][N] */
    double force[3];
    int status;
} ho_sums;

static int ho_pass(const om_mesh *m, const om_params *P, const double *W, const double *dW, double dt, ho_sums *o) {
    int d = m->dim, nv = m->nv, nc = m->ncoef;
    long N = m->n_cell;
    memset(o->F0s, 0, sizeof(double) * nv * N);
    memset(o->Fts, 0, sizeof(double) * nv * N);
    memset(o->G0s, 0, sizeof(double) * d * nv * N);
    memset(o->Gts, 0, sizeof(double) * d * nv * N);
    o->force[0] = o->force[1] = o->force[2] = 0;
    o->status = 0;
    double *coef = (double *)malloc(sizeof(double) * N * nc * nv);
    for (long i = 0; i < N; i++)
        if (recon_cell(m, P, i, W, dW, coef + i * nc * nv) < 0) { o->status = -2; free(coef); return -2; }
    for (long f = 0; f < m->n_face; f++) {
        long L = m->owner[f], R = m->neigh[f];
        for (int g = 0; g < m->ngp[f]; g++) {
            const double *x = m->gx + (f * MAXGP + g) * d;
            const double *n = m->gn + (f * MAXGP + g) * d;
            double wJ = m->gw[f * MAXGP + g];
            double e[3][3];
            local_frame(d, n, e);
            double WLg[NVMAX], dWLg[DMAX * NVMAX], WL[NVMAX], dWL[DMAX * NVMAX];
            recon_eval(m, L, W, coef + L * nc * nv, x, WLg, dWLg);
            state_to_local(d, e, WLg, WL);
            grad_to_local(d, e, dWLg, dWL);
            double Wc[NVMAX], dWc[DMAX * NVMAX], WR[NVMAX], dWR[DMAX * NVMAX];
            int wall = 0;
            if (R >= 0) {
                double xr[3], WRg[NVMAX], dWRg[DMAX * NVMAX];
                for (int a = 0; a < d; a++) xr[a] = x[a] - m->shift[f * d + a];
                recon_eval(m, R, W, coef + R * nc * nv, xr, WRg, dWRg);
                state_to_local(d, e, WRg, WR);
                grad_to_local(d, e, dWRg, dWR);
            } else if (m->bc[f] == BC_SLIP) {
                /* mirror state: normal velocity reversed; normal derivatives of the
                   mirrored field change sign except for the normal momentum */
                vcopy(WR, WL, nv);
                WR[1] = -WL[1];
                for (int a = 0; a < d; a++)
                    for (int v = 0; v < nv; v++) {
                        double sgn = (a == 0) ? -1.0 : 1.0;
                        if (v == 1) sgn = -sgn;
                        dWR[a * nv + v] = sgn * dWL[a * nv + v];
                    }
            } else if (m->bc[f] == BC_FARFIELD) {
                double Winf_l[NVMAX];
                state_to_local(d, e, P->W_inf, Winf_l);
                farfield_state(d, P->gamma, WL, Winf_l, WR);
                memset(dWR, 0, sizeof(double) * d * nv);
            } else if (m->bc[f] == BC_ADIABATIC) {
                /* no-slip adiabatic wall (Sec. 4 viscous cases): the mirror
                   ghost with every velocity component reversed.  A derivative
                   of the ghost field changes sign when exactly one of (normal
                   direction, momentum component) applies to it, so in the
                   average the normal derivatives of rho and E and the
                   tangential derivatives of the momentum vanish: zero velocity
                   and zero heat flux at the wall. */
                vcopy(WR, WL, nv);
                for (int a = 0; a < d; a++) WR[1 + a] = -WL[1 + a];
                for (int a = 0; a < d; a++)
                    for (int v = 0; v < nv; v++) {
                        double sgn = (a == 0) ? -1.0 : 1.0;
                        if (v >= 1 && v <= d) sgn = -sgn;
                        dWR[a * nv + v] = sgn * dWL[a * nv + v];
                    }
            } else if (m->bc[f] == BC_ISOTHERMAL) {
                wall = 1;
            } else {
                o->status = -3;
                free(coef);
                return -3;
            }
            if (wall) {
                /* no-slip isothermal wall: interface state (p_L / T_w, 0, p_L), gradient
                   of the interior side, no mass flux */
                prim q = to_prim(WL, d, P->gamma);
                memset(Wc, 0, sizeof(double) * nv);
                Wc[0] = q.p / P->T_wall;
                Wc[nv - 1] = q.p / (P->gamma - 1.0);
                vcopy(dWc, dWL, d * nv);
            } else {
                if (om_halfspace_state(d, P->gamma, WL, WR, Wc)) { o->status = -1; free(coef); return -1; }
                for (int k = 0; k < d * nv; k++) dWc[k] = 0.5 * (dWL[k] + dWR[k]);
            }
            double F0l[NVMAX], Ftl[NVMAX], Wtl[NVMAX];
            if (P->flux_kind == 1 && !wall) {
                /* full solution: the interface state of the Gauss-Green sums is
                   its time fit W0 in place of W^c */
                if (om_gks_flux_full(d, P->gamma, P->mu, P->Pr, dt, WL, dWL, WR, dWR, F0l, Ftl, Wc, Wtl)) {
                    o->status = -1; free(coef); return -1;
                }
            } else if (om_gks_flux(d, P->gamma, P->mu, P->Pr, Wc, dWc, F0l, Ftl, Wtl)) {
                o->status = -1; free(coef); return -1;
            }
            if (wall) {
                F0l[0] = 0.0;
                Ftl[0] = 0.0;
                memset(Wtl, 0, sizeof(double) * nv);
            }
            double F0[NVMAX], Ft[NVMAX], Wg[NVMAX], Wt[NVMAX];
            vec_to_global(d, e, F0l, F0);
            vec_to_global(d, e, Ftl, Ft);
            vec_to_global(d, e, Wc, Wg);
            vec_to_global(d, e, Wtl, Wt);
            if (R < 0 && (m->bc[f] == BC_SLIP || m->bc[f] == BC_ISOTHERMAL || m->bc[f] == BC_ADIABATIC))
                for (int a = 0; a < d; a++) o->force[a] += wJ * F0[1 + a];
            for (int side = 0; side < 2; side++) {
                long c = side ? R : L;
                if (c < 0) continue;
                double s = side ? -1.0 : 1.0;
                for (int v = 0; v < nv; v++) {
                    o->F0s[v * N + c] += s * wJ * F0[v];
                    o->Fts[v * N + c] += s * wJ * Ft[v];
                    for (int a = 0; a < d; a++) {
                        o->G0s[(a * nv + v) * N + c] += s * wJ * Wg[v] * n[a];
                        o->Gts[(a * nv + v) * N + c] += s * wJ * Wt[v] * n[a];
                    }
                }
            }
        }
    }
    free(coef);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Time step.  The paper gives CFL 0.3-0.5 on the high-order level and  */
/* 1000 (local) on the low-order level (Sec. 4).  Reading:               */
/*   dt = CFL min_i h_i / (|U_i| + c_i + 2 nu_i / h_i),  nu = mu / rho.   */
/* ------------------------------------------------------------------ */
static double cell_dt(const om_mesh *m, const om_params *P, const double *W, long i, double cfl) {
    int d = m->dim, nv = m->nv;
    long N = m->n_cell;
    double Wi[NVMAX];
    for (int v = 0; v < nv; v++) Wi[v] = W[v * N + i];
    prim q = to_prim(Wi, d, P->gamma);
    double un = 0;
    for (int a = 0; a < d; a++) un += q.U[a] * q.U[a];
    un = sqrt(un);
    double c = sqrt(P->gamma * q.p / q.rho);
    double h = m->h[i];
    return cfl * h / (un + c + 2.0 * P->mu / q.rho / h);
}

double om_dt(const om_mesh *m, const om_params *P, const double *W) {
    if (P->dt_fixed > 0) return P->dt_fixed;
    double dt = INFINITY;
    for (long i = 0; i < m->n_cell; i++) {
        double t = cell_dt(m, P, W, i, P->cfl_high);
        if (t < dt) dt = t;
    }
    return dt;
}

/* ------------------------------------------------------------------ */
/* Context holding the work arrays of a cycle                            */
/* ------------------------------------------------------------------ */
typedef struct {
    const om_mesh *m;
    om_params P;
    ho_sums hs;
    double *Wn, *L0, *Lt0, *G0, *Gt0; /* stage-one data */
    double dt;
    double force[3];
} om_ctx;

om_ctx *om_ctx_create(const om_mesh *m, const om_params *P) {
    om_ctx *c = (om_ctx *)calloc(1, sizeof(om_ctx));
    long N = m->n_cell;
    int nv = m->nv, d = m->dim;
    c->m = m;
    c->P = *P;
    c->hs.F0s = (double *)calloc(nv * N, sizeof(double));
    c->hs.Fts = (double *)calloc(nv * N, sizeof(double));
    c->hs.G0s = (double *)calloc(d * nv * N, sizeof(double));
    c->hs.Gts = (double *)calloc(d * nv * N, sizeof(double));
    c->Wn = (double *)calloc(nv * N, sizeof(double));
    c->L0 = (double *)calloc(nv * N, sizeof(double));
    c->Lt0 = (double *)calloc(nv * N, sizeof(double));
    c->G0 = (double *)calloc(d * nv * N, sizeof(double));
    c->Gt0 = (double *)calloc(d * nv * N, sizeof(double));
    return c;
}

void om_ctx_destroy(om_ctx *c) {
    if (!c) return;
    free(c->hs.F0s); free(c->hs.Fts); free(c->hs.G0s); free(c->hs.Gts);
    free(c->Wn); free(c->L0); free(c->Lt0); free(c->G0); free(c->Gt0);
    free(c);
}

double om_ctx_dt(const om_ctx *c) { return c->dt; }
void om_ctx_force(const om_ctx *c, double *f) { f[0] = c->force[0]; f[1] = c->force[1]; f[2] = c->force[2]; }

/* ------------------------------------------------------------------ */
/* High-order stages (Sec. 2.4 and the two-stage fourth-order marching   */
/* cited in Sec. 1).                                                     */
/*  S1O2: W^{n+1} = W^n + dt L + dt^2/2 L_t; the interface distribution  */
/*        advances as f^{n+1} = f^n + dt f_t, so the new cell gradient is */
/*        the Gauss-Green sum of W_g + dt W_t.                            */
/*  S2O4 (reading of the cited two-stage scheme):                         */
/*    W*      = W^n + dt/2 L^n + dt^2/8 L_t^n,  grad W* = GG(W_g + dt/2 W_t) */
/*    W^{n+1} = W^n + dt L^n + dt^2/6 (L_t^n + 2 L_t^*),                  */
/*    grad W^{n+1} = GG(W_g^n) + dt GG(W_t^*).                            */
/* Gauss-Green: |V| grad W = sum_f sum_g wJ W_g n (Sec. 2.3).            */
/* stage 0 computes dt and the first stage; stage 1 finishes S2O4.       */
/* ------------------------------------------------------------------ */
/* The stage formulas on one value, used by om_stage for every cell and
   exported for the closed-form time-marching pins.  Cell averages: from
   W^n, L^n, L_t^n (and L_t^* at stage 1).  Gradients: from the Gauss-Green
   sums G = GG(W_g), Gt = GG(W_t) of the current pass (and G0 = GG(W_g^n)
   at stage 1). */
void om_stage_combine(int scheme, int stage, double dt, double Wn, double L0, double Lt0, double Lt1, double *out) {
    if (stage == 0) *out = scheme == 0 ? Wn + 0.5 * dt * L0 + 0.125 * dt * dt * Lt0 : Wn + dt * L0 + 0.5 * dt * dt * Lt0;
    else *out = Wn + dt * L0 + dt * dt / 6.0 * (Lt0 + 2.0 * Lt1);
}

void om_grad_combine(int scheme, int stage, double dt, double G0, double G, double Gt, double *out) {
    if (stage == 0) *out = scheme == 0 ? G + 0.5 * dt * Gt : G + dt * Gt;
    else *out = G0 + dt * Gt;
}

int om_stage(om_ctx *c, int stage, double *W, double *dW) {
    const om_mesh *m = c->m;
    const om_params *P = &c->P;
    long N = m->n_cell;
    int nv = m->nv, d = m->dim;
    if (stage == 0) {
        c->dt = om_dt(m, P, W);
        vcopy(c->Wn, W, (int)(nv * N));
    }
    double dt = c->dt;
    int st = ho_pass(m, P, W, dW, dt, &c->hs);
    if (st) return st;
    if (stage == 0) for (int a = 0; a < 3; a++) c->force[a] = c->hs.force[a];
    for (long i = 0; i < N; i++) {
        double V = m->vol[i];
        for (int v = 0; v < nv; v++) {
            double L = -c->hs.F0s[v * N + i] / V;
            double Lt = -c->hs.Fts[v * N + i] / V;
            if (stage == 0) {
                c->L0[v * N + i] = L;
                c->Lt0[v * N + i] = Lt;
                om_stage_combine(P->time_scheme, 0, dt, c->Wn[v * N + i], L, Lt, 0.0, &W[v * N + i]);
            } else {
                om_stage_combine(P->time_scheme, 1, dt, c->Wn[v * N + i], c->L0[v * N + i], c->Lt0[v * N + i], Lt,
                                 &W[v * N + i]);
            }
            for (int a = 0; a < d; a++) {
                long k = (a * nv + v) * N + i;
                double G = c->hs.G0s[k] / V, Gt = c->hs.Gts[k] / V;
                if (stage == 0) {
                    c->G0[k] = G;
                    c->Gt0[k] = Gt;
                }
                om_grad_combine(P->time_scheme, stage, dt, c->G0[k], G, Gt, &dW[k]);
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* High-order residual transferred to the low level (Sec. 3, step 2):   */
/* the time average over [t^{n+1}, t^{n+1}+dt] of the net flux of a      */
/* flux linear in time.  Extensive, with the sign of -oint F.n:          */
/*   R1_i = -sum_f s sum_g wJ (F0 + dt/2 Ft).                             */
/* ------------------------------------------------------------------ */
int om_residual_high(om_ctx *c, const double *W, const double *dW, double *R1) {
    const om_mesh *m = c->m;
    long N = m->n_cell;
    int nv = m->nv;
    int st = ho_pass(m, &c->P, W, dW, c->dt, &c->hs);
    if (st) return st;
    for (long i = 0; i < N; i++)
        for (int v = 0; v < nv; v++) R1[v * N + i] = -(c->hs.F0s[v * N + i] + 0.5 * c->dt * c->hs.Fts[v * N + i]);
    return 0;
}

/* exported: raw per-cell sums of one high-order pass (for parity tests) */
int om_ho_sums(om_ctx *c, const double *W, const double *dW, double *F0s, double *Fts, double *G0s, double *Gts) {
    const om_mesh *m = c->m;
    long N = m->n_cell;
    int nv = m->nv, d = m->dim;
    int st = ho_pass(m, &c->P, W, dW, c->dt, &c->hs);
    if (st) return st;
    vcopy(F0s, c->hs.F0s, (int)(nv * N));
    vcopy(Fts, c->hs.Fts, (int)(nv * N));
    vcopy(G0s, c->hs.G0s, (int)(d * nv * N));
    vcopy(Gts, c->hs.Gts, (int)(d * nv * N));
    return 0;
}

/* ------------------------------------------------------------------ */
/* Low-order level (Sec. 3).                                            */
/* ------------------------------------------------------------------ */
/* ghost state of a boundary face for the first-order scheme (local frame) */
static int ghost_state(const om_mesh *m, const om_params *P, int bc, double e[3][3], const double *Ul, double *Ug) {
    int d = m->dim, nv = m->nv;
    if (bc == BC_SLIP) {
        vcopy(Ug, Ul, nv);
        Ug[1] = -Ul[1];
    } else if (bc == BC_FARFIELD) {
        double Winf_l[NVMAX];
        state_to_local(d, e, P->W_inf, Winf_l);
        farfield_state(d, P->gamma, Ul, Winf_l, Ug);
    } else if (bc == BC_ISOTHERMAL || bc == BC_ADIABATIC) {
        /* no slip: every velocity component reversed */
        vcopy(Ug, Ul, nv);
        for (int a = 0; a < d; a++) Ug[1 + a] = -Ul[1 + a];
    } else {
        return -3;
    }
    return 0;
}

static void euler_flux(int dim, double gamma, const double *U, const double *n, double *F);
static double side_radius(const om_mesh *m, const om_params *P, const double *U, long i, long f);

/* First-order Lax-Friedrichs flux in the face frame (the low-order flux the
   paper compares with KFVS in Sec. 4):
     F = 1/2 (F_n(U_l) + F_n(U_r)) - 1/2 lam (U_r - U_l),
   lam the spectral radius the implicit operator uses on this face, so that
   the operator's splitting A+- = 1/2 (A +- lam I) is the flux's own
   Jacobian at frozen lam. */
static int lf_flux(int dim, double gamma, const double *Ul, const double *Ur, double lam, double *F) {
    int nv = dim + 2;
    prim a = to_prim(Ul, dim, gamma), b = to_prim(Ur, dim, gamma);
    if (!(a.rho > 0) || !(a.p > 0) || !(b.rho > 0) || !(b.p > 0)) return -1;
    const double e0[3] = {1.0, 0.0, 0.0};
    double Fa[NVMAX], Fb[NVMAX];
    euler_flux(dim, gamma, Ul, e0, Fa);
    euler_flux(dim, gamma, Ur, e0, Fb);
    for (int v = 0; v < nv; v++) F[v] = 0.5 * (Fa[v] + Fb[v]) - 0.5 * lam * (Ur[v] - Ul[v]);
    return 0;
}

/* R0_i = -sum_f s S_f F(U_L, U_R; n_f), first order, one flux per face; F is
   KFVS, or Lax-Friedrichs with the face's spectral radius (low_flux = 1) */
int om_residual_low(const om_mesh *m, const om_params *P, const double *U, double *R0) {
    int d = m->dim, nv = m->nv;
    long N = m->n_cell;
    memset(R0, 0, sizeof(double) * nv * N);
    for (long f = 0; f < m->n_face; f++) {
        long L = m->owner[f], R = m->neigh[f];
        double n[3];
        for (int a = 0; a < d; a++) n[a] = m->avec[f * d + a] / m->S[f];
        double e[3][3];
        local_frame(d, n, e);
        double UL[NVMAX], UR[NVMAX], Ug[NVMAX], Ul[NVMAX], Ur[NVMAX];
        for (int v = 0; v < nv; v++) Ug[v] = U[v * N + L];
        state_to_local(d, e, Ug, Ul);
        if (R >= 0) {
            for (int v = 0; v < nv; v++) UR[v] = U[v * N + R];
            state_to_local(d, e, UR, Ur);
        } else if (ghost_state(m, P, m->bc[f], e, Ul, Ur)) {
            return -3;
        }
        (void)UL;
        double Fl[NVMAX], F[NVMAX];
        if (P->low_flux == 1) {
            double lam = side_radius(m, P, U, L, f);
            if (R >= 0) {
                double r = side_radius(m, P, U, R, f);
                if (r > lam) lam = r;
            }
            if (lf_flux(d, P->gamma, Ul, Ur, lam, Fl)) return -1;
        } else if (om_kfvs(d, P->gamma, Ul, Ur, Fl)) {
            return -1;
        }
        vec_to_global(d, e, Fl, F);
        for (int v = 0; v < nv; v++) {
            R0[v * N + L] -= m->S[f] * F[v];
            if (R >= 0) R0[v * N + R] += m->S[f] * F[v];
        }
    }
    return 0;
}

/* normal Euler flux of U along unit n (global frame) */
static void euler_flux(int dim, double gamma, const double *U, const double *n, double *F) {
    int nv = dim + 2;
    prim q = to_prim(U, dim, gamma);
    double un = 0;
    for (int a = 0; a < dim; a++) un += q.U[a] * n[a];
    F[0] = q.rho * un;
    for (int a = 0; a < dim; a++) F[1 + a] = U[1 + a] * un + q.p * n[a];
    F[nv - 1] = (U[nv - 1] + q.p) * un;
}

/* spectral radius of one side: |U.n| + c + 2 (mu/rho) S_f / |V|
   (reading of the modified radius, made dimensionally consistent) */
static double side_radius(const om_mesh *m, const om_params *P, const double *U, long i, long f) {
    int d = m->dim, nv = m->nv;
    long N = m->n_cell;
    double Ui[NVMAX];
    for (int v = 0; v < nv; v++) Ui[v] = U[v * N + i];
    prim q = to_prim(Ui, d, P->gamma);
    double un = 0;
    for (int a = 0; a < d; a++) un += q.U[a] * m->avec[f * d + a] / m->S[f];
    return fabs(un) + sqrt(P->gamma * q.p / q.rho) + 2.0 * P->mu / q.rho * m->S[f] / m->vol[i];
}

/* The low-order solve: W_p0 = W (copy), S = R1 - R0(W_p0), n_implicit
   backward-Euler steps of the first-order scheme with local time steps,
   each solved by point relaxation (Algorithm 1) in the multicolour order:
   every sweep visits the colours ascending, then descending.  The cell
   update is
     dU_i [V_i/dt_i + 1/2 sum_f lam_f S_f]
        + sum_f S_f [F-(U_m + dU_m) - F-(U_m)] = R0_i(U) + S_i,
   F-(U) = 1/2 (F_n(U) - lam_f U) with n outward from i, lam_f the larger
   side radius; boundary faces carry no increment.  Finally the correction
   C = U - W_p0 is added to W. */
int om_lowlevel(const om_mesh *m, const om_params *P, double *W, const double *R1) {
    int d = m->dim, nv = m->nv;
    long N = m->n_cell, NF = m->n_face;
    double *Wp0 = (double *)malloc(sizeof(double) * nv * N);
    double *S = (double *)malloc(sizeof(double) * nv * N);
    double *U = (double *)malloc(sizeof(double) * nv * N);
    double *RHS = (double *)malloc(sizeof(double) * nv * N);
    double *dU = (double *)malloc(sizeof(double) * nv * N);
    double *D = (double *)malloc(sizeof(double) * N);
    double *lam = (double *)malloc(sizeof(double) * NF);
    int st = 0;
    vcopy(Wp0, W, (int)(nv * N));
    st = om_residual_low(m, P, Wp0, S);
    if (st) goto done;
    for (long k = 0; k < nv * N; k++) S[k] = R1[k] - S[k];
    vcopy(U, Wp0, (int)(nv * N));
    for (int step = 0; step < P->n_implicit; step++) {
        st = om_residual_low(m, P, U, RHS);
        if (st) goto done;
        for (long k = 0; k < nv * N; k++) RHS[k] += S[k];
        for (long f = 0; f < NF; f++) {
            double l = side_radius(m, P, U, m->owner[f], f);
            if (m->neigh[f] >= 0) {
                double r = side_radius(m, P, U, m->neigh[f], f);
                if (r > l) l = r;
            }
            lam[f] = l;
        }
        for (long i = 0; i < N; i++) {
            double sum = 0;
            for (long q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; q++) sum += lam[m->cf_face[q]] * m->S[m->cf_face[q]];
            D[i] = m->vol[i] / cell_dt(m, P, U, i, P->cfl_low) + 0.5 * sum;
        }
        memset(dU, 0, sizeof(double) * nv * N);
        for (int sw = 0; sw < P->n_sweeps; sw++)
            for (int dir = 0; dir < 2; dir++)
                for (int cc = 0; cc < m->n_colour; cc++) {
                    int col = dir == 0 ? cc : m->n_colour - 1 - cc;
                    for (long i = 0; i < N; i++) {
                        if (m->colour[i] != col) continue;
                        double acc[NVMAX];
                        for (int v = 0; v < nv; v++) acc[v] = RHS[v * N + i];
                        for (long q = m->cf_ptr[i]; q < m->cf_ptr[i + 1]; q++) {
                            long f = m->cf_face[q];
                            long nb = m->cf_sign[q] > 0 ? m->neigh[f] : m->owner[f];
                            if (nb < 0) continue;
                            double n[3], Um[NVMAX], Up[NVMAX], Fa[NVMAX], Fb[NVMAX];
                            for (int a = 0; a < d; a++) n[a] = m->cf_sign[q] * m->avec[f * d + a] / m->S[f];
                            for (int v = 0; v < nv; v++) {
                                Um[v] = U[v * N + nb];
                                Up[v] = Um[v] + dU[v * N + nb];
                            }
                            euler_flux(d, P->gamma, Up, n, Fa);
                            euler_flux(d, P->gamma, Um, n, Fb);
                            for (int v = 0; v < nv; v++) {
                                double dFm = 0.5 * (Fa[v] - lam[f] * Up[v]) - 0.5 * (Fb[v] - lam[f] * Um[v]);
                                acc[v] -= m->S[f] * dFm;
                            }
                        }
                        for (int v = 0; v < nv; v++) dU[v * N + i] = acc[v] / D[i];
                    }
                }
        for (long k = 0; k < nv * N; k++) U[k] += dU[k];
    }
    for (long k = 0; k < nv * N; k++) W[k] = W[k] + (U[k] - Wp0[k]);
done:
    free(Wp0); free(S); free(U); free(RHS); free(dU); free(D); free(lam);
    return st;
}

/* Res = sum |rho_new - rho_old| / sum rho_old (Sec. 4) */
double om_res(long N, const double *Wold, const double *Wnew) {
    double a = 0, b = 0;
    for (long i = 0; i < N; i++) {
        a += fabs(Wnew[i] - Wold[i]);
        b += Wold[i];
    }
    return a / b;
}

/* ------------------------------------------------------------------ */
/* One two-level V-cycle (Sec. 3): high-order step, restriction of W and */
/* of the residual, forcing, low-order solve, prolongation of the        */
/* correction.  Returns Res of the cycle in *res.                         */
/* ------------------------------------------------------------------ */
int om_cycle(om_ctx *c, double *W, double *dW, double *res) {
    const om_mesh *m = c->m;
    long N = m->n_cell;
    int nv = m->nv;
    double *Wold = (double *)malloc(sizeof(double) * N);
    double *R1 = NULL;
    int st;
    vcopy(Wold, W, (int)N);
    st = om_stage(c, 0, W, dW);
    if (!st && c->P.time_scheme == 0) st = om_stage(c, 1, W, dW);
    if (!st && !c->P.explicit_only) {
        R1 = (double *)malloc(sizeof(double) * nv * N);
        st = om_residual_high(c, W, dW, R1);
        if (!st) st = om_lowlevel(m, &c->P, W, R1);
    }
    if (!st) *res = om_res(N, Wold, W);
    free(Wold);
    free(R1);
    return st;
}
