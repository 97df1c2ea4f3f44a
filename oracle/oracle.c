/*
 * oracle.c -- plain FP64 CPU oracle of the linearized Poisson-Boltzmann grid method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header, table or constant with the GPU library.
 *
 * What it computes (reduced Gaussian units: lengths in Angstrom, charges in e, the
 * potential in e/Angstrom; multiply by the Bjerrum length for kT/e):
 *
 *   -div(eps grad phi) + eps_s kD^2 chi_s phi = 4 pi sum_i q_i delta(x - x_i)
 *
 * which is the linearized PBE of Sect. 2.1 (eq. LPBE) with 4 pi eps_0 = 1.
 *
 *  1. Geometry: a node is solute iff it lies strictly inside one of the atom balls
 *     (the solute is the union of atom balls, Sect. 2.1).  An edge whose two end
 *     nodes lie in different media is "cut"; alpha is the fraction of the edge, measured
 *     from its solute end, up to the first point where the walk leaves the union of
 *     balls (WHA weight, Sect. 3.2 eq. WHA).  The crossing point r_p and the analytic
 *     sphere normal n_p of the ball that is left there are recorded.
 *  2. Operator: cell-by-cell assembly of the primal-mixed FEM condensed with vertex
 *     quadrature (Sect. 3.1, eq. matrixequation): every cell edge adds (h/4) eps_e to the
 *     edge Laplacian, every cell vertex adds (h^3/8) kbar^2 to the diagonal.  eps_e is
 *     eps_in or eps_out for edges inside one medium and the weighted harmonic average
 *     1/(alpha/eps_in + (1-alpha)/eps_out) for cut edges (Sect. 3.2, eq. WHA).
 *  3. Load: trilinear deposition of the point charges, R(w_n) = sum q_i w_n(r_i)
 *     (Sect. 3.1, eq. RVop_), scaled by 4 pi; Dirichlet box nodes are eliminated into
 *     the right-hand side (homogeneous, Debye-Hueckel or user values, Sect. 2.3).
 *  4. Jacobi-preconditioned CG on the assembled CSR matrix (the paper uses CG, Sect. 4).
 *  5. Energy: flux through each cut edge F_p = K_e (phi_s - phi_w) gives the polarization
 *     charge q_p = (1/eps_out - 1/eps_in) F_p / (4 pi) at r_p (Sect. 3.3.1); the ionic
 *     term is the surface formula of eq. energy_ion with the surface potential of
 *     eq. phi0 (second form) and marching-cubes area weights (Sect. 3.3.2); the
 *     Coulomb term is the analytic pair sum without self energy (Sect. 3.3).
 *
 * Built with -ffp-contract=off so that node coordinates and squared distances are
 * evaluated exactly as written (x = origin + h*i; d2 = (dx*dx + dy*dy) + dz*dz).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* physical constants (CODATA 2018) and derived reduced-unit parameters       */
/* ------------------------------------------------------------------------- */

/* Bjerrum length in vacuum, e^2/(4 pi eps0 kB T), in Angstrom; and the ionic
 * screening factor kD^2 in 1/Angstrom^2 for a 1:1 salt of ionic strength I (mol/L),
 * kD^2 = e^2 sum_j z_j^2 rho_j / (eps_s kB T) (Sect. 2.1, after eq. LPBE). */
void orc_constants(double temp_K, double ionic_M, double eps_out, double* lB, double* kD2)
{
    const double e = 1.602176634e-19, kB = 1.380649e-23, NA = 6.02214076e23;
    const double eps0 = 8.8541878128e-12;
    double lb_m = e * e / (4.0 * ORC_PI * eps0 * kB * temp_K);
    double lb = lb_m * 1e10;
    *lB = lb;
    /* rho_j = I * NA * 1000 per m^3 for each of the two species, z = +-1:
     * kD^2 = 2 I NA 1e3 e^2/(eps0 eps_s kB T) = 8 pi lB I NA 1e3 / eps_s  [1/m^2] */
    double kd2_m = 8.0 * ORC_PI * lb_m * ionic_M * NA * 1e3 / eps_out;
    *kD2 = kd2_m * 1e-20;
}

/* ------------------------------------------------------------------------- */
/* grid and atom bins                                                          */
/* ------------------------------------------------------------------------- */

static inline int64_t nid(const int32_t* n, int64_t i, int64_t j, int64_t k)
{
    return (i * n[1] + j) * n[2] + k;
}

static inline double coord(const double* origin, double h, int ax, int64_t i)
{
    return origin[ax] + h * (double)i;
}

typedef struct {
    double lo[3];
    double bs;
    int64_t nb[3];
    int64_t* start; /* nb0*nb1*nb2 + 1 */
    int64_t* ids;
} bins_t;

/* Each atom is listed, in ascending index order, in every bin that its bounding box
 * [c - R, c + R] touches. */
static int bins_build(bins_t* B, int64_t na, const double* xyz, const double* rad, double bs)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t a = 0; a < na; ++a)
        for (int d = 0; d < 3; ++d) {
            double l = xyz[3 * a + d] - rad[a], u = xyz[3 * a + d] + rad[a];
            if (l < lo[d]) lo[d] = l;
            if (u > hi[d]) hi[d] = u;
        }
    B->bs = bs;
    int64_t nbt = 1;
    for (int d = 0; d < 3; ++d) {
        if (na == 0) { lo[d] = 0; hi[d] = 0; }
        B->lo[d] = lo[d];
        B->nb[d] = (int64_t)floor((hi[d] - lo[d]) / bs) + 1;
        nbt *= B->nb[d];
    }
    B->start = (int64_t*)calloc((size_t)nbt + 1, sizeof(int64_t));
    if (!B->start) return -1;
    for (int pass = 0; pass < 2; ++pass) {
        int64_t* fill = NULL;
        if (pass == 1) {
            for (int64_t b = 0; b < nbt; ++b) B->start[b + 1] += B->start[b];
            B->ids = (int64_t*)malloc(sizeof(int64_t) * (size_t)(B->start[nbt] + 1));
            fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nbt + 1));
            if (!B->ids || !fill) return -1;
            memcpy(fill, B->start, sizeof(int64_t) * (size_t)nbt);
        }
        for (int64_t a = 0; a < na; ++a) {
            int64_t b0[3], b1[3];
            for (int d = 0; d < 3; ++d) {
                b0[d] = (int64_t)floor((xyz[3 * a + d] - rad[a] - B->lo[d]) / bs);
                b1[d] = (int64_t)floor((xyz[3 * a + d] + rad[a] - B->lo[d]) / bs);
                if (b0[d] < 0) b0[d] = 0;
                if (b1[d] > B->nb[d] - 1) b1[d] = B->nb[d] - 1;
            }
            for (int64_t x = b0[0]; x <= b1[0]; ++x)
                for (int64_t y = b0[1]; y <= b1[1]; ++y)
                    for (int64_t z = b0[2]; z <= b1[2]; ++z) {
                        int64_t b = (x * B->nb[1] + y) * B->nb[2] + z;
                        if (pass == 0) B->start[b + 1]++;
                        else B->ids[fill[b]++] = a;
                    }
        }
        free(fill);
    }
    return 0;
}

static void bins_free(bins_t* B)
{
    free(B->start);
    free(B->ids);
}

/* bin holding point p, or -1 when p is outside every atom's bounding box */
static int64_t bins_find(const bins_t* B, const double* p)
{
    int64_t b[3];
    for (int d = 0; d < 3; ++d) {
        double f = floor((p[d] - B->lo[d]) / B->bs);
        if (f < 0 || f >= (double)B->nb[d]) return -1;
        b[d] = (int64_t)f;
    }
    return (b[0] * B->nb[1] + b[1]) * B->nb[2] + b[2];
}

/* ------------------------------------------------------------------------- */
/* 1. node classification                                                     */
/* ------------------------------------------------------------------------- */

/* solute[n] = 1 iff node n is strictly inside some atom ball (ties count as solvent). */
int orc_classify(const int32_t* n, const double* origin, double h, int64_t na,
                 const double* xyz, const double* rad, uint8_t* solute)
{
    bins_t B;
    memset(&B, 0, sizeof(B));
    if (bins_build(&B, na, xyz, rad, 2.0 > h ? 2.0 : h)) return -1;
    int64_t N = (int64_t)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n[0]; ++i)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t k = 0; k < n[2]; ++k) {
                double p[3] = {coord(origin, h, 0, i), coord(origin, h, 1, j),
                               coord(origin, h, 2, k)};
                uint8_t s = 0;
                int64_t b = bins_find(&B, p);
                if (b >= 0)
                    for (int64_t t = B.start[b]; t < B.start[b + 1] && !s; ++t) {
                        int64_t a = B.ids[t];
                        double dx = p[0] - xyz[3 * a], dy = p[1] - xyz[3 * a + 1],
                               dz = p[2] - xyz[3 * a + 2];
                        double d2 = dx * dx + dy * dy + dz * dz;
                        if (d2 < rad[a] * rad[a]) s = 1;
                    }
                solute[nid(n, i, j, k)] = s;
            }
    (void)N;
    bins_free(&B);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* 1b. cut edges: alpha, crossing point, normal, owner atom                    */
/* ------------------------------------------------------------------------- */

/* Number of edges whose end nodes are in different media.  Edge keys are
 * key = 3 * n_low + axis with n_low the end with the smaller coordinate. */
int64_t orc_count_cut(const int32_t* n, const uint8_t* solute)
{
    int64_t c = 0;
    for (int64_t i = 0; i < n[0]; ++i)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t k = 0; k < n[2]; ++k) {
                int64_t a = nid(n, i, j, k);
                if (i + 1 < n[0] && solute[a] != solute[nid(n, i + 1, j, k)]) c++;
                if (j + 1 < n[1] && solute[a] != solute[nid(n, i, j + 1, k)]) c++;
                if (k + 1 < n[2] && solute[a] != solute[nid(n, i, j, k + 1)]) c++;
            }
    return c;
}

/* First exit from the union of balls along the edge from its solute end s toward
 * its solvent end w.  t runs from 0 (at s) to h (at w).  Each candidate ball whose
 * axis line distance is below its radius gives a chord [lo, hi]; starting at t = 0
 * we jump to the far end of any chord that contains t until no chord does. */
static void first_exit(const double* s, int ax, double dir, double h, const bins_t* B,
                       const double* w, const double* xyz, const double* rad,
                       double* t_out, int64_t* owner_out)
{
    int64_t bl[2] = {bins_find(B, s), bins_find(B, w)};
    int nbl = (bl[1] == bl[0]) ? 1 : 2;
    double t = 0.0;
    int64_t owner = -1;
    for (;;) {
        double tn = t;
        for (int q = 0; q < nbl; ++q) {
            if (bl[q] < 0) continue;
            for (int64_t u = B->start[bl[q]]; u < B->start[bl[q] + 1]; ++u) {
                int64_t a = B->ids[u];
                double dperp2 = 0.0;
                for (int d = 0; d < 3; ++d) {
                    if (d == ax) continue;
                    double dd = s[d] - xyz[3 * a + d];
                    dperp2 = dperp2 + dd * dd;
                }
                double R2 = rad[a] * rad[a];
                if (!(dperp2 < R2)) continue;
                double half = sqrt(R2 - dperp2);
                double tc = (xyz[3 * a + ax] - s[ax]) * dir;
                double lo = tc - half, hi = tc + half;
                if (lo <= t && t < hi && hi > tn) tn = hi;
            }
        }
        if (tn == t) break;
        t = tn;
    }
    /* owner: lowest-index ball whose chord ends exactly at t and starts before it */
    for (int q = 0; q < nbl; ++q) {
        if (bl[q] < 0) continue;
        for (int64_t u = B->start[bl[q]]; u < B->start[bl[q] + 1]; ++u) {
            int64_t a = B->ids[u];
            double dperp2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                if (d == ax) continue;
                double dd = s[d] - xyz[3 * a + d];
                dperp2 = dperp2 + dd * dd;
            }
            double R2 = rad[a] * rad[a];
            if (!(dperp2 < R2)) continue;
            double half = sqrt(R2 - dperp2);
            double tc = (xyz[3 * a + ax] - s[ax]) * dir;
            double lo = tc - half, hi = tc + half;
            if (hi == t && lo < t && (owner < 0 || a < owner)) owner = a;
        }
    }
    if (t > h) t = h;
    *t_out = t;
    *owner_out = owner;
}

/* Fill the cut-edge list (ncut entries, in ascending key order). */
int orc_cut_edges(const int32_t* n, const double* origin, double h, int64_t na,
                  const double* xyz, const double* rad, const uint8_t* solute, int64_t ncut,
                  int64_t* key, double* alpha, double* rp, double* np, int64_t* owner)
{
    bins_t B;
    memset(&B, 0, sizeof(B));
    if (bins_build(&B, na, xyz, rad, 2.0 > h ? 2.0 : h)) return -1;
    /* ordered pass to collect keys */
    int64_t c = 0;
    for (int64_t i = 0; i < n[0]; ++i)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t k = 0; k < n[2]; ++k) {
                int64_t a = nid(n, i, j, k);
                if (i + 1 < n[0] && solute[a] != solute[nid(n, i + 1, j, k)]) key[c++] = 3 * a + 0;
                if (j + 1 < n[1] && solute[a] != solute[nid(n, i, j + 1, k)]) key[c++] = 3 * a + 1;
                if (k + 1 < n[2] && solute[a] != solute[nid(n, i, j, k + 1)]) key[c++] = 3 * a + 2;
            }
    if (c != ncut) { bins_free(&B); return -2; }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t e = 0; e < ncut; ++e) {
        int64_t a = key[e] / 3;
        int ax = (int)(key[e] % 3);
        int64_t k = a % n[2], j = (a / n[2]) % n[1], i = a / ((int64_t)n[1] * n[2]);
        int64_t ijk[3] = {i, j, k};
        int64_t ijk2[3] = {i, j, k};
        ijk2[ax] += 1;
        double pa[3], pb[3];
        for (int d = 0; d < 3; ++d) {
            pa[d] = coord(origin, h, d, ijk[d]);
            pb[d] = coord(origin, h, d, ijk2[d]);
        }
        int a_is_solute = solute[a] != 0;
        const double* s = a_is_solute ? pa : pb;
        const double* w = a_is_solute ? pb : pa;
        double dir = a_is_solute ? 1.0 : -1.0;
        double t;
        int64_t ow;
        first_exit(s, ax, dir, h, &B, w, xyz, rad, &t, &ow);
        if (ow < 0) {
#pragma omp atomic write
            err = 1;
            ow = 0;
        }
        alpha[e] = t / h;
        for (int d = 0; d < 3; ++d) rp[3 * e + d] = s[d];
        rp[3 * e + ax] = s[ax] + dir * t;
        for (int d = 0; d < 3; ++d) np[3 * e + d] = (rp[3 * e + d] - xyz[3 * ow + d]) / rad[ow];
        owner[e] = ow;
    }
    bins_free(&B);
    return err ? -3 : 0;
}

/* binary search of a key in the ascending cut-key list; -1 when absent */
static int64_t find_key(const int64_t* key, int64_t ncut, int64_t k)
{
    int64_t lo = 0, hi = ncut - 1;
    while (lo <= hi) {
        int64_t m = (lo + hi) / 2;
        if (key[m] == k) return m;
        if (key[m] < k) lo = m + 1;
        else hi = m - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* 2. cell-by-cell assembly into CSR over the interior unknowns               */
/* ------------------------------------------------------------------------- */

static inline double edge_eps(const uint8_t* solute, int64_t a, int64_t b, int64_t ekey,
                              const int64_t* key, const double* alpha, int64_t ncut,
                              double eps_in, double eps_out, int* missing)
{
    if (solute[a] && solute[b]) return eps_in;
    if (!solute[a] && !solute[b]) return eps_out;
    int64_t c = find_key(key, ncut, ekey);
    if (c < 0) { *missing = 1; return eps_out; }
    double al = alpha[c];
    return 1.0 / (al / eps_in + (1.0 - al) / eps_out);
}

/* interior unknown number of node (i,j,k), or -1 for a box (Dirichlet) node */
static inline int64_t unk(const int32_t* n, int64_t i, int64_t j, int64_t k)
{
    if (i <= 0 || j <= 0 || k <= 0 || i >= n[0] - 1 || j >= n[1] - 1 || k >= n[2] - 1) return -1;
    return ((i - 1) * (n[1] - 2) + (j - 1)) * (int64_t)(n[2] - 2) + (k - 1);
}

/*
 * Row-by-row gather of the cell contributions: the row of interior node v collects,
 * from each of the (up to 8) cells having v as a vertex, the cell's edge terms on
 * edges incident to v and the cell's lumped mass at v.  The cell edge weight is
 * (h/4) eps_e and the cell vertex mass is (h^3/8) kbar2(v).  Columns of box nodes
 * are moved to the right-hand side as lift[v] += w * g[box node].
 * CSR arrays: rowptr[nu+1], col[7*nu], val[7*nu] (capacity), *nnz_out.
 */
int orc_assemble(const int32_t* n, double h, double eps_in, double eps_out, double kbar2_out,
                 const uint8_t* solute, int64_t ncut, const int64_t* key, const double* alpha,
                 const double* g, int64_t* rowptr, int64_t* col, double* val, double* lift,
                 int64_t* nnz_out)
{
    int64_t nx = n[0] - 2, ny = n[1] - 2, nz = n[2] - 2;
    int64_t nu = nx * ny * nz;
    int missing = 0;
    double we = 0.25 * h;             /* per-cell edge factor h/4 */
    double wm = h * h * h / 8.0;      /* per-cell vertex mass factor h^3/8 */
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < nu; ++u) {
        int64_t k = u % nz + 1, j = (u / nz) % ny + 1, i = u / (nz * ny) + 1;
        int64_t v = nid(n, i, j, k);
        /* local row: slot 0 = diagonal, slots 1..6 = -x,+x,-y,+y,-z,+z neighbours */
        double rowv[7] = {0, 0, 0, 0, 0, 0, 0};
        int64_t nb[7];
        nb[0] = v;
        nb[1] = nid(n, i - 1, j, k); nb[2] = nid(n, i + 1, j, k);
        nb[3] = nid(n, i, j - 1, k); nb[4] = nid(n, i, j + 1, k);
        nb[5] = nid(n, i, j, k - 1); nb[6] = nid(n, i, j, k + 1);
        /* loop over the 8 cells with v as a vertex: cell lower corner (i-a, j-b, k-c) */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    int64_t ci = i - a, cj = j - b, ck = k - c;
                    /* v is the corner (a, b, c) of this cell; its 3 cell edges run to the
                     * corners differing in one bit */
                    for (int ax = 0; ax < 3; ++ax) {
                        int64_t oi = i, oj = j, ok = k;
                        int bit = (ax == 0) ? a : (ax == 1) ? b : c;
                        int slot;
                        if (ax == 0) { oi = bit ? i - 1 : i + 1; slot = bit ? 1 : 2; }
                        else if (ax == 1) { oj = bit ? j - 1 : j + 1; slot = bit ? 3 : 4; }
                        else { ok = bit ? k - 1 : k + 1; slot = bit ? 5 : 6; }
                        int64_t o = nid(n, oi, oj, ok);
                        int64_t lowi = oi < i ? oi : i, lowj = oj < j ? oj : j, lowk = ok < k ? ok : k;
                        int64_t ekey = 3 * nid(n, lowi, lowj, lowk) + ax;
                        double eps = edge_eps(solute, v, o, ekey, key, alpha, ncut, eps_in,
                                              eps_out, &missing);
                        double w = we * eps;
                        rowv[0] += w;
                        rowv[slot] -= w;
                    }
                    (void)ci; (void)cj; (void)ck;
                    rowv[0] += wm * (solute[v] ? 0.0 : kbar2_out);
                }
        /* write the row: diagonal, then neighbours in slot order; box columns -> lift */
        int64_t base = 7 * u, m = 0;
        double lf = 0.0;
        col[base + m] = u;
        val[base + m] = rowv[0];
        m++;
        for (int s = 1; s < 7; ++s) {
            int64_t o = nb[s];
            int64_t ok = o % n[2], oj = (o / n[2]) % n[1], oi = o / ((int64_t)n[1] * n[2]);
            int64_t cu = unk(n, oi, oj, ok);
            if (cu < 0) {
                lf += -rowv[s] * g[o];
            } else {
                col[base + m] = cu;
                val[base + m] = rowv[s];
                m++;
            }
        }
        for (; m < 7; ++m) { col[base + m] = -1; val[base + m] = 0.0; }
        lift[u] = lf;
    }
    /* compact into CSR */
    int64_t nnz = 0;
    for (int64_t u = 0; u < nu; ++u) {
        rowptr[u] = nnz;
        for (int s = 0; s < 7; ++s) {
            if (col[7 * u + s] < 0) continue;
            col[nnz] = col[7 * u + s];
            val[nnz] = val[7 * u + s];
            nnz++;
        }
    }
    rowptr[nu] = nnz;
    *nnz_out = nnz;
    return missing ? -4 : 0;
}

/*
 * The assembled operator as node fields over the full grid: K[ax] at node (i,j,k) is the
 * total weight of the edge to the next node along ax (4 cells x (h/4) eps_e = h eps_e, the
 * same eps_e as the assembly), zero on the last layer where that edge leaves the box;
 * m at node v is its total mass (8 cells x (h^3/8) kbar2(v)).  For every interior node,
 * the assembled row is diagonal sum(K of its 6 edges) + m and -K towards each neighbour.
 */
int orc_edge_coeffs(const int32_t* n, double h, double eps_in, double eps_out, double kbar2_out,
                    const uint8_t* solute, int64_t ncut, const int64_t* key, const double* alpha,
                    double* Kx, double* Ky, double* Kz, double* m)
{
    int missing = 0;
    const int64_t N = (int64_t)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(static) reduction(| : missing)
    for (int64_t v = 0; v < N; ++v) {
        int64_t k = v % n[2], j = (v / n[2]) % n[1], i = v / ((int64_t)n[1] * n[2]);
        double* out[3] = {Kx, Ky, Kz};
        int64_t idx[3] = {i, j, k};
        for (int ax = 0; ax < 3; ++ax) {
            if (idx[ax] + 1 >= n[ax]) {
                out[ax][v] = 0.0;
                continue;
            }
            int64_t o = nid(n, i + (ax == 0), j + (ax == 1), k + (ax == 2));
            int miss = 0;
            double eps = edge_eps(solute, v, o, 3 * v + ax, key, alpha, ncut, eps_in, eps_out, &miss);
            missing |= miss;
            out[ax][v] = 4.0 * (0.25 * h) * eps;
        }
        m[v] = 8.0 * (h * h * h / 8.0) * (solute[v] ? 0.0 : kbar2_out);
    }
    return missing ? -4 : 0;
}

/* ------------------------------------------------------------------------- */
/* 3. load vector and boundary values                                          */
/* ------------------------------------------------------------------------- */

/* Trilinear deposition: b[node] += 4 pi q w(node), over the full grid.  The host
 * cell is floor((r - origin)/h) clamped to [0, n-2]. */
int orc_deposit(const int32_t* n, const double* origin, double h, int64_t na,
                const double* xyz, const double* q, double* b_full)
{
    for (int64_t a = 0; a < na; ++a) {
        int64_t c[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            double f = (xyz[3 * a + d] - origin[d]) / h;
            double fl = floor(f);
            if (fl < 0) fl = 0;
            if (fl > n[d] - 2) fl = n[d] - 2;
            c[d] = (int64_t)fl;
            t[d] = f - fl;
        }
        for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y)
                for (int z = 0; z < 2; ++z) {
                    double w = (x ? t[0] : 1.0 - t[0]) * (y ? t[1] : 1.0 - t[1]) *
                               (z ? t[2] : 1.0 - t[2]);
                    b_full[nid(n, c[0] + x, c[1] + y, c[2] + z)] += 4.0 * ORC_PI * q[a] * w;
                }
    }
    return 0;
}

/* Debye-Hueckel boundary values (Sect. 2.3):  g(x) = sum_i q_i exp(-kD r)/(eps_out r),
 * on every box node; interior entries are left untouched. */
int orc_bc_dh(const int32_t* n, const double* origin, double h, int64_t na, const double* xyz,
              const double* q, double eps_out, double kD, double* g_full)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n[0]; ++i)
        for (int64_t j = 0; j < n[1]; ++j)
            for (int64_t k = 0; k < n[2]; ++k) {
                if (!(i == 0 || j == 0 || k == 0 || i == n[0] - 1 || j == n[1] - 1 || k == n[2] - 1))
                    continue;
                double p[3] = {coord(origin, h, 0, i), coord(origin, h, 1, j), coord(origin, h, 2, k)};
                double s = 0.0;
                for (int64_t a = 0; a < na; ++a) {
                    double dx = p[0] - xyz[3 * a], dy = p[1] - xyz[3 * a + 1], dz = p[2] - xyz[3 * a + 2];
                    double r = sqrt(dx * dx + dy * dy + dz * dz);
                    s += q[a] * exp(-kD * r) / (eps_out * r);
                }
                g_full[nid(n, i, j, k)] = s;
            }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* 4. Jacobi-preconditioned conjugate gradients on CSR                         */
/* ------------------------------------------------------------------------- */

static void spmv(int64_t nu, const int64_t* rp, const int64_t* ci, const double* v,
                 const double* x, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nu; ++r) {
        double s = 0.0;
        for (int64_t t = rp[r]; t < rp[r + 1]; ++t) s += v[t] * x[ci[t]];
        y[r] = s;
    }
}

/* dot product with a fixed partition into 256 chunks summed in order */
static double dot(int64_t nu, const double* a, const double* b)
{
    enum { NC = 256 };
    double part[NC];
    int64_t chunk = (nu + NC - 1) / NC;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < NC; ++c) {
        double s = 0.0;
        int64_t lo = (int64_t)c * chunk, hi = lo + chunk;
        if (hi > nu) hi = nu;
        for (int64_t r = lo; r < hi; ++r) s += a[r] * b[r];
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < NC; ++c) s += part[c];
    return s;
}

/* Solve A x = b (x starts at 0).  Stops when ||r||_2 <= rtol ||b||_2 with r the
 * recursive residual.  Returns 0 on convergence, 1 when max_iter is reached,
 * 2 on breakdown (p.Ap <= 0). */
int orc_pcg(int64_t nu, const int64_t* rp, const int64_t* ci, const double* v, const double* b,
            double* x, double rtol, int32_t max_iter, int32_t* iters, double* relres)
{
    double* r = (double*)malloc(sizeof(double) * (size_t)nu);
    double* z = (double*)malloc(sizeof(double) * (size_t)nu);
    double* p = (double*)malloc(sizeof(double) * (size_t)nu);
    double* q = (double*)malloc(sizeof(double) * (size_t)nu);
    double* dinv = (double*)malloc(sizeof(double) * (size_t)nu);
    if (!r || !z || !p || !q || !dinv) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < nu; ++u) {
        double d = 0.0;
        for (int64_t t = rp[u]; t < rp[u + 1]; ++t)
            if (ci[t] == u) d += v[t];
        dinv[u] = 1.0 / d;
        x[u] = 0.0;
        r[u] = b[u];
        z[u] = dinv[u] * r[u];
        p[u] = z[u];
    }
    double bnorm = sqrt(dot(nu, b, b));
    double rz = dot(nu, r, z);
    int status = 1, it = 0;
    double rn = bnorm;
    if (bnorm == 0.0) { status = 0; rn = 0.0; }
    for (it = 0; status == 1 && it < max_iter; ++it) {
        spmv(nu, rp, ci, v, p, q);
        double pq = dot(nu, p, q);
        if (!(pq > 0.0)) { status = 2; break; }
        double al = rz / pq;
#pragma omp parallel for schedule(static)
        for (int64_t u = 0; u < nu; ++u) {
            x[u] += al * p[u];
            r[u] -= al * q[u];
        }
        rn = sqrt(dot(nu, r, r));
        if (rn <= rtol * bnorm) { status = 0; it++; break; }
#pragma omp parallel for schedule(static)
        for (int64_t u = 0; u < nu; ++u) z[u] = dinv[u] * r[u];
        double rz2 = dot(nu, r, z);
        double be = rz2 / rz;
        rz = rz2;
#pragma omp parallel for schedule(static)
        for (int64_t u = 0; u < nu; ++u) p[u] = z[u] + be * p[u];
    }
    *iters = it;
    *relres = bnorm > 0 ? rn / bnorm : 0.0;
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/* ------------------------------------------------------------------------- */
/* 5. energy read-back                                                         */
/* ------------------------------------------------------------------------- */

/* Marching-cubes area weights.  For every cell whose corners are not all in one medium,
 * the crossing points on its cut edges are joined face by face: on a face with two cut
 * edges those two are joined; on a face with four (diagonal solute corners) each solute
 * corner's two face edges are joined, which keeps solute corners apart.  Every cut edge
 * then has two partners and the joins form closed loops.  A loop of m crossing points is
 * triangulated as a fan from each of its m vertices in turn; every fan triangle gives a
 * third of its area, divided by m, to each of its three vertices (the average of the m
 * fans, so that the weights do not depend on how the cell edges are numbered).  Local edges: 0..3 along x at (y,z) = 00,10,01,11; 4..7 along y at
 * (x,z) = 00,10,01,11; 8..11 along z at (x,y) = 00,10,01,11. */
static void cell_edge_info(int e, int* ax, int* c0, int* c1)
{
    /* corner id = x + 2y + 4z */
    int g = e / 4, m = e % 4, u = m & 1, v = (m >> 1) & 1;
    *ax = g;
    if (g == 0) { *c0 = 0 + 2 * u + 4 * v; *c1 = 1 + 2 * u + 4 * v; }
    else if (g == 1) { *c0 = u + 0 + 4 * v; *c1 = u + 2 + 4 * v; }
    else { *c0 = u + 2 * v + 0; *c1 = u + 2 * v + 4; }
}

int orc_mc_weights(const int32_t* n, const uint8_t* solute, int64_t ncut, const int64_t* key,
                   const double* rp, double* wp)
{
    for (int64_t e = 0; e < ncut; ++e) wp[e] = 0.0;
    int err = 0;
    for (int64_t ci = 0; ci + 1 < n[0]; ++ci)
        for (int64_t cj = 0; cj + 1 < n[1]; ++cj)
            for (int64_t ck = 0; ck + 1 < n[2]; ++ck) {
                int s[8], ns = 0;
                for (int c = 0; c < 8; ++c) {
                    s[c] = solute[nid(n, ci + (c & 1), cj + ((c >> 1) & 1), ck + ((c >> 2) & 1))] ? 1 : 0;
                    ns += s[c];
                }
                if (ns == 0 || ns == 8) continue;
                int cut[12];
                int64_t gidx[12];
                int link[12][2];
                for (int e = 0; e < 12; ++e) {
                    int ax, c0, c1;
                    cell_edge_info(e, &ax, &c0, &c1);
                    cut[e] = s[c0] != s[c1];
                    link[e][0] = link[e][1] = -1;
                    gidx[e] = -1;
                    if (cut[e]) {
                        int64_t li = ci + (c0 & 1), lj = cj + ((c0 >> 1) & 1), lk = ck + ((c0 >> 2) & 1);
                        gidx[e] = find_key(key, ncut, 3 * nid(n, li, lj, lk) + ax);
                        if (gidx[e] < 0) err = 1;
                    }
                }
                if (err) continue;
                /* faces: fixed axis fa, side sd; its edges are the cell edges whose both
                 * corners have bit fa equal to sd */
                for (int fa = 0; fa < 3; ++fa)
                    for (int sd = 0; sd < 2; ++sd) {
                        int fe[4], nf = 0, ncf = 0;
                        for (int e = 0; e < 12; ++e) {
                            int ax, c0, c1;
                            cell_edge_info(e, &ax, &c0, &c1);
                            if (ax == fa) continue;
                            if (((c0 >> fa) & 1) == sd && ((c1 >> fa) & 1) == sd) fe[nf++] = e;
                        }
                        for (int t = 0; t < 4; ++t) ncf += cut[fe[t]];
                        int pairs[2][2], np_ = 0;
                        if (ncf == 2) {
                            int a = -1, b = -1;
                            for (int t = 0; t < 4; ++t)
                                if (cut[fe[t]]) { if (a < 0) a = fe[t]; else b = fe[t]; }
                            pairs[0][0] = a; pairs[0][1] = b; np_ = 1;
                        } else if (ncf == 4) {
                            /* for each solute corner on this face, its two face edges */
                            for (int c = 0; c < 8; ++c) {
                                if (((c >> fa) & 1) != sd || !s[c]) continue;
                                int a = -1, b = -1;
                                for (int t = 0; t < 4; ++t) {
                                    int ax, c0, c1;
                                    cell_edge_info(fe[t], &ax, &c0, &c1);
                                    if (c0 == c || c1 == c) { if (a < 0) a = fe[t]; else b = fe[t]; }
                                }
                                pairs[np_][0] = a; pairs[np_][1] = b; np_++;
                            }
                        }
                        for (int t = 0; t < np_; ++t) {
                            int a = pairs[t][0], b = pairs[t][1];
                            if (link[a][0] < 0) link[a][0] = b; else link[a][1] = b;
                            if (link[b][0] < 0) link[b][0] = a; else link[b][1] = a;
                        }
                    }
                /* walk the loops */
                int seen[12] = {0};
                for (int e0 = 0; e0 < 12; ++e0) {
                    if (!cut[e0] || seen[e0]) continue;
                    int loop[12], m = 0, prev = -1, cur = e0;
                    for (;;) {
                        loop[m++] = cur;
                        seen[cur] = 1;
                        int nxt = (link[cur][0] != prev) ? link[cur][0] : link[cur][1];
                        if (m == 2 && link[cur][0] == link[cur][1]) nxt = link[cur][0];
                        if (nxt == e0 || nxt < 0 || m >= 12) break;
                        prev = cur;
                        cur = nxt;
                    }
                    /* average of the m fans, one from each vertex of the loop */
                    for (int st = 0; st < m; ++st) {
                        const double* v0 = rp + 3 * gidx[loop[st]];
                        for (int t = 1; t + 1 < m; ++t) {
                            int i1 = loop[(st + t) % m], i2 = loop[(st + t + 1) % m];
                            const double* v1 = rp + 3 * gidx[i1];
                            const double* v2 = rp + 3 * gidx[i2];
                            double a1[3], a2[3], cr[3];
                            for (int d = 0; d < 3; ++d) { a1[d] = v1[d] - v0[d]; a2[d] = v2[d] - v0[d]; }
                            cr[0] = a1[1] * a2[2] - a1[2] * a2[1];
                            cr[1] = a1[2] * a2[0] - a1[0] * a2[2];
                            cr[2] = a1[0] * a2[1] - a1[1] * a2[0];
                            double T = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
                            double share = T / (3.0 * (double)m);
                            wp[gidx[loop[st]]] += share;
                            wp[gidx[i1]] += share;
                            wp[gidx[i2]] += share;
                        }
                    }
                }
            }
    return err ? -5 : 0;
}

/* Per cut edge: flux F = K_e (phi_s - phi_w) with K_e = h eps_eff, and the surface
 * potential phi_p = phi_s + (alpha/eps_in) eps_eff (phi_w - phi_s)  (eq. phi0, second
 * form, with medium 1 the solute). */
int orc_edge_fields(const int32_t* n, double h, double eps_in, double eps_out,
                    const uint8_t* solute, int64_t ncut, const int64_t* key, const double* alpha,
                    const double* phi, double* F, double* phip)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ncut; ++e) {
        int64_t a = key[e] / 3;
        int ax = (int)(key[e] % 3);
        int64_t b = a + (ax == 0 ? (int64_t)n[1] * n[2] : ax == 1 ? n[2] : 1);
        int64_t s = solute[a] ? a : b, w = solute[a] ? b : a;
        double al = alpha[e];
        double ee = 1.0 / (al / eps_in + (1.0 - al) / eps_out);
        F[e] = h * ee * (phi[s] - phi[w]);
        phip[e] = phi[s] + (al / eps_in) * ee * (phi[w] - phi[s]);
    }
    return 0;
}

/* For each selected atom i: S_F(i) = sum_p F_p/(4 pi |r_p - r_i|) and
 * S_D(i) = sum_p w_p phi_p (r_p - r_i).n_p / (4 pi |r_p - r_i|^3), summed over p in order. */
int orc_surface_sums(int64_t nsel, const int64_t* sel, const double* xyz, int64_t ncut,
                     const double* rp, const double* np, const double* F, const double* wp,
                     const double* phip, double* SF, double* SD)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nsel; ++t) {
        int64_t i = sel[t];
        double sf = 0.0, sd = 0.0;
        for (int64_t p = 0; p < ncut; ++p) {
            double d[3] = {rp[3 * p] - xyz[3 * i], rp[3 * p + 1] - xyz[3 * i + 1],
                           rp[3 * p + 2] - xyz[3 * i + 2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r = sqrt(r2);
            sf += F[p] / (4.0 * ORC_PI * r);
            double dn = d[0] * np[3 * p] + d[1] * np[3 * p + 1] + d[2] * np[3 * p + 2];
            sd += wp[p] * phip[p] * dn / (4.0 * ORC_PI * r2 * r);
        }
        SF[t] = sf;
        SD[t] = sd;
    }
    return 0;
}

/* Coulomb energy without self terms, sum_{i<j} q_i q_j /(eps_in r_ij), in e^2/Angstrom. */
double orc_coulomb(int64_t na, const double* xyz, const double* q, double eps_in)
{
    enum { NC = 256 };
    double part[NC];
    for (int c = 0; c < NC; ++c) part[c] = 0.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < NC; ++c) {
        double s = 0.0;
        for (int64_t i = c; i < na; i += NC)
            for (int64_t j = 0; j < i; ++j) {
                double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
                       dz = xyz[3 * i + 2] - xyz[3 * j + 2];
                s += q[i] * q[j] / (eps_in * sqrt(dx * dx + dy * dy + dz * dz));
            }
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < NC; ++c) s += part[c];
    return s;
}

/* ------------------------------------------------------------------------- */
/* local refinement: which coarse cells are split into 2x2x2 fine cells        */
/* ------------------------------------------------------------------------- */

/* Coarse cell c (index per axis in [0, n-2]) covers the closed box
 * [origin + H c, origin + H (c+1)].  It is flagged when a surface crossing point lies
 * within distance delta of that box; flags are then rounded up to aligned bricks of
 * brick^3 cells (a brick is refined as a whole when any of its cells is flagged).
 * refined[] is indexed ((ci*(n1-1) + cj)*(n2-1) + ck).  Returns the number of refined
 * cells. */
int64_t orc_refine_cells(const int32_t* n, const double* origin, double H, double delta,
                         int32_t brick, int64_t np, const double* rp, uint8_t* refined)
{
    const int64_t nc[3] = {n[0] - 1, n[1] - 1, n[2] - 1};
    const int64_t ncell = nc[0] * nc[1] * nc[2];
    uint8_t* flag = (uint8_t*)calloc((size_t)ncell, 1);
    if (!flag) return -1;
    const double d2max = delta * delta;
    for (int64_t p = 0; p < np; ++p) {
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            double a = floor((rp[3 * p + d] - delta - origin[d]) / H) - 1;
            double b = floor((rp[3 * p + d] + delta - origin[d]) / H) + 1;
            lo[d] = a < 0 ? 0 : (int64_t)a;
            hi[d] = b > nc[d] - 1 ? nc[d] - 1 : (int64_t)b;
        }
        for (int64_t i = lo[0]; i <= hi[0]; ++i)
            for (int64_t j = lo[1]; j <= hi[1]; ++j)
                for (int64_t k = lo[2]; k <= hi[2]; ++k) {
                    const int64_t c[3] = {i, j, k};
                    double dd[3];
                    for (int d = 0; d < 3; ++d) {
                        double blo = origin[d] + H * (double)c[d];
                        double bhi = origin[d] + H * (double)(c[d] + 1);
                        double x = rp[3 * p + d];
                        double e = blo - x > x - bhi ? blo - x : x - bhi;
                        dd[d] = e > 0.0 ? e : 0.0;
                    }
                    double d2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
                    if (d2 <= d2max) flag[(i * nc[1] + j) * nc[2] + k] = 1;
                }
    }
    /* bricks */
    const int64_t nb[3] = {(nc[0] + brick - 1) / brick, (nc[1] + brick - 1) / brick, (nc[2] + brick - 1) / brick};
    uint8_t* bf = (uint8_t*)calloc((size_t)(nb[0] * nb[1] * nb[2]), 1);
    if (!bf) {
        free(flag);
        return -1;
    }
    for (int64_t i = 0; i < nc[0]; ++i)
        for (int64_t j = 0; j < nc[1]; ++j)
            for (int64_t k = 0; k < nc[2]; ++k)
                if (flag[(i * nc[1] + j) * nc[2] + k])
                    bf[((i / brick) * nb[1] + j / brick) * nb[2] + k / brick] = 1;
    int64_t cnt = 0;
    for (int64_t i = 0; i < nc[0]; ++i)
        for (int64_t j = 0; j < nc[1]; ++j)
            for (int64_t k = 0; k < nc[2]; ++k) {
                uint8_t r = bf[((i / brick) * nb[1] + j / brick) * nb[2] + k / brick];
                refined[(i * nc[1] + j) * nc[2] + k] = r;
                cnt += r;
            }
    free(flag);
    free(bf);
    return cnt;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
