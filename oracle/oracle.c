/*
 * oracle.c -- plain, slow FP64 CPU reference ("the oracle") for Barnes-Hut
 * tree forces with monopole and traceless-quadrupole cell terms, evaluated
 * over per-group interaction lists.
 *
 * Follows Kodama & Ishiyama, "Acceleration of the tree method with SIMD
 * instruction set" (arXiv:1812.07313):
 *   - Sec. 1: the oct-tree and the opening criterion l/d < theta;
 *   - Sec. 3, eq. (1): monopole + quadrupole potential of a cell;
 *   - Sec. 3, eq. (2)-(3): the traceless quadrupole tensor Q of a cell,
 *     all six components stored;
 *   - Sec. 3, eqs. (4)-(7): phi_mono, phi_quad, a = -grad phi and the
 *     resulting acceleration;
 *   - Sec. 3.4 (List 4 and its text): groups of at most n_crit particles
 *     sharing one interaction list of j-particles and j-cells; the
 *     particle-particle part is summed first, the cell part is added.
 *   - Sec. 4, eq. (8): relative force error against direct summation.
 * The Gaussian-split short-range kernel (periodic box, cutoff) is not from
 * the paper; it is the standard split Phi(r) = -erfc(r / 2 r_s) / r expanded
 * to second order about the cell centre of mass, including the trace term.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the checker.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the GPU library, and
 * the GPU library never calls it.
 *
 * Everything is computed in double precision, in the plain order in which
 * the definitions are written.  OpenMP only distributes independent groups
 * (or particles) over threads; it never changes the order of any sum.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_NOMEM (-5)

enum { ORC_MONO = 0, ORC_QUAD = 1, ORC_SPLIT_QUAD = 2, ORC_SPLIT_MONO = 3,
       ORC_QUAD_SOFT = 4 };

/* ------------------------------------------------------------------------ */
/* Pair and cell interaction terms                                           */
/* ------------------------------------------------------------------------ */

/* Plummer-softened point mass m at separation d = r_j - r_i (Sec. 3, eq. 1
 * first term; eq. 7 with Q = 0).  Adds the attractive acceleration and the
 * (negative) potential. */
void orc_pp_plummer(const double d[3], double m, double eps2, double a[3],
                    double *phi)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
    double rhat = sqrt(r2);
    double rhat3 = rhat * rhat * rhat;
    a[0] += m * d[0] / rhat3;
    a[1] += m * d[1] / rhat3;
    a[2] += m * d[2] / rhat3;
    *phi -= m / rhat;
}

/* One j-cell on one i-particle, monopole + traceless quadrupole, eq. (1)
 * for the potential and eq. (7) for the acceleration, with
 * d = r_ij = r_j - r_i (centre of mass minus i-position),
 * rhat^2 = |d|^2 + eps^2, phi_mono = M / rhat (eq. 4),
 * phi_quad = d.Q.d / (2 rhat^5) (eq. 5), a = -grad phi (eq. 6).
 * Sign convention: a is attractive (points along +d for Q = 0), phi < 0.
 * q = (q00, q01, q02, q11, q12, q22) (List 1 order). */
void orc_pc_quad(const double d[3], double M, const double q[6], double eps2,
                 double a[3], double *phi)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
    double rhat = sqrt(r2);
    double Qd[3];
    Qd[0] = q[0] * d[0] + q[1] * d[1] + q[2] * d[2];
    Qd[1] = q[1] * d[0] + q[3] * d[1] + q[4] * d[2];
    Qd[2] = q[2] * d[0] + q[4] * d[1] + q[5] * d[2];
    double dQd = d[0] * Qd[0] + d[1] * Qd[1] + d[2] * Qd[2];
    double rhat2 = r2;
    double rhat5 = rhat2 * rhat2 * rhat;
    double phi_mono = M / rhat;
    double phi_quad = dQd / (2.0 * rhat5);
    double c = (phi_mono + 5.0 * phi_quad) / rhat2;
    for (int k = 0; k < 3; ++k)
        a[k] += c * d[k] - Qd[k] / rhat5;
    *phi -= phi_mono + phi_quad;
}

/* One j-cell on one i-particle, the complete second-order expansion of the
 * Plummer-softened potential -1/rhat about the cell's centre of mass.
 * Because the softened potential is not harmonic, the second moment
 * contributes through its trace T = sum m |x - com|^2 as well as through
 * the traceless Q.  With the radial derivative functions of
 * Phi(r) = -1/rhat, rhat^2 = r^2 + eps^2:
 *   D1 = Phi'/r = rhat^-3,  D2 = D1'/r = -3 rhat^-5,  D3 = D2'/r = 15 rhat^-7,
 * the expansion of sum_p m_p Phi(|r_p - r_i|) to second order in r_p - com
 * (Taylor's theorem, second moment (Q + T 1)/3) is
 *   phi = M Phi + D2 (d.Q.d) / 6 + T (D2 r^2 + 3 D1) / 6
 *   a   = -grad_i phi
 *       = M D1 d + [D3 (d.Q.d) d + 2 D2 Q d] / 6 + T (D3 r^2 + 5 D2) d / 6
 * with d = com - r_i, r = |d|.  With T = 0 this is orc_pc_quad; the T part
 * is T eps^2 / (2 rhat^5) in phi, the term eq. (1) leaves out. */
void orc_pc_quad_soft(const double d[3], double M, const double q[6], double T,
                      double eps2, double a[3], double *phi)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double rhat = sqrt(r2 + eps2);
    double Phi = -1.0 / rhat;
    double D1 = 1.0 / (rhat * rhat * rhat);
    double D2 = -3.0 * D1 / (rhat * rhat);
    double D3 = -5.0 * D2 / (rhat * rhat);
    double Qd[3];
    Qd[0] = q[0] * d[0] + q[1] * d[1] + q[2] * d[2];
    Qd[1] = q[1] * d[0] + q[3] * d[1] + q[4] * d[2];
    Qd[2] = q[2] * d[0] + q[4] * d[1] + q[5] * d[2];
    double dQd = d[0] * Qd[0] + d[1] * Qd[1] + d[2] * Qd[2];
    double pot = M * Phi + D2 * dQd / 6.0 + T / 6.0 * (D2 * r2 + 3.0 * D1);
    double coef = M * D1 + D3 * dQd / 6.0 + T / 6.0 * (D3 * r2 + 5.0 * D2);
    double qterm = 2.0 * D2 / 6.0;
    for (int k = 0; k < 3; ++k)
        a[k] += coef * d[k] + qterm * Qd[k];
    *phi += pot;
}

/* Monopole-only cell: the cell is a point of mass M at its centre of mass
 * (the paper's "monopole" program, Sec. 5.1, Table 2). */
void orc_pc_mono(const double d[3], double M, double eps2, double a[3],
                 double *phi)
{
    orc_pp_plummer(d, M, eps2, a, phi);
}

/* Gaussian-split short-range kernel (not from the paper; see file header).
 * Phi(r) = -erfc(u)/r with u = r / (2 rs).  Radial derivative functions
 * D1 = Phi'/r, D2 = D1'/r, D3 = D2'/r, derived by hand:
 *   g(u) = erfc(u) + (2u/sqrt(pi)) exp(-u^2)
 *   h(u) = (4u^3/sqrt(pi)) exp(-u^2)
 *   D1 = g / r^3
 *   D2 = -(3g + h) / r^5
 *   D3 = (15g + 5h + (8u^5/sqrt(pi)) exp(-u^2)) / r^7                      */
void orc_split_derivs(double r, double rs, double *Phi, double *D1, double *D2,
                      double *D3)
{
    const double rsqpi = 0.56418958354775628694807945156; /* 1/sqrt(pi) */
    double u = r / (2.0 * rs);
    double e = exp(-u * u);
    double ec = erfc(u);
    double g = ec + 2.0 * u * rsqpi * e;
    double h = 4.0 * u * u * u * rsqpi * e;
    double r2 = r * r;
    double r3 = r2 * r;
    double r5 = r3 * r2;
    double r7 = r5 * r2;
    *Phi = -ec / r;
    *D1 = g / r3;
    *D2 = -(3.0 * g + h) / r5;
    *D3 = (15.0 * g + 5.0 * h + 8.0 * u * u * u * u * u * rsqpi * e) / r7;
}

/* The cutoff of the split kernel is a discrete decision: a term is kept iff
 * its separation is non-zero and below rcut.  By definition that is decided
 * on d = r_j - r_i in FP64 (mode ORC_MASK_ABS).  An implementation that
 * forms the separation from positions relative to a group centre c decides
 * the same way except where |d| lies within rounding (~1e-16 relative) of
 * rcut; mode ORC_MASK_F64_OFS takes the decision that way:
 *   positions relative to c in FP64 (periodic: v - box * rint(v * (1/box))),
 *   their difference, r^2 = fma(dz, dz, fma(dy, dy, dx * dx)),
 *   kept iff 0 < r^2 < rcut * rcut.
 * orc_mask_flips counts the terms of a set of lists on which the two modes
 * disagree, so that a comparison made with ORC_MASK_F64_OFS can be shown to
 * be one with the definition's decisions. */
enum { ORC_MASK_ABS = 0, ORC_MASK_F64_OFS = 1 };

static double wrap_ofs(double v, double box)
{
    return box > 0.0 ? v - box * nearbyint(v * (1.0 / box)) : v;
}

int orc_split_keep(int mode, const double xj[3], const double xi[3],
                   const double c[3], double box, double rcut)
{
    if (mode == ORC_MASK_F64_OFS) {
        double d[3];
        for (int k = 0; k < 3; ++k)
            d[k] = wrap_ofs(xj[k] - c[k], box) - wrap_ofs(xi[k] - c[k], box);
        double r2 = fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
        return r2 > 0.0 && r2 < rcut * rcut;
    }
    double d[3];
    for (int k = 0; k < 3; ++k) {
        d[k] = xj[k] - xi[k];
        if (box > 0.0) d[k] -= box * nearbyint(d[k] / box);
    }
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    return r2 > 0.0 && sqrt(r2) < rcut;
}

/* Number of (i, list entry) terms of the lists (arguments as orc_eval) on
 * which ORC_MASK_ABS and ORC_MASK_F64_OFS decide differently. */
int64_t orc_mask_flips(int64_t ng, const int64_t *i_idx, const int64_t *i_off,
                       const double *x, const int64_t *jp_off, const double *jp_x,
                       const int64_t *jc_off, const double *jc_x, double box, double rcut,
                       const double *gcenter)
{
    int64_t flips = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : flips)
    for (int64_t g = 0; g < ng; ++g) {
        const double *c = &gcenter[3 * g];
        for (int64_t k = i_off[g]; k < i_off[g + 1]; ++k) {
            const double *xi = &x[3 * i_idx[k]];
            for (int64_t j = jp_off[g]; j < jp_off[g + 1]; ++j)
                flips += orc_split_keep(ORC_MASK_ABS, &jp_x[3 * j], xi, c, box, rcut) !=
                         orc_split_keep(ORC_MASK_F64_OFS, &jp_x[3 * j], xi, c, box, rcut);
            for (int64_t j = jc_off[g]; j < jc_off[g + 1]; ++j)
                flips += orc_split_keep(ORC_MASK_ABS, &jc_x[3 * j], xi, c, box, rcut) !=
                         orc_split_keep(ORC_MASK_F64_OFS, &jc_x[3 * j], xi, c, box, rcut);
        }
    }
    return flips;
}

/* Number of (i, list entry) terms of the lists (arguments as orc_eval)
 * that the cutoff keeps under decision `mode`: out[0] for the particle
 * entries, out[1] for the cell entries. */
void orc_count_keep(int mode, int64_t ng, const int64_t *i_idx, const int64_t *i_off,
                    const double *x, const int64_t *jp_off, const double *jp_x,
                    const int64_t *jc_off, const double *jc_x, double box, double rcut,
                    const double *gcenter, int64_t out[2])
{
    int64_t kp = 0, kc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : kp, kc)
    for (int64_t g = 0; g < ng; ++g) {
        const double *c = &gcenter[3 * g];
        for (int64_t k = i_off[g]; k < i_off[g + 1]; ++k) {
            const double *xi = &x[3 * i_idx[k]];
            for (int64_t j = jp_off[g]; j < jp_off[g + 1]; ++j)
                kp += orc_split_keep(mode, &jp_x[3 * j], xi, c, box, rcut);
            for (int64_t j = jc_off[g]; j < jc_off[g + 1]; ++j)
                kc += orc_split_keep(mode, &jc_x[3 * j], xi, c, box, rcut);
        }
    }
    out[0] = kp;
    out[1] = kc;
}

/* Short-range point mass without the cutoff test: a = m D1(r) d,
 * phi = m Phi(r). */
static void split_pair_value(const double d[3], double m, double rs,
                             double a[3], double *phi)
{
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double Phi, D1, D2, D3;
    orc_split_derivs(r, rs, &Phi, &D1, &D2, &D3);
    a[0] += m * D1 * d[0];
    a[1] += m * D1 * d[1];
    a[2] += m * D1 * d[2];
    *phi += m * Phi;
}

/* Short-range point mass: a = m D1(r) d, phi = m Phi(r); zero for r >= rcut
 * and for r == 0 (the self pair; no softening in the split kernel). */
void orc_pp_split(const double d[3], double m, double rs, double rcut,
                  double a[3], double *phi)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return;
    double r = sqrt(r2);
    if (r >= rcut) return;
    double Phi, D1, D2, D3;
    orc_split_derivs(r, rs, &Phi, &D1, &D2, &D3);
    a[0] += m * D1 * d[0];
    a[1] += m * D1 * d[1];
    a[2] += m * D1 * d[2];
    *phi += m * Phi;
}

/* Short-range cell, second order about the centre of mass, with
 * second moment I = (Q + T 1)/3, T = sum m |x - com|^2, d = com - r_i:
 *   phi = M Phi + (1/6) D2 (d.Q.d) + (T/6)(D2 r^2 + 3 D1)
 *   a   = M D1 d + (1/6)(D3 (d.Q.d) d + 2 D2 Q.d) + (T/6)(D3 r^2 + 5 D2) d
 * The cell contributes only when its centre of mass is closer than rcut.
 * With use_quad == 0 only the M terms are kept (split monopole). */
/* The split cell term without the cutoff test. */
static void split_cell_value(const double d[3], double M, const double q[6],
                             double T, double rs, int use_quad, double a[3],
                             double *phi)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r = sqrt(r2);
    double Phi, D1, D2, D3;
    orc_split_derivs(r, rs, &Phi, &D1, &D2, &D3);
    double pot = M * Phi;
    double coef = M * D1;
    double Qd[3] = {0.0, 0.0, 0.0};
    double qterm = 0.0;
    if (use_quad) {
        Qd[0] = q[0] * d[0] + q[1] * d[1] + q[2] * d[2];
        Qd[1] = q[1] * d[0] + q[3] * d[1] + q[4] * d[2];
        Qd[2] = q[2] * d[0] + q[4] * d[1] + q[5] * d[2];
        double dQd = d[0] * Qd[0] + d[1] * Qd[1] + d[2] * Qd[2];
        pot += D2 * dQd / 6.0 + T / 6.0 * (D2 * r2 + 3.0 * D1);
        coef += D3 * dQd / 6.0 + T / 6.0 * (D3 * r2 + 5.0 * D2);
        qterm = 2.0 * D2 / 6.0;
    }
    for (int k = 0; k < 3; ++k)
        a[k] += coef * d[k] + qterm * Qd[k];
    *phi += pot;
}

void orc_pc_split(const double d[3], double M, const double q[6], double T,
                  double rs, double rcut, int use_quad, double a[3],
                  double *phi)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return;
    if (sqrt(r2) >= rcut) return;
    split_cell_value(d, M, q, T, rs, use_quad, a, phi);
}

/* ------------------------------------------------------------------------ */
/* Cell moments (Sec. 3, eq. 2): computed directly from member particles     */
/* ------------------------------------------------------------------------ */

/* M = sum m, com = sum m x / M,
 * Q_ab = sum m (3 x_a x_b - r^2 delta_ab) with x = position - com,
 * T = sum m r^2.  All six Q components are computed (q22 is not derived
 * from q00 + q11), so that tracelessness can be checked.
 * idx == NULL means particles 0..n-1. */
void orc_moments(int64_t n, const int64_t *idx, const double *x,
                 const double *m, double *M_out, double com[3], double q[6],
                 double *T_out)
{
    double M = 0.0, s[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = idx ? idx[k] : k;
        M += m[p];
        for (int c = 0; c < 3; ++c) s[c] += m[p] * x[3 * p + c];
    }
    for (int c = 0; c < 3; ++c) com[c] = (M > 0.0) ? s[c] / M : 0.0;
    for (int c = 0; c < 6; ++c) q[c] = 0.0;
    double T = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = idx ? idx[k] : k;
        double dx = x[3 * p + 0] - com[0];
        double dy = x[3 * p + 1] - com[1];
        double dz = x[3 * p + 2] - com[2];
        double r2 = dx * dx + dy * dy + dz * dz;
        q[0] += m[p] * (3.0 * dx * dx - r2);
        q[1] += m[p] * (3.0 * dx * dy);
        q[2] += m[p] * (3.0 * dx * dz);
        q[3] += m[p] * (3.0 * dy * dy - r2);
        q[4] += m[p] * (3.0 * dy * dz);
        q[5] += m[p] * (3.0 * dz * dz - r2);
        T += m[p] * r2;
    }
    *M_out = M;
    *T_out = T;
}

/* ------------------------------------------------------------------------ */
/* Oct-tree (Sec. 1)                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    double center[3];
    double side;
    int64_t first, count; /* contiguous range of perm[] */
    int32_t child[8];     /* -1 when the octant is empty */
    int32_t parent;
    int32_t depth;
    int32_t leaf;
    double mass, com[3], q[6], trace;
} onode;

typedef struct {
    int64_t n;
    double box; /* > 0: periodic cube [0, box)^3; 0: open boundary */
    int64_t *perm;
    onode *nodes;
    int64_t nnodes, cap;
    /* groups (Sec. 3.4) */
    int64_t ngroups;
    int32_t *group_node;
    /* interaction lists (CSR over groups) */
    int64_t *jp_off, *jp_idx; /* j-particles: original particle indices */
    int64_t *jc_off;
    int32_t *jc_node;         /* j-cells: node ids */
} orc_tree;

static int32_t new_node(orc_tree *t)
{
    if (t->nnodes == t->cap) {
        int64_t nc = t->cap ? 2 * t->cap : 1024;
        onode *p = (onode *)realloc(t->nodes, (size_t)nc * sizeof(onode));
        if (!p) return -1;
        t->nodes = p;
        t->cap = nc;
    }
    onode *nd = &t->nodes[t->nnodes];
    memset(nd, 0, sizeof(*nd));
    for (int k = 0; k < 8; ++k) nd->child[k] = -1;
    nd->parent = -1;
    return (int32_t)t->nnodes++;
}

/* Octant of x in a node: bit k set iff x_k >= centre_k (x -> bit 0,
 * y -> bit 1, z -> bit 2). */
static int octant(const double *xp, const double *c)
{
    return (xp[0] >= c[0] ? 1 : 0) | (xp[1] >= c[1] ? 2 : 0) |
           (xp[2] >= c[2] ? 4 : 0);
}

/* Recursive top-down split of node id: any node with more than nleaf
 * particles below maxdepth is divided into its non-empty octants, in
 * octant order; the split is stable, so particles keep their input order
 * inside each octant. */
static int split_node(orc_tree *t, const double *x, int32_t id, int nleaf,
                      int maxdepth, int64_t *tmp)
{
    int64_t first = t->nodes[id].first, count = t->nodes[id].count;
    if (count <= nleaf || t->nodes[id].depth >= maxdepth) {
        t->nodes[id].leaf = 1;
        return ORC_OK;
    }
    double c[3] = {t->nodes[id].center[0], t->nodes[id].center[1],
                   t->nodes[id].center[2]};
    double side = t->nodes[id].side;
    int64_t cnt[8] = {0}, start[8];
    for (int64_t k = first; k < first + count; ++k)
        cnt[octant(&x[3 * t->perm[k]], c)]++;
    start[0] = first;
    for (int o = 1; o < 8; ++o) start[o] = start[o - 1] + cnt[o - 1];
    int64_t pos[8];
    memcpy(pos, start, sizeof(pos));
    for (int64_t k = first; k < first + count; ++k) {
        int o = octant(&x[3 * t->perm[k]], c);
        tmp[pos[o]++] = t->perm[k];
    }
    memcpy(&t->perm[first], &tmp[first], (size_t)count * sizeof(int64_t));
    for (int o = 0; o < 8; ++o) {
        if (cnt[o] == 0) continue;
        int32_t ch = new_node(t);
        if (ch < 0) return ORC_E_NOMEM;
        onode *nd = &t->nodes[ch];
        double quarter = side * 0.25;
        nd->center[0] = c[0] + ((o & 1) ? quarter : -quarter);
        nd->center[1] = c[1] + ((o & 2) ? quarter : -quarter);
        nd->center[2] = c[2] + ((o & 4) ? quarter : -quarter);
        nd->side = side * 0.5;
        nd->first = start[o];
        nd->count = cnt[o];
        nd->parent = id;
        nd->depth = t->nodes[id].depth + 1;
        t->nodes[id].child[o] = ch;
        int rc = split_node(t, x, ch, nleaf, maxdepth, tmp);
        if (rc) return rc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Groups and the walk (Sec. 3.4; Sec. 1 opening criterion)                  */
/* ------------------------------------------------------------------------ */

static void collect_groups(orc_tree *t, int32_t id, int ncrit, int64_t *ng,
                           int32_t *out)
{
    const onode *nd = &t->nodes[id];
    if (nd->count <= ncrit || nd->leaf) {
        if (out) out[*ng] = id;
        (*ng)++;
        return;
    }
    for (int o = 0; o < 8; ++o)
        if (nd->child[o] >= 0) collect_groups(t, nd->child[o], ncrit, ng, out);
}

/* Minimum-image component (periodic box) or identity. */
static double wrap(double v, double box)
{
    if (box > 0.0) v -= box * nearbyint(v / box);
    return v;
}

/* Squared distance from point p to the cube of centre c and side s. */
static double dist2_point_cube(const double p[3], const double c[3], double s,
                               double box)
{
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double v = fabs(wrap(p[k] - c[k], box)) - 0.5 * s;
        if (v > 0.0) d2 += v * v;
    }
    return d2;
}

/* Squared distance between two cubes. */
static double dist2_cube_cube(const double c1[3], double s1, const double c2[3],
                              double s2, double box)
{
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double v = fabs(wrap(c1[k] - c2[k], box)) - 0.5 * (s1 + s2);
        if (v > 0.0) d2 += v * v;
    }
    return d2;
}

/* Squared distance from point p to the box [lo, hi] (minimum image),
 * formed about the box centre. */
static double dist2_point_box(const double *p, const double *lo,
                              const double *hi, double box)
{
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        double c = 0.5 * (lo[k] + hi[k]), h = 0.5 * (hi[k] - lo[k]);
        double v = fabs(wrap(p[k] - c, box)) - h;
        if (v > 0.0) d2 += v * v;
    }
    return d2;
}

typedef struct {
    double theta2; /* theta^2 */
    double rcut;   /* > 0: prune nodes farther than rcut from the group */
    double rdrop2; /* > 0: drop accepted nodes whose centre of mass lies at
                      least sqrt(rdrop2) from the group's particles' box */
    const double *gbox; /* that box: lo[3], hi[3] */
    int64_t njp, njc;
    int64_t *jp;   /* NULL on the counting pass */
    int32_t *jc;
} walk_state;

static void append_particles(const orc_tree *t, const onode *nd, walk_state *w)
{
    for (int64_t k = nd->first; k < nd->first + nd->count; ++k) {
        if (w->jp) w->jp[w->njp] = t->perm[k];
        w->njp++;
    }
}

/* Walk the tree from node id for group node g.  A node that contains the
 * group is opened.  Otherwise, with d the distance from the node's centre
 * of mass to the nearest point of the group cube and l the node side, the
 * node is accepted as a j-cell iff l^2 < theta^2 d^2 (Sec. 1; theta is
 * passed squared as in List 4).  An accepted one-particle node is entered
 * as a j-particle.  A rejected leaf contributes its particles.
 * With a cutoff, a node whose cube lies farther than rcut from the group
 * cube is skipped with its subtree, and an accepted node whose centre of
 * mass lies at least rcut (1 + 2^-16) from the bounding box of the group's
 * particles is dropped: every particle of the group lies in that box, so
 * each pair such an entry would form is beyond the cutoff, where the
 * short-range terms vanish (the margin keeps the drop exact when r^2 is
 * formed in single precision). */
static void walk_node(const orc_tree *t, int32_t id, const onode *g,
                      walk_state *w)
{
    const onode *nd = &t->nodes[id];
    int contains = nd->first <= g->first &&
                   g->first + g->count <= nd->first + nd->count;
    if (!contains) {
        if (w->rcut > 0.0 &&
            dist2_cube_cube(nd->center, nd->side, g->center, g->side, t->box) >
                w->rcut * w->rcut)
            return;
        double d2 = dist2_point_cube(nd->com, g->center, g->side, t->box);
        if (nd->side * nd->side < w->theta2 * d2) {
            if (w->rdrop2 > 0.0 &&
                dist2_point_box(nd->com, w->gbox, w->gbox + 3, t->box) >= w->rdrop2)
                return;
            if (nd->count == 1) {
                append_particles(t, nd, w);
            } else {
                if (w->jc) w->jc[w->njc] = id;
                w->njc++;
            }
            return;
        }
    }
    if (nd->leaf) {
        append_particles(t, nd, w);
        return;
    }
    for (int o = 0; o < 8; ++o)
        if (nd->child[o] >= 0) walk_node(t, nd->child[o], g, w);
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                       */
/* ------------------------------------------------------------------------ */

void orc_free(orc_tree *t)
{
    if (!t) return;
    free(t->perm);
    free(t->nodes);
    free(t->group_node);
    free(t->jp_off);
    free(t->jp_idx);
    free(t->jc_off);
    free(t->jc_node);
    free(t);
}

/* Build the tree, moments, groups and interaction lists.
 *   n, x[3n], m[n]  particles (FP64)
 *   theta, ncrit    opening angle and group size bound
 *   nleaf           leaf size bound (nodes with more particles are split)
 *   maxdepth        nodes at this depth are leaves regardless of count
 *   box             > 0: periodic cube [0, box)^3 as the root; 0: the root
 *                   is centred on the midpoint of the bounding box, with
 *                   side = largest extent * (1 + 2^-20)
 *   rcut            > 0: prune nodes farther than rcut (min-image)
 *   walk_stride     >= 1: lists are built for groups g with g % walk_stride
 *                   == 0 only (the others get empty lists), to sample very
 *                   large inputs */
int orc_build(int64_t n, const double *x, const double *m, double theta,
              int ncrit, int nleaf, int maxdepth, double box, double rcut,
              int walk_stride, orc_tree **out)
{
    if (!out || n < 1 || !x || !m || ncrit < 1 || nleaf < 1 || theta < 0.0 ||
        maxdepth < 0 || walk_stride < 1)
        return ORC_E_ARG;
    *out = NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    if (!t) return ORC_E_NOMEM;
    t->n = n;
    t->box = box;
    t->perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!t->perm || !tmp) {
        free(tmp);
        orc_free(t);
        return ORC_E_NOMEM;
    }
    for (int64_t k = 0; k < n; ++k) t->perm[k] = k;

    int32_t root = new_node(t);
    if (root < 0) {
        free(tmp);
        orc_free(t);
        return ORC_E_NOMEM;
    }
    if (box > 0.0) {
        for (int k = 0; k < 3; ++k) t->nodes[root].center[k] = 0.5 * box;
        t->nodes[root].side = box;
    } else {
        double lo[3], hi[3];
        for (int k = 0; k < 3; ++k) lo[k] = hi[k] = x[k];
        for (int64_t p = 1; p < n; ++p)
            for (int k = 0; k < 3; ++k) {
                if (x[3 * p + k] < lo[k]) lo[k] = x[3 * p + k];
                if (x[3 * p + k] > hi[k]) hi[k] = x[3 * p + k];
            }
        double ext = 0.0;
        for (int k = 0; k < 3; ++k) {
            t->nodes[root].center[k] = 0.5 * (lo[k] + hi[k]);
            if (hi[k] - lo[k] > ext) ext = hi[k] - lo[k];
        }
        t->nodes[root].side = (ext > 0.0) ? ext * (1.0 + ldexp(1.0, -20)) : 1.0;
    }
    t->nodes[root].first = 0;
    t->nodes[root].count = n;
    int rc = split_node(t, x, root, nleaf, maxdepth, tmp);
    free(tmp);
    if (rc) {
        orc_free(t);
        return rc;
    }

    /* moments of every node, directly from its member particles */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t id = 0; id < t->nnodes; ++id) {
        onode *nd = &t->nodes[id];
        orc_moments(nd->count, &t->perm[nd->first], x, m, &nd->mass, nd->com,
                    nd->q, &nd->trace);
    }

    /* groups */
    int64_t ng = 0;
    collect_groups(t, root, ncrit, &ng, NULL);
    t->ngroups = ng;
    t->group_node = (int32_t *)malloc((size_t)ng * sizeof(int32_t));
    t->jp_off = (int64_t *)calloc((size_t)ng + 1, sizeof(int64_t));
    t->jc_off = (int64_t *)calloc((size_t)ng + 1, sizeof(int64_t));
    if (!t->group_node || !t->jp_off || !t->jc_off) {
        orc_free(t);
        return ORC_E_NOMEM;
    }
    ng = 0;
    collect_groups(t, root, ncrit, &ng, t->group_node);

    /* counting pass, then filling pass */
    double theta2 = theta * theta;
    double rdrop = rcut * (1.0 + 0x1p-16);
    double rdrop2 = rcut > 0.0 ? rdrop * rdrop : 0.0;
    /* bounding box of each group's particles */
    double *gbox = (double *)malloc((size_t)ng * 6 * sizeof(double));
    if (!gbox) {
        orc_free(t);
        return ORC_E_NOMEM;
    }
    for (int64_t g = 0; g < ng; ++g) {
        const onode *gn = &t->nodes[t->group_node[g]];
        double *b = &gbox[6 * g];
        for (int k = 0; k < 3; ++k) {
            b[k] = INFINITY;
            b[3 + k] = -INFINITY;
        }
        for (int64_t q = gn->first; q < gn->first + gn->count; ++q) {
            const double *xp = &x[3 * t->perm[q]];
            for (int k = 0; k < 3; ++k) {
                if (xp[k] < b[k]) b[k] = xp[k];
                if (xp[k] > b[3 + k]) b[3 + k] = xp[k];
            }
        }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < ng; ++g) {
        walk_state w = {theta2, rcut, rdrop2, &gbox[6 * g], 0, 0, NULL, NULL};
        if (g % walk_stride == 0)
            walk_node(t, root, &t->nodes[t->group_node[g]], &w);
        t->jp_off[g + 1] = w.njp;
        t->jc_off[g + 1] = w.njc;
    }
    for (int64_t g = 0; g < ng; ++g) {
        t->jp_off[g + 1] += t->jp_off[g];
        t->jc_off[g + 1] += t->jc_off[g];
    }
    t->jp_idx = (int64_t *)malloc((size_t)(t->jp_off[ng] + 1) * sizeof(int64_t));
    t->jc_node = (int32_t *)malloc((size_t)(t->jc_off[ng] + 1) * sizeof(int32_t));
    if (!t->jp_idx || !t->jc_node) {
        free(gbox);
        orc_free(t);
        return ORC_E_NOMEM;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < ng; ++g) {
        walk_state w = {theta2, rcut, rdrop2, &gbox[6 * g], 0, 0,
                        &t->jp_idx[t->jp_off[g]], &t->jc_node[t->jc_off[g]]};
        if (g % walk_stride == 0)
            walk_node(t, root, &t->nodes[t->group_node[g]], &w);
    }
    free(gbox);
    *out = t;
    return ORC_OK;
}

/* sizes[0..3] = ngroups, total j-particle entries, total j-cell entries,
 * number of nodes. */
void orc_sizes(const orc_tree *t, int64_t sizes[4])
{
    sizes[0] = t->ngroups;
    sizes[1] = t->jp_off[t->ngroups];
    sizes[2] = t->jc_off[t->ngroups];
    sizes[3] = t->nnodes;
}

/* Copy out the groups and lists.  Any pointer may be NULL.
 *   perm[n]           particle order of the tree (groups are contiguous)
 *   i_off[ng+1]       group g owns perm[i_off[g] .. i_off[g+1])
 *   gnode[ng]         node id of each group
 *   jp_off[ng+1], jp_idx[njp]   j-particles (original indices)
 *   jc_off[ng+1], jc_node[njc]  j-cells (node ids) */
void orc_export_lists(const orc_tree *t, int64_t *perm, int64_t *i_off,
                      int32_t *gnode, int64_t *jp_off, int64_t *jp_idx,
                      int64_t *jc_off, int32_t *jc_node)
{
    int64_t ng = t->ngroups;
    if (perm) memcpy(perm, t->perm, (size_t)t->n * sizeof(int64_t));
    if (i_off) {
        for (int64_t g = 0; g < ng; ++g)
            i_off[g] = t->nodes[t->group_node[g]].first;
        i_off[ng] = t->n;
    }
    if (gnode) memcpy(gnode, t->group_node, (size_t)ng * sizeof(int32_t));
    if (jp_off) memcpy(jp_off, t->jp_off, (size_t)(ng + 1) * sizeof(int64_t));
    if (jp_idx)
        memcpy(jp_idx, t->jp_idx, (size_t)t->jp_off[ng] * sizeof(int64_t));
    if (jc_off) memcpy(jc_off, t->jc_off, (size_t)(ng + 1) * sizeof(int64_t));
    if (jc_node)
        memcpy(jc_node, t->jc_node, (size_t)t->jc_off[ng] * sizeof(int32_t));
}

/* Copy out node data (arrays of nnodes; any pointer may be NULL).
 * ints[8*k ..] = first, count, parent, depth, leaf, 0, 0, 0. */
void orc_export_nodes(const orc_tree *t, double *center, double *side,
                      double *mass, double *com, double *q, double *trace,
                      int64_t *ints)
{
    for (int64_t k = 0; k < t->nnodes; ++k) {
        const onode *nd = &t->nodes[k];
        for (int c = 0; c < 3; ++c) {
            if (center) center[3 * k + c] = nd->center[c];
            if (com) com[3 * k + c] = nd->com[c];
        }
        if (side) side[k] = nd->side;
        if (mass) mass[k] = nd->mass;
        if (trace) trace[k] = nd->trace;
        if (q)
            for (int c = 0; c < 6; ++c) q[6 * k + c] = nd->q[c];
        if (ints) {
            int64_t *o = &ints[8 * k];
            o[0] = nd->first;
            o[1] = nd->count;
            o[2] = nd->parent;
            o[3] = nd->depth;
            o[4] = nd->leaf;
            o[5] = o[6] = o[7] = 0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Evaluation of the interaction lists                                       */
/* ------------------------------------------------------------------------ */

/* The result given the lists: for each i of group g (in perm order),
 *   first the j-particles of g in list order, then the j-cells of g in list
 *   order (the particle-particle part is assigned, the cell part added:
 *   Sec. 3.4, List 4).
 * Inputs are explicit arrays so that any lists (not only this tree's) can
 * be evaluated:
 *   n, x[3n], eps2[n]                 i-particles (original indexing)
 *   ng, i_idx[], i_off[ng+1]          group g owns i_idx[i_off[g]..)
 *   jp_off[ng+1]; jp_x[3*], jp_m[]    materialised j-particles
 *   jc_off[ng+1]; jc_x[3*], jc_m[], jc_q[6*], jc_t[]  j-cells
 *   kind   ORC_MONO / ORC_QUAD / ORC_SPLIT_QUAD / ORC_SPLIT_MONO /
 *          ORC_QUAD_SOFT (Plummer cells with the trace term; needs jc_t)
 *   box    > 0: minimum image separations (periodic)
 *   rs, rcut  split-kernel parameters
 *   mask_mode, gcenter[3 ng]  how the split kernel's cutoff is decided (see
 *             orc_split_keep; gcenter may be NULL for ORC_MASK_ABS)
 * Writes a[3 i], phi[i] for every i listed. */
void orc_eval(int kind, int64_t ng, const int64_t *i_idx, const int64_t *i_off,
              const double *x, const double *eps2, const int64_t *jp_off,
              const double *jp_x, const double *jp_m, const int64_t *jc_off,
              const double *jc_x, const double *jc_m, const double *jc_q,
              const double *jc_t, double box, double rs, double rcut,
              int mask_mode, const double *gcenter, double *a, double *phi)
{
    int split = (kind == ORC_SPLIT_QUAD || kind == ORC_SPLIT_MONO);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < ng; ++g) {
        for (int64_t k = i_off[g]; k < i_off[g + 1]; ++k) {
            int64_t i = i_idx[k];
            const double *xi = &x[3 * i];
            double acc[3] = {0.0, 0.0, 0.0}, pot = 0.0;
            for (int64_t j = jp_off[g]; j < jp_off[g + 1]; ++j) {
                double d[3];
                for (int c = 0; c < 3; ++c)
                    d[c] = wrap(jp_x[3 * j + c] - xi[c], box);
                if (split) {
                    if (orc_split_keep(mask_mode, &jp_x[3 * j], xi,
                                       gcenter ? &gcenter[3 * g] : xi, box,
                                       rcut))
                        split_pair_value(d, jp_m[j], rs, acc, &pot);
                } else {
                    orc_pp_plummer(d, jp_m[j], eps2[i], acc, &pot);
                }
            }
            for (int64_t j = jc_off[g]; j < jc_off[g + 1]; ++j) {
                double d[3];
                for (int c = 0; c < 3; ++c)
                    d[c] = wrap(jc_x[3 * j + c] - xi[c], box);
                switch (kind) {
                case ORC_MONO:
                    orc_pc_mono(d, jc_m[j], eps2[i], acc, &pot);
                    break;
                case ORC_QUAD:
                    orc_pc_quad(d, jc_m[j], &jc_q[6 * j], eps2[i], acc, &pot);
                    break;
                case ORC_QUAD_SOFT:
                    orc_pc_quad_soft(d, jc_m[j], &jc_q[6 * j], jc_t ? jc_t[j] : 0.0,
                                     eps2[i], acc, &pot);
                    break;
                default:
                    if (orc_split_keep(mask_mode, &jc_x[3 * j], xi,
                                       gcenter ? &gcenter[3 * g] : xi, box,
                                       rcut))
                        split_cell_value(d, jc_m[j], &jc_q[6 * j],
                                         (kind == ORC_SPLIT_QUAD && jc_t)
                                             ? jc_t[j] : 0.0,
                                         rs, kind == ORC_SPLIT_QUAD, acc, &pot);
                    break;
                }
            }
            for (int c = 0; c < 3; ++c) a[3 * i + c] = acc[c];
            phi[i] = pot;
        }
    }
}

/* Direct summation over all n particles for the nt targets tgt[] (all when
 * tgt == NULL): Plummer softening with the target's eps2, or the split
 * kernel (split != 0) with minimum image in a periodic box and the cutoff.
 * The self pair is included: it adds no force and -m_i/eps_i to the
 * Plummer potential, and nothing to the split kernel (r = 0 is masked).
 * Writes a[3 k], phi[k] for the k-th target (Sec. 4, eq. 8 reference). */
void orc_direct(int64_t n, const double *x, const double *m,
                const double *eps2, int64_t nt, const int64_t *tgt, int split,
                double box, double rs, double rcut, double *a, double *phi)
{
    if (!tgt) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tgt ? tgt[k] : k;
        double acc[3] = {0.0, 0.0, 0.0}, pot = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double d[3];
            for (int c = 0; c < 3; ++c)
                d[c] = wrap(x[3 * j + c] - x[3 * i + c], box);
            if (split)
                orc_pp_split(d, m[j], rs, rcut, acc, &pot);
            else
                orc_pp_plummer(d, m[j], eps2[i], acc, &pot);
        }
        for (int c = 0; c < 3; ++c) a[3 * k + c] = acc[c];
        phi[k] = pot;
    }
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_num_threads(void)
{
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            nt = omp_get_num_threads();
#endif
        }
    }
    return nt;
}

/* Number of OpenMP threads for the oracle's later parallel loops (n >= 1;
 * it distributes independent groups or particles only, so results do not
 * depend on it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
