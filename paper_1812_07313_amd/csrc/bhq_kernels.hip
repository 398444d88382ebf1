// bhq_kernels.hip -- force kernels for gfx950 (CDNA4).
//
// One block (256 or 128 threads) evaluates one group's interaction list (the
// modified tree algorithm of Kodama & Ishiyama, Sec. 3.4: all i-particles of
// a group share one list).  Each active thread owns one or two i-particles
// (two: every LDS broadcast feeds two interactions).  The list is
// streamed through LDS in tiles of up to 256 entries: every thread loads one
// entry with coalesced FP64 SoA reads, forms its position relative to the
// group's FP64 reference point, converts it to the working precision and
// stores it in LDS; the threads then read entries back as broadcasts.
//
// Small groups (ni < 256) split each tile between S = 256 / ni slices of
// ni threads.  A tile then holds T = S * floor(256 / S) entries and slice s
// takes the contiguous chunk [s * it, (s + 1) * it) of it (the cell loop
// of the split kernels: the interleaved entries s, s + S, ...); the last
// tile is padded to a multiple of S with zero-mass entries, so every thread
// runs the same trip count.  The slices' partial sums are combined in a
// fixed order at the end, so results are deterministic run to run.
//
// Lists are either materialised (SoA FP64 copies of every entry) or
// index lists into shared particle and cell pools (AoS FP64 records); the
// staging step gathers either kind into the same LDS tile.
//
// Interaction arithmetic (per i-particle, per list entry, d = x_j - x_i):
//   particle:  rinv = rsq(|d|^2 + eps^2); a += m rinv^3 d; -phi += m rinv
//   cell (monopole + traceless quadrupole, Sec. 3 eqs. 1 and 7):
//     Qd = Q d, dQd = d.Qd, rinv5 = rinv^5,
//     -phi += M rinv + dQd rinv5 / 2,
//     a += (M rinv + 2.5 dQd rinv5) rinv^2 d - rinv5 Qd
//   This is the paper's per-cell sequence with the constant factors folded
//   (0.5 and 5 phi_q become 0.5 and 2.5 on dQd rinv5), 34 VALU operations.
//   The complete softened expansion (cells carry their trace T) replaces
//   dQd by dQd - T eps^2 in both terms: 35 operations.
// The particle-particle part is summed before the cell part (List 4).
// Accumulation is tile-blocked: each tile is summed into fresh registers
// that are then added to the running sums.
#include <hip/hip_runtime.h>

#include "bhq_internal.h"
#include "bhq_terms.h"
#include "split_table.h"
#include "split_table64.h"

#include <mutex>
#include <type_traits>

namespace bhq {

namespace {

__device__ __forceinline__ double erfc_r(double v) { return ::erfc(v); }
__device__ __forceinline__ double exp_r(double v) { return ::exp(v); }

// Minimum image v - box rint(v / box), rounded as written (no contraction of
// the product into the subtraction), so that every kernel forms the same
// FP64 offsets.
__device__ __forceinline__ double wrap(double v, double box, double ibox)
{
    return box > 0.0 ? __dsub_rn(v, __dmul_rn(box, ::rint(__dmul_rn(v, ibox)))) : v;
}

constexpr int kMono = 0, kQuad = 1, kSplitQuad = 2, kSplitMono = 3, kQuadSoft = 4;

// Constants of the Gaussian split, uniform over a launch: u = r i2rs with
// i2rs = 1 / (2 r_s); the FP32 table variable is t = r ct = u N / U.
template <typename R>
struct SplitK {
    R i2rs;
    R ct;
};

template <typename R>
__device__ __forceinline__ SplitK<R> split_k(double rs)
{
    SplitK<R> K;
    const double i2rs = 0.5 / rs;
    K.i2rs = R(i2rs);
    K.ct = R(i2rs * ((double)kSplitIntervals / (double)kSplitDomain));
    return K;
}

// The FP32 table of the split radial functions (split_table.h) in device
// memory, one V4 {c0, c1, c2, c3} per function and interval; each block of
// a split kernel copies it to LDS, where lanes read their own intervals.
struct SplitTab {
    V4<float> v[kSplitFuncs * kSplitEntries];
};

constexpr SplitTab make_split_tab()
{
    SplitTab t{};
    for (int f = 0; f < kSplitFuncs; ++f)
        for (int q = 0; q < kSplitEntries; ++q)
            t.v[f * kSplitEntries + q] = {kSplitTable[f][q][0], kSplitTable[f][q][1],
                                          kSplitTable[f][q][2], kSplitTable[f][q][3]};
    return t;
}

__device__ const SplitTab kSplitTabDev = make_split_tab();

// The FP64 kernels' table of exp(-u^2) and erfcx (split_table64.h),
// likewise copied to LDS by each block of an FP64 split kernel.
struct Tab64 {
    double v[kTab64Intervals * kTab64Stride];
};

constexpr Tab64 make_tab64()
{
    Tab64 t{};
    for (int q = 0; q < kTab64Intervals; ++q)
        for (int k = 0; k < kTab64Stride; ++k) t.v[q * kTab64Stride + k] = kTab64[q][k];
    return t;
}

__device__ const Tab64 kTab64Dev = make_tab64();

// Element type of the LDS table of a precision.
template <typename R>
struct SplitTabT {
    using type = V4<float>;
};
template <>
struct SplitTabT<double> {
    using type = double;
};
template <typename R>
using TabT = typename SplitTabT<R>::type;

// Gaussian-split radial functions at r (r2 = r^2), u = r / (2 r_s):
//   ec = erfc(u), g = erfc(u) + (2u/sqrt(pi)) e^{-u^2},
//   G2 = 3g + h, G3 = 15g + 5h + k, with h = (4u^3/sqrt(pi)) e^{-u^2} and
//   k = 2 u^2 h (G2, G3 only for cells with the quadrupole).
// FP64 takes E = exp(-u^2) and erfcx(u) from the polynomials of
// split_table64.h (interval q = floor(t), t = u 64 / 4, f = t - q, Horner's
// rule; degree 9 for E, 7 for erfcx) and forms erfc(u) = E erfcx(u); past
// u = 4, that is for cutoffs beyond 8 r_s, it calls the library's exp and
// erfc.  FP32 reads the
// piecewise cubics of the table at t = r ct: interval q = floor(t), local
// variable f = t - q, Horner's rule (valid for u up to kSplitDomain and one
// interval beyond; the host refuses FP32 split kernels with a longer
// cutoff).
template <typename R>
struct SplitG {
    R ec, g, g2, g3;
};

__device__ __forceinline__ float horner(const V4<float> &c, float f)
{
    return fmaf(fmaf(fmaf(c.w, f, c.z), f, c.y), f, c.x);
}

template <typename R, bool CELL>
__device__ __forceinline__ SplitG<R> split_g(R r, const SplitK<R> &K, const TabT<R> *tab)
{
    SplitG<R> s;
    if constexpr (std::is_same<R, float>::value) {
        const float t = r * K.ct;
        const int q = (int)t;  // t >= 0
        const float f = __builtin_amdgcn_fractf(t);
        s.ec = horner(tab[q], f);
        s.g = horner(tab[kSplitEntries + q], f);
        if (CELL) {
            s.g2 = horner(tab[2 * kSplitEntries + q], f);
            s.g3 = horner(tab[3 * kSplitEntries + q], f);
        }
    } else {
        const R rsqpi = R(0.56418958354775628694807945156);
        const R u = r * K.i2rs;
        const R u2 = u * u;
        R E;
        if (u < R(kTab64Domain)) {
            // t < 64 exactly: the scale 64 / 4 is a power of two
            const R t = u * R(kTab64Intervals / kTab64Domain);
            const int q = (int)t;
            const R f = t - R(q);
            const double *c = tab + q * kTab64Stride;
            E = c[kExpDegree];
#pragma unroll
            for (int k = kExpDegree - 1; k >= 0; --k) E = fma(E, f, c[k]);
            const double *cx = c + kExpDegree + 1;
            R x = cx[kErfcxDegree];
#pragma unroll
            for (int k = kErfcxDegree - 1; k >= 0; --k) x = fma(x, f, cx[k]);
            s.ec = E * x;
        } else {
            E = exp_r(-u2);
            s.ec = erfc_r(u);
        }
        const R e = E * rsqpi;
        s.g = fma(R(2) * u, e, s.ec);
        if (CELL) {
            const R h = R(4) * u * u2 * e;
            const R k = R(2) * u2 * h;
            s.g2 = fma(R(3), s.g, h);
            s.g3 = fma(R(15), s.g, fma(R(5), h, k));
        }
    }
    return s;
}

// The cutoff is a decision on r^2, which the FP32 kernels form from FP32
// offsets.  It is taken as the FP64 kernel takes it: FP64 offsets
// X = wrap(v - c) from the group centre c, D = X_j - X_i, r^2 =
// fma(Dz, Dz, fma(Dy, Dy, Dx Dx)), kept iff 0 < r^2 < rcut * rcut in FP64.
// Outside a band around fl32(rcut^2) the FP32 r^2 decides the same way; a
// term inside the band (rare) is decided again from the FP64 positions.
//
// Band: with u = 2^-24, FP32 offsets x = X (1 + e), |e| <= u, the FP32
// difference and the three-term FMA chain give, to first order in u,
// |r2_32 - |D|^2| <= 7 u |D|^2 + 4 u |X_i| |D|, and fl32(rcut^2) is within
// u rcut^2 of rcut^2 (the FP64 side is exact to 2^-50).  Near the cutoff
// |D| ~ rcut, so u (8 rcut^2 + 4 |X_i| rcut) bounds the difference;
// band_i = u (16 rcut^2 + 8 |X_i| rcut) doubles it.  A term with
// |r2_32 - fl32(rcut^2)| >= band_i is on the same side in both precisions.
__device__ __forceinline__ float cut_band(float xi, float yi, float zi, float rcut)
{
    const float xn = __builtin_sqrtf(fmaf(zi, zi, fmaf(yi, yi, xi * xi)));
    return 0x1p-21f * rcut * fmaf(2.0f, rcut, xn);  // u (16 rcut^2 + 8 |X_i| rcut)
}

// FP64 cutoff decision of the FP64 kernel for the FP64 offsets xj - xi
// (each already wrapped relative to the group centre).
__device__ __forceinline__ bool keep_f64(double djx, double djy, double djz, double rcut)
{
    const double r2 = fma(djz, djz, fma(djy, djy, djx * djx));
    return r2 > 0.0 && r2 < rcut * rcut;
}

// Separation of a list entry from an i-particle and its squared length.
template <typename R>
struct Sep {
    R dx, dy, dz, r2;
};

template <typename R>
__device__ __forceinline__ Sep<R> separation(const V4<R> &j, R xi, R yi, R zi)
{
    Sep<R> s;
    s.dx = j.x - xi;
    s.dy = j.y - yi;
    s.dz = j.z - zi;
    s.r2 = fma(s.dz, s.dz, fma(s.dy, s.dy, s.dx * s.dx));
    return s;
}

// Short-range particle at separation s, kept by the cutoff decision:
// a += m g/r^3 d, -phi += m erfc(u)/r.
template <typename R>
__device__ __forceinline__ void pp_split(const V4<R> &j, const Sep<R> &s, const SplitK<R> &K,
                                         const TabT<R> *tab, R &ax, R &ay, R &az, R &pt)
{
    const R rinv = rsq(s.r2);
    const R r = s.r2 * rinv;
    const SplitG<R> f = split_g<R, false>(r, K, tab);
    const R mr = j.w * rinv;
    const R c = mr * f.g * (rinv * rinv);
    pt = fma(mr, f.ec, pt);
    ax = fma(c, s.dx, ax);
    ay = fma(c, s.dy, ay);
    az = fma(c, s.dz, az);
}

// Short-range cell expanded to second order about its centre of mass
// (with the trace T):
//   phi = M Phi + D2 dQd / 6 + T/6 (D2 r^2 + 3 D1)
//   a   = [M D1 + D3 dQd / 6 + T/6 (D3 r^2 + 5 D2)] d + D2/3 Qd
// with D1 = g/r^3, D2 = -(3g + h)/r^5, D3 = (15g + 5h + k)/r^7.
template <typename R, bool QUAD>
__device__ __forceinline__ void pc_split(const V4<R> &a, const V4<R> &b, const V4<R> &c,
                                         const Sep<R> &s, const SplitK<R> &K,
                                         const TabT<R> *tab, R &ax, R &ay, R &az, R &pt)
{
    const R dx = s.dx, dy = s.dy, dz = s.dz, r2 = s.r2;
    const R rinv = rsq(r2);
    const R r = r2 * rinv;
    const R rinv2 = rinv * rinv;
    const SplitG<R> f = split_g<R, QUAD>(r, K, tab);
    const R D1 = f.g * rinv2 * rinv;
    R phi = -a.w * f.ec * rinv;  // M Phi
    R coef = a.w * D1;
    if (QUAD) {
        const R rinv5 = rinv2 * rinv2 * rinv;
        const R D2 = -f.g2 * rinv5;
        const R D3 = f.g3 * rinv5 * rinv2;
        const R qx = fma(b.z, dz, fma(b.y, dy, b.x * dx));
        const R qy = fma(c.x, dz, fma(b.w, dy, b.y * dx));
        const R qz = fma(c.y, dz, fma(c.x, dy, b.z * dx));
        const R dqd = fma(dz, qz, fma(dy, qy, dx * qx));
        const R t6 = c.z * R(1.0 / 6.0);
        phi = fma(D2, dqd * R(1.0 / 6.0), phi);
        phi = fma(t6, fma(D2, r2, R(3) * D1), phi);
        coef = fma(D3, dqd * R(1.0 / 6.0), coef);
        coef = fma(t6, fma(D3, r2, R(5) * D2), coef);
        const R d23 = D2 * R(1.0 / 3.0);
        ax = fma(d23, qx, ax);
        ay = fma(d23, qy, ay);
        az = fma(d23, qz, az);
    }
    pt -= phi;
    ax = fma(coef, dx, ax);
    ay = fma(coef, dy, ay);
    az = fma(coef, dz, az);
}

// Compile-time tuning: unroll depth of the cell loop and of the particle
// loop (whose shorter body leaves more room for independent work: 4 measured
// 3 % faster than 2 on the quadrupole kernel) and list entries staged per
// thread per tile (2 doubles the LDS tile; slower for the split kernels).
// The occupancy (waves per SIMD) the register allocator must allow is a
// launch knob: kernel instances for 6 and 8 waves besides the compiler's
// own choice.
#ifndef BHQ_UNROLL
#define BHQ_UNROLL 2
#endif
#ifndef BHQ_UNROLL_PP
#define BHQ_UNROLL_PP 4
#endif
#ifndef BHQ_TILE_DEPTH
#define BHQ_TILE_DEPTH 1
#endif

// Far position for padding entries: zero mass (and zero moments) at a
// finite distance, so that a padded entry adds exactly +0 to every sum.
constexpr float kPadPos = 1.0e15f;

template <typename R, int KIND>
struct Smem {
    static constexpr bool kCellQ = (KIND == kQuad || KIND == kSplitQuad || KIND == kQuadSoft);
};

// Evaluate group g with a block of BS threads, each owning IB i-particles;
// sa, sb, sc are LDS tiles of BS entries (sb, sc only for the quadrupole
// kinds); tab is the FP32 split table in LDS (FP32 split kinds only).
// Part js of nj of each list (cross-block j-split; nj == 1: the whole
// lists): the results go to the part buffer instead of the outputs.
template <typename R, int KIND, bool PERIODIC, int BS, int IB>
__device__ __forceinline__ void process_group(const ForceArgs &A, int64_t g, int js, int nj,
                                              V4<R> *sa, V4<R> *sb, V4<R> *sc,
                                              const TabT<R> *tab)
{
    constexpr bool kSplit = (KIND == kSplitQuad || KIND == kSplitMono);
    constexpr bool kCellQ = Smem<R, KIND>::kCellQ;
    const int t = threadIdx.x;
    const int64_t i0 = A.i_off[g];
    const int64_t ni = A.i_off[g + 1] - i0;
    const double cx = A.gcx[g], cy = A.gcy[g], cz = A.gcz[g];
    const int64_t npg = A.jp_off[g + 1] - A.jp_off[g], ncg = A.jc_off[g + 1] - A.jc_off[g];
    const int64_t pb = npg * js / nj, cb = ncg * js / nj;
    const int64_t np = npg * (js + 1) / nj - pb, nc = ncg * (js + 1) / nj - cb;
    const int64_t p0 = (A.jp_slot > 0 ? g * A.jp_slot : A.jp_off[g]) + pb;
    const int64_t c0 = (A.jc_slot > 0 ? g * A.jc_slot : A.jc_off[g]) + cb;
    const double box = A.box;
    const double ibox = PERIODIC ? 1.0 / box : 0.0;
    const SplitK<R> K = split_k<R>(kSplit ? A.rs : 1.0);
    const R rcut2 = kSplit ? R(A.rcut * A.rcut) : R(0);
    const bool indexed = A.jp_idx != nullptr;
    auto rel64 = [&](double v, double c) -> double {
        return PERIODIC ? wrap(v - c, box, ibox) : v - c;
    };
    auto rel = [&](double v, double c) -> R { return R(rel64(v, c)); };

    for (int64_t ib = 0; ib < ni; ib += (int64_t)BS * IB) {
        // nic i-particles in this pass, P threads per slice owning IB each
        // (thread islot owns islot, islot + P, ...).  S slices; a tile holds
        // T = S * floor(BS / S) entries and slice s takes the contiguous
        // chunk [s*it, (s+1)*it) of it.
        const int nic = (int)(ni - ib < (int64_t)BS * IB ? ni - ib : BS * IB);
        const int P = (nic + IB - 1) / IB;
        const int S = BS / P;
        constexpr int TD = BHQ_TILE_DEPTH;  // list entries staged per thread
        const int T = S * (TD * BS / S);
        const int slice = t / P;
        const int islot = t - slice * P;
        const bool active = slice < S;

        // Cutoff limits per owned i-particle (split kernels): a term with
        // r^2 < lim is kept, one with lim <= r^2 < hi lies in the FP32 band
        // and is decided again in FP64 after the tile (FP32 only; FP64 keeps
        // r^2 < rcut^2 directly).
        R xi[IB], yi[IB], zi[IB], e2[IB], lim[IB], hi[IB];
#pragma unroll
        for (int u = 0; u < IB; ++u) {
            // an i-slot past the end repeats a valid particle; its sums are
            // computed but never written
            const int li = islot + u * P < nic ? islot + u * P : islot;
            xi[u] = yi[u] = zi[u] = R(0);
            e2[u] = R(1);
            if (active) {
                const int64_t i = i0 + ib + li;
                xi[u] = rel(A.xi[i], cx);
                yi[u] = rel(A.yi[i], cy);
                zi[u] = rel(A.zi[i], cz);
                e2[u] = R(A.e2i[i]);
            }
            lim[u] = hi[u] = rcut2;
            if constexpr (kSplit && std::is_same<R, float>::value) {
                const float band = cut_band(xi[u], yi[u], zi[u], float(A.rcut));
                lim[u] = rcut2 - band;
                hi[u] = rcut2 + band;
            }
        }
        // FP64 cutoff decision for i-slot u and entry e of the current tile
        // (list position first + e).
        auto exact = [&](int u, int64_t first, int e, bool cells) -> bool {
            // the empty asm keeps the compiler from computing these
            // addresses ahead of the tile loops (they would stay live there)
            int lu = islot + u * P;
            asm volatile("" : "+v"(lu), "+v"(e));
            const int64_t i = i0 + ib + (lu < nic ? lu : islot);
            const int64_t j = first + e;
            double x, y, z;
            if (cells) {
                if (indexed) {
                    const CellRec *C = A.pool_c + A.jc_idx[j];
                    x = C->x, y = C->y, z = C->z;
                } else {
                    x = A.jcx[j], y = A.jcy[j], z = A.jcz[j];
                }
            } else {
                if (indexed) {
                    const PartRec *Q = A.pool_p + A.jp_idx[j];
                    x = Q->x, y = Q->y, z = Q->z;
                } else {
                    x = A.jpx[j], y = A.jpy[j], z = A.jpz[j];
                }
            }
            return keep_f64(rel64(x, cx) - rel64(A.xi[i], cx), rel64(y, cy) - rel64(A.yi[i], cy),
                            rel64(z, cz) - rel64(A.zi[i], cz), A.rcut);
        };
        // Separations of entry jv from every owned i-particle and the
        // cutoff decisions of the tile loops (split kernels); near collects
        // whether a term fell in the FP32 band.
        auto decide = [&](const V4<R> &jv, Sep<R> (&sp)[IB], bool (&keep)[IB], bool &near) {
#pragma unroll
            for (int u = 0; u < IB; ++u) {
                sp[u] = separation(jv, xi[u], yi[u], zi[u]);
                const bool lo = sp[u].r2 < lim[u];
                keep[u] = sp[u].r2 > R(0) && lo;
                if constexpr (std::is_same<R, float>::value) near |= !lo && sp[u].r2 < hi[u];
            }
        };
        R ax[IB], ay[IB], az[IB], pt[IB];
#pragma unroll
        for (int u = 0; u < IB; ++u) ax[u] = ay[u] = az[u] = pt[u] = R(0);

        // Staging of list entries: the FP64 data of entry j (pool record ix
        // for index lists), then its LDS form relative to the group centre.
        auto load_p = [&](int64_t j, int32_t ix) -> PartRec {
            if (indexed) return A.pool_p[ix];
            return PartRec{A.jpx[j], A.jpy[j], A.jpz[j], A.jpm[j]};
        };
        auto stage_p = [&](const PartRec &q, bool real) -> V4<R> {
            V4<R> v;
            if (real) {
                v.x = rel(q.x, cx);
                v.y = rel(q.y, cy);
                v.z = rel(q.z, cz);
                v.w = R(q.m);
            } else {
                v.x = v.y = v.z = R(kPadPos);
                v.w = R(0);
            }
            return v;
        };
        auto load_c = [&](int64_t j, int32_t ix) -> CellRec {
            if (indexed) {
                const CellRec *C = A.pool_c + ix;
                CellRec c;
                c.x = C->x, c.y = C->y, c.z = C->z, c.m = C->m;
                if (kCellQ) {
                    c.q00 = C->q00, c.q01 = C->q01, c.q02 = C->q02, c.q11 = C->q11;
                    c.q12 = C->q12, c.q22 = C->q22;
                    c.t = (KIND == kSplitQuad || KIND == kQuadSoft) ? C->t : 0.0;
                }
                return c;
            }
            CellRec c;
            c.x = A.jcx[j], c.y = A.jcy[j], c.z = A.jcz[j], c.m = A.jcm[j];
            if (kCellQ) {
                c.q00 = A.q00[j], c.q01 = A.q01[j], c.q02 = A.q02[j], c.q11 = A.q11[j];
                c.q12 = A.q12[j], c.q22 = A.q22[j];
                c.t = (KIND == kSplitQuad || KIND == kQuadSoft) ? A.jct[j] : 0.0;
            }
            return c;
        };
        auto stage_c = [&](const CellRec &c, bool real, int e) {
            V4<R> v, w, u;
            if (real) {
                v.x = rel(c.x, cx);
                v.y = rel(c.y, cy);
                v.z = rel(c.z, cz);
                v.w = R(c.m);
                if (kCellQ) {
                    w.x = R(c.q00);
                    w.y = R(c.q01);
                    w.z = R(c.q02);
                    w.w = R(c.q11);
                    u.x = R(c.q12);
                    u.y = R(c.q22);
                    u.z = R(c.t);
                    u.w = R(0);
                }
            } else {
                v.x = v.y = v.z = R(kPadPos);
                v.w = R(0);
                w.x = w.y = w.z = w.w = R(0);
                u.x = u.y = u.z = u.w = R(0);
            }
            sa[e] = v;
            if (kCellQ) {
                sb[e] = w;
                sc[e] = u;
            }
        };
        // j-particles
        for (int64_t base = 0; base < np; base += T) {
            const int cnt = (int)(np - base < T ? np - base : T);
            const int it = (cnt + S - 1) / S;  // entries per slice
            __syncthreads();
#pragma unroll
            for (int r = 0; r < TD; ++r) {
                const int te = t + r * BS;
                if (te < it * S) {
                    const int64_t j = p0 + base + te;
                    sa[te] = te < cnt ? stage_p(load_p(j, indexed ? A.jp_idx[j] : 0), true)
                                      : stage_p(PartRec{}, false);
                }
            }
            __syncthreads();
            if (active) {
                R bx[IB], by[IB], bz[IB], bp[IB];
#pragma unroll
                for (int u = 0; u < IB; ++u) bx[u] = by[u] = bz[u] = bp[u] = R(0);
                const V4<R> *pa = sa + slice * it;
                bool near = false;
#pragma unroll BHQ_UNROLL_PP
                for (int k = 0; k < it; ++k) {
                    const V4<R> jv = pa[k];
                    if constexpr (kSplit) {
                        Sep<R> sp[IB];
                        bool keep[IB];
                        decide(jv, sp, keep, near);
#pragma unroll
                        for (int u = 0; u < IB; ++u)
                            if (keep[u]) pp_split(jv, sp[u], K, tab, bx[u], by[u], bz[u], bp[u]);
                    } else {
#pragma unroll
                        for (int u = 0; u < IB; ++u)
                            pp_plummer(jv, xi[u], yi[u], zi[u], e2[u], bx[u], by[u], bz[u],
                                       bp[u]);
                    }
                }
                if constexpr (kSplit && std::is_same<R, float>::value) {
                    // Band terms (rare): a lane that flagged one goes over
                    // its entries again, decides each band term in FP64 and
                    // adds the kept ones after the tile's other terms.
                    if (__builtin_expect(near, 0)) {
#pragma unroll 1
                        for (int k = 0; k < it; ++k) {
                            const V4<R> jv = pa[k];
#pragma unroll
                            for (int u = 0; u < IB; ++u) {
                                const Sep<R> sp = separation(jv, xi[u], yi[u], zi[u]);
                                if (sp.r2 >= lim[u] && sp.r2 < hi[u] &&
                                    exact(u, p0 + base, slice * it + k, false))
                                    pp_split(jv, sp, K, tab, bx[u], by[u], bz[u], bp[u]);
                            }
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < IB; ++u) {
                    ax[u] += bx[u];
                    ay[u] += by[u];
                    az[u] += bz[u];
                    pt[u] += bp[u];
                }
            }
        }

        // j-cells
        for (int64_t base = 0; base < nc; base += T) {
            const int cnt = (int)(nc - base < T ? nc - base : T);
            const int it = (cnt + S - 1) / S;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < TD; ++r) {
                const int te = t + r * BS;
                if (te < it * S) {
                    const int64_t j = c0 + base + te;
                    if (te < cnt)
                        stage_c(load_c(j, indexed ? A.jc_idx[j] : 0), true, te);
                    else
                        stage_c(CellRec{}, false, te);
                }
            }
            __syncthreads();
            if (active) {
                R bx[IB], by[IB], bz[IB], bp[IB];
#pragma unroll
                for (int u = 0; u < IB; ++u) bx[u] = by[u] = bz[u] = bp[u] = R(0);
                const int e0 = slice * it;
                bool near = false;
                if constexpr (kSplit) {
                    // Most cell terms of a split kernel lie beyond the
                    // cutoff, and which ones differs from lane to lane.  A
                    // lane first decides a chunk of up to 32 of its
                    // entries, keeping the live ones as bits of a mask per
                    // owned i-particle, and then evaluates only those, in
                    // list order; the wave loops until its busiest lane is
                    // done.  Slices take interleaved entries (slice, slice
                    // + S, ...): consecutive list entries lie close together,
                    // so a contiguous chunk would be live mostly for the
                    // lanes on one side of the group.
                    for (int kc = 0; kc < it; kc += 32) {
                        const int n = it - kc < 32 ? it - kc : 32;
                        uint32_t live[IB];
#pragma unroll
                        for (int u = 0; u < IB; ++u) live[u] = 0u;
#pragma unroll BHQ_UNROLL_PP
                        for (int k = 0; k < n; ++k) {
                            Sep<R> sp[IB];
                            bool keep[IB];
                            decide(sa[slice + (kc + k) * S], sp, keep, near);
#pragma unroll
                            for (int u = 0; u < IB; ++u) live[u] |= keep[u] ? 1u << k : 0u;
                        }
#pragma unroll
                        for (int u = 0; u < IB; ++u)
                            for (uint32_t m = live[u]; m != 0u; m &= m - 1u) {
                                const int e = slice + (kc + __builtin_ctz(m)) * S;
                                const V4<R> ja = sa[e];
                                V4<R> jb, jc;
                                if (kCellQ) {
                                    jb = sb[e];
                                    jc = sc[e];
                                }
                                pc_split<R, KIND == kSplitQuad>(
                                    ja, jb, jc, separation(ja, xi[u], yi[u], zi[u]), K, tab, bx[u],
                                    by[u], bz[u], bp[u]);
                            }
                    }
                } else {
#pragma unroll BHQ_UNROLL
                    for (int k = 0; k < it; ++k) {
                        const int e = e0 + k;
                        const V4<R> ja = sa[e];
                        V4<R> jb, jc;
                        if (kCellQ) {
                            jb = sb[e];
                            jc = sc[e];
                        }
#pragma unroll
                        for (int u = 0; u < IB; ++u) {
                            if (KIND == kQuad || KIND == kQuadSoft)
                                pc_quad<R, KIND == kQuadSoft>(ja, jb, jc, xi[u], yi[u], zi[u],
                                                              e2[u], bx[u], by[u], bz[u], bp[u]);
                            else
                                pp_plummer(ja, xi[u], yi[u], zi[u], e2[u], bx[u], by[u], bz[u],
                                           bp[u]);
                        }
                    }
                }
                if constexpr (kSplit && std::is_same<R, float>::value) {
                    // band terms, as for the particles
                    if (__builtin_expect(near, 0)) {
#pragma unroll 1
                        for (int k = 0; k < it; ++k) {
                            const int e = slice + k * S;
                            const V4<R> ja = sa[e];
                            V4<R> jb, jc;
                            if (kCellQ) {
                                jb = sb[e];
                                jc = sc[e];
                            }
#pragma unroll
                            for (int u = 0; u < IB; ++u) {
                                const Sep<R> sp = separation(ja, xi[u], yi[u], zi[u]);
                                if (sp.r2 >= lim[u] && sp.r2 < hi[u] &&
                                    exact(u, c0 + base, e, true))
                                    pc_split<R, KIND == kSplitQuad>(ja, jb, jc, sp, K, tab,
                                                                    bx[u], by[u], bz[u], bp[u]);
                            }
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < IB; ++u) {
                    ax[u] += bx[u];
                    ay[u] += by[u];
                    az[u] += bz[u];
                    pt[u] += bp[u];
                }
            }
        }

        // combine the slices in a fixed order, one owned i-slot at a time
#pragma unroll
        for (int u = 0; u < IB; ++u) {
            __syncthreads();
            if (active) {
                V4<R> v;
                v.x = ax[u];
                v.y = ay[u];
                v.z = az[u];
                v.w = pt[u];
                sa[t] = v;
            }
            __syncthreads();
            const int li = t + u * P;
            if (t < P && li < nic) {
                R sx = R(0), sy = R(0), sz = R(0), sp = R(0);
                for (int s = 0; s < S; ++s) {
                    const V4<R> v = sa[s * P + t];
                    sx += v.x;
                    sy += v.y;
                    sz += v.z;
                    sp += v.w;
                }
                const int64_t i = i0 + ib + li;
                if (nj > 1) {
                    V4<R> v;
                    v.x = sx;
                    v.y = sy;
                    v.z = sz;
                    v.w = sp;
                    static_cast<V4<R> *>(A.part)[js * A.ni + i] = v;
                } else {
                    const int64_t o = i * A.out_stride;
                    A.ax[o] = (double)sx;
                    A.ay[o] = (double)sy;
                    A.az[o] = (double)sz;
                    if (A.pot) A.pot[i] = -(double)sp;
                }
            }
        }
    }
}

// The split kinds keep the table of their radial functions in LDS (FP32:
// split_table.h; FP64: the exp(-u^2) and erfcx polynomials of
// split_table64.h).
template <typename R, int KIND>
constexpr int split_tab_size()
{
    return KIND != kSplitQuad && KIND != kSplitMono ? 1
           : std::is_same<R, float>::value          ? kSplitFuncs * kSplitEntries
                                                    : kTab64Intervals * kTab64Stride;
}

template <typename R, int KIND, int BS>
__device__ __forceinline__ void load_split_tab(TabT<R> *tab)
{
    if constexpr (split_tab_size<R, KIND>() > 1) {
        if constexpr (std::is_same<R, float>::value) {
            for (int k = threadIdx.x; k < kSplitFuncs * kSplitEntries; k += BS)
                tab[k] = kSplitTabDev.v[k];
        } else {
            for (int k = threadIdx.x; k < kTab64Intervals * kTab64Stride; k += BS)
                tab[k] = kTab64Dev.v[k];
        }
        __syncthreads();
    }
}

// Waves per SIMD the register allocation must allow: WPE > 0 asks for at
// least WPE (registers capped to fit).  Otherwise the FP64 split kinds ask
// for BHQ_F64_SPLIT_WAVES: left alone the compiler takes 188 VGPRs (2
// waves); capped for 3, 4 and 5 waves (registers spilled to scratch) they
// ran the 2^24 lattice in 49.2, 47.5 and 50.8 ms against 56.7, with exp
// from the library.  A minimum of 1 leaves the compiler's choice.
#ifndef BHQ_F64_SPLIT_WAVES
#define BHQ_F64_SPLIT_WAVES 4
#endif
template <typename R, int KIND, int WPE>
constexpr int min_waves()
{
    return WPE > 0 ? WPE
                   : (std::is_same<R, double>::value && (KIND == kSplitQuad || KIND == kSplitMono)
                          ? BHQ_F64_SPLIT_WAVES
                          : 1);
}

template <typename R, int KIND, bool PERIODIC, int BS, int IB, int WPE>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(min_waves<R, KIND, WPE>())))
void force_kernel(const ForceArgs A)
{
    constexpr bool kCellQ = Smem<R, KIND>::kCellQ;
    __shared__ V4<R> sa[BHQ_TILE_DEPTH * BS];
    __shared__ V4<R> sb[kCellQ ? BHQ_TILE_DEPTH * BS : 1];
    __shared__ V4<R> sc[kCellQ ? BHQ_TILE_DEPTH * BS : 1];
    __shared__ __align__(16) TabT<R> st[split_tab_size<R, KIND>()];
    // block b: slot b % nslots, part b / nslots of its group's lists (the
    // slot of a block keeps its XCD, b % 8, when nslots is a multiple of 8)
    const int nj = (int)(gridDim.x / A.nslots);
    const int js = (int)(blockIdx.x / A.nslots);
    const int64_t slot = blockIdx.x - (int64_t)js * A.nslots;
    const int64_t g = A.order ? A.order[slot] : slot;
    if (g < 0) return;  // empty slot (uniform over the block)
    load_split_tab<R, KIND, BS>(st);
    process_group<R, KIND, PERIODIC, BS, IB>(A, g, js, nj, sa, sb, sc, st);
}

// Id of the XCD this wave runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcd_id()
{
    constexpr int kHwRegXccId = 20;
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | kHwRegXccId) & 0xfu);
}

// Persistent variant: a grid sized to the machine pulls slots of A.order
// from the counters in A.queue (zeroed before the launch).  With xcds == 0
// one counter runs over all slots; otherwise counter x runs over the slots
// of XCD x (b % xcds == x) and a block drains its own XCD's counter first,
// then the others' in turn.  Every counter only grows, and a block leaves a
// counter once it has passed that counter's slot count, so every block
// exits.
template <typename R, int KIND, bool PERIODIC, int BS, int IB, int WPE>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(min_waves<R, KIND, WPE>())))
void force_kernel_persistent(const ForceArgs A, int nj)
{
    constexpr bool kCellQ = Smem<R, KIND>::kCellQ;
    __shared__ V4<R> sa[BHQ_TILE_DEPTH * BS];
    __shared__ V4<R> sb[kCellQ ? BHQ_TILE_DEPTH * BS : 1];
    __shared__ V4<R> sc[kCellQ ? BHQ_TILE_DEPTH * BS : 1];
    __shared__ __align__(16) TabT<R> st[split_tab_size<R, KIND>()];
    __shared__ int64_t next;
    load_split_tab<R, KIND, BS>(st);
    const int nq = A.xcds > 0 ? A.xcds : 1;
    const int64_t per_q = A.nslots / nq;  // nslots is a multiple of nq
    const int home = A.xcds > 0 ? xcd_id() % nq : 0;
    // counter q hands out per_q * nj items: item k is local slot k % per_q
    // of queue q (launch slot (k % per_q) * nq + q), list part k / per_q
    for (int r = 0; r < nq; ++r) {
        const int q = (home + r) % nq;
        for (;;) {
            if (threadIdx.x == 0) next = (int64_t)atomicAdd(A.queue + q, 1u);
            __syncthreads();
            const int64_t k = next;
            __syncthreads();
            if (k >= per_q * nj) break;
            const int js = (int)(k / per_q);
            const int64_t slot = (k - js * per_q) * nq + q;
            const int64_t g = A.order ? A.order[slot] : slot;
            if (g >= 0) process_group<R, KIND, PERIODIC, BS, IB>(A, g, js, nj, sa, sb, sc, st);
        }
    }
}

// Sum of the nj parts of every i-particle in the order s = 0, 1, ... (in
// the working precision), written to the outputs.
template <typename R>
__global__ __launch_bounds__(256) void reduce_parts(const ForceArgs A, int nj)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= A.ni) return;
    const V4<R> *part = static_cast<const V4<R> *>(A.part);
    V4<R> s = part[i];
    for (int k = 1; k < nj; ++k) {
        const V4<R> v = part[k * A.ni + i];
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
    }
    const int64_t o = i * A.out_stride;
    A.ax[o] = (double)s.x;
    A.ay[o] = (double)s.y;
    A.az[o] = (double)s.z;
    if (A.pot) A.pot[i] = -(double)s.w;
}

__global__ void reset_queue(unsigned int *q)
{
    if (blockIdx.x == 0 && threadIdx.x < kQueueWords) q[threadIdx.x] = 0u;
}

template <typename R, int KIND, bool P, int BS, int IB, int WPE>
hipError_t launch_one(const ForceArgs &A, const LaunchCfg &cfg, hipStream_t s)
{
    const int nj = cfg.jsplit;
    const int64_t items = A.nslots * nj;
    if (cfg.persistent) {
        hipLaunchKernelGGL(reset_queue, dim3(1), dim3(kQueueWords), 0, s, A.queue);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        int per_cu = cfg.blocks_per_cu;
        if (per_cu <= 0) {
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, force_kernel_persistent<R, KIND, P, BS, IB, WPE>, BS, 0);
            if (e != hipSuccess) return e;
            if (per_cu < 1) per_cu = 1;
        }
        const int64_t want = (int64_t)per_cu * cfg.num_cu;
        const unsigned grid = (unsigned)(want < items ? want : items);
        hipLaunchKernelGGL((force_kernel_persistent<R, KIND, P, BS, IB, WPE>),
                           dim3(grid), dim3(BS), 0, s, A, nj);
    } else {
        hipLaunchKernelGGL((force_kernel<R, KIND, P, BS, IB, WPE>),
                           dim3((unsigned)items), dim3(BS), 0, s, A);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nj == 1 || A.ni == 0) return e;
    hipLaunchKernelGGL(reduce_parts<R>, dim3((unsigned)((A.ni + 255) / 256)), dim3(256), 0, s,
                       A, nj);
    return hipGetLastError();
}

// Block 256 in FP32 has instances for 6 and 8 waves per SIMD; the other
// shapes and FP64 run the compiler's choice whatever cfg.waves_per_eu says.
template <typename R, int KIND, bool P, int IB>
hipError_t launch_wpe(const ForceArgs &A, const LaunchCfg &cfg, hipStream_t s)
{
    if constexpr (std::is_same<R, float>::value) {
        if (cfg.waves_per_eu == 6) return launch_one<R, KIND, P, 256, IB, 6>(A, cfg, s);
        if (cfg.waves_per_eu == 8) return launch_one<R, KIND, P, 256, IB, 8>(A, cfg, s);
    }
    return launch_one<R, KIND, P, 256, IB, 0>(A, cfg, s);
}

template <typename R, int KIND, bool P>
hipError_t launch_bs(const ForceArgs &A, const LaunchCfg &cfg, hipStream_t s)
{
    if (cfg.i_per_thread == 2)
        return cfg.block == 128 ? launch_one<R, KIND, P, 128, 2, 0>(A, cfg, s)
                                : launch_wpe<R, KIND, P, 2>(A, cfg, s);
    return cfg.block == 128 ? launch_one<R, KIND, P, 128, 1, 0>(A, cfg, s)
                            : launch_wpe<R, KIND, P, 1>(A, cfg, s);
}

template <typename R>
hipError_t launch_prec(int kernel, const ForceArgs &A, const LaunchCfg &cfg,
                       hipStream_t s)
{
    // periodic minimum image only for the split kernels in a box
    const bool periodic = A.box > 0.0;
    switch (kernel) {
    case kMono:
        return launch_bs<R, kMono, false>(A, cfg, s);
    case kQuad:
        return launch_bs<R, kQuad, false>(A, cfg, s);
    case kQuadSoft:
        return launch_bs<R, kQuadSoft, false>(A, cfg, s);
    case kSplitQuad:
        return periodic ? launch_bs<R, kSplitQuad, true>(A, cfg, s)
                        : launch_bs<R, kSplitQuad, false>(A, cfg, s);
    case kSplitMono:
        return periodic ? launch_bs<R, kSplitMono, true>(A, cfg, s)
                        : launch_bs<R, kSplitMono, false>(A, cfg, s);
    default:
        return hipErrorInvalidValue;
    }
}

// Number of (i-particle, list entry) pairs of the split kernels' lists
// inside the cutoff, with the FP64 decision of the kernels (FP64 offsets to
// the group centre, 0 < r^2 < rcut^2): one block per group, its threads
// over the i-particles, every list entry read by all of them.  Adds to
// out[0] (particles) and out[1] (cells).
__global__ __launch_bounds__(256) void count_live(const ForceArgs A, unsigned long long *out)
{
    __shared__ unsigned long long red[2][4];
    const int64_t g = blockIdx.x;
    const int64_t i0 = A.i_off[g], ni = A.i_off[g + 1] - i0;
    const double cx = A.gcx[g], cy = A.gcy[g], cz = A.gcz[g];
    const double box = A.box, ibox = box > 0.0 ? 1.0 / box : 0.0;
    auto rel = [&](double v, double c) { return box > 0.0 ? wrap(v - c, box, ibox) : v - c; };
    const int64_t np = A.jp_off[g + 1] - A.jp_off[g], nc = A.jc_off[g + 1] - A.jc_off[g];
    const int64_t p0 = A.jp_slot > 0 ? g * A.jp_slot : A.jp_off[g];
    const int64_t c0 = A.jc_slot > 0 ? g * A.jc_slot : A.jc_off[g];
    const bool indexed = A.jp_idx != nullptr;
    unsigned long long lp = 0, lc = 0;
    for (int64_t k = threadIdx.x; k < ni; k += 256) {
        const int64_t i = i0 + k;
        const double xi = rel(A.xi[i], cx), yi = rel(A.yi[i], cy), zi = rel(A.zi[i], cz);
        for (int64_t e = 0; e < np; ++e) {
            const int64_t j = p0 + e;
            double x, y, z;
            if (indexed) {
                const PartRec &q = A.pool_p[A.jp_idx[j]];
                x = q.x, y = q.y, z = q.z;
            } else {
                x = A.jpx[j], y = A.jpy[j], z = A.jpz[j];
            }
            lp += keep_f64(rel(x, cx) - xi, rel(y, cy) - yi, rel(z, cz) - zi, A.rcut);
        }
        for (int64_t e = 0; e < nc; ++e) {
            const int64_t j = c0 + e;
            double x, y, z;
            if (indexed) {
                const CellRec &q = A.pool_c[A.jc_idx[j]];
                x = q.x, y = q.y, z = q.z;
            } else {
                x = A.jcx[j], y = A.jcy[j], z = A.jcz[j];
            }
            lc += keep_f64(rel(x, cx) - xi, rel(y, cy) - yi, rel(z, cz) - zi, A.rcut);
        }
    }
    // per wave, then per block, then one atomic per block and kind
    for (int m = 32; m >= 1; m >>= 1) {
        lp += __shfl_xor(lp, m, 64);
        lc += __shfl_xor(lc, m, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = lp;
        red[1][threadIdx.x >> 6] = lc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(out, red[0][0] + red[0][1] + red[0][2] + red[0][3]);
        atomicAdd(out + 1, red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    }
}

// The shader clock of one CU over a wall-clock window: one wave reads the
// shader-clock counter (s_memtime) and the constant-rate counter
// (s_memrealtime) at the start, waits until the latter has advanced by
// `ticks`, and reads both again (out[0..3] = clock start, real start,
// clock end, real end).
__global__ __launch_bounds__(64) void clock_window(unsigned long long ticks,
                                                   unsigned long long *out)
{
    const unsigned long long c0 = __builtin_amdgcn_s_memtime();
    const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
    unsigned long long r = r0;
    while (r - r0 < ticks) {
        __builtin_amdgcn_s_sleep(2);
        r = __builtin_amdgcn_s_memrealtime();
    }
    const unsigned long long c1 = __builtin_amdgcn_s_memtime();
    if (threadIdx.x == 0) {
        out[0] = c0;
        out[1] = r0;
        out[2] = c1;
        out[3] = r;
    }
}

// Working memory of bhq_compute_noalloc: queue counters, then j-split
// parts.  In host code this name is a stand-in, not a device address; the
// address comes from hipGetSymbolAddress (scratch_init).
static __device__ __align__(256) unsigned char scratch[kScratchQueueBytes + kScratchPartBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t launch_count_live(const ForceArgs &A, unsigned long long *out, hipStream_t s)
{
    if (A.ng <= 0) return hipSuccess;
    if (A.ng > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(count_live, dim3((unsigned)A.ng), dim3(256), 0, s, A, out);
    return hipGetLastError();
}

hipError_t launch_clock_window(unsigned long long ticks, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(clock_window, dim3(1), dim3(64), 0, s, ticks, out);
    return hipGetLastError();
}

hipError_t scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_ptr[device];
}

hipError_t launch_force(int kernel, int precision, const ForceArgs &A,
                        const LaunchCfg &cfg, hipStream_t stream)
{
    if (A.ng <= 0 || A.nslots <= 0) return hipSuccess;
    if (A.ng > 0x7fffffff || A.nslots > 0x7fffffff) return hipErrorInvalidValue;
    if (A.xcds < 0 || A.xcds > kQueueWords) return hipErrorInvalidValue;
    if (A.xcds > 0 && A.nslots % A.xcds != 0) return hipErrorInvalidValue;
    if (cfg.block != 128 && cfg.block != 256) return hipErrorInvalidValue;
    if (cfg.i_per_thread != 1 && cfg.i_per_thread != 2) return hipErrorInvalidValue;
    if (cfg.persistent && (!A.queue || cfg.num_cu <= 0))
        return hipErrorInvalidValue;
    if (cfg.jsplit < 1 || cfg.jsplit > kMaxJsplit || (cfg.jsplit > 1 && !A.part))
        return hipErrorInvalidValue;
    if (A.nslots * cfg.jsplit > 0x7fffffff) return hipErrorInvalidValue;
    if (A.out_stride != 1 && A.out_stride != 3) return hipErrorInvalidValue;
    return precision == 1 ? launch_prec<double>(kernel, A, cfg, stream)
                          : launch_prec<float>(kernel, A, cfg, stream);
}

}  // namespace bhq
