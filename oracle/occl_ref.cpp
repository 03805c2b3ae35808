/*
 * occl_ref.cpp -- CPU oracle of the fast edge-aware occlusion detector
 * (Sippel, Seiler, Kaup, "Fast Edge-Aware Occlusion Detection in the Context
 * of Multispectral Camera Arrays", ICIP 2024), Sec. 3, Eqs. (1)-(6).
 *
 * TEST INFRASTRUCTURE.  This file is the plain, slow, single-threaded
 * statement of what the detector computes.  It is used only by the tests,
 * by the package's smoke check and by the benchmark's CPU-baseline leg.  It
 * shares no code, header or constant with the GPU library; the product path
 * never links or calls it.
 *
 * Arithmetic: IEEE fp32 on SSE (no excess precision), built with
 * -ffp-contract=off and without fast-math, so every product and sum below is
 * rounded exactly as written.  Each function follows the paper's steps in
 * the paper's order; the readings taken where the paper is silent or garbled
 * are stated next to the step they affect:
 *
 *  R1  alpha is the angle of the centre->peripheral baseline, x to the right,
 *      y down.  A centre pixel at scanline offset g with disparity V lands at
 *      W = g - r*V in that view (Sec. 3, the warp after Eq. (4); the printed
 *      "+" is read with the sign fixed by the camera geometry of Sec. 1 so
 *      that the edges Eq. (2) keeps are the occluding ones).
 *  R2  Eq. (1): forward difference anchored at (x, y); E_x = 0 on the last
 *      column and E_y = 0 on the last row.
 *  R3  Eq. (2): the angle test |A - alpha| < pi/2 is evaluated as the
 *      equivalent sign test E_x*cos(alpha) + E_y*sin(alpha) > 0 (A is the
 *      two-argument arctangent; the difference is wrapped).  E > gamma strict.
 *  R4  Eq. (3)/(4): L is a parameter, G = {-floor(L/2), ..., +floor(L/2)}.
 *  R5  Eq. (4): scanline coordinates are rounded to the nearest pixel
 *      (fp32 multiply, then add, then round half to even); samples outside
 *      the frame are dropped from the scanline.
 *  R6  Sort of W ascending; equal W keep ascending g (stable sort).
 *  R7  Eq. (5): d ranges over +-1 .. +-max(1, ceil(N/2)); a hit needs
 *      |W_k - W_{k+d}| < zeta and V_{k+d} - V_k > beta (the larger disparity
 *      occludes; the printed "+ beta" is read as "- beta").
 *  R8  Eq. (6): the mask starts at 0 and a scanline only ever sets pixels.
 *  R9  Direction vector: octant-exact fp32 cos/sin (see ref_direction).
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

const float kTightEps = 1e-4f;

struct Sample {
    float W;   // warped position along the baseline (R1)
    float V;   // sampled disparity
    int g;     // offset inside the general scanline G
    int ix, iy;
    float px, py;
};

// R9: (cos alpha, sin alpha) in fp32.  alpha is reduced modulo 360 degrees;
// multiples of 90 degrees are exact; otherwise the angle is reduced to its
// octant reference angle psi in (0, 45], cos/sin of psi are computed in
// double, rounded to fp32 and mapped back by the octant's swap and sign
// symmetries.  This makes dir(a + 180) = -dir(a) and dir(90 - a) = swap(dir(a))
// exactly whenever those angles are exact in double.
void ref_direction(double angle_deg, float* c, float* s) {
    double a = std::fmod(angle_deg, 360.0);
    if (a < 0.0) a += 360.0;
    if (a >= 360.0) a = 0.0;
    int q = (int)std::floor(a / 90.0);
    if (q > 3) q = 3;
    double b = a - 90.0 * q;  // in [0, 90)
    float cb, sb;
    const double deg = 3.14159265358979323846 / 180.0;
    if (b == 0.0) {
        cb = 1.0f; sb = 0.0f;
    } else if (b <= 45.0) {
        cb = (float)std::cos(b * deg);
        sb = (float)std::sin(b * deg);
    } else {
        double p = 90.0 - b;
        cb = (float)std::sin(p * deg);
        sb = (float)std::cos(p * deg);
    }
    switch (q) {
        case 0: *c = cb;  *s = sb;  break;
        case 1: *c = -sb; *s = cb;  break;
        case 2: *c = -cb; *s = -sb; break;
        default: *c = sb; *s = -cb; break;
    }
}

// Eq. (1) with R2: forward differences, zero on the last column / row.
inline float edge_x(const float* D, int H, int W, int x, int y) {
    (void)H;
    return (x + 1 < W) ? (D[(size_t)y * W + x + 1] - D[(size_t)y * W + x]) : 0.0f;
}
inline float edge_y(const float* D, int H, int W, int x, int y) {
    return (y + 1 < H) ? (D[(size_t)(y + 1) * W + x] - D[(size_t)y * W + x]) : 0.0f;
}
// magnitude of the edge maps, correctly rounded square root
inline float edge_mag(float ex, float ey) {
    float sx = ex * ex;
    float sy = ey * ey;
    float q = sx + sy;
    return std::sqrt(q);
}
// Eq. (2) direction part via R3
inline float edge_dot(float ex, float ey, float c, float s) {
    float a = ex * c;
    float b = ey * s;
    return a + b;
}
// Eq. (2): both tests strict, as printed
inline bool is_candidate(float E, float dot, float gamma) {
    return (E > gamma) && (dot > 0.0f);
}

// Eq. (4) + the sampling step: the samples of one scanline, in g order.
// Variant (not the paper's): V read by bilinear interpolation of D at the
// scanline's real position (px, py) instead of at its nearest pixel.  The
// four taps around (px, py) are clamped into the frame; with fx = px -
// floor(px), fy = py - floor(py) (exact in fp32):
//     top = (1 - fx) D(x0, y0) + fx D(x0 + 1, y0)
//     bot = (1 - fx) D(x0, y0 + 1) + fx D(x0 + 1, y0 + 1)
//     V   = (1 - fy) top + fy bot
// (each product and sum rounded to fp32 in this order).  Which samples are
// kept, and which pixel a hit marks, stay those of the nearest pixel (R5).
float bilinear_sample(const float* D, int H, int W, float px, float py) {
    const float fx0 = std::floor(px), fy0 = std::floor(py);
    const float fx = px - fx0, fy = py - fy0;
    const int x0 = (int)fx0, y0 = (int)fy0;
    auto at = [&](int x, int y) {
        x = std::min(std::max(x, 0), W - 1);
        y = std::min(std::max(y, 0), H - 1);
        return D[(size_t)y * W + x];
    };
    const float a = at(x0, y0), b = at(x0 + 1, y0), c = at(x0, y0 + 1), d = at(x0 + 1, y0 + 1);
    const float top = (1.0f - fx) * a + fx * b;
    const float bot = (1.0f - fx) * c + fx * d;
    return (1.0f - fy) * top + fy * bot;
}

// The window is g = -h .. hi (hi = h except in the thinning variant).
void build_scanline(const float* D, int H, int W, int cx, int cy, float c, float s,
                    float r, int h, std::vector<Sample>& out, bool bilinear = false, int hi = -1) {
    out.clear();
    if (hi < 0) hi = h;
    for (int g = -h; g <= hi; ++g) {
        float gf = (float)g;
        float tx = c * gf;
        float ty = s * gf;
        float px = (float)cx + tx;
        float py = (float)cy + ty;
        int ix = (int)std::rint(px);
        int iy = (int)std::rint(py);
        if (ix < 0 || ix >= W || iy < 0 || iy >= H) continue;  // R5: dropped
        Sample sm;
        sm.V = bilinear ? bilinear_sample(D, H, W, px, py) : D[(size_t)iy * W + ix];
        float rv = r * sm.V;
        float w = gf - rv;          // R1: W = g - r*V
        sm.W = w + 0.0f;            // -0 -> +0
        sm.g = g;
        sm.ix = ix; sm.iy = iy;
        sm.px = px; sm.py = py;
        out.push_back(sm);
    }
}

// Sort (R6) and Eq. (5) (R7).  Returns the sorted samples and O_k > 0 flags.
void sort_and_test(std::vector<Sample>& smp, float zeta, float beta, int ns,
                   std::vector<unsigned char>& hit) {
    std::stable_sort(smp.begin(), smp.end(),
                     [](const Sample& a, const Sample& b) { return a.W < b.W; });
    const int n = (int)smp.size();
    hit.assign(n, 0);
    for (int k = 0; k < n; ++k) {
        int O = 0;
        for (int d = -ns; d <= ns; ++d) {
            if (d == 0) continue;
            int j = k + d;
            if (j < 0 || j >= n) continue;
            float dw = std::fabs(smp[k].W - smp[j].W);
            float dv = smp[j].V - smp[k].V;
            if (dw < zeta && dv > beta) ++O;
        }
        hit[k] = (O > 0) ? 1 : 0;
    }
}

// Eq. (5) at sorted position k of an ordered scanline: O_k > 0.
bool hit_at(const std::vector<Sample>& smp, int k, float zeta, float beta, int ns) {
    const int n = (int)smp.size();
    for (int d = -ns; d <= ns; ++d) {
        const int j = k + d;
        if (d == 0 || j < 0 || j >= n) continue;
        if (std::fabs(smp[k].W - smp[j].W) < zeta && smp[j].V - smp[k].V > beta) return true;
    }
    return false;
}

// Pixel of scanline offset g of candidate (cx, cy) (Eq. (4), R5); false
// when it falls outside the frame.
bool scanline_pixel(int cx, int cy, float c, float s, int g, int H, int W, int* ix, int* iy) {
    float gf = (float)g;
    float tx = c * gf;
    float ty = s * gf;
    float px = (float)cx + tx;
    float py = (float)cy + ty;
    *ix = (int)std::rint(px);
    *iy = (int)std::rint(py);
    return *ix >= 0 && *ix < W && *iy >= 0 && *iy < H;
}

inline int neighbours_per_side(int N) {
    int ns = (N + 1) / 2;  // ceil(N/2)
    return ns < 1 ? 1 : ns;
}

// The tight map (parity exemption): the pixels whose mask value rests on a
// decision taken within kTightEps of its threshold.  A margin that is
// exactly 0 is not tight: it comes from exact operands (a zero factor,
// integer offsets, equal disparities), every implementation that rounds
// each operation as written decides it the same way, and the paper's
// strict tests and the stable sort's tie rule decide it.
//   (i)   Eq. (2): 0 < |dot| < eps for a strong edge, or dot == 0 as the sum
//         of two non-zero products that cancel (a rounding artefact).  The
//         magnitude test E > gamma is no margin: E and the comparison are
//         fixed by the definition (correctly rounded square root).
//   (ii)  Eq. (4): a scanline coordinate within eps of a half pixel (the
//         exact half included: its tie rule is a reading).
//   (iii) the sort: 0 < |W_a - W_b| < eps for sorted neighbours.
//   (iv)  Eq. (5): 0 < |zeta - |dW|| < eps or 0 < |dV - beta| < eps in a
//         comparison that could decide a hit.
inline bool in_margin(float m) { return m != 0.0f && std::fabs(m) < kTightEps; }

inline bool dot_margin_tight(float ex, float ey, float c, float s) {
    float a = ex * c;
    float b = ey * s;
    float dot = a + b;
    if (dot == 0.0f) return a != 0.0f && b != 0.0f;
    return std::fabs(dot) < kTightEps;
}

// (iv) for sorted sample k: a comparison within eps of zeta or beta could
// flip, and no comparison outside the margins already makes it a hit.
bool decision_fragile(const std::vector<Sample>& smp, int k, float zeta, float beta, int ns) {
    const int n = (int)smp.size();
    bool near = false, robust_hit = false;
    for (int d = -ns; d <= ns; ++d) {
        const int j = k + d;
        if (d == 0 || j < 0 || j >= n) continue;
        const float dw = std::fabs(smp[k].W - smp[j].W);
        const float dv = smp[j].V - smp[k].V;
        const bool m = (in_margin(zeta - dw) && dv > beta - kTightEps) ||
                       (in_margin(dv - beta) && dw < zeta + kTightEps);
        if (m) near = true;
        else if (dw < zeta && dv > beta) robust_hit = true;
    }
    return near && !robust_hit;
}

inline bool near_half(float p) {
    float f = p - std::floor(p);
    return std::fabs(f - 0.5f) < kTightEps;
}

}  // namespace

extern "C" {

/* Direction vector of a baseline angle (R9). */
int occl_ref_direction(double angle_deg, float* c, float* s) {
    if (!c || !s || !std::isfinite(angle_deg)) return -1;
    ref_direction(angle_deg, c, s);
    return 0;
}

/* Eq. (1) and the magnitude / angle maps.  Any output may be NULL.
 * A = atan2f(E_y, E_x) (the two-argument reading of tan^-1(E_y/E_x)). */
int occl_ref_edges(const float* D, int H, int W, float* ex, float* ey, float* E, float* A) {
    if (!D || H < 1 || W < 1) return -1;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            float gx = edge_x(D, H, W, x, y);
            float gy = edge_y(D, H, W, x, y);
            if (ex) ex[i] = gx;
            if (ey) ey[i] = gy;
            if (E) E[i] = edge_mag(gx, gy);
            if (A) A[i] = std::atan2(gy, gx);
        }
    return 0;
}

/* Eq. (2): candidate map for one direction (1 = candidate). */
int occl_ref_candidates(const float* D, int H, int W, double angle_deg, float gamma,
                        unsigned char* C, long long* count) {
    if (!D || !C || H < 1 || W < 1) return -1;
    float c, s;
    ref_direction(angle_deg, &c, &s);
    long long n = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            float gx = edge_x(D, H, W, x, y);
            float gy = edge_y(D, H, W, x, y);
            float E = edge_mag(gx, gy);
            bool cand = is_candidate(E, edge_dot(gx, gy, c, s), gamma);
            C[(size_t)y * W + x] = cand ? 1 : 0;
            n += cand ? 1 : 0;
        }
    if (count) *count = n;
    return 0;
}

/* One scanline given directly as its depth-line values (for unit tests of
 * the warp/sort/occlusion steps).  Sample i has offset g = g0 + i and value
 * V[i]; valid[i] == 0 drops it (NULL: all valid).  hit[i] = 1 iff O_i > 0. */
int occl_ref_line(int n, const float* V, const unsigned char* valid, int g0, float r,
                  float zeta, float beta, int neighbours, unsigned char* hit) {
    if (n < 0 || (n > 0 && (!V || !hit)) || neighbours < 1) return -1;
    std::vector<Sample> smp;
    for (int i = 0; i < n; ++i) {
        hit[i] = 0;
        if (valid && !valid[i]) continue;
        Sample sm;
        int g = g0 + i;
        float gf = (float)g;
        sm.V = V[i];
        float rv = r * sm.V;
        float w = gf - rv;
        sm.W = w + 0.0f;
        sm.g = g; sm.ix = i; sm.iy = 0; sm.px = 0; sm.py = 0;
        smp.push_back(sm);
    }
    std::vector<unsigned char> h;
    sort_and_test(smp, zeta, beta, neighbours_per_side(neighbours), h);
    for (size_t k = 0; k < smp.size(); ++k)
        if (h[k]) hit[smp[k].ix] = 1;
    return 0;
}

/* The pixels that the scanline of a candidate at (cx, cy) samples, in g
 * order (Eq. (4) with R4/R5); out-of-frame samples are dropped.  xy receives
 * 2 ints per sample and g the offsets; returns the number of samples or -1. */
int occl_ref_scanline_pixels(int cx, int cy, double angle_deg, int L, int H, int W,
                             int* xy, int* g, int cap) {
    if (L < 1 || H < 1 || W < 1 || !xy || !g) return -1;
    float c, s;
    ref_direction(angle_deg, &c, &s);
    std::vector<float> D((size_t)H * W, 0.0f);
    std::vector<Sample> smp;
    build_scanline(D.data(), H, W, cx, cy, c, s, 1.0f, L / 2, smp);
    int n = (int)smp.size();
    if (n > cap) return -1;
    for (int k = 0; k < n; ++k) {
        xy[2 * k] = smp[k].ix;
        xy[2 * k + 1] = smp[k].iy;
        g[k] = smp[k].g;
    }
    return n;
}

/* Scan length rules: mode 0: ceil(max(D) * r) + 2 (product in fp32);
 * mode 1: Eq. (3) with the ratio, ceil(2 * r * (max(D) - min(D))). */
int occl_ref_scan_len(const float* D, int H, int W, int n_views, const float* ratios,
                      int mode, int* L) {
    if (!D || !ratios || !L || H < 1 || W < 1 || n_views < 1) return -1;
    float mx = D[0], mn = D[0];
    for (size_t i = 0; i < (size_t)H * W; ++i) {
        mx = std::max(mx, D[i]);
        mn = std::min(mn, D[i]);
    }
    for (int v = 0; v < n_views; ++v) {
        float r = ratios[v];
        long long l;
        if (mode == 0) {
            float p = mx * r;
            l = (long long)std::ceil(p) + 2;
        } else {
            float span = mx - mn;
            float t = span * r;
            float p = t * 2.0f;
            l = (long long)std::ceil(p);
        }
        if (l < 1) l = 1;
        if (l > (1 << 30)) l = 1 << 30;
        L[v] = (int)l;
    }
    return 0;
}

/* The whole detector for n_views peripheral views (Eqs. (1)-(6)).
 *   D        host fp32 [H][W] row-major
 *   angles   host double [n_views], degrees (R1, R9)
 *   ratios   host float  [n_views], baseline ratio r > 0
 *   scan_len host int    [n_views], L >= 1
 *   M        host uint8  [n_views][H][W], written with {0, 1}
 *   tight    optional host uint8 [n_views][H][W]: 1 where the value could
 *            flip under a perturbation below 1e-4 px of any threshold margin
 *   n_cand   optional host int64 [n_views]: candidates per view
 * Returns 0, or -1 on an invalid argument. */
int occl_ref_detect_ex(const float* D, int H, int W, int n_views, const double* angles,
                       const float* ratios, const int* scan_len, float gamma, float beta,
                       float zeta, int neighbours, unsigned char* M, unsigned char* tight,
                       long long* n_cand, int flags);

int occl_ref_detect(const float* D, int H, int W, int n_views, const double* angles,
                    const float* ratios, const int* scan_len, float gamma, float beta,
                    float zeta, int neighbours, unsigned char* M, unsigned char* tight,
                    long long* n_cand) {
    return occl_ref_detect_ex(D, H, W, n_views, angles, ratios, scan_len, gamma, beta, zeta,
                              neighbours, M, tight, n_cand, 0);
}

/* occl_ref_detect with variant flags: bit 0 = bilinear V sampling (see
 * bilinear_sample; the tight map then covers the nearest-pixel decisions
 * only); bit 1 = candidate thinning (below; needs tight == NULL).
 *
 * Candidate thinning (variant, not the paper's method: its summary, Sec. 6, names
 * a thinner candidate list as future work).  Collinear candidates share most of their
 * scanline, so their scanlines are merged:
 *   - a candidate whose scanline pixel at g = -1 is itself a candidate of the
 *     same view (Eq. (2)) is a follower and is not scanned;
 *   - every other candidate scans g = -h .. h + m instead of -h .. h, where m
 *     is the number of consecutive candidates of the view at g = 1, 2, ...
 *     (m <= h; a pixel outside the frame ends the run).
 * Everything else (sampling, warp, sort, Eq. (5), Eq. (6)) is unchanged.  On
 * axis directions the merged window is exactly the union of the followers'
 * windows; in other directions the followers' rounded pixels can differ
 * from the head's, so the result is an approximation of the method's mask. */
int occl_ref_detect_ex(const float* D, int H, int W, int n_views, const double* angles,
                       const float* ratios, const int* scan_len, float gamma, float beta,
                       float zeta, int neighbours, unsigned char* M, unsigned char* tight,
                       long long* n_cand, int flags) {
    const bool bilinear = (flags & 1) != 0;
    const bool thin = (flags & 2) != 0;
    if (!D || !angles || !ratios || !scan_len || !M || H < 1 || W < 1 || n_views < 1 ||
        neighbours < 1 || (thin && tight))
        return -1;
    for (int v = 0; v < n_views; ++v)
        if (scan_len[v] < 1 || !(ratios[v] > 0.0f) || !std::isfinite(angles[v])) return -1;
    const size_t HW = (size_t)H * W;
    const int ns = neighbours_per_side(neighbours);
    std::memset(M, 0, HW * n_views);
    if (tight) std::memset(tight, 0, HW * n_views);

    // Eq. (1): edge maps (view independent)
    std::vector<float> ex(HW), ey(HW), E(HW);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t i = (size_t)y * W + x;
            ex[i] = edge_x(D, H, W, x, y);
            ey[i] = edge_y(D, H, W, x, y);
            E[i] = edge_mag(ex[i], ey[i]);
        }

    std::vector<Sample> smp;
    std::vector<unsigned char> hit;
    std::vector<unsigned char> candv(thin ? HW : 0);
    std::vector<unsigned char> fragile_px, robust_px;
    for (int v = 0; v < n_views; ++v) {
        float c, s;
        ref_direction(angles[v], &c, &s);
        const float r = ratios[v];
        const int h = scan_len[v] / 2;
        unsigned char* Mv = M + HW * v;
        unsigned char* Tv = tight ? tight + HW * v : nullptr;
        // tight bookkeeping: Fv = some sample of the pixel could flip its hit,
        // Rv = some hit of the pixel is robust
        if (Tv) {
            fragile_px.assign(HW, 0);
            robust_px.assign(HW, 0);
        }
        unsigned char* Fv = Tv ? fragile_px.data() : nullptr;
        unsigned char* Rv = Tv ? robust_px.data() : nullptr;
        long long nc = 0;
        if (thin)  // Eq. (2) over the whole frame, for the follower / run tests
            for (size_t i = 0; i < HW; ++i)
                candv[i] = is_candidate(E[i], edge_dot(ex[i], ey[i], c, s), gamma) ? 1 : 0;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                size_t i = (size_t)y * W + x;
                float dot = edge_dot(ex[i], ey[i], c, s);
                bool cand = is_candidate(E[i], dot, gamma);  // Eq. (2)
                // tight (i): a strong edge whose direction test rests on a dot
                // product within eps of 0 (the magnitude test is not a margin)
                const bool cand_tight = Tv && E[i] > gamma && dot_margin_tight(ex[i], ey[i], c, s);
                if (!cand && !cand_tight) continue;
                int hi = h;
                if (thin) {
                    int px, py;
                    if (scanline_pixel(x, y, c, s, -1, H, W, &px, &py) && candv[(size_t)py * W + px]) {
                        ++nc;  // a follower: counted as a candidate, not scanned
                        continue;
                    }
                    int m = 0;
                    while (m < h && scanline_pixel(x, y, c, s, m + 1, H, W, &px, &py) &&
                           candv[(size_t)py * W + px])
                        ++m;
                    hi = h + m;
                }
                build_scanline(D, H, W, x, y, c, s, r, h, smp, bilinear, hi);  // Eq. (4) + V
                if (cand) ++nc;
                bool round_tight = false;
                if (Tv)
                    for (const Sample& sm : smp) round_tight |= near_half(sm.px) || near_half(sm.py);
                if (round_tight && cand) {  // (ii): the alternative pixels could be sampled
                    for (const Sample& sm : smp) {
                        int ax = sm.ix, ay = sm.iy;
                        if (near_half(sm.px)) ax = (sm.px >= (float)sm.ix) ? sm.ix + 1 : sm.ix - 1;
                        if (near_half(sm.py)) ay = (sm.py >= (float)sm.iy) ? sm.iy + 1 : sm.iy - 1;
                        if ((ax != sm.ix || ay != sm.iy) && ax >= 0 && ax < W && ay >= 0 && ay < H)
                            Fv[(size_t)ay * W + ax] = 1;
                    }
                }
                sort_and_test(smp, zeta, beta, ns, hit);  // sort + Eq. (5)
                const int n = (int)smp.size();
                if (cand)
                    for (int k = 0; k < n; ++k)            // Eq. (6) (R8)
                        if (hit[k]) Mv[(size_t)smp[k].iy * W + smp[k].ix] = 1;
                if (!Tv) continue;
                // which samples' hit status could flip (see the tight map rules)
                std::vector<unsigned char> frag(n, 0);
                if (round_tight && cand) {
                    frag.assign(n, 1);       // any sample's V, hence any test, could change
                } else if (cand_tight) {
                    for (int k = 0; k < n; ++k) frag[k] = hit[k];  // hits that could (dis)appear
                } else {
                    for (int k = 0; k < n; ++k) frag[k] = decision_fragile(smp, k, zeta, beta, ns) ? 1 : 0;
                    for (int k = 0; k + 1 < n; ++k) {  // (iii) near-ties: test the swapped order
                        if (!in_margin(smp[k + 1].W - smp[k].W)) continue;
                        std::swap(smp[k], smp[k + 1]);
                        for (int j = std::max(0, k - ns); j <= std::min(n - 1, k + 1 + ns); ++j) {
                            const int orig = (j == k) ? k + 1 : (j == k + 1) ? k : j;
                            if (hit_at(smp, j, zeta, beta, ns) != (hit[orig] != 0)) frag[orig] = 1;
                        }
                        std::swap(smp[k], smp[k + 1]);
                    }
                }
                for (int k = 0; k < n; ++k) {
                    const size_t p = (size_t)smp[k].iy * W + smp[k].ix;
                    if (frag[k]) Fv[p] = 1;
                    else if (hit[k] && cand) Rv[p] = 1;  // a hit no single margin can remove
                }
            }
        if (Tv)  // tight: some decision could flip the pixel and no robust hit holds it at 1
            for (size_t i = 0; i < HW; ++i) Tv[i] = (Fv[i] && !Rv[i]) ? 1 : 0;
        if (n_cand) n_cand[v] = nc;
    }
    return 0;
}

/* The same detector restricted to a window [x0, x1) x [y0, y1) of the mask:
 * every candidate whose scanline can reach the window (it lies within
 * floor(L/2) + 1 pixels of it) is processed exactly as in occl_ref_detect and
 * only hits inside the window are written to Mw [n_views][y1-y0][x1-x0].
 * Lets large frames be checked on sampled windows. */
int occl_ref_detect_window(const float* D, int H, int W, int n_views, const double* angles,
                           const float* ratios, const int* scan_len, float gamma, float beta,
                           float zeta, int neighbours, int x0, int y0, int x1, int y1,
                           unsigned char* Mw) {
    if (!D || !angles || !ratios || !scan_len || !Mw || H < 1 || W < 1 || n_views < 1 ||
        neighbours < 1 || x0 < 0 || y0 < 0 || x1 > W || y1 > H || x0 >= x1 || y0 >= y1)
        return -1;
    const int ww = x1 - x0, wh = y1 - y0;
    const int ns = neighbours_per_side(neighbours);
    std::memset(Mw, 0, (size_t)ww * wh * n_views);
    std::vector<Sample> smp;
    std::vector<unsigned char> hit;
    for (int v = 0; v < n_views; ++v) {
        if (scan_len[v] < 1 || !(ratios[v] > 0.0f)) return -1;
        float c, s;
        ref_direction(angles[v], &c, &s);
        const float r = ratios[v];
        const int h = scan_len[v] / 2;
        unsigned char* Mv = Mw + (size_t)ww * wh * v;
        const int ya = std::max(0, y0 - h - 1), yb = std::min(H, y1 + h + 1);
        const int xa = std::max(0, x0 - h - 1), xb = std::min(W, x1 + h + 1);
        for (int y = ya; y < yb; ++y)
            for (int x = xa; x < xb; ++x) {
                float ex = edge_x(D, H, W, x, y), ey = edge_y(D, H, W, x, y);
                if (!is_candidate(edge_mag(ex, ey), edge_dot(ex, ey, c, s), gamma)) continue;
                build_scanline(D, H, W, x, y, c, s, r, h, smp);
                sort_and_test(smp, zeta, beta, ns, hit);
                for (size_t k = 0; k < smp.size(); ++k) {
                    const Sample& sm = smp[k];
                    if (hit[k] && sm.ix >= x0 && sm.ix < x1 && sm.iy >= y0 && sm.iy < y1)
                        Mv[(size_t)(sm.iy - y0) * ww + (sm.ix - x0)] = 1;
                }
            }
    }
    return 0;
}

/* Occlusion-mask quality counts (Eq. (7) inputs): pred vs ref over n bytes.
 * out[0] = TP, out[1] = FP, out[2] = FN, out[3] = TN. */
int occl_ref_confusion(const unsigned char* pred, const unsigned char* ref, long long n,
                       long long* out) {
    if (!pred || !ref || !out || n < 0) return -1;
    long long tp = 0, fp = 0, fn = 0, tn = 0;
    for (long long i = 0; i < n; ++i) {
        bool p = pred[i] != 0, t = ref[i] != 0;
        if (p && t) ++tp;
        else if (p && !t) ++fp;
        else if (!p && t) ++fn;
        else ++tn;
    }
    out[0] = tp; out[1] = fp; out[2] = fn; out[3] = tn;
    return 0;
}

/* Ground truth by forward warping (z-buffer): the reference the quality
 * counts of Eq. (7) are taken against.  Under R1 a centre pixel p = (x, y)
 * with disparity D(p) lands at p - r*D(p)*u in the peripheral view of
 * direction u = (c, s); the target pixel is the nearest one:
 *     t = r*D(p) (fp32),  tx = rint(x - t*c),  ty = rint(y - t*s)
 * (fp32, round half to even).  p is occluded in that view iff some pixel q
 * (p itself included) lands on the same target pixel with D(q) - D(p) > beta
 * (fp32 subtraction).  The target may lie outside the peripheral frame: two
 * centre pixels landing on the same outside position still occlude each other.
 * M: [n_views][H][W] bytes 0 / 1. */
int occl_ref_zbuffer(const float* D, int H, int W, int n_views, const double* angles,
                     const float* ratios, float beta, unsigned char* M) {
    if (!D || !M || H < 1 || W < 1 || n_views < 1 || !angles || !ratios) return -1;
    const size_t HW = (size_t)H * W;
    for (int v = 0; v < n_views; ++v) {
        float c, s;
        if (occl_ref_direction(angles[v], &c, &s) != 0) return -1;
        const float r = ratios[v];
        std::vector<long long> key(HW);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const float t = r * D[(size_t)y * W + x];
                const long long tx = (long long)std::nearbyint((float)x - t * c);
                const long long ty = (long long)std::nearbyint((float)y - t * s);
                key[(size_t)y * W + x] = (ty << 32) ^ (tx & 0xffffffffLL);
            }
        // largest disparity landing on each target: pixel indices sorted by
        // target key, then the maximum of each run of equal keys
        std::vector<size_t> order(HW);
        for (size_t i = 0; i < HW; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return key[a] < key[b]; });
        std::vector<float> best(HW);
        for (size_t i = 0; i < HW;) {
            size_t j = i;
            float m = D[order[i]];
            while (j < HW && key[order[j]] == key[order[i]]) {
                m = std::max(m, D[order[j]]);
                ++j;
            }
            for (size_t k = i; k < j; ++k) best[order[k]] = m;
            i = j;
        }
        for (size_t i = 0; i < HW; ++i) M[(size_t)v * HW + i] = (best[i] - D[i] > beta) ? 1 : 0;
    }
    return 0;
}

/* The V of one scanline sample at real position (px, py): nearest pixel
 * (bilinear = 0; the position must round into the frame) or the bilinear
 * variant (bilinear = 1). */
int occl_ref_sample(const float* D, int H, int W, float px, float py, int bilinear, float* V) {
    if (!D || !V || H < 1 || W < 1) return -1;
    if (bilinear) {
        *V = bilinear_sample(D, H, W, px, py);
        return 0;
    }
    const int ix = (int)std::rint(px), iy = (int)std::rint(py);
    if (ix < 0 || ix >= W || iy < 0 || iy >= H) return -1;
    *V = D[(size_t)iy * W + ix];
    return 0;
}

/* Pixel-wise median fusion of K per-view disparity maps into the centre
 * map D (the step before the method, Sec. 4's multispectral pipeline):
 * D[i] = median of the non-NaN values maps[k][i], k = 0..K-1; for an even
 * count the mean of the two middle values, (a + b) * 0.5 in fp32; NaN if
 * every value is NaN.  maps: [K][H*W]. */
int occl_ref_median_fuse(const float* maps, int K, long long n, float* D) {
    if (!maps || !D || K < 1 || K > 64 || n < 0) return -1;
    std::vector<float> v;
    for (long long i = 0; i < n; ++i) {
        v.clear();
        for (int k = 0; k < K; ++k) {
            const float x = maps[(size_t)k * n + i];
            if (!std::isnan(x)) v.push_back(x);
        }
        if (v.empty()) {
            D[i] = std::nanf("");
            continue;
        }
        std::sort(v.begin(), v.end());
        const size_t m = v.size();
        D[i] = (m % 2) ? v[m / 2] : (v[m / 2 - 1] + v[m / 2]) * 0.5f;
    }
    return 0;
}

}  // extern "C"
