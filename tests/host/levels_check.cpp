// Host check of the affine level estimates (test_host_sanitizers.py).
//
// Replays, in float32 on the CPU, the arithmetic the kernels use to turn a
// float value into a level with the margins of affine_levels: the bin form of
// the 2D and z-marching kernels (first pass window with eps, later windows with
// eps_far) and the level form of the tile, batched-volume, 4D and class-count
// kernels, each followed by the settle step where the estimate is flagged.
// Every value at, just below and just above every threshold, and many random
// values, must land on the level min{l : x <= t_l} (L when none).  The host and
// the device both round fma, add and subtract to nearest, so the replay is
// exact.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "ecc_levels.h"

using namespace ecc;

#define CHECK(c, ...)                                                                  \
    do {                                                                               \
        if (!(c)) {                                                                    \
            std::fprintf(stderr, "check failed: %s (line %d): ", #c, __LINE__);        \
            std::fprintf(stderr, __VA_ARGS__);                                         \
            std::fprintf(stderr, "\n");                                                \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

static const float kMagicF = 12582912.0f;  // 1.5 * 2^23: adding it rounds to an integer
static const uint32_t kMagicBitsF = 0x4B400000u;

static uint32_t bits_of(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}
// median of three (the device's fmed3 on non-NaN inputs)
static float med3(float a, float lo, float hi) { return std::fmin(std::fmax(a, lo), hi); }

static int true_level(const std::vector<float> &t, float x) {
    int lo = 0, hi = (int)t.size();
    while (lo < hi) {
        const int m = (lo + hi) / 2;
        if (x <= t[m])
            hi = m;
        else
            lo = m + 1;
    }
    return lo;
}

// the settle step: the level is within one of the estimate g
static int settle(const std::vector<float> &t, float x, int g) {
    const int L = (int)t.size();
    const float a = t[g > 0 ? g - 1 : 0], b = t[g < L ? g : L - 1];
    const int dec = (g > 0 && x <= a) ? 1 : 0;
    const int inc = (g < L && !(x <= b)) ? 1 : 0;
    return g - dec + inc;
}

struct Stats {
    long n = 0, flagged = 0;
};

// bin form for the pass window [lo, lo + W): returns the bin the kernel adds
// the cell to (kBinOff + level - lo inside the window; below kBinOff for levels
// below it, at least kBinOff + W above it or never)
static int bin_form(const std::vector<float> &t, const AffineFit &f, float x, bool neg, int lo, int W, Stats &st) {
    const int L = (int)t.size();
    const float eps = lo == 0 ? f.eps : f.eps_far;
    const float c = pass_constant(f.u0d, lo);
    // superlevel: the kernel keeps the raw value and the negated slope
    const float y = neg ? std::fmaf(-x, -f.inv_step, c) : std::fmaf(x, f.inv_step, c);
    CHECK(bits_of(y) == bits_of(std::fmaf(x, f.inv_step, c)), "negated slope changes the estimate");
    const float m = y + kMagicF;
    const float r = y - (m - kMagicF);
    const int below = 5, never = W + kBinOff + 5;  // the bins of lane 5
    const float mlo = kMagicF + (float)(lo == 0 ? kBinOff : below), mhi = kMagicF + (float)never;
    int k = (int)(bits_of(med3(m, mlo, mhi)) - kMagicBitsF);
    ++st.n;
    if (!(std::fabs(r) <= 0.5f - eps)) {
        ++st.flagged;
        if (k >= kBinOff - 1 && k <= W + kBinOff) {
            const int g0 = k + lo - kBinOff < 0 ? 0 : k + lo - kBinOff;
            const int g = settle(t, x, g0 > L ? L : g0);
            k = g < lo ? below : (g >= lo + W ? never : g - lo + kBinOff);
        }
    }
    (void)L;
    return k;
}

// level form: the level of x
static int level_form(const std::vector<float> &t, const AffineFit &f, float x, Stats &st) {
    const int L = (int)t.size();
    const float u = std::fmaf(x, f.inv_step, f.u0);
    const float fr = std::fmin(u - std::floor(u), 0x1.fffffep-1f);
    const float uc = med3(u, -2.0f, (float)L + 2.0f);
    int g = (int)std::floor(uc) + 1;
    g = g < 0 ? 0 : (g > L ? L : g);
    ++st.n;
    if (!(std::fabs(fr - 0.5f) <= 0.5f - f.eps)) {
        ++st.flagged;
        g = settle(t, x, g);
    }
    return g;
}

static void check_value(const std::vector<float> &t, const AffineFit &f, float x, Stats &sa, Stats &sb,
                        Stats &sf) {
    const int L = (int)t.size();
    const int lt = true_level(t, x);
    // first pass window (all levels when L <= kMaxWindow; here the window of the
    // first pass is min(L, 4096))
    const int W0 = L < 4096 ? L : 4096;
    const int b0 = bin_form(t, f, x, false, 0, W0, sa);
    if (lt < W0)
        CHECK(b0 == lt + kBinOff, "bin form, first pass: x=%a level %d bin %d", (double)x, lt, b0);
    else
        CHECK(b0 >= W0 + kBinOff, "bin form, first pass: x=%a level %d bin %d", (double)x, lt, b0);
    bin_form(t, f, x, true, 0, W0, sa);
    // later windows of several widths, with the far margin
    for (int Wmax : {4096, 1366, 1000}) {
        for (int lo = Wmax; lo < L; lo += Wmax) {
            const int W = L - lo < Wmax ? L - lo : Wmax;
            const int b = bin_form(t, f, x, false, lo, W, sf);
            if (lt < lo)
                CHECK(b < kBinOff, "bin form, lo=%d: x=%a level %d bin %d", lo, (double)x, lt, b);
            else if (lt >= lo + W)
                CHECK(b >= W + kBinOff, "bin form, lo=%d: x=%a level %d bin %d", lo, (double)x, lt, b);
            else
                CHECK(b == lt - lo + kBinOff, "bin form, lo=%d: x=%a level %d bin %d", lo, (double)x, lt, b);
        }
    }
    const int g = level_form(t, f, x, sb);
    CHECK(g == lt, "level form: x=%a level %d got %d", (double)x, lt, g);
}

static std::vector<float> linspace(double a, double b, int n) {
    std::vector<float> t(n);
    for (int i = 0; i < n; ++i) t[i] = (float)(a + (b - a) * i / (n - 1));
    return t;
}

int main() {
    std::mt19937_64 rng(12345);
    struct Case {
        const char *name;
        std::vector<float> t;
    };
    std::vector<Case> cases;
    cases.push_back({"linspace(-4,4,1024)", linspace(-4, 4, 1024)});
    cases.push_back({"linspace(-3,3,200)", linspace(-3, 3, 200)});
    cases.push_back({"linspace(-3,3,300)", linspace(-3, 3, 300)});
    cases.push_back({"linspace(-3,3,400)", linspace(-3, 3, 400)});
    cases.push_back({"linspace(0,1,4096)", linspace(0, 1, 4096)});
    cases.push_back({"linspace(-1,1,5000)", linspace(-1, 1, 5000)});
    cases.push_back({"linspace(-2,2,10000)", linspace(-2, 2, 10000)});
    cases.push_back({"linspace(1000,1001,1024)", linspace(1000, 1001, 1024)});
    cases.push_back({"linspace(-1e-3,1e-3,777)", linspace(-1e-3, 1e-3, 777)});
    cases.push_back({"linspace(-255,0,256)", linspace(-255, 0, 256)});
    cases.push_back({"linspace(1,2,2)", linspace(1, 2, 2)});
    {
        // a grid with small deviations
        std::uniform_real_distribution<double> d(-0.01, 0.01);
        std::vector<float> t(600);
        for (int i = 0; i < 600; ++i) t[i] = (float)(-2.0 + 0.007 * (i + d(rng)));
        cases.push_back({"perturbed grid (600)", t});
    }
    int fitted = 0;
    for (const Case &cs : cases) {
        const std::vector<float> &t = cs.t;
        AffineFit f;
        if (!affine_levels(t.data(), (int)t.size(), &f)) {
            std::printf("%-28s not affine\n", cs.name);
            continue;
        }
        ++fitted;
        CHECK(f.eps > 0.f && f.eps <= f.eps_far && f.eps_far < 0.25f, "margins %g %g", (double)f.eps,
              (double)f.eps_far);
        Stats sa, sb, sf;
        const int L = (int)t.size();
        for (int l = 0; l < L; ++l) {
            float x = t[l];
            check_value(t, f, x, sa, sb, sf);
            float up = x, dn = x;
            for (int k = 0; k < 4; ++k) {
                up = std::nextafterf(up, INFINITY);
                dn = std::nextafterf(dn, -INFINITY);
                check_value(t, f, up, sa, sb, sf);
                check_value(t, f, dn, sa, sb, sf);
            }
        }
        Stats ra, rb, rf;
        const double span = (double)t[L - 1] - t[0];
        std::uniform_real_distribution<double> ux((double)t[0] - 0.01 * span, (double)t[L - 1] + 0.01 * span);
        for (int i = 0; i < 200000; ++i) check_value(t, f, (float)ux(rng), ra, rb, rf);
        for (float x : {-1e30f, 1e30f, -INFINITY, INFINITY, 0.0f, -0.0f}) check_value(t, f, x, ra, rb, rf);
        std::printf("%-28s eps %.3g (far %.3g): flagged at random values %.5f (bin form) %.5f (level form), "
                    "%.5f with the far margin\n",
                    cs.name, (double)f.eps, (double)f.eps_far, (double)ra.flagged / ra.n,
                    (double)rb.flagged / rb.n, rf.n ? (double)rf.flagged / rf.n : 0.0);
    }
    CHECK(fitted >= 10, "%d threshold sets fitted", fitted);
    std::printf("level estimates OK\n");
    return 0;
}
