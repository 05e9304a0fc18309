// Host check of the table layouts that the kernels read with paired loads
// (built and run by test_table_layout.py; no GPU):
//  * level_index: every level's entries are distinct and fill the table, and
//    the powers (1, 2), (3, 4), (5, 6) of one k sit side by side at an even
//    entry (one 16-byte load);
//  * mirror_pair_index: a bijection of the points onto the entries, and for
//    every plan (N, W) each lane's two loads per slot pair plus the lane-0
//    selects (the rule that load_mirror_pairs applies) yield exactly the
//    points of that lane's slots.
#include <cstdio>
#include <vector>

#include "../paper_2107_06147_amd/csrc/qt_internal.h"

using qt::level_index;
using qt::level_table_len;
using qt::mirror_pair_index;

static int failures = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            if (failures++ < 20) {                     \
                std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
                std::printf(__VA_ARGS__);              \
                std::printf("\n");                     \
            }                                          \
        }                                              \
    } while (0)

static void check_level_table(int n)
{
    const int len = level_table_len(n);
    std::vector<int> seen(len, 0);
    for (int L = 4; L <= n; L *= 2)
        for (int r = 1; r <= 7; ++r)
            for (int k = 0; k < L / 2; ++k) {
                const int i = level_index(L, r, k);
                CHECK(i >= 0 && i < len, "n=%d L=%d r=%d k=%d index %d outside [0,%d)", n, L, r, k, i, len);
                if (i < 0 || i >= len) continue;
                ++seen[i];
                if (r % 2 == 1 && r <= 5) {
                    CHECK(i % 2 == 0, "n=%d L=%d r=%d k=%d: pair at odd entry %d", n, L, r, k, i);
                    CHECK(level_index(L, r + 1, k) == i + 1, "n=%d L=%d r=%d k=%d: r+1 not adjacent", n, L, r, k);
                }
            }
    for (int i = 0; i < len; ++i) CHECK(seen[i] == 1, "n=%d entry %d used %d times", n, i, seen[i]);
}

static void check_mirror_pairs(int N, int W)
{
    const int P = N / W, R1 = P / 2, T = 2 * W, Q = R1 / 2;
    std::vector<int> point(N, -1);   // entry element -> point
    for (int m = 0; m < N; ++m) {
        const int i = mirror_pair_index(N, m);
        CHECK(i >= 0 && i < N, "N=%d m=%d element %d", N, m, i);
        if (i < 0 || i >= N) continue;
        CHECK(point[i] < 0, "N=%d element %d taken twice", N, i);
        point[i] = m;
    }
    for (int t = 0; t < W; ++t) {
        const int ja = t, jb = t == 0 ? W : T - t;
        std::vector<int> ax(Q), ay(Q), bx(Q), by(Q), v(2 * R1, -1);
        for (int r = 0; r < Q; ++r) {
            const int ea = 2 * (ja + r * T), eb = 2 * (jb + r * T);
            CHECK(ea + 1 < N && eb + 1 < N, "N=%d W=%d t=%d r=%d: entry beyond the table", N, W, t, r);
            if (ea + 1 >= N || eb + 1 >= N) return;
            ax[r] = point[ea];
            ay[r] = point[ea + 1];
            bx[r] = point[eb];
            by[r] = point[eb + 1];
        }
        for (int r = 0; r < Q; ++r) {
            v[r] = ax[r];
            v[R1 + r] = bx[r];
            v[R1 - 1 - r] = t == 0 ? ay[(r + 1) % Q] : by[r];
            v[2 * R1 - 1 - r] = t == 0 ? by[r] : ay[r];
        }
        for (int r = 0; r < R1; ++r) {
            CHECK(v[r] == ja + r * T, "N=%d W=%d lane %d slot a[%d]: point %d, wanted %d", N, W, t, r, v[r], ja + r * T);
            CHECK(v[R1 + r] == jb + r * T, "N=%d W=%d lane %d slot b[%d]: point %d, wanted %d", N, W, t, r, v[R1 + r], jb + r * T);
        }
    }
}

int main()
{
    for (int n = 4; n <= 8192; n *= 2) check_level_table(n);
    int plans = 0;
    for (int N = 256; N <= 16384; N *= 2)
        for (int P = 4; P <= 32; P *= 2)
            if (N / P >= 64) {
                check_mirror_pairs(N, N / P);
                ++plans;
            }
    std::printf("%s: level tables up to 8192, mirror pairs for %d plans, %d failures\n",
                failures ? "FAIL" : "ok", plans, failures);
    return failures ? 1 : 0;
}
