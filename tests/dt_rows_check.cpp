// Host check of the device triangulation's building blocks (lf_delaunay.h):
// on random point sets laid out as the prior's (points on rows, the four
// frame corners), the row strips and side pockets must tile the frame with
// positively oriented triangles (Euler's count, the frame's area), and
// rounds of independent flips - the device kernels' rules, replayed here one
// round at a time - must end at a Delaunay triangulation (no point strictly
// inside any triangle's circumcircle).  Prints "ok <cases> <max rounds>".
#include "../paper_2003_11076_amd/csrc/lf_delaunay.h"

#include <algorithm>
#include <climits>
#include <cstdio>
#include <map>
#include <random>
#include <vector>

using namespace lfem::dt;
struct Tri {
    int v[3];
};

static std::vector<Tri> initial(const std::vector<Pt> &P, int W) {
    const int n = (int)P.size();
    std::vector<int> rs, idx(n);
    for (int i = 0; i < n; ++i) {
        idx[i] = i;
        if (i == 0 || P[i].y != P[i - 1].y) rs.push_back(i);
    }
    rs.push_back(n);
    const int nr = (int)rs.size() - 1;
    std::vector<Tri> T;
    auto emit = [&](int a, int b, int c) { T.push_back({{a, b, c}}); };
    for (int r = 0; r + 1 < nr; ++r)
        zip_strip(P.data(), idx.data() + rs[r], rs[r + 1] - rs[r], idx.data() + rs[r + 1], rs[r + 2] - rs[r + 1], emit);
    std::vector<int> C(nr), work(3 * nr);
    for (int r = 0; r < nr; ++r) C[r] = rs[r];
    side_pocket(P.data(), C.data(), nr, 0, -1, work.data(), emit);
    for (int r = 0; r < nr; ++r) C[r] = rs[r + 1] - 1;
    side_pocket(P.data(), C.data(), nr, W - 1, 1, work.data(), emit);
    return T;
}

// Rounds of flips: an illegal edge claims the six triangles its flip
// rewrites with its slot number, and flips when it holds all six.
static int flip_rounds(const std::vector<Pt> &P, std::vector<Tri> &T) {
    const int m = 3 * (int)T.size();
    std::map<std::pair<int, int>, int> first;
    std::vector<int> nb(m, -1);
    for (int s = 0; s < m; ++s) {
        const int t = s / 3, e = s % 3;
        const int a = T[t].v[(e + 1) % 3], b = T[t].v[(e + 2) % 3];
        const auto key = std::make_pair(std::min(a, b), std::max(a, b));
        auto it = first.find(key);
        if (it == first.end()) {
            first[key] = s;
        } else {
            nb[s] = it->second;
            nb[it->second] = s;
        }
    }
    auto parts = [&](int te, int other, int (&tri)[6]) {
        const int t = te / 3, e = te % 3, u = other / 3, f = other % 3;
        tri[0] = t;
        tri[1] = u;
        const int o[4] = {nb[3 * t + (e + 1) % 3], nb[3 * t + (e + 2) % 3], nb[3 * u + (f + 1) % 3],
                          nb[3 * u + (f + 2) % 3]};
        for (int k = 0; k < 4; ++k) tri[2 + k] = o[k] < 0 ? -1 : o[k] / 3;
    };
    for (int round = 0;; ++round) {
        if (round > 100000) return -1;
        std::vector<int> claim(T.size(), INT_MAX), marked;
        for (int te = 0; te < m; ++te) {
            const int other = nb[te];
            if (other < te) continue;
            const int t = te / 3, u = other / 3, f = other % 3;
            if (incircle(P[T[t].v[0]], P[T[t].v[1]], P[T[t].v[2]], P[T[u].v[f]]) <= 0) continue;
            marked.push_back(te);
            int tri[6];
            parts(te, other, tri);
            for (int k = 0; k < 6; ++k)
                if (tri[k] >= 0) claim[tri[k]] = std::min(claim[tri[k]], te);
        }
        if (marked.empty()) return round;
        for (int te : marked) {
            const int other = nb[te];
            int tri[6];
            parts(te, other, tri);
            bool win = true;
            for (int k = 0; k < 6; ++k) win = win && (tri[k] < 0 || claim[tri[k]] == te);
            if (!win) continue;
            const int t = te / 3, e = te % 3, u = other / 3, f = other % 3;
            const int a = T[t].v[e], b = T[t].v[(e + 1) % 3], c = T[t].v[(e + 2) % 3], d = T[u].v[f];
            const int n_ca = nb[3 * t + (e + 1) % 3], n_ab = nb[3 * t + (e + 2) % 3];
            const int n_bd = nb[3 * u + (f + 1) % 3], n_dc = nb[3 * u + (f + 2) % 3];
            T[t] = {{a, b, d}};
            T[u] = {{a, d, c}};
            nb[3 * t + 0] = n_bd;
            nb[3 * t + 1] = 3 * u + 2;
            nb[3 * t + 2] = n_ab;
            nb[3 * u + 0] = n_dc;
            nb[3 * u + 1] = n_ca;
            nb[3 * u + 2] = 3 * t + 1;
            if (n_bd >= 0) nb[n_bd] = 3 * t + 0;
            if (n_ab >= 0) nb[n_ab] = 3 * t + 2;
            if (n_dc >= 0) nb[n_dc] = 3 * u + 0;
            if (n_ca >= 0) nb[n_ca] = 3 * u + 1;
        }
    }
}

int main() {
    std::mt19937 rng(2003);
    int max_rounds = 0;
    const int cases = 1500;
    for (int trial = 0; trial < cases; ++trial) {
        const int W = 2 + rng() % 50, H = 2 + rng() % 50, step = 1 + rng() % 6;
        const double dens = (rng() % 100) / 100.0;
        std::vector<Pt> P;
        std::map<std::pair<int, int>, int> seen;
        auto add = [&](int x, int y) {
            if (!seen.count({y, x})) {
                seen[{y, x}] = 1;
                P.push_back({x, y});
            }
        };
        for (int y = step / 2; y < H; y += step)
            for (int x = 0; x < W; ++x)
                if ((rng() % 1000) / 1000.0 < dens * (x % step == step / 2 ? 1.0 : 0.15)) add(x, y);
        add(0, 0);
        add(W - 1, 0);
        add(0, H - 1);
        add(W - 1, H - 1);
        std::sort(P.begin(), P.end(), [](Pt a, Pt b) { return a.y != b.y ? a.y < b.y : a.x < b.x; });
        const int n = (int)P.size();
        int h = 0;
        for (const Pt &p : P) h += p.x == 0 || p.x == W - 1 || p.y == 0 || p.y == H - 1;
        std::vector<Tri> T = initial(P, W);
        for (int pass = 0; pass < 2; ++pass) {
            long long area = 0;
            for (const Tri &t : T) {
                const long long o = orient(P[t.v[0]], P[t.v[1]], P[t.v[2]]);
                if (o <= 0) {
                    printf("case %d (W=%d H=%d): triangle with orientation %lld\n", trial, W, H, o);
                    return 1;
                }
                area += o;
            }
            if ((int)T.size() != 2 * n - h - 2 || area != 2LL * (W - 1) * (H - 1)) {
                printf("case %d (W=%d H=%d): %zu triangles (Euler %d), area %lld of %lld\n", trial, W, H, T.size(),
                       2 * n - h - 2, area, 2LL * (W - 1) * (H - 1));
                return 1;
            }
            if (pass == 0) {
                const int rounds = flip_rounds(P, T);
                if (rounds < 0) {
                    printf("case %d: flips did not settle\n", trial);
                    return 1;
                }
                max_rounds = std::max(max_rounds, rounds);
            }
        }
        for (const Tri &t : T)
            for (int i = 0; i < n; ++i)
                if (incircle(P[t.v[0]], P[t.v[1]], P[t.v[2]], P[i]) > 0) {
                    printf("case %d (W=%d H=%d): point %d inside a circumcircle\n", trial, W, H, i);
                    return 1;
                }
    }
    printf("ok %d %d\n", cases, max_rounds);
    return 0;
}
