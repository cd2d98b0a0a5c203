// Delaunay triangulation of the prior's points (Sec. III-C, disparity prior)
// for the device: an initial triangulation built from the points' rows, then
// edge flips until every edge is locally Delaunay (Lawson's flip algorithm:
// from any triangulation of a point set, flipping edges whose opposite
// vertex lies strictly inside the circumcircle ends at a Delaunay
// triangulation).
//
// Every prior point lies on a horizontal row (support points on grid rows,
// moved points along their row, the four image corners on the first and last
// rows), and the corners make the convex hull the frame rectangle.  The
// initial triangulation covers it with
//   * one strip between each two consecutive rows: a ladder of triangles
//     whose rungs join the rows, advancing along the row whose next point is
//     further left; every such triangle has two vertices on one row and one
//     on the other, so its area is positive;
//   * two side pockets: the region between the rows' first points and the
//     frame's left edge, and between their last points and the right edge,
//     each cut at the points that lie on that edge into y-monotone polygons
//     whose other side is one straight edge, triangulated by one pass with a
//     stack (a vertex is cut off when the turn there is strictly convex).
// The functions here are plain sequential code, shared by the device kernels
// and the host-side checks.
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#define LF_HD __host__ __device__ __forceinline__
#else
#define LF_HD inline
#endif

namespace lfem {
namespace dt {

struct Pt {
    int x, y;
};

// Twice the signed area of (a, b, c); > 0 for the triangle order the
// triangulation keeps (counter-clockwise with y pointing up).
LF_HD long long orient(Pt a, Pt b, Pt c) {
    return (long long)(b.x - a.x) * (c.y - a.y) - (long long)(b.y - a.y) * (c.x - a.x);
}

// > 0 when d lies strictly inside the circle through a, b, c (orient > 0).
// Coordinates below 2^15: every term fits 64 bits.
LF_HD int incircle(Pt a, Pt b, Pt c, Pt d) {
    const long long adx = a.x - d.x, ady = a.y - d.y, bdx = b.x - d.x, bdy = b.y - d.y, cdx = c.x - d.x,
                    cdy = c.y - d.y;
    const long long det = (adx * adx + ady * ady) * (bdx * cdy - bdy * cdx) -
                          (bdx * bdx + bdy * bdy) * (adx * cdy - ady * cdx) +
                          (cdx * cdx + cdy * cdy) * (adx * bdy - ady * bdx);
    return det > 0 ? 1 : (det < 0 ? -1 : 0);
}

// Triangles of the strip between row A (na points, indices A[0..na) into P,
// increasing x) and the row B below it (larger y): na + nb - 2 of them.  Of
// the two possible next triangles, the one whose circumcircle does not hold
// the other's new vertex is taken (the merge step of divide-and-conquer
// Delaunay), so the strip is Delaunay on its own and few flips remain.
template <typename Emit>
LF_HD void zip_strip(const Pt *P, const int *A, int na, const int *B, int nb, Emit emit) {
    int i = 0, j = 0;
    while (i < na - 1 || j < nb - 1) {
        const bool adv_a =
            j == nb - 1 || (i < na - 1 && incircle(P[A[i]], P[A[i + 1]], P[B[j]], P[B[j + 1]]) <= 0);
        if (adv_a) {
            emit(A[i], A[i + 1], B[j]);
            ++i;
        } else {
            emit(A[i], B[j + 1], B[j]);
            ++j;
        }
    }
}

// One pass of the stack triangulation over chain vertices V[0..n) (monotone
// in y), cutting off every stack top whose turn is strictly convex for the
// pocket (sign: the sign of orient(u, w, v) at a convex w for this walking
// direction and side).  Leaves the reflex chain that remains on `stack` and
// returns its length.
template <typename Emit>
LF_HD int stack_pass(const Pt *P, const int *V, int n, int sign, int *stack, Emit emit) {
    int top = 0;
    for (int k = 0; k < n; ++k) {
        const int v = V[k];
        while (top >= 2) {
            const int u = stack[top - 2], w = stack[top - 1];
            const long long o = orient(P[u], P[w], P[v]);
            if (sign > 0 ? o > 0 : o < 0) {
                if (o > 0) emit(u, w, v);
                else emit(u, v, w);
                --top;
            } else {
                break;
            }
        }
        stack[top++] = v;
    }
    return top;
}

// Triangles of one side pocket: chain C[0..m) (one point per row, top to
// bottom) between the chain and the vertical frame edge x = edge_x, which
// the chain's first and last points lie on (side < 0: the left edge; side >
// 0: the right edge).  `work` holds 3 m ints.  The pocket is cut at the chain
// points on the edge into sub-pockets, each a y-monotone polygon closed by
// one straight edge.  With orient's sign convention (y up) a left pocket's
// boundary runs counter-clockwise down the chain, a right pocket's
// clockwise, so a chain vertex is convex where the chain turns with
// orient > 0 (left, walking down) or < 0 (right); walking up reverses the
// sign.  Each sub-pocket is triangulated from both ends toward the chain
// point halfway down (so that its triangles fan out from both edge points,
// not one: fewer flips), then the two reflex chains that remain are joined
// and closed by one more pass.  Every cut is an ear: the vertices not yet
// passed lie beyond it in y and the pocket's other side is the straight
// edge.  Emits one triangle per chain point off the edge.
template <typename Emit>
LF_HD void side_pocket(const Pt *P, const int *C, int m, int edge_x, int side, int *work, Emit emit) {
    const int down = side < 0 ? 1 : -1;
    int a = 0;
    while (a < m - 1) {
        int b = a + 1;
        while (b < m - 1 && P[C[b]].x != edge_x) ++b;   // the last chain point is on the edge
        if (b > a + 1) {
            // the chain point nearest halfway between the two edge points
            const long long y2 = (long long)P[C[a]].y + P[C[b]].y;
            int mid = a + 1;
            for (int k = a + 2; k < b; ++k)
                if (2LL * P[C[k]].y <= y2) mid = k;
            int *s1 = work, *s2 = work + m, *chain = work + 2 * m;
            const int n1 = stack_pass(P, C + a, mid - a + 1, down, s1, emit);
            // bottom-up: the chain from C[b] up to C[mid]
            int n2 = 0;
            for (int k = b; k >= mid; --k) chain[n2++] = C[k];
            n2 = stack_pass(P, chain, n2, -down, s2, emit);
            // what remains: s1 (C[a] .. C[mid]) then s2 back down (.. C[b])
            int n = 0;
            for (int k = 0; k < n1; ++k) chain[n++] = s1[k];
            for (int k = n2 - 2; k >= 0; --k) chain[n++] = s2[k];
            (void)stack_pass(P, chain, n, down, s1, emit);
        }
        a = b;
    }
}

}  // namespace dt
}  // namespace lfem
