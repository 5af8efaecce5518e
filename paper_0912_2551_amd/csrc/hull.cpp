// hull.cpp -- 3-D convex hull of the surrogate's training points (host).
//
// Incremental construction: start from a non-degenerate tetrahedron, then add
// points one by one; the faces a new point sees are removed and the hole is
// closed with faces from the point to the horizon edges.  The result is a
// list of outward half-spaces n.x <= d; a query point is inside the training
// hull when it satisfies all of them.
#include <algorithm>
#include <cmath>
#include <map>
#include <utility>
#include <vector>

#include "smc_internal.h"

namespace smc {

namespace {

struct V3 {
    double x, y, z;
};
V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
double norm(V3 a) { return std::sqrt(dot(a, a)); }

struct Face {
    int a, b, c;
    V3 n;
    double d;
    bool alive;
};

Face make_face(const std::vector<V3> &p, int a, int b, int c, V3 inside)
{
    Face f{a, b, c, {0, 0, 0}, 0.0, true};
    V3 n = cross(sub(p[b], p[a]), sub(p[c], p[a]));
    double len = norm(n);
    n = {n.x / len, n.y / len, n.z / len};
    double d = dot(n, p[a]);
    if (dot(n, inside) > d) {   // orient outward
        std::swap(f.b, f.c);
        n = {-n.x, -n.y, -n.z};
        d = -d;
    }
    f.n = n;
    f.d = d;
    return f;
}

}  // namespace

// Returns planes (nx, ny, nz, d) with n.x <= d inside; empty if the points
// are degenerate (fewer than 4 affinely independent points).
std::vector<double> convex_hull_planes(const float *pts, size_t n)
{
    std::vector<V3> p(n);
    for (size_t i = 0; i < n; ++i) p[i] = {pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]};
    std::vector<double> out;
    if (n < 4) return out;
    double scale = 0.0;
    for (auto &q : p) scale = std::max({scale, std::fabs(q.x), std::fabs(q.y), std::fabs(q.z)});
    const double eps = 1e-10 * std::max(scale, 1.0);
    // initial tetrahedron: extreme point, farthest point, farthest from the
    // line, farthest from the plane
    int i0 = 0;
    for (size_t i = 1; i < n; ++i)
        if (p[i].x < p[i0].x) i0 = (int)i;
    int i1 = -1;
    double best = -1.0;
    for (size_t i = 0; i < n; ++i) {
        const double dd = norm(sub(p[i], p[i0]));
        if (dd > best) best = dd, i1 = (int)i;
    }
    int i2 = -1;
    best = -1.0;
    for (size_t i = 0; i < n; ++i) {
        const double dd = norm(cross(sub(p[i1], p[i0]), sub(p[i], p[i0])));
        if (dd > best) best = dd, i2 = (int)i;
    }
    if (best <= eps) return out;
    int i3 = -1;
    best = -1.0;
    const V3 nrm = cross(sub(p[i1], p[i0]), sub(p[i2], p[i0]));
    for (size_t i = 0; i < n; ++i) {
        const double dd = std::fabs(dot(nrm, sub(p[i], p[i0])));
        if (dd > best) best = dd, i3 = (int)i;
    }
    if (best <= eps * norm(nrm)) return out;
    const V3 c = {(p[i0].x + p[i1].x + p[i2].x + p[i3].x) / 4, (p[i0].y + p[i1].y + p[i2].y + p[i3].y) / 4,
                  (p[i0].z + p[i1].z + p[i2].z + p[i3].z) / 4};
    std::vector<Face> F;
    F.push_back(make_face(p, i0, i1, i2, c));
    F.push_back(make_face(p, i0, i1, i3, c));
    F.push_back(make_face(p, i0, i2, i3, c));
    F.push_back(make_face(p, i1, i2, i3, c));
    for (size_t q = 0; q < n; ++q) {
        if ((int)q == i0 || (int)q == i1 || (int)q == i2 || (int)q == i3) continue;
        std::vector<int> vis;
        for (size_t f = 0; f < F.size(); ++f)
            if (F[f].alive && dot(F[f].n, p[q]) - F[f].d > eps) vis.push_back((int)f);
        if (vis.empty()) continue;
        // directed edges of the visible faces; horizon = edges whose reverse is not visible
        std::map<std::pair<int, int>, int> edges;
        for (int f : vis) {
            const int v[3] = {F[f].a, F[f].b, F[f].c};
            for (int e = 0; e < 3; ++e) edges[{v[e], v[(e + 1) % 3]}] += 1;
            F[f].alive = false;
        }
        for (auto &kv : edges) {
            const int a = kv.first.first, b = kv.first.second;
            if (edges.count({b, a})) continue;
            Face nf{a, b, (int)q, {0, 0, 0}, 0.0, true};
            V3 nn = cross(sub(p[b], p[a]), sub(p[q], p[a]));
            const double len = norm(nn);
            if (len <= 0.0) continue;
            nf.n = {nn.x / len, nn.y / len, nn.z / len};
            nf.d = dot(nf.n, p[a]);
            F.push_back(nf);
        }
    }
    for (auto &f : F)
        if (f.alive) {
            out.push_back(f.n.x);
            out.push_back(f.n.y);
            out.push_back(f.n.z);
            out.push_back(f.d);
        }
    return out;
}

}  // namespace smc
