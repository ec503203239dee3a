// Host-side mesh topology, RWG/BC tables and barycentric refinement.
//
// Sec. II-C: RWG f_n = (r - r+)/(2A+) on c+, (r- - r)/(2A-) on c- (unit flux,
// no edge-length factor); BC g_n on the barycentric refinement.
// Sec. II-D: Lambda (vertex-edge, +1 at v+, -1 at v-), Sigma (face-edge, +1 at
// c+, -1 at c-).
//
// Rules fixed here because the paper leaves them open (the same written rules
// drive the independent CPU reference): edges are sorted by (min, max) vertex
// and oriented min -> max; c+ is the triangle whose counter-clockwise vertex
// cycle traverses v- -> v+.  BC coefficients (cited, not printed): flux 1/2
// through each of the two fine edges of the dual edge of e_n, from the dual
// cell of v- into that of v+, and charge +-1 spread equally, 1/(2 N_v) per
// fine triangle, over each dual cell; around v+ the radial fine-edge fluxes
// are (N - j)/(2N), j = 1..2N-1, counted from the half-edge (v+, mid e_n),
// with zero on that half-edge; the v- side is the negative mirror.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <numeric>

#include "qhp_internal.h"

namespace qhp {

// q_0 of temporal order p spans p + 2 intervals: it reaches p + 1 shells past
// the largest distance (the 1e-9 guard keeps an integer D/dt stable)
int64_t n_lags(double diameter, double dt, int order)
{
    return (int64_t)std::ceil(diameter / dt - 1e-9) + (order > 1 ? order : 1);
}

static int fail(std::string &err, const std::string &msg)
{
    err = msg;
    return QHP_EMESH;
}

int build_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nc, Mesh &m,
               std::string &err)
{
    if (nv < 4 || nc < 4) return fail(err, "mesh too small for a closed surface");
    m = Mesh();
    m.nv = nv;
    m.nc = nc;
    m.xyz.assign(xyz, xyz + 3 * nv);
    m.tri.assign(tri, tri + 3 * nc);
    for (int64_t i = 0; i < 3 * nc; ++i)
        if (tri[i] < 0 || tri[i] >= nv) return fail(err, "triangle vertex index out of range");

    // ---- edges: key (min, max) -> uses (triangle, local index, first vertex)
    struct Use { int32_t c, i, a; };
    std::map<std::pair<int32_t, int32_t>, std::vector<Use>> emap;
    for (int64_t c = 0; c < nc; ++c)
        for (int i = 0; i < 3; ++i) {
            int32_t a = tri[3 * c + (i + 1) % 3], b = tri[3 * c + (i + 2) % 3];
            if (a == b) return fail(err, "degenerate triangle");
            emap[{std::min(a, b), std::max(a, b)}].push_back({(int32_t)c, i, a});
        }
    m.ne = (int64_t)emap.size();
    m.edges.resize(2 * m.ne);
    m.cells.resize(2 * m.ne);
    m.tri_edge.assign(3 * nc, -1);
    m.tri_sign.assign(3 * nc, 0);
    int64_t e = 0;
    for (auto &kv : emap) {
        const auto &uses = kv.second;
        if (uses.size() != 2) return fail(err, "edge not shared by exactly two triangles (open or non-manifold)");
        const Use *plus = nullptr, *minus = nullptr;
        for (const auto &u : uses) {
            if (u.a == kv.first.first) plus = &u;   // traverses v- -> v+
            else minus = &u;
        }
        if (!plus || !minus) return fail(err, "inconsistently oriented triangles");
        m.edges[2 * e] = kv.first.first;
        m.edges[2 * e + 1] = kv.first.second;
        m.cells[2 * e] = plus->c;
        m.cells[2 * e + 1] = minus->c;
        m.tri_edge[3 * plus->c + plus->i] = (int32_t)e;
        m.tri_sign[3 * plus->c + plus->i] = 1;
        m.tri_edge[3 * minus->c + minus->i] = (int32_t)e;
        m.tri_sign[3 * minus->c + minus->i] = -1;
        ++e;
    }
    // ---- connectivity of the triangle adjacency graph
    {
        std::vector<int32_t> parent(nc);
        std::iota(parent.begin(), parent.end(), 0);
        auto find = [&](int32_t x) {
            while (parent[x] != x) { parent[x] = parent[parent[x]]; x = parent[x]; }
            return x;
        };
        for (int64_t k = 0; k < m.ne; ++k) {
            int32_t a = find(m.cells[2 * k]), b = find(m.cells[2 * k + 1]);
            if (a != b) parent[a] = b;
        }
        int32_t r0 = find(0);
        for (int64_t c = 1; c < nc; ++c)
            if (find((int32_t)c) != r0) return fail(err, "surface is not connected");
    }
    // ---- geometry
    m.area.resize(nc);
    for (int64_t c = 0; c < nc; ++c) {
        const double *p0 = &xyz[3 * tri[3 * c]], *p1 = &xyz[3 * tri[3 * c + 1]], *p2 = &xyz[3 * tri[3 * c + 2]];
        double u[3], v[3], w[3];
        for (int k = 0; k < 3; ++k) { u[k] = p1[k] - p0[k]; v[k] = p2[k] - p0[k]; }
        w[0] = u[1] * v[2] - u[2] * v[1];
        w[1] = u[2] * v[0] - u[0] * v[2];
        w[2] = u[0] * v[1] - u[1] * v[0];
        m.area[c] = 0.5 * std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        // zero up to rounding: below 1e-12 of the square of the longest edge
        double l2 = 0.0;
        for (const double *e : {u, v}) l2 = std::max(l2, e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        l2 = std::max(l2, (u[0] - v[0]) * (u[0] - v[0]) + (u[1] - v[1]) * (u[1] - v[1]) + (u[2] - v[2]) * (u[2] - v[2]));
        if (!(m.area[c] > 1e-12 * l2)) return fail(err, "zero-area triangle");
    }
    double dmax = 0.0;
    for (int64_t a = 0; a < nv; ++a)
        for (int64_t b = a + 1; b < nv; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) { double d = xyz[3 * a + k] - xyz[3 * b + k]; s += d * d; }
            dmax = std::max(dmax, s);
        }
    m.diameter = std::sqrt(dmax);
    m.n_harmonic = 2 - (nv - m.ne + nc);

    // ---- barycentric refinement: fine vertices = vertices, midpoints, centroids
    m.nfv = nv + m.ne + nc;
    m.nf = 6 * nc;
    m.fxyz.resize(3 * m.nfv);
    for (int64_t i = 0; i < 3 * nv; ++i) m.fxyz[i] = xyz[i];
    for (int64_t k = 0; k < m.ne; ++k)
        for (int q = 0; q < 3; ++q)
            m.fxyz[3 * (nv + k) + q] = 0.5 * (xyz[3 * m.edges[2 * k] + q] + xyz[3 * m.edges[2 * k + 1] + q]);
    for (int64_t c = 0; c < nc; ++c)
        for (int q = 0; q < 3; ++q)
            m.fxyz[3 * (nv + m.ne + c) + q] =
                (xyz[3 * tri[3 * c] + q] + xyz[3 * tri[3 * c + 1] + q] + xyz[3 * tri[3 * c + 2] + q]) / 3.0;
    m.ftri.resize(3 * m.nf);
    m.fparent.resize(m.nf);
    m.fowner.resize(m.nf);
    for (int64_t c = 0; c < nc; ++c) {
        int32_t g = (int32_t)(nv + m.ne + c);
        for (int i = 0; i < 3; ++i) {
            int32_t vi = tri[3 * c + i];
            int32_t m_next = (int32_t)nv + m.tri_edge[3 * c + (i + 2) % 3];  // {v_i, v_i+1}
            int32_t m_prev = (int32_t)nv + m.tri_edge[3 * c + (i + 1) % 3];  // {v_i-1, v_i}
            int64_t f0 = 6 * c + 2 * i, f1 = f0 + 1;
            m.ftri[3 * f0] = vi; m.ftri[3 * f0 + 1] = m_next; m.ftri[3 * f0 + 2] = g;
            m.ftri[3 * f1] = vi; m.ftri[3 * f1 + 1] = g; m.ftri[3 * f1 + 2] = m_prev;
            m.fparent[f0] = m.fparent[f1] = (int32_t)c;
            m.fowner[f0] = m.fowner[f1] = vi;
        }
    }

    // ---- fans around each vertex, BC fluxes
    std::vector<std::vector<std::pair<int32_t, int32_t>>> inc(nv);  // (triangle, local index)
    for (int64_t c = 0; c < nc; ++c)
        for (int i = 0; i < 3; ++i) inc[tri[3 * c + i]].push_back({(int32_t)c, i});
    m.valence.resize(nv);
    std::vector<std::vector<std::pair<int32_t, std::array<double, 3>>>> entries(m.nf);
    m.vcell_off.assign(nv + 1, 0);
    m.vedge_off.assign(nv + 1, 0);
    std::vector<std::vector<int32_t>> vcell(nv), vedges(nv);
    for (int64_t v = 0; v < nv; ++v) {
        const auto &fan = inc[v];
        int nvv = (int)fan.size();
        if (nvv < 3) return fail(err, "vertex with fewer than three triangles");
        m.valence[v] = nvv;
        std::vector<int32_t> ring_tris, ring_mid;
        int32_t c0 = fan[0].first, c = c0;
        for (int s = 0; s < nvv; ++s) {
            int li = -1;
            for (const auto &pr : fan)
                if (pr.first == c) li = pr.second;
            int32_t b = tri[3 * c + (li + 2) % 3];
            ring_mid.push_back(m.tri_edge[3 * c + (li + 2) % 3]);  // {v, a}
            ring_tris.push_back((int32_t)(6 * c + 2 * li));
            ring_tris.push_back((int32_t)(6 * c + 2 * li + 1));
            int32_t nxt = -1;
            for (const auto &pr : fan)
                if (tri[3 * pr.first + (pr.second + 1) % 3] == b) nxt = pr.first;
            if (nxt < 0) return fail(err, "broken vertex fan (non-manifold vertex)");
            c = nxt;
        }
        {
            std::vector<int32_t> chk(ring_tris);
            std::sort(chk.begin(), chk.end());
            if (c != c0 || std::unique(chk.begin(), chk.end()) != chk.end())
                return fail(err, "vertex fan is not a single disc (non-manifold vertex)");
        }
        int two_n = 2 * nvv;
        vcell[v] = ring_tris;
        for (int jm = 0; jm < nvv; ++jm) {
            int32_t edge = ring_mid[jm];
            vedges[v].push_back(edge);
            double s = (m.edges[2 * edge + 1] == v) ? 1.0 : -1.0;  // v+ is the sink
            int i0 = 2 * jm;
            std::vector<double> F(two_n + 1, 0.0);
            for (int j = 1; j < two_n; ++j) F[j] = (nvv - j) / (2.0 * nvv);
            for (int j = 1; j <= two_n; ++j) {
                int32_t t = ring_tris[(i0 + j - 1) % two_n];
                std::array<double, 3> fl = {((j == 1 || j == two_n) ? -0.5 : 0.0) * s, F[j] * s,
                                            -F[j - 1] * s};
                entries[t].push_back({edge, fl});
            }
        }
    }
    for (int64_t v = 0; v < nv; ++v) {
        m.vcell_off[v + 1] = m.vcell_off[v] + (int32_t)vcell[v].size();
        m.vedge_off[v + 1] = m.vedge_off[v] + (int32_t)vedges[v].size();
        m.vcell_tri.insert(m.vcell_tri.end(), vcell[v].begin(), vcell[v].end());
        m.vedge.insert(m.vedge.end(), vedges[v].begin(), vedges[v].end());
    }
    m.bc_off.assign(m.nf + 1, 0);
    for (int64_t t = 0; t < m.nf; ++t) {
        int32_t v = m.fowner[t];
        for (const auto &en : entries[t]) {
            m.bc_edge.push_back(en.first);
            int rank = -1;
            for (int32_t q = m.vedge_off[v]; q < m.vedge_off[v + 1]; ++q)
                if (m.vedge[q] == en.first) rank = q - m.vedge_off[v];
            m.bc_local.push_back(rank);
            for (int q = 0; q < 3; ++q) m.bc_flux.push_back(en.second[q]);
        }
        m.bc_off[t + 1] = (int32_t)m.bc_edge.size();
    }
    return QHP_OK;
}

}  // namespace qhp
