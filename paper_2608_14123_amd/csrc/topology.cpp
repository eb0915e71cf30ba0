// Subdomain tables of the Schwarz method on unstructured hexahedral meshes (Sec. 4.3.1 design
// principles 4-6, neighbour data of Sec. 5.1).
//
// Nodes of an element are addressed by integer coordinates (q1, q2, q3) in 0..n-1; the same
// coordinates extended beyond an element address the neighbour across the face: layer l of the
// neighbour (l = 0 at the shared face) sits at n + l beyond the + face and at -1 - l beyond the
// - face.  Crossing a face maps these coordinates into the neighbour's own through its face and
// the relative orientation.
//   * face blocks of a subdomain take the face neighbour's layers;
//   * an edge block is mapped when the elements around the edge close a ring of four and both
//     walking orders reach the same nodes; with no element beyond the two face neighbours it
//     is zero-filled; otherwise the surplus elements' nodes on the edge are averaged into the
//     block's innermost row (the rest stays zero);
//   * a vertex block is mapped when exactly one element around the vertex is not the element,
//     a face neighbour or around one of the three edges there, and all six walking orders
//     reach it alike; zero-filled when none is left; else the vertex nodes of those left are
//     averaged into the innermost slot.
#include "topology.hpp"

#include <algorithm>
#include <numeric>
#include <map>
#include <set>
#include <stdexcept>

namespace dgfas {
namespace {

// face-node layout (first axis, second axis) of face phi
const int kLay[6][2] = {{2, 1}, {2, 1}, {2, 0}, {2, 0}, {1, 0}, {1, 0}};

struct P3 {
  int q[3];
};

bool same_pts(const std::vector<P3>& a, const std::vector<P3>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    for (int c = 0; c < 3; ++c)
      if (a[i].q[c] != b[i].q[c]) return false;
  return true;
}

struct Walker {
  const TopoMesh& m;
  int n;
  explicit Walker(const TopoMesh& mm) : m(mm), n(mm.n) {}

  int face_of(int e, int phi) const { return m.nface ? m.nface[e * 6 + phi] : (phi ^ 1); }
  int orient_of(int e, int phi) const { return m.norient ? m.norient[e * 6 + phi] : 0; }

  // move the points across face phi of e into the neighbour's coordinates; amap (optional)
  // receives, for each of e's axes, the neighbour's axis it runs along.  -1 at a boundary.
  int cross(int e, int phi, P3* p, size_t np, int* amap) const {
    const int en = m.nbr[e * 6 + phi];
    if (en < 0) return -1;
    const int f2 = face_of(e, phi), o = orient_of(e, phi);
    const int c = phi >> 1, s = phi & 1, c2 = f2 >> 1, s2 = f2 & 1;
    const int fa = kLay[phi][0], fb = kLay[phi][1], ga = kLay[f2][0], gb = kLay[f2][1];
    for (size_t i = 0; i < np; ++i) {
      const int l = s ? p[i].q[c] - n : -1 - p[i].q[c];
      const int a = p[i].q[fa], b = p[i].q[fb];
      const int x = (o & 1) ? b : a, y = (o & 1) ? a : b;
      P3 r;
      r.q[c2] = s2 ? n - 1 - l : l;
      r.q[ga] = (o & 2) ? n - 1 - x : x;
      r.q[gb] = (o & 4) ? n - 1 - y : y;
      p[i] = r;
    }
    if (amap) {
      amap[c] = c2;
      amap[fa] = (o & 1) ? gb : ga;
      amap[fb] = (o & 1) ? ga : gb;
    }
    return en;
  }

  // nodes of e on face phi -> the same physical nodes of the neighbour
  int onto_face(int e, int phi, std::vector<P3>& p) const {
    const int f2 = face_of(e, phi);
    const int en = cross(e, phi, p.data(), p.size(), nullptr);
    if (en < 0) return -1;
    for (P3& x : p) x.q[f2 >> 1] = (f2 & 1) ? n - 1 : 0;
    return en;
  }

  // walk the points of one block (all beyond e along the same axes) across faces, taking e's
  // axes in `order`; returns the element reached, or -1 at a boundary
  int locate(int e, std::vector<P3>& p, const int* order, int k) const {
    int cur = e, ax[3] = {0, 1, 2};
    for (int t = 0; t < k; ++t) {
      const int a = ax[order[t]];
      const int v = p[0].q[a];
      if (v >= 0 && v < n) continue;
      const int phi = 2 * a + (v >= n ? 1 : 0);
      int amap[3];
      const int en = cross(cur, phi, p.data(), p.size(), amap);
      if (en < 0) return -1;
      for (int i = 0; i < 3; ++i) ax[i] = amap[ax[i]];
      cur = en;
    }
    return cur;
  }

  bool at_end(const std::vector<P3>& p, int a, int& side) const {
    const int v = p[0].q[a];
    if (v != 0 && v != n - 1) return false;
    for (const P3& x : p)
      if (x.q[a] != v) return false;
    side = v == n - 1 ? 1 : 0;
    return true;
  }

  struct Member {
    int e;
    std::vector<P3> pts;   // the element's nodes on the edge, in the order of e's edge nodes
  };

  // around the edge of e from face (fax, fside): true when the walk returns to e
  bool ring_walk(int e, int fax, int fside, const std::vector<P3>& pts0, std::vector<Member>& seq) const {
    int cur = e, ax = fax, sd = fside;
    std::vector<P3> pts = pts0;
    for (int step = 0; step < 64; ++step) {
      const int phi = 2 * ax + sd;
      if (m.nbr[cur * 6 + phi] < 0) return false;
      const int entry = face_of(cur, phi) >> 1;
      const int en = onto_face(cur, phi, pts);
      if (en == e && same_pts(pts, pts0)) return true;
      seq.push_back({en, pts});
      int nxt = -1, nside = 0, cnt = 0;
      for (int a = 0; a < 3; ++a) {
        int side;
        if (a != entry && at_end(pts, a, side)) { nxt = a; nside = side; ++cnt; }
      }
      if (cnt != 1) throw std::runtime_error("edge walk lost the edge at element " + std::to_string(en));
      cur = en; ax = nxt; sd = nside;
    }
    throw std::runtime_error("an edge ring longer than 64 elements");
  }

  struct EdgeInfo {
    int kind = 0;                // 2 mapped, 3 zero-filled, 4 merged
    std::vector<Member> others;  // mapped: the edge neighbour; merged: the surplus elements
    std::set<int> ring;          // every element around the edge but e
  };

  EdgeInfo edge(int e, int a1, int s1, int a2, int s2) const {
    const int c3 = 3 - a1 - a2;
    std::vector<P3> pts0(n);
    for (int t = 0; t < n; ++t) {
      pts0[t].q[a1] = s1 ? n - 1 : 0;
      pts0[t].q[a2] = s2 ? n - 1 : 0;
      pts0[t].q[c3] = t;
    }
    std::vector<Member> side1, side2;
    const bool closed = ring_walk(e, a1, s1, pts0, side1);
    if (!closed) ring_walk(e, a2, s2, pts0, side2);
    EdgeInfo info;
    std::set<int> faces;
    if (!side1.empty()) faces.insert(side1.front().e);
    if (closed) faces.insert(side1.back().e);
    else if (!side2.empty()) faces.insert(side2.front().e);
    std::vector<Member> cand;
    if (closed) {
      if (side1.size() > 2) cand.assign(side1.begin() + 1, side1.end() - 1);
    } else {
      if (side1.size() > 1) cand.insert(cand.end(), side1.begin() + 1, side1.end());
      if (side2.size() > 1) cand.insert(cand.end(), side2.begin() + 1, side2.end());
    }
    for (const Member& x : cand)
      if (!faces.count(x.e) && x.e != e) info.others.push_back(x);
    for (const Member& x : side1) info.ring.insert(x.e);
    for (const Member& x : side2) info.ring.insert(x.e);
    if (closed && side1.size() == 3 && info.others.size() == 1) info.kind = 2;
    else if (info.others.empty()) info.kind = 3;
    else info.kind = 4;
    return info;
  }

  // elements around the vertex of e at `corner` (side per axis) with their vertex node, in
  // discovery order (depth first)
  std::vector<std::pair<int, P3>> star(int e, const int* corner) const {
    P3 q0;
    for (int a = 0; a < 3; ++a) q0.q[a] = corner[a] ? n - 1 : 0;
    std::vector<std::pair<int, P3>> seen{{e, q0}};
    std::vector<std::pair<int, P3>> todo{{e, q0}};
    while (!todo.empty()) {
      const auto cur = todo.back();
      todo.pop_back();
      for (int a = 0; a < 3; ++a) {
        const int phi = 2 * a + (cur.second.q[a] == n - 1 ? 1 : 0);
        if (m.nbr[cur.first * 6 + phi] < 0) continue;
        std::vector<P3> p{cur.second};
        const int en = onto_face(cur.first, phi, p);
        bool have = false;
        for (const auto& s : seen) have = have || s.first == en;
        if (!have) {
          seen.push_back({en, p[0]});
          todo.push_back({en, p[0]});
        }
      }
    }
    return seen;
  }
};

}  // namespace

std::string topo_check(const TopoMesh& m) {
  const int n = m.n;
  for (int e = 0; e < m.E; ++e)
    for (int phi = 0; phi < 6; ++phi) {
      const int en = m.nbr[e * 6 + phi];
      if (en < 0) continue;
      if (en >= m.E) return "neighbour id out of range at element " + std::to_string(e);
      const int f2 = m.nface ? m.nface[e * 6 + phi] : (phi ^ 1);
      const int o = m.norient ? m.norient[e * 6 + phi] : 0;
      if (f2 < 0 || f2 > 5 || o < 0 || o > 7)
        return "neighbour face or orientation out of range at element " + std::to_string(e);
      if (m.nbr[en * 6 + f2] != e || (m.nface ? m.nface[en * 6 + f2] : (f2 ^ 1)) != phi)
        return "element " + std::to_string(e) + " face " + std::to_string(phi) +
               ": the neighbour does not see it back through the same face";
      const int ob = m.norient ? m.norient[en * 6 + f2] : 0;
      // the two orientations must be inverse maps of the face nodes
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          int x = (o & 1) ? b : a, y = (o & 1) ? a : b;
          const int a1 = (o & 2) ? n - 1 - x : x, b1 = (o & 4) ? n - 1 - y : y;
          x = (ob & 1) ? b1 : a1; y = (ob & 1) ? a1 : b1;
          const int a2 = (ob & 2) ? n - 1 - x : x, b2 = (ob & 4) ? n - 1 - y : y;
          if (a2 != a || b2 != b)
            return "element " + std::to_string(e) + " face " + std::to_string(phi) +
                   ": the orientations of the two sides are not inverse";
        }
    }
  return std::string();
}

TopoTables topo_tables(const TopoMesh& m, int ns, const int8_t* var, const int* map1d, const double* W,
                       bool normalise) {
  const int n = m.n, E = m.E, nt = ns * ns * ns;
  const int64_t n3 = (int64_t)n * n * n, ndof = (int64_t)E * n3;
  if (ndof >= ((int64_t)1 << 31) || (int64_t)E * nt >= ((int64_t)1 << 31))
    throw std::runtime_error("unstructured mesh too large for 32-bit node and slot indices");
  Walker w(m);
  TopoTables T;
  T.nt = nt;
  T.gather.assign((size_t)E * nt, -1);
  T.mptr.push_back(0);
  // contributions (node, subdomain slot, share) in subdomain and slot order
  struct Contrib {
    int node, slot;
    double share;
  };
  std::vector<Contrib> con;
  auto node_of = [&](int el, const P3& p) { return (int)(el * n3 + ((int64_t)p.q[2] * n + p.q[1]) * n + p.q[0]); };

  for (int e = 0; e < E; ++e) {
    // tile positions per direction: block -1/0/1 and coordinate, or padding
    int blk[3][16], crd[3][16];
    bool ok[3][16];
    for (int d = 0; d < 3; ++d) {
      const int v = var[(size_t)e * 3 + d];
      for (int s = 0; s < ns; ++s) {
        const int mp = map1d[v * ns + s];
        ok[d][s] = mp >= 0;
        blk[d][s] = mp >= 0 ? (mp >> 6) - 1 : 0;
        crd[d][s] = mp >= 0 ? blk[d][s] * n + (mp & 63) : 0;
      }
    }
    auto slot_of = [&](int s1, int s2, int s3) { return (s3 * ns + s2) * ns + s1; };
    std::vector<std::pair<int, std::vector<std::pair<int, double>>>> entries;   // slot -> (node, share)
    auto put1 = [&](int slot, int node) { entries.push_back({slot, {{node, 1.0}}}); };
    std::map<std::pair<int, int>, std::set<int>> rings;   // edge (face1, face2) -> its ring

    for (int b3 = -1; b3 <= 1; ++b3)
      for (int b2 = -1; b2 <= 1; ++b2)
        for (int b1 = -1; b1 <= 1; ++b1) {
          const int bb[3] = {b1, b2, b3};
          std::vector<int> sl;
          std::vector<P3> pts;
          for (int s3 = 0; s3 < ns; ++s3)
            for (int s2 = 0; s2 < ns; ++s2)
              for (int s1 = 0; s1 < ns; ++s1) {
                if (!ok[0][s1] || !ok[1][s2] || !ok[2][s3]) continue;
                if (blk[0][s1] != b1 || blk[1][s2] != b2 || blk[2][s3] != b3) continue;
                sl.push_back(slot_of(s1, s2, s3));
                pts.push_back({{crd[0][s1], crd[1][s2], crd[2][s3]}});
              }
          if (sl.empty()) continue;
          int nz[3], k = 0;
          for (int a = 0; a < 3; ++a)
            if (bb[a]) nz[k++] = a;
          if (k <= 1) {
            const int el = w.locate(e, pts, nz, k);
            if (el < 0) throw std::runtime_error("a face block beyond a boundary");
            for (size_t i = 0; i < sl.size(); ++i) put1(sl[i], node_of(el, pts[i]));
            T.blocks[k == 0 ? 0 : 1]++;
            continue;
          }
          if (k == 2) {
            const int a1 = nz[0], a2 = nz[1];
            Walker::EdgeInfo info = w.edge(e, a1, bb[a1] > 0, a2, bb[a2] > 0);
            rings[{2 * a1 + (bb[a1] > 0), 2 * a2 + (bb[a2] > 0)}] = info.ring;
            int kind = info.kind;
            if (kind == 2) {
              std::vector<P3> p1 = pts, p2 = pts;
              const int o1[2] = {a1, a2}, o2[2] = {a2, a1};
              const int x1 = w.locate(e, p1, o1, 2), x2 = w.locate(e, p2, o2, 2);
              if (x1 >= 0 && x1 == x2 && same_pts(p1, p2)) {
                for (size_t i = 0; i < sl.size(); ++i) put1(sl[i], node_of(x1, p1[i]));
                T.blocks[2]++;
                continue;
              }
              kind = 4;
            }
            if (kind == 3) { T.blocks[3]++; continue; }
            T.blocks[4]++;
            const int c3 = 3 - a1 - a2;
            const int in1 = bb[a1] > 0 ? n : -1, in2 = bb[a2] > 0 ? n : -1;
            const double share = 1.0 / (double)info.others.size();
            for (size_t i = 0; i < sl.size(); ++i) {
              if (pts[i].q[a1] != in1 || pts[i].q[a2] != in2) continue;
              const int t = pts[i].q[c3];
              std::vector<std::pair<int, double>> list;
              for (const auto& x : info.others) list.push_back({node_of(x.e, x.pts[t]), share});
              entries.push_back({sl[i], list});
            }
            continue;
          }
          // vertex block
          const int corner[3] = {b1 > 0, b2 > 0, b3 > 0};
          std::set<int> used{e};
          for (int a = 0; a < 3; ++a) {
            const int nb = m.nbr[e * 6 + 2 * a + corner[a]];
            if (nb >= 0) used.insert(nb);
          }
          const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
          for (const auto& pr : pairs) {
            const std::pair<int, int> key{2 * pr[0] + corner[pr[0]], 2 * pr[1] + corner[pr[1]]};
            auto it = rings.find(key);
            const std::set<int> ring =
                it != rings.end() ? it->second : w.edge(e, pr[0], corner[pr[0]], pr[1], corner[pr[1]]).ring;
            used.insert(ring.begin(), ring.end());
          }
          std::vector<std::pair<int, P3>> others;
          for (const auto& s : w.star(e, corner))
            if (!used.count(s.first)) others.push_back(s);
          if (others.empty()) { T.blocks[3]++; continue; }
          if (others.size() == 1) {
            int perm[3] = {0, 1, 2};
            bool agree = true;
            std::vector<P3> first;
            int el0 = -1;
            do {
              std::vector<P3> p = pts;
              const int el = w.locate(e, p, perm, 3);
              if (el < 0 || el != others[0].first) { agree = false; break; }
              if (first.empty()) { first = p; el0 = el; }
              else if (!same_pts(first, p)) { agree = false; break; }
            } while (std::next_permutation(perm, perm + 3));
            if (agree) {
              for (size_t i = 0; i < sl.size(); ++i) put1(sl[i], node_of(el0, first[i]));
              T.blocks[2]++;
              continue;
            }
          }
          T.blocks[4]++;
          const double share = 1.0 / (double)others.size();
          for (size_t i = 0; i < sl.size(); ++i) {
            bool inner = true;
            for (int a = 0; a < 3; ++a) inner = inner && pts[i].q[a] == (bb[a] > 0 ? n : -1);
            if (!inner) continue;
            std::vector<std::pair<int, double>> list;
            for (const auto& x : others) list.push_back({node_of(x.first, x.second), share});
            entries.push_back({sl[i], list});
          }
        }
    std::sort(entries.begin(), entries.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    for (const auto& en : entries) {
      int& g = T.gather[(size_t)e * nt + en.first];
      if (en.second.size() == 1 && en.second[0].second == 1.0) {
        g = en.second[0].first;
      } else {
        g = -2 - (int)(T.mptr.size() - 1);
        for (const auto& x : en.second) T.midx.push_back(x.first);
        T.mptr.push_back((int)T.midx.size());
      }
      for (const auto& x : en.second) con.push_back({x.first, e * nt + en.first, x.second});
    }
  }
  // tensor weights, the weight sum per node and the per-node lists
  auto weight = [&](int gslot) {
    const int e = gslot / nt, s = gslot - e * nt;
    const int s1 = s % ns, s2 = (s / ns) % ns, s3 = s / (ns * ns);
    const double* w1 = W + var[(size_t)e * 3 + 0] * ns;
    const double* w2 = W + var[(size_t)e * 3 + 1] * ns;
    const double* w3 = W + var[(size_t)e * 3 + 2] * ns;
    return w3[s3] * w2[s2] * w1[s1];
  };
  std::vector<double> C((size_t)ndof, 0.0);
  for (const Contrib& c : con) C[c.node] += c.share * weight(c.slot);
  T.sptr.assign((size_t)ndof + 1, 0);
  for (const Contrib& c : con) T.sptr[c.node + 1]++;
  for (int64_t g = 0; g < ndof; ++g) T.sptr[g + 1] += T.sptr[g];
  T.sslot.resize(con.size());
  T.scoef.resize(con.size());
  std::vector<int64_t> fillp(T.sptr.begin(), T.sptr.end() - 1);
  for (const Contrib& c : con) {
    if (normalise && !(C[c.node] > 0)) throw std::runtime_error("a node without a covering subdomain");
    const int64_t k = fillp[c.node]++;
    T.sslot[k] = c.slot;
    T.scoef[k] = c.share * weight(c.slot) * (normalise ? 1.0 / C[c.node] : 1.0);
  }
  return T;
}

}  // namespace dgfas
