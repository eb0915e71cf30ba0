// Host-side subdomain tables of the Schwarz method on unstructured meshes (Sec. 4.3.1 with the
// oriented neighbour data of Sec. 5.1).
#pragma once
#include <stdint.h>
#include <string>
#include <vector>

namespace dgfas {

// One uniform-degree mesh level: n = p + 1; nface / norient may be null (aligned neighbours).
struct TopoMesh {
  int E = 0, n = 0;
  const int* nbr = nullptr;          // [E][6], -1 on the boundary
  const int8_t* nface = nullptr;     // [E][6] the neighbour's face across each interior face
  const int8_t* norient = nullptr;   // [E][6] relative orientation code 0..7
};

struct TopoTables {
  int nt = 0;                        // slots per subdomain tile, ns^3
  std::vector<int> gather;           // [E][nt] node of each slot, -1 zero, -2 - j merged slot j
  std::vector<int> mptr, midx;       // merged slot j averages midx[mptr[j] .. mptr[j + 1])
  std::vector<int64_t> sptr;         // [ndof + 1] contributions per node
  std::vector<int> sslot;            // subdomain * nt + slot
  std::vector<double> scoef;         // merge share x tensor weight (x 1 / weight sum)
  int64_t blocks[5] = {0, 0, 0, 0, 0};   // subdomain blocks: own, face, mapped, zero-filled, merged
};

// var: [E][3] 1D variant per direction; map1d: [variants][ns] tile position -> ((block + 1) << 6) |
// layer, or -1 for padding; W: [variants][ns] 1D weights.  normalise: divide every contribution by
// the weight sum at its node.  Throws std::runtime_error on inconsistent neighbour data.
TopoTables topo_tables(const TopoMesh& m, int ns, const int8_t* var, const int* map1d, const double* W,
                       bool normalise);

// Checks that every interior face is seen back from its neighbour through the same face with
// the inverse orientation; returns an empty string or the first problem found.
std::string topo_check(const TopoMesh& m);

}  // namespace dgfas
