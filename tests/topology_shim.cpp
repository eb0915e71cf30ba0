// Test shim: the library's host-side subdomain table builder (topology.cpp) behind a C call, so
// that the CPU tests can compare its tables with the oracle's without a GPU.
#include <cstring>
#include <stdexcept>

#include "../paper_2608_14123_amd/csrc/topology.hpp"

extern "C" int shim_topo_tables(int E, int n, const int* nbr, const int8_t* nface, const int8_t* norient, int ns,
                                const int8_t* var, const int* map1d, const double* W, int normalise,
                                int64_t* blocks, int* gather, int* nmerge, int* mptr, int mcap, int* midx,
                                int icap, int64_t* sptr, int* sslot, double* scoef, int64_t ccap) {
  try {
    dgfas::TopoMesh m;
    m.E = E; m.n = n; m.nbr = nbr; m.nface = nface; m.norient = norient;
    const std::string bad = dgfas::topo_check(m);
    if (!bad.empty()) return -2;
    dgfas::TopoTables T = dgfas::topo_tables(m, ns, var, map1d, W, normalise != 0);
    if ((int)T.mptr.size() > mcap || (int)T.midx.size() > icap || (int64_t)T.sslot.size() > ccap) return -3;
    std::memcpy(blocks, T.blocks, sizeof(T.blocks));
    std::memcpy(gather, T.gather.data(), T.gather.size() * sizeof(int));
    *nmerge = (int)T.mptr.size() - 1;
    std::memcpy(mptr, T.mptr.data(), T.mptr.size() * sizeof(int));
    if (!T.midx.empty()) std::memcpy(midx, T.midx.data(), T.midx.size() * sizeof(int));
    std::memcpy(sptr, T.sptr.data(), T.sptr.size() * sizeof(int64_t));
    std::memcpy(sslot, T.sslot.data(), T.sslot.size() * sizeof(int));
    std::memcpy(scoef, T.scoef.data(), T.scoef.size() * sizeof(double));
    return 0;
  } catch (const std::exception&) {
    return -1;
  }
}
