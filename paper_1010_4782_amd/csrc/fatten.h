// Link fattening (fatten.hip): asqtad one-hop links and three-hop products from a thin gauge field.
#pragma once

#include <hip/hip_runtime.h>

namespace stag {

constexpr int kFattenWsFields = 6;  // link-matrix fields of workspace (144 B per site each)

size_t fatten_workspace_bytes(const int dims[4]);
// thin, fat, lng: device complex128 [4][Lt][Lz][Ly][Lx][3][3]; ws: fatten_workspace_bytes(dims).
hipError_t fatten_links(const int dims[4], const void* thin, double u0, void* fat, void* lng, void* ws,
                        hipStream_t st);

}  // namespace stag
