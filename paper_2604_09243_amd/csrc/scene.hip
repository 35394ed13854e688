// Multi-scene arena support: the BVHs of several meshes are copied into one
// node array and one triangle array so that a single traversal kernel serves
// every scene of a batch; a ray finds its scene's root in its angle plan.
// Node references are relocated on the device: an internal child c >= 0
// becomes c + node_off, a leaf code ~(first * 8 + count - 1) moves its first
// slot by slot_off, and triangle ids move by id_off (ids keep their order
// within a scene, so the smaller-id tie rule is unchanged).
#include "sbr_internal.hpp"

namespace sbr {
namespace {

__global__ void k_zero_u32(uint32_t *p, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__device__ __forceinline__ int reloc_ref(int c, int32_t node_off, int32_t slot_off)
{
    if (c >= 0) return c + node_off;
    return ~((~c) + slot_off * 8);
}

__global__ void k_relocate_nodes(const BNode *__restrict__ src, int64_t n, BNode *__restrict__ dst, int32_t node_off,
                                 int32_t slot_off)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    BNode b = src[i];
    b.ch.x = reloc_ref(b.ch.x, node_off, slot_off);
    b.ch.y = reloc_ref(b.ch.y, node_off, slot_off);
    dst[i] = b;
}

__global__ void k_relocate_tris(const BTri *__restrict__ src, int64_t n, BTri *__restrict__ dst, int32_t id_off)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    BTri t = src[i];
    t.p0.w = __int_as_float(__float_as_int(t.p0.w) + id_off);
    dst[i] = t;
}

}  // namespace

int launch_zero_u32(hipStream_t s, uint32_t *p, int64_t n)
{
    if (n <= 0) return SBR_OK;
    k_zero_u32<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(p, n);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

int launch_relocate(hipStream_t s, const BNode *src_nodes, int64_t n_nodes, BNode *dst_nodes, int32_t node_off,
                    const BTri *src_tris, int64_t n_slots, BTri *dst_tris, int32_t slot_off, int32_t id_off)
{
    if (n_nodes > 0)
        k_relocate_nodes<<<static_cast<unsigned>((n_nodes + 255) / 256), 256, 0, s>>>(src_nodes, n_nodes, dst_nodes,
                                                                                     node_off, slot_off);
    if (n_slots > 0)
        k_relocate_tris<<<static_cast<unsigned>((n_slots + 255) / 256), 256, 0, s>>>(src_tris, n_slots, dst_tris,
                                                                                    id_off);
    SBR_HIP(hipGetLastError());
    return SBR_OK;
}

}  // namespace sbr
