// Uniform (red) refinement of a mesh on the GPU: the routine the paper calls
// before assembling, which splits every triangle at its edge midpoints into
// four (section 2.1), so that h-convergence studies refine on the device.
//
// Numbering: the nodes keep their indices; the midpoint of edge e gets index
// n_nodes + e, with the edge ids fixed at mesh creation (the order in which a
// walk over the elements and their edges (v0 v1), (v1 v2), (v2 v0) first meets
// each edge).  Triangle (a, b, c) with midpoints ab, bc, ca becomes, at rows
// 4K .. 4K + 3, (a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca): all
// counter-clockwise when the parent is.  Listed boundary edge (a, b) becomes
// (a, m), (m, b) in place 2i, 2i + 1, keeping its Dirichlet or Neumann list.
// Every output entry has one writer, so the result is deterministic.
#include <hip/hip_runtime.h>

#include "dg_internal.h"

namespace dg {
namespace {

constexpr int RB = 256;

// old nodes copied; each edge's midpoint written by its first half-edge
__global__ __launch_bounds__(RB) void refine_nodes_kernel(const double* __restrict__ nodes, int64_t n_nodes,
                                                          const int32_t* __restrict__ elems,
                                                          const int32_t* __restrict__ eid,
                                                          const int32_t* __restrict__ owner, int64_t T,
                                                          double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i < n_nodes) {
        out[2 * i] = nodes[2 * i];
        out[2 * i + 1] = nodes[2 * i + 1];
    }
    if (i < 3 * T && owner[i]) {
        const int64_t K = i / 3;
        const int l = (int)(i - 3 * K);
        const int64_t a = elems[3 * K + l], b = elems[3 * K + (l == 2 ? 0 : l + 1)];
        const int64_t m = n_nodes + eid[i];
        out[2 * m] = 0.5 * (nodes[2 * a] + nodes[2 * b]);
        out[2 * m + 1] = 0.5 * (nodes[2 * a + 1] + nodes[2 * b + 1]);
    }
}

__global__ __launch_bounds__(RB) void refine_elems_kernel(const int32_t* __restrict__ elems,
                                                          const int32_t* __restrict__ eid, int64_t T,
                                                          int32_t n_nodes, int32_t* __restrict__ out)
{
    const int64_t K = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (K >= T) return;
    const int32_t a = elems[3 * K], b = elems[3 * K + 1], c = elems[3 * K + 2];
    const int32_t ab = n_nodes + eid[3 * K], bc = n_nodes + eid[3 * K + 1], ca = n_nodes + eid[3 * K + 2];
    const int32_t ch[12] = {a, ab, ca, ab, b, bc, ca, bc, c, ab, bc, ca};
    int32_t* o = out + 12 * K;
#pragma unroll
    for (int q = 0; q < 12; ++q) o[q] = ch[q];
}

__global__ __launch_bounds__(RB) void refine_edges_kernel(const int32_t* __restrict__ e,
                                                          const int32_t* __restrict__ ids, int64_t cnt,
                                                          int32_t n_nodes, int32_t* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
    if (i >= cnt) return;
    const int32_t m = n_nodes + ids[i];
    out[4 * i] = e[2 * i];
    out[4 * i + 1] = m;
    out[4 * i + 2] = m;
    out[4 * i + 3] = e[2 * i + 1];
}

unsigned blocks(int64_t n) { return (unsigned)((n + RB - 1) / RB); }

}  // namespace
}  // namespace dg

using namespace dg;

extern "C" int32_t dg_mesh_refine_sizes(const dg_mesh* m, int64_t* sizes)
{
    if (!m || !sizes) return DG_ERR_ARG;
    sizes[0] = m->n_nodes + m->n_edges;
    sizes[1] = 4 * m->T;
    sizes[2] = 2 * m->n_dir;
    sizes[3] = 2 * m->n_neu;
    return DG_OK;
}

extern "C" int32_t dg_mesh_refine(const dg_mesh* m, double* dev_nodes, int32_t* dev_elems, int32_t* dev_dir,
                                  int32_t* dev_neu, void* stream)
{
    if (!m || !dev_nodes || !dev_elems) return DG_ERR_ARG;
    if ((m->n_dir > 0 && !dev_dir) || (m->n_neu > 0 && !dev_neu)) return DG_ERR_ARG;
    if (m->n_nodes + m->n_edges > INT32_MAX || 4 * m->T > INT32_MAX) return DG_ERR_ARG;  // int32 node and element ids
    hipStream_t st = (hipStream_t)stream;
    const int32_t nn = (int32_t)m->n_nodes;
    hipLaunchKernelGGL(refine_nodes_kernel, dim3(blocks(std::max(m->n_nodes, 3 * m->T))), dim3(RB), 0, st,
                       m->d_nodes, m->n_nodes, m->d_elems, m->d_eid, m->d_owner, m->T, dev_nodes);
    hipLaunchKernelGGL(refine_elems_kernel, dim3(blocks(m->T)), dim3(RB), 0, st, m->d_elems, m->d_eid, m->T, nn,
                       dev_elems);
    if (m->n_dir > 0)
        hipLaunchKernelGGL(refine_edges_kernel, dim3(blocks(m->n_dir)), dim3(RB), 0, st, m->d_dir, m->d_dir_eid,
                           m->n_dir, nn, dev_dir);
    if (m->n_neu > 0)
        hipLaunchKernelGGL(refine_edges_kernel, dim3(blocks(m->n_neu)), dim3(RB), 0, st, m->d_neu, m->d_neu_eid,
                           m->n_neu, nn, dev_neu);
    return hipGetLastError() == hipSuccess ? DG_OK : DG_ERR_HIP;
}
