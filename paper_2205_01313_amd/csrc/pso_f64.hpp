// pso_f64.hpp -- the binary64 path: the same method in double (the paper's
// own precision, Sec. 5), from the same binary32 parameters and the same
// 24-bit uniforms.  Host side of the kernels in pso_f64.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pso {

// Control block of a binary64 swarm (device memory).
struct alignas(256) Ctrl64 {
    unsigned long long gord; // order bits of the gbest fitness (see ord64)
    uint32_t gidx;           // gbest particle
    uint32_t arrive;         // workgroups that finished the current launch
    long long giter;         // iteration of the last gbest change
    long long t;             // iterations completed
    uint32_t stop;           // stop rule met
    uint32_t err;            // a bounded wait of the gang kernel gave up
    double tol, fstar;       // stop rule |gbest - fstar| < tol (tol <= 0: off)
    unsigned long long gang_arrive; // gang kernel: workgroup arrivals (monotonic within a launch)
    unsigned char pad2[184];
};
static_assert(sizeof(Ctrl64) == 256, "Ctrl64 layout");

struct Swarm64Args {
    double *x, *v, *p, *pf;        // D*Np, D*Np, D*Np, Np; element (d, i) at d*Np + i
    double *gpos;                  // D
    const double *shift;           // D
    unsigned long long *slot_ord;  // one per grid workgroup (gang: two per workgroup by parity; staged gang: six tagged words)
    uint32_t *slot_idx;            // as slot_ord
    double *cand_pos;              // gang: [parity][workgroup][D] candidate positions (staged gang: tagged words)
    uint8_t *pend;                 // Np: 1 = pbest position of i is x, not yet in p (wide grid step)
    Ctrl64 *ctrl;
    uint32_t N, Np;
    int32_t D;
    double lo, hi, w, c1, c2, vmax;
    uint32_t k0, k1;
};

struct Layout64 {
    size_t ctrl, gpos, shift, slot_ord, slot_idx, cand_pos, pf, pend, x, v, p, total;
    uint64_t Np;
    uint32_t nblocks;
};

Layout64 layout64_of(uint64_t N, int D);
Swarm64Args bind64(void *base, const Layout64 &L, uint64_t N, int D);

// Step 1 (grid), one iteration (grid), or up to T iterations in one
// workgroup (block).  All honour and update the control block's stop rule.
hipError_t launch64_reset(const Swarm64Args &a, hipStream_t stream);
hipError_t launch64_init(int fitness, const Swarm64Args &a, hipStream_t stream);
hipError_t launch64_step(int fitness, const Swarm64Args &a, hipStream_t stream);
hipError_t launch64_block_run(int fitness, const Swarm64Args &a, long long T, hipStream_t stream);
// The swarm's state fits the LDS of the one-workgroup run (and staging is on).
bool block64_staged_fits(const Swarm64Args &a);
// The grid step of the swarm is the split one (lanes share a particle).
bool step64_split(int fitness, const Swarm64Args &a);
hipError_t launch64_arm(const Swarm64Args &a, double tol, double fstar, hipStream_t stream);
// Copies every pending pbest position (wide grid step) from x to p and
// clears the marks: before the state is read or another path runs.
hipError_t launch64_flush(const Swarm64Args &a, hipStream_t stream);
// out[m] = F(pts[m]) in binary64 for M device-resident points (row-major M x D).
hipError_t launch64_eval(int fitness, const Swarm64Args &a, const double *pts, uint64_t M, double *out,
                         hipStream_t stream);
// Up to T iterations by a persistent gang of co-resident workgroups that meet
// once per iteration (bit-identical to T grid steps); ctrl->gang_arrive must
// be zero.  *launched = false if the swarm needs more workgroups than can be
// co-resident (nothing is enqueued then).
// staged_only: launch only the gang with its slices in LDS (*launched false otherwise).
hipError_t launch64_gang(int fitness, const Swarm64Args &a, long long T, hipStream_t stream, bool *launched,
                         bool staged_only = false);

} // namespace pso
