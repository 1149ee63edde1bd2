// Batched uneven meshblock packs: three launches per RK2 stage advance every
// block of a pack -- face fluxes of every block along x1..x3, edge EMFs,
// then the zone update with the inversion -- each launch covering the work
// items of all blocks (one workgroup per item, in XCD order), so uneven
// block sizes fill the whole GPU together and every phase keeps the
// register budget of its own single-grid kernel.  Tile shapes (T1 x T2 x T3
// <= BLOCK threads, or linear runs of BLOCK positions) are chosen per block
// size (an autotuner picks them); the per-face, per-edge and per-zone work
// is the same device code as the single-block kernels, so a block advanced
// in a pack matches the same block advanced alone bit for bit (with the
// linear tile shape the x1 faces come from the same shared-edge sweep as the
// single grid's).  Ghost zones are frozen (Dirichlet) unless the ghost
// exchange fills them before each stage.
//
// Included inside the anonymous namespace of grmhd.hip.

struct BlockView {
  Dev g;
  double *P, *P1, *V;
  double *F[3], *E[3];
  double *tabC, *tabF1, *tabF2, *corner, *dgs;
  int t1, t2, t3;  // tile shape
  int o1, o2, o3;  // offset of the block's first interior zone in the global grid
};

enum { PH_FLUX = 0, PH_EMF = 1, PH_UPDATE = 2, PH_N = 3 };

// Boxes of the three phases of a block (flux boxes per direction).
__host__ __device__ inline Box phase_box(const Dev& g, int ph, int d) {
  if (ph == PH_FLUX) {
    if (d == 1) return Box{0, -1, -1, g.n1 + 1, g.n2 + 2, g.n3 + 2};
    if (d == 2) return Box{-1, 0, -1, g.n1 + 2, g.n2 + 1, g.n3 + 2};
    return Box{-1, -1, 0, g.n1 + 2, g.n2 + 2, g.n3 + 1};
  }
  if (ph == PH_EMF) return Box{0, 0, 0, g.n1 + 1, g.n2 + 1, g.n3 + 1};
  return Box{0, 0, 0, g.n1, g.n2, g.n3};
}

// Tiles of a box: t1 x t2 x t3 sub-boxes, or, for the linear shape
// (t1 = 0), runs of BLOCK consecutive positions in x1-fastest order (no
// thread idles except in a box's last run, whatever the box extents).
__host__ __device__ inline int tiles_of(const Box& b, int t1, int t2, int t3) {
  if (t1 == 0) return (int)((b.count() + BLOCK - 1) / BLOCK);
  return ((b.n1 + t1 - 1) / t1) * ((b.n2 + t2 - 1) / t2) * ((b.n3 + t3 - 1) / t3);
}

// Work items of a block's x1 faces: with the linear tile shape, workgroups
// of the shared-edge sweep (sweep_x1: BLOCK / 64 wavefronts of 63 new zones
// each over the zones i in [-1, n1], j in [-1, n2], k in [-1, n3]); with a
// t1 x t2 x t3 shape, tiles of faces.
__host__ __device__ inline int x1_items(const BlockView& b) {
  if (b.t1 == 0) {
    const long n1z = (long)(b.g.n1 + 2) * (b.g.n2 + 2) * (b.g.n3 + 2);
    return (int)(((n1z + 62) / 63 + BLOCK / 64 - 1) / (BLOCK / 64));
  }
  return tiles_of(phase_box(b.g, PH_FLUX, 1), b.t1, b.t2, b.t3);
}

// Work items of a block in a phase (the flux phase holds all three directions).
__host__ __device__ inline int block_items(const BlockView& b, int ph) {
  if (ph == PH_FLUX)
    return x1_items(b) + tiles_of(phase_box(b.g, PH_FLUX, 2), b.t1, b.t2, b.t3) +
           tiles_of(phase_box(b.g, PH_FLUX, 3), b.t1, b.t2, b.t3);
  return tiles_of(phase_box(b.g, ph, 0), b.t1, b.t2, b.t3);
}

// Position of this thread in tile `lt` of box b, if inside.
__device__ __forceinline__ bool tile_pos(const Box& b, int t1, int t2, int t3, int lt, int& i, int& j,
                                         int& k) {
  if (t1 == 0) {  // 32-bit index arithmetic: a block's boxes hold far fewer than 2^31 positions
    const unsigned t = (unsigned)lt * BLOCK + threadIdx.x;
    const unsigned n1 = (unsigned)b.n1, n12 = n1 * (unsigned)b.n2;
    if (t >= n12 * (unsigned)b.n3) return false;
    const unsigned kk = t / n12, r = t - kk * n12, jj = r / n1;
    i = b.lo1 + (int)(r - jj * n1);
    j = b.lo2 + (int)jj;
    k = b.lo3 + (int)kk;
    return true;
  }
  int nt1 = (b.n1 + t1 - 1) / t1, nt2 = (b.n2 + t2 - 1) / t2;
  int a = lt % nt1, rest = lt / nt1;
  int bb = rest % nt2, cc = rest / nt2;
  int th = threadIdx.x;
  int x = th % t1, y = (th / t1) % t2, z = th / (t1 * t2);
  int ii = a * t1 + x, jj = bb * t2 + y, kk = cc * t3 + z;
  if (z >= t3 || ii >= b.n1 || jj >= b.n2 || kk >= b.n3) return false;
  i = b.lo1 + ii;
  j = b.lo2 + jj;
  k = b.lo3 + kk;
  return true;
}

// One work item of a block's flux phase: x1 faces, then x2, then x3.  With
// LINEAR every block of the pack uses the linear tile shape (the x1 faces
// from the sweep), which keeps the general tile arithmetic out of the
// kernel.
template <int RECON, bool LINEAR>
__device__ __forceinline__ void pack_flux_item(const BlockView& b, const double* __restrict__ Pin, int lt) {
  const Dev& g = b.g;
  const int t1 = LINEAR ? 0 : b.t1, t2 = LINEAR ? 0 : b.t2, t3 = LINEAR ? 0 : b.t3;
  int i, j, k;
  const int n1t = x1_items(b);
  if (lt < n1t) {
    if (LINEAR || t1 == 0) {  // every thread of the workgroup takes part (cross-lane shift)
      sweep_x1<RECON, double, double, false>(g, (unsigned)lt, Pin, b.tabF1, b.F[0], nullptr);
      return;
    }
    if (tile_pos(phase_box(g, PH_FLUX, 1), t1, t2, t3, lt, i, j, k))
      flux_face<1, RECON, double, double>(g, Pin, b.tabF1, b.F[0], i, j, k);
    return;
  }
  lt -= n1t;
  const Box b2 = phase_box(g, PH_FLUX, 2);
  const int n2t = tiles_of(b2, t1, t2, t3);
  if (lt < n2t) {
    if (tile_pos(b2, t1, t2, t3, lt, i, j, k)) flux_face<2, RECON, double, double>(g, Pin, b.tabF2, b.F[1], i, j, k);
    return;
  }
  lt -= n2t;
  if (tile_pos(phase_box(g, PH_FLUX, 3), t1, t2, t3, lt, i, j, k))
    flux_face<3, RECON, double, double>(g, Pin, b.tabC, b.F[2], i, j, k);
}

// Block of a work item: the last block whose item offset is <= item.
__device__ __forceinline__ int find_block(const int* __restrict__ pre, int nb, int item) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (pre[mid] <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Work item of this workgroup in a phase (pre holds, per phase, nb + 1 item
// offsets, the last being the phase's total, which is the launch's
// workgroup count): its block and its item within that block.
__device__ __forceinline__ int pack_item(int nb, const int* __restrict__ pre, int ph, int& lt) {
  const int* p = pre + ph * (nb + 1);
  const int item = (int)xcd_order(blockIdx.x, gridDim.x);
  const int blk = find_block(p, nb, item);
  lt = item - p[blk];
  return blk;
}

template <int STAGE, int RECON, bool LINEAR>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(FLUX_WAVES, 8)))
k_pack_flux(const BlockView* __restrict__ bv, int nb, const int* __restrict__ pre) {
  int lt;
  const BlockView& b = bv[pack_item(nb, pre, PH_FLUX, lt)];
  pack_flux_item<RECON, LINEAR>(b, STAGE == 1 ? b.P : b.P1, lt);
}

__global__ void __launch_bounds__(BLOCK) k_pack_emf(const BlockView* __restrict__ bv, int nb,
                                                    const int* __restrict__ pre) {
  int lt, i, j, k;
  const BlockView& b = bv[pack_item(nb, pre, PH_EMF, lt)];
  if (tile_pos(phase_box(b.g, PH_EMF, 0), b.t1, b.t2, b.t3, lt, i, j, k))
    emf_edge<double>(b.g, b.F[0], b.F[1], b.F[2], b.E[0], b.E[1], b.E[2], i, j, k);
}

template <int STAGE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(UPDATE_WAVES, 8)))
k_pack_update(const BlockView* __restrict__ bv, int nb, const int* __restrict__ pre, double dt,
              unsigned long long* fails) {
  int lt, i, j, k;
  const BlockView& b = bv[pack_item(nb, pre, PH_UPDATE, lt)];
  if (tile_pos(phase_box(b.g, PH_UPDATE, 0), b.t1, b.t2, b.t3, lt, i, j, k))
    update_zone<STAGE, double>(b.g, STAGE == 1 ? b.P : b.P1, STAGE == 1 ? b.P1 : b.P, b.V, b.F[0], b.F[1],
                               b.F[2], b.E[0], b.E[1], b.E[2], b.tabC, b.dgs, dt, fails, nullptr, i, j, k);
}

// Ghost exchange between the blocks of a pack (the blocks tile part or all
// of one global grid).  Grid: x over the padded positions of the largest
// block, y over blocks.  A ghost zone of block b at global position G (its
// local position plus the block offset) takes the value the single global
// grid would hold there: G is mapped by the global boundary conditions
// (periodic, outflow, polar mirror with u~2 and B2 flipped; frozen axes and
// zones no block owns keep their values) to a global interior zone, whose
// owner block supplies it.  Reads touch interior zones only and writes ghost
// zones only, so no value read here is written here.
struct PackGlobal {
  int n1, n2, n3;
  int bc[6];
};

__global__ void __launch_bounds__(BLOCK) k_pack_exchange(const BlockView* __restrict__ views,
                                                         const int* __restrict__ owner, PackGlobal G,
                                                         int stage) {
  const BlockView& b = views[blockIdx.y];
  const long t = blockIdx.x * (long)BLOCK + threadIdx.x;
  if (t >= b.g.nz) return;
  const int s1 = b.g.s1;
  const int i = (int)(t % s1) - NG, j = (int)((t / s1) % s1) - NG, k = (int)(t / b.g.plane) - NG;
  const int n = b.g.n1;
  if (i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n) return;  // interior
  bool f1 = false, f2 = false, f3 = false;
  const int gi = bc_map(i + b.o1, G.n1, G.bc[0], G.bc[1], f1);
  const int gj = bc_map(j + b.o2, G.n2, G.bc[2], G.bc[3], f2);
  const int gk = bc_map(k + b.o3, G.n3, G.bc[4], G.bc[5], f3);
  if (gi < 0 || gi >= G.n1 || gj < 0 || gj >= G.n2 || gk < 0 || gk >= G.n3) return;  // frozen
  const int ob = owner[((long)gk * G.n2 + gj) * G.n1 + gi];
  if (ob < 0) return;  // no block holds that zone
  const BlockView& src = views[ob];
  const long sidx = zid(src.g, gi - src.o1, gj - src.o2, gk - src.o3), didx = zid(b.g, i, j, k);
  const double* Ps = stage == 1 ? src.P : src.P1;
  double* Pd = stage == 1 ? b.P : b.P1;
#pragma unroll
  for (int v = 0; v < NVAR; v++) {
    double x = Ps[v * src.g.nz + sidx];
    if (f2 && (v == U2 || v == B2)) x = -x;
    Pd[v * b.g.nz + didx] = x;
  }
}
