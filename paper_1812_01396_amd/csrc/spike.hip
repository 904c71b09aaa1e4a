// Step 1 through partitions and the recursive SPIKE merge (Sec. 3B: the partitioned pre-processing and
// its recursive merge, which distribute one device over several GPUs in the paper).
//
// The nb blocks of a device are cut into p = nparts consecutive partitions.  Every partition j is a
// closed device of its own, A_j (the blocks of A on its rows, without the couplings to its neighbours),
// with the absorbing shift i*absorb*I of Step 1 on both of its end blocks (the device's own ends and the
// cuts alike: at a cut it broadens the resonances of the closed partition as it does at the device's
// ends, and the merge below takes it out again).  Alg. 1 gives the first and last block columns of
// A_j^{-1} for all partitions of all instances in one lockstep batch (p times as many systems, nb/p steps
// each).  Adjacent partitions a (above) and b (below) are then merged into the first and last block
// columns of their union, level by level (log2 p levels):
//
//   with C = A_{la,fb} (la = last block of a, fb = first block of b), B = A_{fb,la} = C^H, and the corner
//   blocks Ga_LL = (A_a^{-1})_{la,la}, Ga_LF = (A_a^{-1})_{la,fa}, Gb_FF = (A_b^{-1})_{fb,fb},
//   Gb_FL = (A_b^{-1})_{fb,lb}, the union is D + U K U^T with D = diag(A_a, A_b), U the block selector of
//   rows (la, fb) and K = [[-i absorb I, C], [B, -i absorb I]] (the couplings, and the shifts of the two
//   cut blocks removed); the Woodbury identity in the form
//   M^{-1} = D^{-1} - D^{-1} U K (I + W K)^{-1} U^T D^{-1}, W = U^T D^{-1} U = diag(Ga_LL, Gb_FF), needs no
//   inverse of K.  With Z = I + W K = [[I - i absorb Ga_LL, Ga_LL C], [Gb_FF B, I - i absorb Gb_FF]] and
//       [Y | Y'] = Z^{-1} [[Ga_LF, 0], [0, Gb_FL]]                 (one LU solve of order 2s)
//       V = K [Y | Y'] = [[C Y_2 - i absorb Y_1, ...], [B Y_1 - i absorb Y_2, ...]]
//                                                                   (Y_1, Y_2: the top and bottom s rows)
//   the merged columns are, on the rows of a:  [Qa_F - Qa_L V_11, -Qa_L V_12]
//                             on the rows of b:  [-Qb_F V_21, Qb_L - Qb_F V_22]
//   (Q_F, Q_L: first and last block columns of the partition's inverse on its own rows).
// Each level reads one Q buffer and writes the other (no update in place); the partition recursion
// starts in the buffer that makes the last level end in the caller's Q.
#include <algorithm>
#include <climits>
#include <vector>

#include "drivers.hpp"
#include "lu.hpp"
#include "tile.hpp"

namespace ss {

using SpikeTile = TileCfg<64, 64, 16, 2, 2>;

struct SpikePair {
  int inst, a0, la, b1;  // instance; partition a = blocks [a0, la], b = blocks [la + 1, b1)
};

struct SpikeArgs {
  const double2 *Hu, *Su;   // upper blocks of the (H, S) sets
  long kstride_u;
  const int *kidx;
  const double *E;
  double absorb;            // shift of the cut blocks, removed by the merge
  int nk, nb, s;
  const SpikePair *pairs;   // [npairs] of this level
  const double2 *Qs;        // source columns [batch][nb][s][2s]
  double2 *Qd;              // destination columns
  double2 *Maug;            // [npairs][2s][4s]: [Z | RHS]
  double2 *Y;               // [npairs][2s][2s]
  double2 *V;               // [npairs][2s][2s]
};

__device__ __forceinline__ int spike_set(const SpikeArgs &a, int inst) {
  const int k = a.kidx ? a.kidx[inst] : inst % a.nk;
  return min(max(k, 0), a.nk - 1);
}

// Per partition e of the lockstep batch: the block pointers of its instance's set, offset to its first
// block, and its energy.
__global__ void k_spike_tables(const double2 *Hd, const double2 *Hu, const double2 *Sd, const double2 *Su,
                               long kstride_d, long kstride_u, const int *kidx, int nk, const double *E, int s,
                               const int *pinst, const int *pstart, int n, const double2 **tab, double *Ep) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int inst = pinst[e];
  int k = kidx ? kidx[inst] : inst % nk;
  k = min(max(k, 0), nk - 1);
  const long off = (long)pstart[e] * s * s;
  tab[4 * e + 0] = Hd + k * kstride_d + off;
  tab[4 * e + 1] = Hu + k * kstride_u + off;
  tab[4 * e + 2] = Sd + k * kstride_d + off;
  tab[4 * e + 3] = Su + k * kstride_u + off;
  Ep[e] = E[inst];
}

// [Z | RHS] of every pair, one 64 x 64 tile of the 2s x 4s matrix per workgroup; grid (8 tiles^2, npairs)
__global__ void __launch_bounds__(SpikeTile::NT) SS_TILE_WAVES k_spike_form(SpikeArgs a) {
  using T = SpikeTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int p = blockIdx.y, s = a.s;
  const SpikePair pr = a.pairs[p];
  const int tiles = cdiv(s, T::BM);
  const int t = blockIdx.x;
  const int qr = t / (4 * tiles * tiles);          // quadrant row 0 / 1 (rows of a / b)
  const int rem = t % (4 * tiles * tiles);
  const int qc = rem / (tiles * tiles);            // quadrant column 0..3 (Z left, Z right, RHS left, right)
  const int tt = rem % (tiles * tiles);
  const int m0 = (tt / tiles) * T::BM, n0 = (tt % tiles) * T::BN;
  const long ss2 = (long)s * s, ldq = 2L * s, ldm = 4L * s;
  const double2 *q = a.Qs + (long)pr.inst * a.nb * s * ldq;
  double2 *M = a.Maug + (long)p * 2 * s * ldm + (long)qr * s * ldm + (long)qc * s;
  const int ks = spike_set(a, pr.inst);
  const double e = a.E[pr.inst];
  const double2 *hu = a.Hu + ks * a.kstride_u + pr.la * ss2, *su = a.Su + ks * a.kstride_u + pr.la * ss2;
  auto put = [&](int r, int c, double2 v) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < s) M[(long)gr * ldm + gc] = v;
  };
  const bool product = (qr == 0 && qc == 1) || (qr == 1 && qc == 0);
  if (product) {
    Acc<T> acc;
    acc.zero();
    if (qr == 0) {  // Ga_LL C: row block la of a's last column, C = A_{la,la+1}
      LdRow la{q + (long)pr.la * s * ldq + s, ldq};
      LdForm<false> lb{hu, su, s, e};
      mma_loop<T>(la, lb, m0, s, n0, s, 0, s, acc, lds);
    } else {  // Gb_FF B: row block fb of b's first column, B = C^H
      LdRow la{q + (long)(pr.la + 1) * s * ldq, ldq};
      LdForm<true> lb{hu, su, s, e};
      mma_loop<T>(la, lb, m0, s, n0, s, 0, s, acc, lds);
    }
    acc_foreach<T>(acc, put);
    return;
  }
  for (int idx = threadIdx.x; idx < T::BM * T::BN; idx += T::NT) {
    const int r = idx / T::BN, c = idx % T::BN, gr = m0 + r, gc = n0 + c;
    if (gr >= s || gc >= s) continue;
    double2 v = make_double2(0.0, 0.0);
    if ((qr == 0 && qc == 0) || (qr == 1 && qc == 1)) {  // I - i absorb G (G = Ga_LL or Gb_FF)
      const double2 g = qr == 0 ? q[(long)pr.la * s * ldq + (long)gr * ldq + s + gc]
                                : q[(long)(pr.la + 1) * s * ldq + (long)gr * ldq + gc];
      v = make_double2((gr == gc ? 1.0 : 0.0) + a.absorb * g.y, -a.absorb * g.x);
    }
    else if (qr == 0 && qc == 2) v = q[(long)pr.la * s * ldq + (long)gr * ldq + gc];            // Ga_LF
    else if (qr == 1 && qc == 3) v = q[(long)(pr.la + 1) * s * ldq + (long)gr * ldq + s + gc];  // Gb_FL
    M[(long)gr * ldm + gc] = v;
  }
}

// V = K Y = [[C Y_2 - i absorb Y_1], [B Y_1 - i absorb Y_2]] (2s x 2s); grid (2 tiles * 2 tiles, npairs)
__global__ void __launch_bounds__(SpikeTile::NT) SS_TILE_WAVES k_spike_v(SpikeArgs a) {
  using T = SpikeTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int p = blockIdx.y, s = a.s;
  const SpikePair pr = a.pairs[p];
  const int tr = cdiv(s, T::BM), tc = cdiv(2 * s, T::BN);
  const int half = blockIdx.x / (tr * tc), rem = blockIdx.x % (tr * tc);
  const int m0 = (rem / tc) * T::BM, n0 = (rem % tc) * T::BN;
  const long ss2 = (long)s * s, ld = 2L * s;
  const int ks = spike_set(a, pr.inst);
  const double e = a.E[pr.inst];
  const double2 *hu = a.Hu + ks * a.kstride_u + pr.la * ss2, *su = a.Su + ks * a.kstride_u + pr.la * ss2;
  const double2 *y = a.Y + (long)p * 2 * s * ld;
  double2 *v = a.V + (long)p * 2 * s * ld + (long)half * s * ld;
  // the diagonal blocks of K: -i absorb times the other half of Y (top: Y_1, bottom: Y_2)
  const double2 *yd = y + (long)half * s * ld;
  Acc<T> acc;
  acc.zero();
  if (half == 0) {  // C Y_2
    LdForm<false> la{hu, su, s, e};
    LdRow lb{y + (long)s * ld, ld};
    mma_loop<T>(la, lb, m0, s, n0, 2 * s, 0, s, acc, lds);
  } else {  // B Y_1
    LdForm<true> la{hu, su, s, e};
    LdRow lb{y, ld};
    mma_loop<T>(la, lb, m0, s, n0, 2 * s, 0, s, acc, lds);
  }
  acc_foreach<T>(acc, [&](int r, int c, double2 x) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < s && gc < 2 * s) {
      const double2 d = yd[(long)gr * ld + gc];
      v[(long)gr * ld + gc] = make_double2(x.x + a.absorb * d.y, x.y - a.absorb * d.x);
    }
  });
}

// Merged columns of every pair from the source buffer into the destination; grid (row tiles of the
// largest pair * column tiles of 2s, npairs).  Rows of a read their last column (times V's top rows),
// rows of b their first column (times V's bottom rows).
__global__ void __launch_bounds__(SpikeTile::NT) SS_TILE_WAVES k_spike_update(SpikeArgs a) {
  using T = SpikeTile;
  __shared__ double lds[T::LDS_DOUBLES];
  const int p = blockIdx.y, s = a.s;
  const SpikePair pr = a.pairs[p];
  const long ld = 2L * s;
  const int rows_a = (pr.la + 1 - pr.a0) * s, rows_b = (pr.b1 - pr.la - 1) * s;
  const int ta = cdiv(rows_a, T::BM), tb = cdiv(rows_b, T::BM), tc = cdiv(2 * s, T::BN);
  const int rt = blockIdx.x / tc, n0 = (blockIdx.x % tc) * T::BN;
  if (rt >= ta + tb) return;
  const bool in_a = rt < ta;
  const int m0 = (in_a ? rt : rt - ta) * T::BM;
  const int rows = in_a ? rows_a : rows_b;
  const long base = ((long)pr.inst * a.nb + (in_a ? pr.a0 : pr.la + 1)) * s;  // first global row
  const double2 *src = a.Qs + base * ld;
  double2 *dst = a.Qd + base * ld;
  const double2 *v = a.V + (long)p * 2 * s * ld + (in_a ? 0 : (long)s * ld);
  Acc<T> acc;
  acc.zero();
  LdRow la{src + (in_a ? s : 0), ld};
  LdRow lb{v, ld};
  mma_loop<T>(la, lb, m0, rows, n0, 2 * s, 0, s, acc, lds);
  acc_foreach<T>(acc, [&](int r, int c, double2 x) {
    const int gr = m0 + r, gc = n0 + c;
    if (gr < rows && gc < 2 * s) {
      const bool keep = in_a ? gc < s : gc >= s;  // the column the partition already had
      const double2 old = keep ? src[(long)gr * ld + gc] : make_double2(0.0, 0.0);
      dst[(long)gr * ld + gc] = csub(old, x);
    }
  });
}

// info of every instance: the smallest code over its partitions (shifted to global block numbers) and
// over the interface systems of its merges (1 + la * s + c for an exact zero pivot in column c of the
// interface system after block la).
__global__ void k_spike_info_init(int *info, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch) info[i] = INT_MAX;
}
__global__ void k_spike_info_parts(const int *pinfo, const int *pinst, const int *pstart, int n, int s, int *info) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n || pinfo[e] == 0) return;
  atomicMin(info + pinst[e], pinfo[e] + pstart[e] * s);
}
__global__ void k_spike_info_pairs(const int *zp, const SpikePair *pairs, int n, int s, int *info) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || zp[p] == 0) return;
  atomicMin(info + pairs[p].inst, pairs[p].la * s + zp[p]);
}
__global__ void k_spike_info_finish(int *info, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch && info[i] == INT_MAX) info[i] = 0;
}

ss_status precompute_spike(ss_ctx *ctx, const ss_btd *hs, int batch, const int *kidx, const double *E, double absorb,
                           int prec, int nparts, ss_c128 *Q, int *info) {
  const int s = hs->s, nb = hs->nb, p = nparts;
  int levels = 0;
  while ((1 << levels) < p) ++levels;
  const long ss2 = (long)s * s;
  // partitions: the first nb % p of them one block longer; entries sorted by length (longest first,
  // as the lockstep recursion expects), instance-major within a length
  std::vector<int> start(p + 1, 0);
  for (int j = 0; j < p; ++j) start[j + 1] = start[j] + nb / p + (j < nb % p ? 1 : 0);
  const int n = batch * p;
  std::vector<int> pinst, pstart, nbv;
  std::vector<long> boff, xoff;
  for (int pass = 0; pass < 2; ++pass)
    for (int i = 0; i < batch; ++i)
      for (int j = 0; j < p; ++j) {
        const int len = start[j + 1] - start[j];
        if ((pass == 0) != (len == nb / p + 1 && nb % p != 0)) continue;
        pinst.push_back(i);
        pstart.push_back(start[j]);
        nbv.push_back(len);
        const long g = (long)i * nb + start[j];  // global first block: Q rows and recursion slots
        boff.push_back(g);
        xoff.push_back(2 * g * ss2);
        xoff.push_back((2 * g + len) * ss2);
      }
  // pair tables of every level (host), block ranges of the partitions at each level
  std::vector<std::vector<SpikePair>> lv(levels);
  for (int l = 0; l < levels; ++l) {
    const int width = 1 << (l + 1);  // partitions of the original cut per merged partition
    for (int i = 0; i < batch; ++i)
      for (int j = 0; j < p; j += width) {
        SpikePair pr;
        pr.inst = i;
        pr.a0 = start[j];
        pr.la = start[j + width / 2] - 1;
        pr.b1 = start[j + width];
        lv[l].push_back(pr);
      }
  }
  const int npmax = batch * p / 2;
  // device workspace: tables, partition infos, the second Q buffer, [Z | RHS], Y, V, the interface LU
  const size_t b_tab = sizeof(void *) * 4 * n, b_int = sizeof(int) * (4 * (size_t)n + std::max(npmax, 1));
  const size_t b_long = sizeof(long) * 3 * (size_t)n, b_e = sizeof(double) * n;
  const size_t b_pairs = sizeof(SpikePair) * (size_t)std::max(1, batch * (p - 1));
  const size_t b_q = sizeof(double2) * (size_t)batch * nb * s * 2 * s;
  const size_t b_aug = sizeof(double2) * (size_t)npmax * 2 * s * 4 * s;
  const size_t b_y = sizeof(double2) * (size_t)npmax * 4 * ss2;
  const size_t b_perm = sizeof(int) * (size_t)npmax * 2 * s;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t total = al(b_tab) + al(b_int) + al(b_long) + al(b_e) + al(b_pairs) + al(b_q) + al(b_aug) +
                       2 * al(b_y) + al(b_perm);
  void *w;
  SS_TRY(workspace(ctx, kSlotSpike, total, &w));
  char *cp = (char *)w;
  auto take = [&](size_t b) { char *r = cp; cp += al(b); return r; };
  const double2 **tab = (const double2 **)take(b_tab);
  int *ip = (int *)take(b_int);
  int *d_pinst = ip, *d_pstart = ip + n, *d_nbv = ip + 2 * n, *pinfo = ip + 3 * n, *d_zp = ip + 4 * n;
  long *lp = (long *)take(b_long);
  long *d_boff = lp, *d_xoff = lp + n;
  double *d_E = (double *)take(b_e);
  SpikePair *d_pairs = (SpikePair *)take(b_pairs);
  double2 *Qtmp = (double2 *)take(b_q);
  double2 *Maug = (double2 *)take(b_aug);
  double2 *Y = (double2 *)take(b_y);
  double2 *V = (double2 *)take(b_y);
  int *perm = (int *)take(b_perm);
  std::vector<SpikePair> allpairs;
  std::vector<size_t> pair_off;
  for (int l = 0; l < levels; ++l) {
    pair_off.push_back(allpairs.size());
    allpairs.insert(allpairs.end(), lv[l].begin(), lv[l].end());
  }
  if (hipMemcpyAsync(d_pinst, pinst.data(), sizeof(int) * n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(d_pstart, pstart.data(), sizeof(int) * n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(d_nbv, nbv.data(), sizeof(int) * n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(d_boff, boff.data(), sizeof(long) * n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(d_xoff, xoff.data(), sizeof(long) * 2 * n, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
      (!allpairs.empty() && hipMemcpyAsync(d_pairs, allpairs.data(), sizeof(SpikePair) * allpairs.size(),
                                           hipMemcpyHostToDevice, ctx->stream) != hipSuccess))
    return fail(ctx, SS_ERR_DEVICE, "precompute_spike: table upload failed");
  const long kstride_d = (long)nb * ss2, kstride_u = (long)std::max(nb - 1, 0) * ss2;
  hipLaunchKernelGGL(k_spike_tables, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, (const double2 *)hs->H_diag,
                     (const double2 *)hs->H_upper, (const double2 *)hs->S_diag, (const double2 *)hs->S_upper,
                     kstride_d, kstride_u, kidx, hs->nk, E, s, (const int *)d_pinst, (const int *)d_pstart, n, tab,
                     d_E);
  // the partitions' own first and last columns (Alg. 1 on every partition, all in one lockstep batch)
  // (every partition carries the absorbing shift at both ends: the merges take the shifts of the cuts out)
  RaggedBatch rb;
  rb.s = s;
  rb.batch = n;
  rb.nb_max = nbv[0];
  rb.total_blocks = (long)batch * nb;
  rb.tab = (const ss_c128 *const *)tab;
  rb.nbv = d_nbv;
  rb.boff = d_boff;
  rb.xoff = d_xoff;
  rb.E = d_E;
  rb.act.assign(rb.nb_max, 0);
  for (int e = 0; e < n; ++e)
    for (int t = 0; t < nbv[e]; ++t) rb.act[t] = e + 1;
  double2 *bufs[2] = {(double2 *)Q, Qtmp};
  int cur = levels % 2;  // the buffer the recursion writes; after `levels` swaps the result is in Q
  SS_TRY(precompute_ragged(ctx, rb, absorb, prec, (ss_c128 *)bufs[cur], pinfo));
  if (info) {
    hipLaunchKernelGGL(k_spike_info_init, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, info, batch);
    hipLaunchKernelGGL(k_spike_info_parts, dim3(cdiv(n, 256)), dim3(256), 0, ctx->stream, (const int *)pinfo,
                       (const int *)d_pinst, (const int *)d_pstart, n, s, info);
  }
  // merges
  SpikeArgs a;
  a.Hu = (const double2 *)hs->H_upper;
  a.Su = (const double2 *)hs->S_upper;
  a.kstride_u = kstride_u;
  a.kidx = kidx;
  a.E = E;
  a.absorb = absorb;
  a.nk = hs->nk;
  a.nb = nb;
  a.s = s;
  a.Maug = Maug;
  a.Y = Y;
  a.V = V;
  using T = SpikeTile;
  const int tiles = cdiv(s, T::BM);
  for (int l = 0; l < levels; ++l) {
    const int np = (int)lv[l].size();
    a.pairs = d_pairs + pair_off[l];
    a.Qs = bufs[cur];
    a.Qd = bufs[1 - cur];
    hipLaunchKernelGGL(k_spike_form, dim3(8 * tiles * tiles, np), dim3(T::NT), 0, ctx->stream, a);
    LuDesc d;
    d.nmat = np;
    d.n = 2 * s;
    d.nrhs = 2 * s;
    d.M = Maug;
    d.sM = (long)2 * s * 4 * s;
    d.ldm = 4 * s;
    d.perm = perm;
    d.sP = 2 * s;
    d.zp = d_zp;
    d.X = Y;
    d.sX = 4 * ss2;
    d.ldx = 2 * s;
    SS_TRY(lu_identity_perm(ctx, d));
    SS_TRY(lu_solve(ctx, d));
    if (info)
      hipLaunchKernelGGL(k_spike_info_pairs, dim3(cdiv(np, 256)), dim3(256), 0, ctx->stream, (const int *)d_zp,
                         (const SpikePair *)a.pairs, np, s, info);
    hipLaunchKernelGGL(k_spike_v, dim3(2 * tiles * cdiv(2 * s, T::BN), np), dim3(T::NT), 0, ctx->stream, a);
    int rmax = 0;
    for (const SpikePair &pr : lv[l])
      rmax = std::max(rmax, cdiv((pr.la + 1 - pr.a0) * s, T::BM) + cdiv((pr.b1 - pr.la - 1) * s, T::BM));
    hipLaunchKernelGGL(k_spike_update, dim3(rmax * cdiv(2 * s, T::BN), np), dim3(T::NT), 0, ctx->stream, a);
    cur = 1 - cur;
  }
  if (info) hipLaunchKernelGGL(k_spike_info_finish, dim3(cdiv(batch, 256)), dim3(256), 0, ctx->stream, info, batch);
  return check_launch(ctx, "precompute_spike");
}

}  // namespace ss
