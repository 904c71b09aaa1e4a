"""Writes tests/golden/<workload>_transmission.txt: the oracle's transmission for every instance of a
lattice-slab workload (calls only the oracle and the input generators).

Workloads (perfect crystal devices: nb copies of the cell, leads = the same cell, eta = 1e-8):
  dft512:  the 8x8x8 cell of seed 1, nb = 40, momenta k in {pi/8, 3pi/8, 5pi/8, 7pi/8}, 64 energies
           linspace(-5, 5, 64); instance b has momentum index b // 64 and energy index b % 64 (256).
  dft1024: the 8x8x16 cell of seed 2, nb = 60, k = pi/3, 32 energies linspace(-5, 5, 32) (32).

Per instance the file holds the Caroli pair (T_LR, T_RL) of the oracle's direct solve of the open
system (block Thomas on T = A - Sigma, decimation to 1e-14), the decimation passes, and the number of
right-moving Bloch states N_ch(E) from the lead band structure (a perfect crystal transmits exactly
N_ch up to O(eta)) with the smallest distance of E to a band on the q grid.

    python tests/golden/make_golden_slab.py --workload dft512 [--workers 8] [--dense 2]
    python tests/golden/make_golden_slab.py --workload dft1024 --workers 4 --threads 2

--dense n additionally solves the first n instances of the largest |T - N_ch| densely (numpy's LU of
the assembled open-system matrix, N = nb s) and writes tests/golden/<workload>_dense_check.txt: the
block-Thomas and the dense transmissions side by side (a full-size check of the oracle itself).
"""
import argparse
import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

WORKLOADS = {
    "dft512": dict(s=512, nb=40, seed=1, ks=[np.pi / 8, 3 * np.pi / 8, 5 * np.pi / 8, 7 * np.pi / 8], n_e=64),
    "dft1024": dict(s=1024, nb=60, seed=2, ks=[np.pi / 3], n_e=32),
}
ETA, NQ = 1e-8, 1024
S = NB = SEED = None
KS = ENERGIES = OUT = DENSE_OUT = None


def _configure(name):
    global S, NB, SEED, KS, ENERGIES, OUT, DENSE_OUT
    w = WORKLOADS[name]
    S, NB, SEED, KS = w["s"], w["nb"], w["seed"], w["ks"]
    ENERGIES = np.linspace(-5.0, 5.0, w["n_e"])
    OUT = os.path.join(HERE, f"{name}_transmission.txt")
    DENSE_OUT = os.path.join(HERE, f"{name}_dense_check.txt")


def _init_worker(name, threads):
    _configure(name)
    import threadpoolctl
    threadpoolctl.threadpool_limits(threads)

_cells = {}


def _cell(ki):
    import synth

    if ki not in _cells:
        _cells[ki] = synth.DFTLikeCell(synth.SLAB_SHAPES[S], SEED).at(KS[ki])
    return _cells[ki]


def _solve(b):
    import synth
    from oracle import transport

    ki, ei = divmod(b, len(ENERGIES))
    inst = synth.device_from_cell(_cell(ki), NB)
    ref = transport.solve_instance(inst.Hd, inst.Hu, inst.Sd, inst.Su, inst.H00, inst.H01, inst.S00, inst.S01,
                                   float(ENERGIES[ei]), ETA, want_q=False)
    return b, ref["t_lr"], ref["t_rl"], ref["iters"]


def _bands(ki):
    from oracle import bands

    q = np.linspace(-np.pi, np.pi, NQ, endpoint=False)
    return ki, bands.bloch_bands(*_cell(ki), q)


def _dense(b):
    from oracle import linalg, selfenergy, transport
    import synth

    ki, ei = divmod(b, len(ENERGIES))
    E = float(ENERGIES[ei])
    inst = synth.device_from_cell(_cell(ki), NB)
    a0, a1, am1 = selfenergy.lead_blocks(inst.H00, inst.H01, inst.S00, inst.S01, E, ETA)
    sig_l, sig_r, _, _ = selfenergy.decimation(a0, a1, am1)
    ad, au, al = transport.device_blocks(inst.Hd, inst.Hu, inst.Sd, inst.Su, E)
    t = linalg.assemble_dense(transport.open_diag(ad, sig_l, sig_r), au, al)
    n = t.shape[0]
    rhs = np.zeros((n, 2 * S), dtype=np.complex128)
    rhs[:S, :S] = np.eye(S)
    rhs[n - S:, S:] = np.eye(S)
    x = np.linalg.solve(t, rhs)
    del t
    gc = np.vstack([x[:S], x[n - S:]])
    return transport.caroli(gc, sig_l, sig_r)


def main():
    from multiprocessing import Pool

    from oracle import bands

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="dft512", choices=sorted(WORKLOADS))
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--threads", type=int, default=1, help="BLAS threads per worker")
    ap.add_argument("--dense", type=int, default=0)
    ap.add_argument("--skip-transport", action="store_true", help="reuse the existing transmission file")
    args = ap.parse_args()
    _configure(args.workload)
    n = len(KS) * len(ENERGIES)
    if not args.skip_transport:
        with Pool(args.workers, initializer=_init_worker, initargs=(args.workload, args.threads)) as pool:
            band_jobs = pool.map_async(_bands, range(len(KS)))  # beside the solves
            rows = {}
            for b, t_lr, t_rl, it in pool.imap_unordered(_solve, range(n)):
                rows[b] = (t_lr, t_rl, it)
                print(f"instance {b}: T_LR {t_lr:.12f} T_RL {t_rl:.12f}", flush=True)
            bb = dict(band_jobs.get())
        lines = ["# b  E  k  T_LR  T_RL  decimation_passes  N_ch  min|E_n(q)-E|",
                 f"# s={S} nb={NB} seed={SEED} eta={ETA:g} crystal device; bands on {NQ} q points"]
        for b in range(n):
            ki, ei = divmod(b, len(ENERGIES))
            nch, gap = bands.channel_count(*_cell(ki), float(ENERGIES[ei]), bands=bb[ki])
            t_lr, t_rl, it = rows[b]
            lines.append(f"{b} {ENERGIES[ei]:.17g} {KS[ki]:.17g} {t_lr:.17g} {t_rl:.17g} {it} {nch} {gap:.3e}")
        with open(OUT, "w") as f:
            f.write("\n".join(lines) + "\n")
    if args.dense > 0:
        tab = np.loadtxt(OUT)
        dev = np.abs(tab[:, 3] - tab[:, 6])
        pick = [int(b) for b in tab[np.argsort(-dev)[: args.dense], 0]]
        import threadpoolctl

        lines = ["# b  T_LR(dense)  T_RL(dense)  T_LR(block Thomas)  T_RL(block Thomas)",
                 f"# dense LU of the assembled open-system matrix (N = {NB * S}) for the instances of largest "
                 "|T - N_ch|"]
        for b in pick:
            with threadpoolctl.threadpool_limits(args.workers):
                t_lr, t_rl = _dense(b)
            row = tab[b]
            lines.append(f"{b} {t_lr:.17g} {t_rl:.17g} {row[3]:.17g} {row[4]:.17g}")
            print(lines[-1], flush=True)
        with open(DENSE_OUT, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
