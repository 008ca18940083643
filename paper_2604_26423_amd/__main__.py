"""Command line of the simulator.

  python -m paper_2604_26423_amd            build libqs.so (as `build`)
  python -m paper_2604_26423_amd build
  python -m paper_2604_26423_amd run --n 20 --p 3 --delta 0.6 [options]

`run` simulates one LR-QAOA circuit (Sec. II-B) on the GPU and prints one JSON
line: the configuration, <C>, the norm, r = <C>/C(x*) (eq. 5) from the exact
probabilities and from the shots, the gradient with respect to (gamma_k,
beta_k) when asked for, and the time of each step.  The instance is K_n with
weights drawn i.i.d. uniform on {0.1, ..., 1.0} (numpy default_rng(seed), pairs
in lexicographic order) unless --weights gives a file of n(n-1)/2 integers in
tenths.
"""
import argparse
import json
import sys
import time


def _weights(args, np):
    if args.weights:
        with open(args.weights) as f:
            w = np.array([int(t) for t in f.read().split()], dtype=np.int32)
        return w
    if args.n is None:
        raise SystemExit("run: give --n (and --seed) or --weights")
    m = args.n * (args.n - 1) // 2
    return np.random.default_rng(args.seed).integers(1, 11, size=m, dtype=np.int32)


def _run(args) -> int:
    import numpy as np
    import torch

    from . import Simulator, gate_grad_to_schedule, linear_ramp, to_gate_angles

    if not torch.cuda.is_available():
        raise SystemExit("run needs a GPU")
    w = _weights(args, np)
    dg = args.delta if args.delta_gamma is None else args.delta_gamma
    db = args.delta if args.delta_beta is None else args.delta_beta
    gam, bet = linear_ramp(args.p, dg, db, args.ramp)
    tzz, tx = to_gate_angles(gam, bet, args.convention)
    ms = {}

    def timed(name, fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ms[name] = round((time.perf_counter() - t0) * 1e3, 3)
        return out

    sim = timed("setup_and_cost_diagonal",
                lambda: Simulator(w, args.precision, symmetric=args.symmetric))
    e, nrm = timed("forward", lambda: sim.forward(tzz, tx))
    out = {"config": {"n": sim.n, "seed": None if args.weights else args.seed, "weights": args.weights,
                      "p": args.p, "delta_gamma": dg, "delta_beta": db, "ramp": args.ramp,
                      "convention": args.convention, "precision": args.precision,
                      "symmetric": args.symmetric, "shots": args.shots, "shot_seed": args.shot_seed},
           "exp_c": e, "norm_minus_1": nrm - 1.0, "cmax": sim.cmax / 10.0, "w_total": sim.w_total / 10.0,
           "r_exact": sim.ratio(e)}
    if args.shots > 0:
        shots = timed("sample", lambda: sim.sample(args.shots, args.shot_seed))
        out["r_shots"] = sim.shots_ratio(shots)
    if args.adjoint != "none":
        ea, gzz, gx = timed("forward_plus_adjoint", lambda: sim.adjoint(tzz, tx, mode=args.adjoint))
        dgam, dbet = gate_grad_to_schedule(gzz, gx, args.convention)
        out.update({"adjoint": args.adjoint, "exp_c_adjoint": ea, "d_gamma": list(map(float, dgam)),
                    "d_beta": list(map(float, dbet))})
    out["ms"] = ms
    sim.close()
    print(json.dumps(out))
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2604_26423_amd")
    sub = ap.add_subparsers(dest="cmd")
    sub.add_parser("build", help="compile libqs.so for gfx950")
    r = sub.add_parser("run", help="simulate one LR-QAOA circuit on the GPU")
    r.add_argument("--n", type=int, help="qubits (graph K_n)")
    r.add_argument("--seed", type=int, default=0, help="instance seed of the weight draw")
    r.add_argument("--weights", help="file of n(n-1)/2 integer weights in tenths, lexicographic pairs")
    r.add_argument("--p", type=int, required=True, help="layers")
    r.add_argument("--delta", type=float, default=0.6, help="ramp slope for both gamma and beta")
    r.add_argument("--delta-gamma", type=float, help="ramp slope of gamma (default --delta)")
    r.add_argument("--delta-beta", type=float, help="ramp slope of beta (default --delta)")
    r.add_argument("--ramp", choices=["midpoint", "paper"], default="midpoint")
    r.add_argument("--convention", choices=["paper", "literal"], default="paper")
    r.add_argument("--precision", choices=["c64", "c128"], default="c64")
    r.add_argument("--symmetric", action="store_true", help="store the complement-symmetric half state")
    r.add_argument("--shots", type=int, default=1000)
    r.add_argument("--shot-seed", type=int, default=0)
    r.add_argument("--adjoint", choices=["none", "uncompute", "store"], default="none",
                   help="also compute the gradient with respect to (gamma_k, beta_k)")
    args = ap.parse_args(argv)
    if args.cmd in (None, "build"):
        from .build import build
        print(build())
        return 0
    return _run(args)


if __name__ == "__main__":
    sys.exit(main())
