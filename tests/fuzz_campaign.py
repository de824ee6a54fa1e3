"""Large seeded parity campaign of both solvers against the oracle (GPU).

Not collected by pytest (too long for the suite): run it by name,
    BF_N=1000000 BF_SEEDS=101,102,103 python tests/fuzz_campaign.py
Per seed and model: S over ten decades, T from 1e-7 to 80 years, r from
-0.2 to 0.5, q from -0.1 to 0.4 (BSM), sigma from 1e-5 to 20 and strikes up
to 15 standard deviations out, priced by the oracle; both solvers are
compared with the oracle's exact roots under the parity contract of
tests/_helpers.compare_iv.  The first ten failing quotes of a (seed, model,
solver) are saved as .npy files in $FUZZ_OUT (default ./fuzz_failures).  Prints one line per
(seed, model, solver) and the total of failures."""
import os, sys, time
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import numpy as np, torch
import oracle
import paper_2604_27210_amd as fv
from _helpers import compare_iv, forward_discount
fv._native.load()
dev = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
n = int(os.environ.get("BF_N", "1000000"))
bad_total = 0
for seed in tuple(int(s) for s in os.environ.get("BF_SEEDS", "101,102,103").split(",")):
    for model in ("black76", "bs", "bsm"):
        rng = np.random.default_rng(seed * 10 + len(model))
        S = np.exp(rng.uniform(np.log(1e-4), np.log(1e6), n))
        T = np.exp(rng.uniform(np.log(1e-7), np.log(80.0), n))
        r = rng.uniform(-0.2, 0.5, n)
        q = rng.uniform(-0.1, 0.4, n) if model == "bsm" else np.zeros(n)
        sig = np.exp(rng.uniform(np.log(1e-5), np.log(20.0), n))
        z = rng.uniform(-15, 15, n)
        F, D = forward_discount(model, S, T, r, q)
        K = F * np.exp(-z * sig * np.sqrt(T))
        flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
        P = oracle.price(model, S, K, T, r, q, sig, flag)
        for solver in ("lbr", "halley"):
            t0 = time.time()
            s, st = fv.implied_vol(model, dev(P), dev(S), dev(K), dev(T), dev(r), flag=dev(flag, torch.int8),
                                   q=dev(q) if model == "bsm" else None, solver=solver)
            res = compare_iv(model, solver, P, S, K, T, r, q, flag, s.cpu().numpy(), st.cpu().numpy())
            nb = len(res["status_bad"]) + len(res["value_bad"]) + len(res["nan_bad"])
            bad_total += nb
            print("seed %d %s %s: ok=%d status_bad=%d value_bad=%d nan_bad=%d ambiguous=%d max=%.3f (%.1fs)" % (
                seed, model, solver, res["n_ok"], len(res["status_bad"]), len(res["value_bad"]),
                len(res["nan_bad"]), res["ambiguous"], res["max_ratio"], time.time() - t0), flush=True)
            if nb:
                idx = (list(res["status_bad"]) + list(res["value_bad"]) + list(res["nan_bad"]))[:10]
                idx = np.array(idx, dtype=np.int64)
                out_dir = os.environ.get("FUZZ_OUT", "fuzz_failures")
                os.makedirs(out_dir, exist_ok=True)
                np.save(os.path.join(out_dir, "fuzz_%d_%s_%s.npy" % (seed, model, solver)),
                        np.stack([P[idx], S[idx], K[idx], T[idx], r[idx], q[idx], flag[idx].astype(float)]))
print("total bad", bad_total)
sys.exit(1 if bad_total else 0)
