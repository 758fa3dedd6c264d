"""Oracle side of the precision study, run in spawned worker processes (CPU only)."""
import numpy as np

import oracle as O
import synth

_STATE = {}


def init(n, fs, n_seg, seed_cfg, injections):
    g = O.grid(n, fs)
    Sn = O.psd_bins(n, fs, 40.0)
    k_lo = O.band_lo(n, fs, 40.0)
    rngs = synth.rngs(seed_cfg, n_seg)
    segs = []
    for s in range(n_seg):
        x = synth.coloured_noise(Sn[k_lo: n // 2], g["df"], k_lo, n // 2 + 1, rngs[s], dtype=np.complex128)
        for inj in injections.get(s, []):
            mc, eta = map(float, synth.mc_eta(inj["m1"], inj["m2"]))
            h = O.spa_template(n, fs, 40.0, mc, eta)
            sig = np.sqrt(O.sigma_sq(h, Sn, g["df"]))
            x = synth.inject(x, h, inj["snr"] / sig, inj["phi0"], inj["j0"], n)
        segs.append(x.astype(np.complex64).astype(np.complex128))
    _STATE.update(n=n, fs=fs, Sn=Sn, segs=segs)


def segments():
    return [s.astype(np.complex64) for s in _STATE["segs"]]


def unit(task):
    mc, eta, s, j_gpu = task
    d = _STATE
    out = O.filter_unit(d["n"], d["fs"], 40.0, mc, eta, d["segs"][s], d["Sn"], return_series=True)
    rho = out["series"]
    return {"rho": out["rho"], "j": out["j"], "sigma": out["sigma"],
            "rho_at": {k: float(rho[j]) for k, j in j_gpu.items()}}
