"""The sphere of Sec. 7.2 at the paper's size on one GPU: eps_r = 100, diameter 0.2 m, in a
0.2 m box of 105^3 voxels, c dt = h, FIR3 with delta = 105^3 * 1e-7, and the paper's Gaussian
plane wave (sigma = 2 lm, t0 = 3.42 lm, k = (-1, -1, -sqrt 2)/2, p = (1, 1, -sqrt 2)/2).
The current of the centre voxel is recorded every step, and its tapered magnitude response
(eq:Halpha, the last 20 % of the record rolled off as in Sec. 7.1) is compared with the Mie
series at the centre, |d_1|, for the sphere of equal volume.

Not a pytest module (it runs for minutes): python tests/paper_scale_sphere.py [--steps N]
[--out DIR].  Prints one line per chunk of steps, writes centre_current.npy and summary.json;
--analyse FILE repeats the comparison from a saved record without a GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

TESTS = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(TESTS))
sys.path.insert(0, TESTS)

C0 = 299792458.0


def sphere_problem():
    import workloads as wl
    U, L = 105, 0.2
    h = L / U
    X, Y, Z = wl.voxel_centres(U, U, U)
    centre = 0.5 * U
    inside = (X - centre) ** 2 + (Y - centre) ** 2 + (Z - centre) ** 2 <= (0.5 * U) ** 2
    eps = np.where(inside, 100.0, 1.0)
    sigma = 2.0                                   # lm: metres of c t
    k = np.array([-0.5, -0.5, -np.sqrt(2.0) / 2.0])
    p = np.array([0.5, 0.5, -np.sqrt(2.0) / 2.0])
    # eq:GaussPlaneWave read as amp = 4 E0 / (sigma sqrt(pi)), width = sigma / 4
    wave = wl.PlaneWave(khat=k, pol=p, width=sigma / 4.0, t0=3.42, amp=4.0 / (sigma * np.sqrt(np.pi)),
                        r_ref=np.zeros(3))
    fir = wl.binomial_highpass(3, U ** 3 * 1e-7)
    return wl.Problem("sphere105", U, U, U, eps, [wave], 0, fir=fir, h=h, c_dt=h), inside


def analyse(J, prob, inside, fmax_hz=750e6):
    """Tapered magnitude response of the centre current against |d_1| of the equal-volume sphere.
    Above about 750 MHz the incident spectrum falls below 1e-8 of its peak and the ratio shows
    the march's rounding rather than the response, so the band stops there."""
    import mie_series as mie
    from paper_2407_03323_amd import spectral
    h = prob.h
    a_eq = h * (3.0 * inside.sum() / (4.0 * np.pi)) ** (1.0 / 3.0)
    fhz = np.linspace(50e6, fmax_hz, 2801)
    f = fhz / C0
    H = spectral.magnitude_response(J, h, 100.0, prob.waves[0].amp, prob.waves[0].width, f)
    Ht = np.sqrt((H ** 2).sum(axis=1))
    Hm = np.abs([mie.centre_field(100.0, 2.0 * np.pi * fi * a_eq) for fi in f])

    # resonances of the series; the march's counterpart is its largest value within 7 % (the
    # record's truncation adds side lobes 1/T apart, so local maxima alone would not do)
    pm = np.where((Hm[1:-1] > Hm[:-2]) & (Hm[1:-1] >= Hm[2:]))[0] + 1
    pg = []
    for i in pm:
        win = np.where(np.abs(fhz - fhz[i]) <= 0.07 * fhz[i])[0]
        pg.append(int(win[np.argmax(Ht[win])]))
    # amplitude of the ringing centre current over the last 90 % of the record: its decay time
    env = [np.abs(J[i:i + 2000]).max() for i in range(len(J) // 10, len(J) - 2000, 2000)]
    tau_m = (len(env) - 1) * 2000 * h / np.log(env[0] / env[-1]) if env[-1] < env[0] else float("inf")
    out = {"steps": int(len(J)), "a_eq_m": a_eq, "band_MHz": [50.0, fmax_hz / 1e6],
           "record_lm": len(J) * h, "resolution_MHz": C0 / (len(J) * h) / 1e6,
           "ringing_decay_time_lm": tau_m,
           "mie_peaks_MHz": [float(fhz[i] / 1e6) for i in pm], "mie_peak_values": [float(Hm[i]) for i in pm],
           "march_peaks_MHz": [float(fhz[i] / 1e6) for i in pg], "march_peak_values": [float(Ht[i]) for i in pg]}
    for q in range(min(len(pm), len(pg))):
        out["peak%d_shift" % (q + 1)] = float((fhz[pg[q]] - fhz[pm[q]]) / fhz[pm[q]])
    lo = fhz <= 150e6
    out["max_rel_err_50_150MHz"] = float(np.max(np.abs(Ht[lo] - Hm[lo]) / Hm[lo]))
    return out, np.stack([fhz, Ht, Hm], axis=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=52500)       # 100 lm
    ap.add_argument("--chunk", type=int, default=500)
    ap.add_argument("--out", default="sphere105_out")
    ap.add_argument("--analyse", default=None, help="analyse a saved centre_current.npy instead of marching")
    args = ap.parse_args()
    prob, inside = sphere_problem()
    U = prob.U
    os.makedirs(args.out, exist_ok=True)
    if args.analyse:
        J = np.load(args.analyse)
    else:
        import torch
        from paper_2407_03323_amd import solver_for
        t0 = time.time()
        s = solver_for(prob)
        print("setup %.2f s, ell %d, %d voxels inside" % (time.time() - t0, s.ell, inside.sum()), flush=True)
        ic = U // 2
        Jt = torch.zeros((args.chunk, 1, 3, U, U, U), dtype=torch.float64, device="cuda")
        rec = []
        done = 0
        t1 = time.time()
        while done < args.steps:
            n = min(args.chunk, args.steps - done)
            s.run(n, Jt[:n])
            rec.append(Jt[:n, 0, :, ic, ic, ic].cpu().numpy())
            done += n
            print("steps %d  %.1f s  |J_c| %.3e" % (done, time.time() - t1, np.abs(rec[-1]).max()), flush=True)
        s.close()
        J = np.concatenate(rec)
        np.save(os.path.join(args.out, "centre_current.npy"), J)
    out, resp = analyse(J, prob, inside)
    with open(os.path.join(args.out, "summary.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    np.save(os.path.join(args.out, "response.npy"), resp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
