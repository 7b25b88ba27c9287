"""Readers for the hand-worked fixtures in tests/golden/ (no harmonic-sum arithmetic)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _kv(tokens):
    out = {}
    for t in tokens:
        k, v = t.split("=", 1)
        out[k] = v
    return out


def _ints(s):
    return [int(v) for v in s.split(",") if v != ""]


def read_1d(name="hand_1d.txt"):
    spectra, cases = {}, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "spectrum":
                spectra[tok[1]] = np.array([float(v) for v in tok[2:]], dtype=np.float32)
            elif tok[0] == "case":
                kv = _kv(tok[3:])
                mask = 0 if kv["mask"] == "all" else sum(1 << (k - 1) for k in _ints(kv["mask"]))
                cases.append(dict(spectrum=tok[1], mode=tok[2], H=int(kv["H"]), mask=mask,
                                  n=int(kv["n"]), S=_ints(kv["S"]), harm=int(kv["harm"]),
                                  drift=int(kv["drift"])))
    return spectra, cases


def read_2d(name="hand_2d.txt"):
    rows, cases = {}, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "row":
                rows[int(tok[1])] = [float(v) for v in tok[2:]]
            elif tok[0] == "case":
                kv = _kv(tok[2:])
                cases.append(dict(mode=tok[1], H=int(kv["H"]), r=int(kv["r"]), z=int(kv["z"]),
                                  S=_ints(kv["S"]), harm=int(kv["harm"]), drift=int(kv["drift"])))
    zs = sorted(rows)
    plane = np.array([rows[z] for z in zs], dtype=np.float32)
    return plane, zs[0], zs[-1], cases


def read_presto(name="hand_presto.txt"):
    """Spectra, stage cases and the last-bin examples of the PRESTO-style sums."""
    spectra, cases, lastbins = {}, [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "spectrum":
                spectra[tok[1]] = np.array([float(v) for v in tok[2:]], dtype=np.float32)
            elif tok[0] == "lastbin":
                kv = _kv(tok[1:])
                lastbins.append(dict(n=int(kv["n"]), K=int(kv["K"]), fundamental=int(kv["fundamental"])))
            elif tok[0] == "pcase":
                kv = _kv(tok[3:])
                mask = 0 if kv["mask"] == "all" else sum(1 << (k - 1) for k in _ints(kv["mask"]))
                stages = []
                for s in kv["stages"].split(","):
                    if s:
                        K, S, m = (int(v) for v in s.split(":"))
                        stages.append((K, S, m))
                cases.append(dict(spectrum=tok[1], mode=tok[2], H=int(kv["H"]), mask=mask,
                                  first=int(kv["first"]), n=int(kv["n"]), stages=stages,
                                  harm=int(kv["harm"])))
    return spectra, cases, lastbins


def read_peaks(name="hand_peaks.txt"):
    """Offsets, dense snr / harm and the clustering cases of the peak fixture."""
    off = snr = harm = None
    cases = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "spectra":
                off = np.array(_ints(tok[1]), dtype=np.int64)
            elif tok[0] == "snr":
                snr = np.array([float(v) for v in tok[1:]], dtype=np.float32)
            elif tok[0] == "harm":
                harm = np.array([int(v) for v in tok[1:]], dtype=np.uint8)
            elif tok[0] == "case":
                kv = _kv(tok[1:])
                keep = [tuple(int(v) for v in p.split(":")) for p in kv["keep"].split(",") if p]
                cases.append(dict(threshold=float(kv["threshold"]), radius=int(kv["radius"]), keep=keep))
    return off, snr, harm, cases


def read_candidates(name="hand_candidates.txt"):
    """Powers, offsets and the hand-worked candidate cases at the threshold."""
    offsets, values, cases = None, None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "spectra":
                offsets = np.array(_ints(tok[1]), dtype=np.int64)
            elif tok[0] == "values":
                values = np.array([float(v) for v in tok[1:]], dtype=np.float32)
            elif tok[0] == "case":
                kv = _kv(tok[2:])
                mask = 0 if kv["mask"] == "all" else sum(1 << (k - 1) for k in _ints(kv["mask"]))
                recs = []
                for r in kv["cands"].split(","):
                    if r:
                        s, b, h, d, v = r.split(":")
                        recs.append((int(s), int(b), float(v), int(h), int(d)))
                cases.append(dict(mode=tok[1], H=int(kv["H"]), mask=mask, thr=float(kv["thr"]), cands=recs))
    return values, offsets, cases
