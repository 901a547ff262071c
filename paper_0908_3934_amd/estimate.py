"""The inverse problem on the GPU (Sections 1 and 4 of the paper): estimate
which candidate pairs i -> j carry a functional edge from calcium-like
observations of a simulated network.

Argument marshalling around the C-ABI only: the simulation, the
observation, the pair features, the MLP (forward, backward, Adam) and the
simulation-based fit all run in the library's HIP kernels; PyTorch holds
device buffers.

* ``observe``          simulate networks (one ensemble launch) and record
                       fluorescence F = n*cbar + b + gamma*xi per 30 Hz frame.
* ``candidate_pairs``  ordered pairs closer than 150 um and their labels.
* ``features``         64 pair features (``net_features``).
* ``EdgeScorer``       the learned scorer: trained on simulated networks.
* ``auc``              area under the ROC curve (Mann-Whitney, ties 1/2).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _abi
from . import GeonetError, Mlp, Net, NET_OBS_FLUOR, library, _stream_handle, NET_OK

SNR = 5.0
CANDIDATE_RADIUS_UM = 150.0


def observation_gamma(spec, gain: float = 1.0, snr: float = SNR) -> float:
    """Noise level for a given SNR: one spike raises calcium by dt (the
    calcium transition of Section 3.3), observed as gain*dt; gamma is that
    jump divided by the SNR."""
    return gain * spec.dt_ms / snr


def frames_in(n_steps: int, num: int, den: int) -> int:
    """Number of complete frames in steps [0, n_steps)."""
    return (n_steps * num) // den


def candidate_pairs(spec, radius_um: float = CANDIDATE_RADIUS_UM):
    """All ordered pairs (i, j), i != j, with |x_i - x_j| < radius; labels
    mark the pairs that are edges of the network."""
    pos = np.asarray(spec.pos_um, dtype=np.float64)
    d = np.sqrt(((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    i, j = np.nonzero(d < radius_um)
    pairs = np.stack([i, j], 1).astype(np.int32)
    dist = d[i, j].astype(np.float32)
    edge = np.zeros((spec.n, spec.n), dtype=bool)
    edge[spec.src, spec.dst] = True
    return pairs, dist, edge[i, j]


@dataclass
class Observed:
    spec: object
    F: object               # torch float32 [n_frames][n] on the GPU
    pairs: object           # torch int32 [P][2]
    dist: object            # torch float32 [P]
    labels: np.ndarray      # bool [P]
    gain: float
    offset: float
    gamma: float

    @property
    def n_frames(self) -> int:
        return int(self.F.shape[0])


def observe(specs: Sequence, n_steps: int, gain: float = 1.0, offset: float = 0.0,
            gamma: Optional[float] = None, autotune: bool = True) -> List[Observed]:
    """Simulate every network for n_steps (one ensemble launch, its workgroup
    shape timed at build unless autotune is False) and observe it."""
    import torch
    specs = list(specs)
    nf = frames_in(n_steps, specs[0].frame_num, specs[0].frame_den)
    if gamma is None:
        gamma = observation_gamma(specs[0], gain)
    from . import NET_BUILD_AUTOTUNE
    net = Net(specs, frame_capacity=nf, flags=NET_BUILD_AUTOTUNE if autotune and len(specs) > 1 else 0)
    net.step(n_steps)
    F_all = net.observe(NET_OBS_FLUOR, frames=nf, gain=gain, offset=offset, gamma=gamma)
    offs = net.node_offsets()
    out = []
    for k, s in enumerate(specs):
        pairs, dist, labels = candidate_pairs(s)
        out.append(Observed(spec=s, F=F_all[:, offs[k]:offs[k + 1]].contiguous(),
                            pairs=torch.tensor(pairs, device=F_all.device),
                            dist=torch.tensor(dist, device=F_all.device), labels=labels,
                            gain=gain, offset=offset, gamma=gamma))
    torch.cuda.synchronize()
    net.close()
    return out


def obs_desc(o: Observed, keep: list, w_assumed: float = 0.0, w_source=None) -> _abi.ObsDesc:
    s = o.spec
    d = _abi.ObsDesc()
    d.n_nodes = s.n
    d.n_frames = o.n_frames
    d.fluor = o.F.data_ptr()
    d.n_pairs = int(o.pairs.shape[0])
    d.pairs = o.pairs.data_ptr()
    d.pair_dist_um = o.dist.data_ptr()
    d.gain, d.offset, d.gamma = o.gain, o.offset, o.gamma
    d.dt_ms = s.dt_ms
    d.tau_c_ms = s.tau_c_ms
    d.frame_num, d.frame_den = s.frame_num, s.frame_den
    if s.drive_rate_hz is not None:
        rate = np.ascontiguousarray(s.drive_rate_hz, dtype=np.float32)
        keep.append(rate)
        d.drive_rate_hz = rate.ctypes.data
    d.drive_amp = s.drive_amp
    d.control_seed = s.seed
    d.tau_ms, d.v_rest, d.v_reset, d.v_th = s.tau_ms, s.v_rest, s.v_reset, s.v_th
    d.noise_sigma = s.noise_sigma
    d.w_assumed = w_assumed
    d.n_ref = s.n_ref
    if w_source is not None:
        ws = np.ascontiguousarray(w_source, dtype=np.float32)
        if ws.shape != (s.n,):
            raise ValueError("w_source must hold one weight per vertex")
        keep.append(ws)
        d.w_source = ws.ctypes.data
    return d


def source_weights(spec, w0: float, g_inh: float = 1.0):
    """The per-source weights the fit assumes when the cell types are known:
    w0 out of excitatory vertices, -g_inh * w0 out of inhibitory ones."""
    ws = np.full(spec.n, w0, dtype=np.float32)
    if getattr(spec, "inhibitory", None) is not None:
        ws[np.asarray(spec.inhibitory, dtype=bool)] = np.float32(-g_inh * w0)
    return ws


def _echeck(st, where):
    if st != NET_OK:
        raise GeonetError(st, where, library().net_estimate_last_error().decode())


def features(o: Observed, stream=None):
    """64 features per candidate pair (torch float32 [P][64] on the GPU)."""
    import torch
    out = torch.empty((int(o.pairs.shape[0]), 64), dtype=torch.float32, device=o.F.device)
    keep = []
    d = obs_desc(o, keep)
    _echeck(library().net_features(C.byref(d), out.data_ptr(), _stream_handle(stream)), "net_features")
    return out


def simfit(o: Observed, w_assumed: float, realisations: int = 8, sweeps: int = 2, init_fraction: float = 0.3,
           fit_seed: int = 0x5EEDF17, min_gain: float = 1e-3, w_source=None, stream=None):
    """Simulation-based fit scores LL(G + e) - LL(G - e) per candidate pair
    (w_source: optional per-source assumed weights, else w_assumed for all)."""
    import torch
    out = torch.empty(int(o.pairs.shape[0]), dtype=torch.float32, device=o.F.device)
    keep = []
    d = obs_desc(o, keep, w_assumed=w_assumed, w_source=w_source)
    opts = _abi.SimfitOpts(realisations, sweeps, init_fraction, min_gain, fit_seed)
    _echeck(library().net_estimate(C.byref(d), _abi.NET_EST_SIMFIT, None, C.byref(opts), out.data_ptr(),
                                   _stream_handle(stream)), "net_estimate")
    return out


def scorer_scores(o: Observed, scorer: "EdgeScorer", stream=None):
    """Learned scores through the library's single SCORER entry point."""
    import torch
    out = torch.empty(int(o.pairs.shape[0]), dtype=torch.float32, device=o.F.device)
    keep = []
    d = obs_desc(o, keep)
    _echeck(library().net_estimate(C.byref(d), _abi.NET_EST_SCORER, scorer.mlp.h, None, out.data_ptr(),
                                   _stream_handle(stream)), "net_estimate")
    return out


def estimate(o: Observed, scorer: Optional["EdgeScorer"] = None, w_assumed: float = 0.0, w_source=None, stream=None,
             **fit_opts):
    """net_estimate with NET_EST_AUTO: the learned scorer when one is given,
    else the simulation-based fit (fit options as for simfit)."""
    import torch
    out = torch.empty(int(o.pairs.shape[0]), dtype=torch.float32, device=o.F.device)
    keep = []
    d = obs_desc(o, keep, w_assumed=w_assumed, w_source=w_source)
    opts = _abi.SimfitOpts(fit_opts.get("realisations", 8), fit_opts.get("sweeps", 2),
                           fit_opts.get("init_fraction", 0.3), fit_opts.get("min_gain", 1e-3),
                           fit_opts.get("fit_seed", 0x5EEDF17))
    _echeck(library().net_estimate(C.byref(d), _abi.NET_EST_AUTO, scorer.mlp.h if scorer is not None else None,
                                   C.byref(opts), out.data_ptr(), _stream_handle(stream)), "net_estimate")
    return out


def auc(scores, labels) -> float:
    """Mann-Whitney area under the ROC curve, ties counted 1/2."""
    s = np.asarray(scores, dtype=np.float64)
    y = np.asarray(labels).astype(bool)
    n1, n0 = int(y.sum()), int((~y).sum())
    if n1 == 0 or n0 == 0:
        return float("nan")
    order = np.argsort(s, kind="mergesort")
    sv = s[order]
    ranks = np.empty(s.size)
    # average rank of each run of equal scores
    starts = np.r_[0, np.nonzero(np.diff(sv))[0] + 1]
    ends = np.r_[starts[1:], s.size]
    for a, b in zip(starts, ends):
        ranks[order[a:b]] = 0.5 * (a + b - 1) + 1.0
    return float((ranks[y].sum() - n1 * (n1 + 1) / 2.0) / (n1 * n0))


class EdgeScorer:
    """Learned edge scorer: 64 pair features -> MLP 256 -> 256 -> 1 (GPU)."""

    def __init__(self, seed: int = 0):
        self.mlp = Mlp(Mlp.init_params(seed))
        self.seed = seed
        self.history = []
        self.input_norm = None     # (shift, scale) of the features, set by fit

    def fit(self, train: Sequence[Observed], epochs: int = 4, batch: int = 16384, lr: float = 1e-3,
            feats: Optional[list] = None, labels: Optional[list] = None):
        """Standardisation fitted to the training features and `epochs`
        shuffled passes (net_mlp_fit_input_norm, net_mlp_train_epoch: every
        row once per epoch, the last batch of an epoch possibly smaller).
        history holds each epoch's mean batch loss."""
        import torch
        X = torch.cat(feats if feats is not None else [features(o) for o in train])
        lab = labels if labels is not None else [o.labels for o in train]
        y = torch.tensor(np.concatenate(lab).astype(np.float32), device=X.device)
        n = int(X.shape[0])
        if n == 0:
            raise ValueError("EdgeScorer.fit: no training pairs")
        self.mlp.fit_input_norm(X)
        self.input_norm = self.mlp.get_input_norm()
        steps = -(-n // batch)
        losses = torch.zeros(steps, dtype=torch.float32, device=X.device)
        for ep in range(epochs):
            self.mlp.train_epoch(X, y, batch, lr, seed=self.seed, epoch=ep, losses=losses)
            self.history.append(float(losses.cpu().numpy().astype(np.float64).mean()))
        return self

    def score(self, o: Observed, feats=None):
        f = features(o) if feats is None else feats
        return self.mlp.forward(f)
