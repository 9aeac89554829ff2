"""Helpers shared by the GPU tests (no oracle arithmetic here)."""
import numpy as np
import torch

from paper_2311_05646_amd import workloads as W

_SCENES = {}


def api():
    from paper_2311_05646_amd import api as A
    return A


def config(name):
    if name.startswith("zoo"):
        dim = int(name[3])
        root = name.split("_")[1]
        return W.make_zoo(dim=dim, root=root)
    return W.CONFIGS[name]()


def scene_for(name, cfg):
    key = (name, id(cfg["scene"]))
    if key not in _SCENES:
        _SCENES.clear()
        _SCENES[key] = api().Scene(cfg["scene"])
    return _SCENES[key]


def fields_c64(cfg):
    return cfg["E"].astype(np.complex64), cfg["A"].astype(np.complex64)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
