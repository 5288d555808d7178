"""Loader for the hand-derived closed-form fixtures in this folder.

Each JSON file names the paper passage it exercises ("cite") and the
derivation of its expected values; no expected value here was produced by the
code under test.
"""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name: str) -> dict:
    with open(os.path.join(HERE, name)) as f:
        fx = json.load(f)
    if "vertices" in fx:
        fx["vertices"] = np.asarray(fx["vertices"], np.float32)
    if "rays" in fx:
        fx["rays"] = np.asarray([[np.inf if x == "inf" else x for x in r] for r in fx["rays"]],
                                np.float32)
    if "texcoords" in fx:
        fx["texcoords"] = np.asarray(fx["texcoords"], np.float32)
    if "geom_ids" in fx:
        fx["geom_ids"] = np.asarray(fx["geom_ids"], np.uint32)
    return fx


def uniform_alpha_textures(alphas, size):
    h, w = size
    tex = np.zeros((len(alphas), h, w), np.uint32)
    for i, a in enumerate(alphas):
        tex[i] = (np.uint32(a) << np.uint32(24)) | np.uint32(0x00336699)
    return tex
