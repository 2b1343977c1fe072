"""Geometry and colour decoders (oracle side).

Sec. 3.1: a light MLP f_omega maps the concatenated 16-d grid feature to the
SDF (Eq. SDF_MLP).  As the hot path is specified here, the geometry decoder
is 16 -> 32 -> 32 -> 16 with ReLU hidden layers and a linear output whose
first entry is the SDF phi and whose other 15 entries feed the colour
decoder 15 -> 32 -> 3 (ReLU hidden layer, sigmoid output).  Parameters come
packed in one vector, each matrix row-major [out][in], in the order
W1 b1 W2 b2 W3 b3 U1 c1 U2 c2 v (v sets the rendering sharpness s = exp(10 v)).
"""
import torch

_LAYOUT = [("W1", (32, 16)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)),
           ("W3", (16, 32)), ("b3", (16,)), ("U1", (32, 15)), ("c1", (32,)),
           ("U2", (3, 32)), ("c2", (3,)), ("v", (1,))]


def unpack(vec):
    """Named views into the packed parameter vector (keeps autograd links)."""
    out, off = {}, 0
    for name, shp in _LAYOUT:
        n = 1
        for s in shp:
            n *= s
        out[name] = vec[off:off + n].reshape(shp)
        off += n
    if off != vec.numel():
        raise ValueError(f"packed decoder vector has {vec.numel()} entries, expected {off}")
    return out


def numel():
    return sum(torch.Size(s).numel() for _, s in _LAYOUT)


def geometry(z, P):
    """f_omega: z [..., 16] -> o [..., 16]; phi = o[..., 0], features o[..., 1:]."""
    h1 = torch.relu(z @ P["W1"].T + P["b1"])
    h2 = torch.relu(h1 @ P["W2"].T + P["b2"])
    return h2 @ P["W3"].T + P["b3"]


def colour(g, P):
    """Colour decoder: g [..., 15] -> c [..., 3] in (0, 1)."""
    h = torch.relu(g @ P["U1"].T + P["c1"])
    return torch.sigmoid(h @ P["U2"].T + P["c2"])


def sharpness(P):
    """s = exp(10 v)."""
    return torch.exp(10.0 * P["v"][0])


# ---------------------------------------------------------------- the paper's colour path
# Sec. 3.1, Eq. COLOR_MLP and the architecture details: colour is decoded from
# a separate colour grid W_beta at the finest level (h_c = 6 features per
# vertex) and the viewing direction d, by g_gamma with 2 hidden layers of 32:
# (6 + 3) -> 32 -> 32 -> 3, ReLU hidden, sigmoid output (the output
# activation, unstated, as for the other decoder).  Packed
# V1[32][9] e1[32] V2[32][32] e2[32] V3[3][32] e3[3]; inputs ordered as the
# 6 colour features, then d.
COLOUR_FEAT = 6
_COLOUR_LAYOUT = [("V1", (32, 9)), ("e1", (32,)), ("V2", (32, 32)), ("e2", (32,)), ("V3", (3, 32)), ("e3", (3,))]


def colour_unpack(vec):
    out, off = {}, 0
    for name, shp in _COLOUR_LAYOUT:
        n = shp[0] * (shp[1] if len(shp) > 1 else 1)
        out[name] = vec[off:off + n].reshape(shp)
        off += n
    if off != vec.numel():
        raise ValueError(f"packed colour decoder has {vec.numel()} entries, expected {off}")
    return out


def colour_numel():
    return sum(s[0] * (s[1] if len(s) > 1 else 1) for _, s in _COLOUR_LAYOUT)


def colour_from_grid(cf, d, Pc):
    """g_gamma: colour features cf [..., 6] and viewing directions d [..., 3]
    (unit length) -> colour [..., 3] in (0, 1)."""
    x = torch.cat([cf, d], -1)
    h1 = torch.relu(x @ Pc["V1"].T + Pc["e1"])
    h2 = torch.relu(h1 @ Pc["V2"].T + Pc["e2"])
    return torch.sigmoid(h2 @ Pc["V3"].T + Pc["e3"])
