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
