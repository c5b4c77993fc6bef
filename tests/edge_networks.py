"""Degenerate network descriptions for the edge-case tests (oracle pins on the CPU, parity
on the GPU): a network without synapses, a one-neuron network, a network that never
fires, and a network driven so hard that every neuron fires once in every bin (the
longest spike list the method allows, given that a neuron spikes at most once per bin)."""
from netgen import configs
from netgen.desc import NetSpec, PopSpec, RECEPTORS_4


def no_edges(seed: int = 20) -> NetSpec:
    """the 1,000-neuron tiny network with its projection removed: E = 0"""
    s = configs.tiny(seed=seed)
    s.projs = []
    return s


def no_edges_share(seed: int = 21) -> NetSpec:
    """a 20,000-neuron share network (five tiles, the last one ragged) without synapses"""
    s = configs.share(n=20000, indegree=300, seed=seed)
    s.projs = []
    return s


def one_neuron(seed: int = 22) -> NetSpec:
    """N = 1, driven above rheobase (I_ext 600 pA > g_L (V_th - V_L) = 500 pA) plus background"""
    p = PopSpec(1, True, I_ext=600.0, g=configs.SHARE_G, bg_rate_hz=500.0, w_bg=configs.SHARE_W_BG,
                v0_lo=-60.0, v0_hi=-50.0)
    return NetSpec([p], [], seed=seed, receptor_mask=RECEPTORS_4, name="one-neuron")


def silent(seed: int = 23) -> NetSpec:
    """tiny network with no background and every V started near V_L: nothing ever fires"""
    s = configs.tiny(seed=seed, bg_rate_hz=0.0)
    for p in s.pops:
        p.v0_lo, p.v0_hi = -69.0, -68.0
    return s


def saturated(seed: int = 24, n: int = 20000, indegree: int = 100) -> NetSpec:
    """share recipe with a drive no synaptic input can oppose (I_ext = 2e5 pA moves V by
    40 mV per step) and the shortest refractory period allowed (T_ref = bin - dt, r = S - 1):
    every neuron fires once in every bin, so each bin's spike list holds all N neurons"""
    s = configs.share(n=n, indegree=indegree, seed=seed)
    for p in s.pops:
        p.I_ext = 2e5
        p.T_ref = 0.9
    return s
