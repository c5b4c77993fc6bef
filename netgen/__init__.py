"""Seeded synthetic network descriptions and their generator (input generation only).

This package builds the network description that both the GPU library and the
CPU oracle take as input, and loads the C generator (``libdbnet.so``) for tests
that inspect generated networks. It contains none of the simulation arithmetic.
"""
from .desc import (Pop, Proj, Desc, PopSpec, ProjSpec, NetSpec, RECEPTORS_2, RECEPTORS_4,
                   SRC_ALL, SRC_SAME_REGION, SRC_OTHER_REGIONS, SRC_POP,
                   CLASS_ANY, CLASS_EXC, CLASS_INH, W_UNIFORM, W_LOGNORMAL, W_CONST,
                   D_FIXED, D_UNIFORM, D_DISTANCE, load_generator)
from . import configs

__all__ = ["Pop", "Proj", "Desc", "PopSpec", "ProjSpec", "NetSpec", "configs", "load_generator",
           "RECEPTORS_2", "RECEPTORS_4", "SRC_ALL", "SRC_SAME_REGION", "SRC_OTHER_REGIONS", "SRC_POP",
           "CLASS_ANY", "CLASS_EXC", "CLASS_INH", "W_UNIFORM", "W_LOGNORMAL", "W_CONST",
           "D_FIXED", "D_UNIFORM", "D_DISTANCE"]
