"""Seeded synthetic workloads: check matrices, priors, errors and syndromes."""
from .codes import (CheckMatrix, bivariate_bicycle, surface_hgp, random_34_hgp, synthetic_dem, round_dem,
                    repetition_code, hypergraph_product, gf2_rank, css_logicals)
from .noise import sample, sample_errors, syndromes, logical_failures

__all__ = ["CheckMatrix", "bivariate_bicycle", "surface_hgp", "random_34_hgp", "synthetic_dem", "round_dem",
           "repetition_code", "hypergraph_product", "gf2_rank", "css_logicals",
           "sample", "sample_errors", "syndromes", "logical_failures"]
