"""Seeded synthetic corpora shared by the oracle-side tests and the GPU-side tests.

This package draws token streams only. It holds none of the similarity method's
arithmetic (no counting, weighting, signing or comparison), so both the oracle
and the HIP path can take their inputs from it without sharing any of the
computation under test.
"""
from .corpus import CONFIGS, Corpus, generate, generate_queries, config_seed  # noqa: F401
