"""CPU oracle for the 2D toric-code message-passing decoder (arXiv:2506.03266).

TEST INFRASTRUCTURE ONLY: the slow, plain definition the GPU path is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it.  It shares no code with the HIP library in
``paper_2506_03266_amd`` and imports nothing from it.
"""
from .oracle import (  # noqa: F401
    build,
    philox4x32_10,
    noise,
    syndrome_of,
    decode_errors,
    run_steps,
    decode_seeds,
    pack_bits,
    links_from_chains,
    decode_links,
    ring_threshold,
    async_run,
    async_decode_seeds,
    set_reading,
    get_reading,
    decide,
)
