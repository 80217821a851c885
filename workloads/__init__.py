"""Seeded synthetic inputs shared by the CPU oracle and the GPU library."""
from .gen import *  # noqa: F401,F403
