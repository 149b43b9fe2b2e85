"""Seeded synthetic input generators (scenes, cameras, rays)."""
from .scenes import *  # noqa: F401,F403
