// Fake binary16 storage type for the CPU test of the library's host code.
#pragma once
struct __half { unsigned short x; };
